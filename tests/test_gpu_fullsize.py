"""Parity at full size, in the launch configuration the benchmark times.

The headline workload (2^20 Plummer particles, Salpeter masses, theta 0.4,
n_crit 2048) is integrated host-driven through its start-up span and the
all-particle step at t = 1/512; the next 72 block steps are recorded with
their update rows.  They are then replayed through ht_step_async (update,
prediction and force in one call, as bench.py times them) in both forms, and
every step's outputs are compared with the FP64 oracle on a sample of its
active particles (all of them when there are at most 256): the oracle
predicts the whole j-memory of the replay (the recorded snapshot with every
earlier step's rows applied) and sums each sampled particle's list.  For the
mixed form the oracle is given the mass, acceleration and jerk rounded to
FP32, as the mixed records store them.  Tolerances as elsewhere: FP64
1e-12; mixed acc 2e-6, jerk 1e-5, pot 1e-6 (per particle, relative).
"""
import sys

import numpy as np
import pytest

import bench
from paper_1602_02832_amd import binding as B
from paper_1602_02832_amd import driver
from paper_1602_02832_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-12, 1e-12, 1e-12), "mixed": (2e-6, 1e-5, 1e-6)}
SAMPLE = 256


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(got, want):
    got = np.asarray(got).reshape(len(want), -1)
    want = np.asarray(want).reshape(len(want), -1)
    return float((np.linalg.norm(got - want, axis=1) / np.maximum(np.linalg.norm(want, axis=1), 1e-300)).max())


@pytest.fixture(scope="module")
def window():
    cfg = W.config("plummer1m_salpeter")
    x, v, m = W.make_initial_conditions(cfg)
    say("full size: start-up of the headline workload (host-driven)")
    sim = driver.Simulation(x, v, m, eps2=cfg.eps2, dt_tree=cfg.dt_tree, eta=cfg.eta, theta=cfg.theta,
                            n_crit=cfg.n_crit, n_leaf=cfg.n_leaf, precision="mixed")
    while sim.next_time() < cfg.dt_tree:
        sim.step()
    sim.step()   # all particles active, then the rebuild
    rec = bench.Recorded(sim)
    while len(rec.steps) < 72:
        tn, act = sim.step()
        rec.add(sim, tn, act)
    sim.close()
    sizes = [a.size for _, a, _ in rec.steps]
    say(f"full size: recorded 72 steps, active per step {min(sizes)} .. {max(sizes)}")
    return cfg, rec


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_full_size_window_sampled(oracle, window, prec):
    import torch

    cfg, rec = window
    n = rec.n
    snap = rec.snap
    stream = torch.cuda.Stream()
    ctx = bench.make_ctx(B, snap, n, prec, cfg.eps2, stream.cuda_stream)
    dev_upd = bench.device_updates(torch, rec)
    kmax = max(a.size for _, a, _ in rec.steps)
    acc = torch.empty((kmax, 3), dtype=torch.float64, device="cuda")
    jrk = torch.empty((kmax, 3), dtype=torch.float64, device="cuda")
    pot = torch.empty(kmax, dtype=torch.float64, device="cuda")
    # the oracle's mirror of the j-memory
    t0, m, x, v, a, j = (snap[k].copy() for k in ("t0", "m", "x", "v", "a", "j"))
    nm, nx, nv, na, nj = (u.copy() for u in snap["node"])
    gf, lo, en = snap["lists"]
    f32 = (lambda u: u.astype(np.float32).astype(np.float64)) if prec == "mixed" else (lambda u: u)
    rng = np.random.default_rng(17)
    ta, tj, tp = TOL[prec]
    worst = [0.0, 0.0, 0.0]
    for k, (t, act, upd) in enumerate(rec.steps):
        prev = None if k == 0 else (dev_upd[k - 1][0].shape[0],) + tuple(u.data_ptr() for u in dev_upd[k - 1])
        ctx.step_async(prev, t, act, acc, jrk, pot)
        torch.cuda.synchronize()
        if k > 0:   # apply the previous step's rows to the mirror, as the device did
            idx, u_t0, u_m, u_x, u_v, u_a, u_j = rec.steps[k - 1][2]
            t0[idx], m[idx], x[idx], v[idx], a[idx], j[idx] = u_t0, u_m, u_x, u_v, u_a, u_j
        pick = np.arange(act.size) if act.size <= SAMPLE else np.sort(rng.choice(act.size, SAMPLE, replace=False))
        xp, vp = oracle.predict(t, t0, x, v, f32(a), f32(j))
        nxp, nvp = oracle.predict(t, np.full(nm.shape[0], snap["t_tree"]), nx, nv, f32(na), f32(nj))
        wa, wj, wp = oracle.force_list(act[pick], np.vstack([xp, nxp]), np.vstack([vp, nvp]),
                                       f32(np.concatenate([m, nm])), cfg.eps2, gf, lo, en)
        got = [u[:act.size].cpu().numpy()[pick] for u in (acc, jrk, pot)]
        e = (rel(got[0], wa), rel(got[1], wj), rel(got[2], wp))
        worst = [max(p, q) for p, q in zip(worst, e)]
        assert e[0] <= ta and e[1] <= tj and e[2] <= tp, \
            f"{prec} step {k} ({act.size} active): acc {e[0]:.3g} jerk {e[1]:.3g} pot {e[2]:.3g}"
    ctx.close()
    say(f"full size {prec}: 72 steps, worst acc {worst[0]:.3g} jerk {worst[1]:.3g} pot {worst[2]:.3g}")
