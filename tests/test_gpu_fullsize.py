"""Parity at full size, in the launch configuration the benchmark times.

The headline workload (2^20 Plummer particles, Salpeter masses, theta 0.4,
n_crit 2048) is integrated host-driven through its start-up span; the state
before the all-particle step at t = 1/512 is kept, then that step and the
rebuild there are taken and the next 72 block steps are recorded with their
update rows.

  * The 72 steps are replayed through ht_step_async (update, prediction and
    force in one call, as bench.py times them) in both forms, and every
    step's outputs are compared with the FP64 oracle on a sample of its active
    particles (all of them when there are at most 256): the oracle predicts
    the whole j-memory of the replay (the recorded snapshot with every earlier
    step's rows applied) and sums each sampled particle's list.  The gate is
    the unrounded FP64 j-memory, so the mixed form's own storage rounding (a,
    jerk and Salpeter masses in FP32) counts against it; the error against
    the FP32-rounded inputs is reported beside it.
  * The all-particle step at t = 1/512 (every particle active, the largest
    launch) is run as the benchmark runs it and sampled the same way.
  * The direct N^2 sum, the baseline of the speed-up, is run on the same
    replay (j-memory updates, prediction, force over all N particles) and
    compared with the oracle's direct sum on sampled active particles of
    two window steps.

Tolerances as elsewhere: FP64 1e-12; mixed acc 2e-6, jerk 1e-5, pot 1e-6
(per particle, relative).
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
    rec_all = bench.Recorded(sim)     # the state before the all-particle step
    t_all = sim.next_time()
    sim.step()   # all particles active, then the rebuild
    rec = bench.Recorded(sim)
    while len(rec.steps) < 72:
        tn, act = sim.step()
        rec.add(sim, tn, act)
    sim.close()
    sizes = [a.size for _, a, _ in rec.steps]
    say(f"full size: recorded 72 steps, active per step {min(sizes)} .. {max(sizes)}")
    return cfg, rec, rec_all, t_all


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_full_size_window_sampled(oracle, window, prec):
    import torch

    cfg, rec, _, _ = window
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
    worst_rounded = [0.0, 0.0, 0.0]
    for k, (t, act, upd) in enumerate(rec.steps):
        prev = None if k == 0 else (dev_upd[k - 1][0].shape[0],) + tuple(u.data_ptr() for u in dev_upd[k - 1])
        ctx.step_async(prev, t, act, acc, jrk, pot)
        torch.cuda.synchronize()
        if k > 0:   # apply the previous step's rows to the mirror, as the device did
            idx, u_t0, u_m, u_x, u_v, u_a, u_j = rec.steps[k - 1][2]
            t0[idx], m[idx], x[idx], v[idx], a[idx], j[idx] = u_t0, u_m, u_x, u_v, u_a, u_j
        pick = np.arange(act.size) if act.size <= SAMPLE else np.sort(rng.choice(act.size, SAMPLE, replace=False))
        got = [u[:act.size].cpu().numpy()[pick] for u in (acc, jrk, pot)]
        for rounded in ((False, True) if prec == "mixed" else (False,)):
            r = f32 if rounded else (lambda u: u)
            xp, vp = oracle.predict(t, t0, x, v, r(a), r(j))
            nxp, nvp = oracle.predict(t, np.full(nm.shape[0], snap["t_tree"]), nx, nv, r(na), r(nj))
            wa, wj, wp = oracle.force_list(act[pick], np.vstack([xp, nxp]), np.vstack([vp, nvp]),
                                           r(np.concatenate([m, nm])), cfg.eps2, gf, lo, en)
            e = (rel(got[0], wa), rel(got[1], wj), rel(got[2], wp))
            if rounded:      # diagnostic only: the inputs as the mixed records store them
                worst_rounded = [max(p, q) for p, q in zip(worst_rounded, e)]
                continue
            worst = [max(p, q) for p, q in zip(worst, e)]
            assert e[0] <= ta and e[1] <= tj and e[2] <= tp, \
                f"{prec} step {k} ({act.size} active): acc {e[0]:.3g} jerk {e[1]:.3g} pot {e[2]:.3g}"
    ctx.close()
    say(f"full size {prec}: 72 steps, worst against the FP64 j-memory acc {worst[0]:.3g} jerk {worst[1]:.3g} "
        f"pot {worst[2]:.3g}; against FP32-rounded a, jerk, m: acc {worst_rounded[0]:.3g} "
        f"jerk {worst_rounded[1]:.3g} pot {worst_rounded[2]:.3g}")


def sampled(rng, n):
    return np.arange(n) if n <= SAMPLE else np.sort(rng.choice(n, SAMPLE, replace=False))


def test_full_size_all_particle_step_sampled(oracle, window):
    """The largest launch: every one of the 2^20 particles active at
    t = 1/512, run as the benchmark runs it (ht_force_async over all ids)."""
    import torch

    cfg, _, rec_all, t_all = window
    snap, n = rec_all.snap, rec_all.n
    stream = torch.cuda.Stream()
    ctx = bench.make_ctx(B, snap, n, "mixed", cfg.eps2, stream.cuda_stream)
    ids = np.arange(n, dtype=np.int32)
    acc = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    jrk = torch.empty_like(acc)
    pot = torch.empty(n, dtype=torch.float64, device="cuda")
    ctx.predict(t_all)
    ctx.force_async(ids, acc, jrk, pot)
    ctx.sync()
    pick = sampled(np.random.default_rng(23), n)
    nm, nx, nv, na, nj = snap["node"]
    xp, vp = oracle.predict(t_all, snap["t0"], snap["x"], snap["v"], snap["a"], snap["j"])
    nxp, nvp = oracle.predict(t_all, np.full(nm.shape[0], snap["t_tree"]), nx, nv, na, nj)
    gf, lo, en = snap["lists"]
    want = oracle.force_list(ids[pick], np.vstack([xp, nxp]), np.vstack([vp, nvp]), np.concatenate([snap["m"], nm]),
                             cfg.eps2, gf, lo, en)
    got = [u.cpu().numpy()[pick] for u in (acc, jrk, pot)]
    e = [rel(g, w) for g, w in zip(got, want)]
    ctx.close()
    say(f"full size all-particle step: {n} active, sampled {pick.size}: acc {e[0]:.3g} jerk {e[1]:.3g} pot {e[2]:.3g}")
    ta, tj, tp = TOL["mixed"]
    assert e[0] <= ta and e[1] <= tj and e[2] <= tp


def test_full_size_direct_sampled(oracle, window):
    """The direct N^2 sum at full size on the replayed window (the benchmark's
    direct leg: j-memory update, prediction, force over all N particles),
    checked on sampled active particles of the window's largest step and of
    a small one against the oracle's direct sum over all 2^20 particles."""
    import torch

    cfg, rec, _, _ = window
    snap, n = rec.snap, rec.n
    stream = torch.cuda.Stream()
    ctx = bench.make_ctx(B, snap, n, "mixed", cfg.eps2, stream.cuda_stream)
    dev_upd = bench.device_updates(torch, rec)
    kmax = max(a.size for _, a, _ in rec.steps)
    acc = torch.empty((kmax, 3), dtype=torch.float64, device="cuda")
    jrk = torch.empty((kmax, 3), dtype=torch.float64, device="cuda")
    pot = torch.empty(kmax, dtype=torch.float64, device="cuda")
    sizes = np.array([a.size for _, a, _ in rec.steps])
    big = int(np.argmax(sizes))
    small = int(np.flatnonzero(sizes == np.sort(sizes)[len(sizes) // 4])[0])
    t0, m, x, v, a, j = (snap[k].copy() for k in ("t0", "m", "x", "v", "a", "j"))
    rng = np.random.default_rng(29)
    ta, tj, tp = TOL["mixed"]
    checked = 0
    for k, (t, act, upd) in enumerate(rec.steps[:max(big, small) + 1]):
        if k > 0:
            ctx.set_j_particles_async(*((dev_upd[k - 1][0].shape[0],) + tuple(u.data_ptr() for u in dev_upd[k - 1])))
            idx, u_t0, u_m, u_x, u_v, u_a, u_j = rec.steps[k - 1][2]
            t0[idx], m[idx], x[idx], v[idx], a[idx], j[idx] = u_t0, u_m, u_x, u_v, u_a, u_j
        ctx.predict(t)
        ctx.force_direct_async(act, acc, jrk, pot)
        ctx.sync()
        if k not in (big, small):
            continue
        pick = sampled(rng, act.size)
        xp, vp = oracle.predict(t, t0, x, v, a, j)
        want = oracle.force_direct(act[pick], xp, vp, m, cfg.eps2)
        got = [u[:act.size].cpu().numpy()[pick] for u in (acc, jrk, pot)]
        e = [rel(g, w) for g, w in zip(got, want)]
        say(f"full size direct, step {k} ({act.size} active, sampled {pick.size}): acc {e[0]:.3g} "
            f"jerk {e[1]:.3g} pot {e[2]:.3g}")
        assert e[0] <= ta and e[1] <= tj and e[2] <= tp
        checked += 1
    ctx.close()
    assert checked == 2
