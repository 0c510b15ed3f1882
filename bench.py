#!/usr/bin/env python3
"""Block-step throughput of the tree/Hermite force evaluation on one MI355X.

Workload (default "plummer1m_salpeter"): Plummer model of N = 2^20 particles
with a Salpeter mass spectrum (m_max/m_min = 100, total mass 1), theta = 0.4,
eps = 4/N, tree interval 1/512, Aarseth eta = 0.01, n_crit = 2048, mixed
precision, fused prediction.  The run integrates through t = 1/512 (start-up,
including the all-particle step and the tree rebuild there), records the next
W + K block steps, then replays them from the same device state with inputs
resident in HBM:

  step k = j-memory update with the particles corrected at step k-1
           -> predict(t_k) -> force on the active set of step k

W steps warm up; K steps are timed twice from the same snapshot: once with
HIP events on the library's stream before every step (step latency) and
around every force launch (kernel time), and once with nothing but the steps
between two synchronisations, whose wall clock gives the throughput.  The
same K steps are then run with the direct N^2 sum (the original Hermite
scheme) and with the FP64 form.  The all-particle step at t = 1/512 is timed
separately.

One JSON line on stdout; progress on stderr.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FLOPS_PER_PAIR = 57          # Section 3 convention for force + jerk
# MI355X's published FP32 vector peak (packed FP32 dual issue): the roofline's peak
PEAK_FP32_TFLOPS = 157.3
# 256 CU x 64 FMA lanes x 2 flop x 2.4 GHz: the non-packed FP32 (and FP64) issue
# rate, which bounds these kernels (they issue no packed FP32), reported beside it
PEAK_NONPACKED_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0          # MI355X HBM3E, published
METRIC = "Hermite acc+jerk interactions/s at N=2^20 vs direct; p99 block-step latency"
METRIC_ENSEMBLE = "batched ensemble (64 Plummer clusters, N 4096-65536): Hermite acc+jerk interactions/s; p99 engine-step latency"
# HBM traffic of the timed force kernel, from two rocprofv3 --pmc passes over
# one window of this benchmark (FETCH_SIZE, then WRITE_SIZE, KiB summed over
# the L2 channels, mean over the timed launches), each divided by what the
# same counter reads per byte for a plain device copy (--calibrate-copy).  Valid
# only for the kernel source and the window (steps, warmup) it was taken on:
# anything else makes the figure null until the counters are taken again.
TRAFFIC = {
    "kernel_source_sha256": "f75cb0057275a324bd018934f3e91a513de77c7cec83f517ee5f0b78d63e4abc",
    "steps": 20,
    "warmup": 5,
    "fetch_bytes_per_launch": 1.16099e8,   # FETCH_SIZE 56689.2 KiB x 2.000
    "write_bytes_per_launch": 2.5291e5,    # WRITE_SIZE 247.0 KiB x 1.000
    "fetch_scale": 2.000,                  # 1 GiB read by a plain copy reads 524294.5 KiB
    "write_scale": 1.000,                  # 1 GiB written reads 1048576 KiB
    "profile": "profiles/force_kernel_mixed_plummer1m_traffic.md",
}
# Bytes the force evaluation needs at least, per launch: every distinct
# j-entry of the active groups' lists once (the mixed record's payload: x, y,
# z, t0, vx, vy, vz in FP64, m, a, jerk in FP32), each active group's list
# indices once, and per active particle its id and outputs (acc, jerk, pot).
REC_PAYLOAD_BYTES = 7 * 8 + 7 * 4
OUT_BYTES = 7 * 8
METRIC_SERVED = "served stream of cluster runs (N 1024-262144, 256 block steps each): p50/p99 engine-step latency at 80% load"


def kernel_source_sha256():
    path = os.path.join(ROOT, "paper_1602_02832_amd", "csrc", "htree.hip")
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(steps, warmup):
    """HBM bytes per launch of the timed kernel, or None when not measured on
    the kernel source as it stands and on this window."""
    if TRAFFIC["kernel_source_sha256"] != kernel_source_sha256() or TRAFFIC["fetch_bytes_per_launch"] is None:
        return None
    if (TRAFFIC["steps"], TRAFFIC["warmup"]) != (steps, warmup):
        return None
    return TRAFFIC["fetch_bytes_per_launch"] + TRAFFIC["write_bytes_per_launch"]


def calibrate_copy(torch, mib):
    """A plain device copy of known size for scaling the L2 byte counters:
    torch.neg reads mib MiB and writes mib MiB in one elementwise kernel."""
    n = (mib << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    log(f"copy calibration: 3 launches, each reading and writing {mib} MiB")


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


class Recorded:
    """Block steps recorded from a tree/Hermite run, ready for replay."""

    def __init__(self, sim):
        self.n = sim.n
        self.snap = self._snapshot(sim)
        self.steps = []   # (t, active, update tuple of host arrays)

    @staticmethod
    def _snapshot(sim):
        tr = sim.tree
        return dict(t0=sim.t0.copy(), m=sim.m.copy(), x=sim.x.copy(), v=sim.v.copy(), a=sim.a.copy(),
                    j=sim.j.copy(), t_tree=sim.t_tree, node=(tr.node_m, tr.node_x, tr.node_v, tr.node_a, tr.node_j),
                    lists=(tr.group_first, tr.list_off, tr.entries), n_node=tr.n_node, n_group=tr.n_group,
                    n_entries=tr.n_entries)

    def add(self, sim, t, act):
        upd = (act.astype(np.int32), sim.t0[act].copy(), sim.m[act].copy(), sim.x[act].copy(), sim.v[act].copy(),
               sim.a[act].copy(), sim.j[act].copy())
        self.steps.append((t, act.astype(np.int32), upd))


def make_ctx(B, snap, n, precision, eps2, stream, predict_mode="fused", lists="csr", placement=None,
             union_width=None, tuning=None):
    ctx = B.Context(n_max=n, node_max=snap["n_node"] + 64, group_max=snap["n_group"] + 16,
                    list_max=snap["n_entries"] + 1024, active_max=n, eps2=eps2, precision=precision,
                    predict_mode=predict_mode, stream=stream)
    if lists != "csr":
        ctx.set_list_form(lists)
    if union_width is not None:
        ctx.set_union_width(union_width)
    if tuning is not None:
        ctx.set_tuning(*tuning)
    if placement is not None:
        ctx.set_placement(placement)
    load_snapshot(ctx, snap)
    return ctx


def load_snapshot(ctx, snap):
    ctx.set_j_particles(snap["t0"], snap["m"], snap["x"], snap["v"], snap["a"], snap["j"])
    ctx.set_nodes(snap["t_tree"], *snap["node"])
    ctx.set_interaction_lists(*snap["lists"])


def device_updates(torch, rec):
    out = []
    for _, _, upd in rec.steps:
        out.append(tuple(torch.from_numpy(np.ascontiguousarray(u)).cuda() for u in upd))
    return out


def replay(torch, B, rec, ctx, stream, warmup, steps, direct=False, mode="clean", graph=False):
    """Replay recorded steps; returns a timing dict for the last `steps` steps.

    mode "clean": nothing but the steps between the two synchronisations (the
    throughput figure).  "latency": one HIP event on the stream before every
    step, nothing else (step latency).  "kernel": HIP events around every
    force launch (kernel time and launches), the per-step pairs and work
    items, and the host time of each step call.  Addresses of the recorded
    arrays (update rows on the device, active ids on the host) are taken
    before the timed loop, as a driver that keeps them resident would."""
    dev_upd = device_updates(torch, rec)
    kmax = max(a.size for _, a, _ in rec.steps)
    acc = torch.empty((kmax, 3), dtype=torch.float64, device="cuda")
    jrk = torch.empty((kmax, 3), dtype=torch.float64, device="cuda")
    pot = torch.empty(kmax, dtype=torch.float64, device="cuda")
    out_ptrs = (acc.data_ptr(), jrk.data_ptr(), pot.data_ptr())
    upd_ptrs = [None] + [(u[0].shape[0],) + tuple(x.data_ptr() for x in u) for u in dev_upd[:-1]]
    act_ptrs = [(a.size, a.ctypes.data) for _, a, _ in rec.steps]
    times = [t for t, _, _ in rec.steps]

    def run_step(k):
        if direct:
            upd = upd_ptrs[k]
            if upd is not None:
                ctx.set_j_particles_async(*upd)
            ctx.predict(times[k])
            ctx.force_direct_async(rec.steps[k][1], *out_ptrs)
        elif graph:
            ctx.step_graph(upd_ptrs[k], times[k], rec.steps[k][1], *out_ptrs)
        else:
            ctx.step_async(upd_ptrs[k], times[k], act_ptrs[k], *out_ptrs)

    for k in range(warmup):
        run_step(k)
    torch.cuda.synchronize()
    if mode == "clean":
        t_wall = time.perf_counter()
        for k in range(warmup, warmup + steps):
            run_step(k)
        torch.cuda.synchronize()
        return dict(wall_s=time.perf_counter() - t_wall)
    if mode == "latency":
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        t_wall = time.perf_counter()
        for q, k in enumerate(range(warmup, warmup + steps)):
            evs[q].record(stream)
            run_step(k)
        evs[steps].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_wall
        return dict(wall_s=wall, lat_ms=np.array([evs[q].elapsed_time(evs[q + 1]) for q in range(steps)]))
    ctx.set_timing(True)
    pairs = 0
    per_step = []
    t_wall = time.perf_counter()
    for k in range(warmup, warmup + steps):
        th = time.perf_counter()
        run_step(k)
        th = time.perf_counter() - th
        p, w = ctx.last_stats()
        pairs += p
        per_step.append((int(rec.steps[k][1].size), int(p), int(w), 1e6 * th))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    kms, launches, kpairs = ctx.kernel_timing()
    ctx.set_timing(False)
    return dict(wall_s=wall, pairs=pairs, kernel_ms=kms, launches=launches, kernel_pairs=kpairs, per_step=per_step)


def algorithmic_bytes(rec, warmup):
    """Mean over the timed steps of the minimal bytes one force launch moves."""
    gf, lo, entries = rec.snap["lists"]
    n_j = rec.n + rec.snap["n_node"]
    mark = np.zeros(n_j, bool)
    total = 0.0
    for _, act, _ in rec.steps[warmup:]:
        groups = np.unique(np.searchsorted(gf, act, side="right") - 1)
        mark[:] = False
        n_idx = 0
        for g in groups:
            mark[entries[lo[g]:lo[g + 1]]] = True
            n_idx += int(lo[g + 1] - lo[g])
        total += int(mark.sum()) * REC_PAYLOAD_BYTES + 4 * n_idx + act.size * (4 + OUT_BYTES)
    return total / max(len(rec.steps) - warmup, 1)


def tile_mix(rec, warmup):
    """Per recorded step: pairs by i-tile size T (active particles of a group
    in tiles of up to 256, T the next power of two)."""
    gf, lo = rec.snap["lists"][0], rec.snap["lists"][1]
    out = []
    for _, act, _ in rec.steps[warmup:]:
        g = np.searchsorted(gf, act, side="right") - 1
        ug, cnt = np.unique(g, return_counts=True)
        mix = {}
        for gg, c in zip(ug, cnt):
            ln = int(lo[gg + 1] - lo[gg])
            for t0 in range(0, int(c), 256):
                ni = min(256, int(c) - t0)
                T = 1 << (ni - 1).bit_length()
                mix[T] = mix.get(T, 0) + ni * ln
        out.append({str(k): v for k, v in sorted(mix.items())})
    return out


def bench_tree_build(torch, B, x, v, m, cfg, reps=5):
    """Step 1 (keys, order, tree, node moments, groups, lists) on the device
    and with the host builder, from the same particles (a and jerk drawn at
    random: the cost does not depend on their values)."""
    rng = np.random.default_rng(6)
    a, j = rng.standard_normal((2, len(m), 3))
    dev = [torch.from_numpy(np.ascontiguousarray(u)).cuda() for u in (x, v, a, j, m)]
    tree = B.DeviceTree(n_max=len(m))
    tree.build(*dev, cfg.n_leaf, cfg.n_crit, cfg.theta)      # warm-up (allocations)
    walls, phases = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tree.build(*dev, cfg.n_leaf, cfg.n_crit, cfg.theta)
        walls.append(1e3 * (time.perf_counter() - t0))
        phases.append(tree.phase_ms())
    M, G, E, C = tree.sizes()
    tree.close()
    t0 = time.perf_counter()
    B.HostTree(x, v, a, j, m, cfg.n_leaf, cfg.n_crit, cfg.theta)
    host_ms = 1e3 * (time.perf_counter() - t0)
    k = int(np.argsort(walls)[len(walls) // 2])
    return {"n": int(len(m)), "nodes": M, "groups": G, "list_entries": E, "device_ms": walls[k],
            "device_phases_ms": {p: round(q, 3) for p, q in phases[k].items()}, "host_builder_ms": host_ms,
            "host_threads": os.cpu_count(), "speedup": host_ms / walls[k]}


def cpu_baseline(W, cfg, rec, warmup, seconds):
    """The oracle (FP64, OpenMP over active particles), built for this host's
    instruction set, on the timed window itself: the recorded snapshot, every
    step's update rows applied in turn, and at every timed step the oracle's
    prediction of the whole j-memory and its list force on the step's active
    set.  The window is replayed until about `seconds` have been spent."""
    from oracle import oracle as O

    from paper_1602_02832_amd import binding as B

    O.use_native_build()
    snap = rec.snap
    gf, lo, en = snap["lists"]
    nm, nx, nv, na, nj = snap["node"]
    t_node = np.full(nm.shape[0], snap["t_tree"])
    spent, done_pairs, done_steps, passes = 0.0, 0, 0, 0
    while spent < seconds and passes < 64:
        t0, m, x, v, a, j = (snap[k].copy() for k in ("t0", "m", "x", "v", "a", "j"))
        for k, (t, act, _) in enumerate(rec.steps):
            if k > 0:
                idx, u_t0, u_m, u_x, u_v, u_a, u_j = rec.steps[k - 1][2]
                t0[idx], m[idx], x[idx], v[idx], a[idx], j[idx] = u_t0, u_m, u_x, u_v, u_a, u_j
            if k < warmup:
                continue
            tw = time.perf_counter()
            xp, vp = O.predict(t, t0, x, v, a, j)
            nxp, nvp = O.predict(t, t_node, nx, nv, na, nj)
            O.force_list(act, np.vstack([xp, nxp]), np.vstack([vp, nvp]), np.concatenate([m, nm]), cfg.eps2, gf, lo,
                         en)
            spent += time.perf_counter() - tw
            g = np.searchsorted(gf, act, side="right") - 1
            done_pairs += int((lo[g + 1] - lo[g]).sum())
            done_steps += 1
        passes += 1
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    base = dict(value=done_pairs / spent, unit="interactions/s", cores=threads, kind="oracle",
                sample=f"the timed window's {len(rec.steps) - warmup} block steps replayed {passes} times "
                       f"({done_steps} steps: prediction of all {rec.n + nm.shape[0]} j-entries and the list force "
                       f"on each step's active set; {done_pairs:.3g} pairs, {spent:.1f} s)",
                build=O.build_flags(native=True))
    # the direct sum on a random sample of 1024 particles against all N, and the tree builds
    x, v, m = W.make_initial_conditions(cfg)
    z = np.zeros_like(x)
    t = time.perf_counter()
    tr = O.Tree(x, v, z, z, m, cfg.n_leaf, cfg.n_crit, cfg.theta)
    t_oracle_tree = time.perf_counter() - t
    t = time.perf_counter()
    B.HostTree(x, v, z, z, m, cfg.n_leaf, cfg.n_crit, cfg.theta)
    t_product_tree = time.perf_counter() - t
    xs, vs, ms = x[tr.perm], v[tr.perm], m[tr.perm]
    rng = np.random.default_rng(99)
    ids = np.sort(rng.choice(cfg.n, 1024, replace=False)).astype(np.int32)
    t = time.perf_counter()
    O.force_direct(ids, xs, vs, ms, cfg.eps2)
    t_direct = time.perf_counter() - t
    extra = dict(direct_interactions_per_s=1024 * (cfg.n - 1) / t_direct,
                 direct_sample=f"direct sum on 1024 random particles against all {cfg.n} ({t_direct:.2f} s)",
                 tree_build_s={"oracle": t_oracle_tree, "product_host_builder": t_product_tree},
                 cores=threads)
    return base, extra


def parse_tuning(text):
    """'gather_cost,target_items' -> (float, float)."""
    gc, ti = (float(u) for u in text.split(","))
    return gc, ti


def engine_device_tree(args):
    return not args.host_engine and not args.host_rebuild


def engine_name(args):
    if args.host_engine:
        return "host-driven"
    return "resident, host rebuilds" if args.host_rebuild else "resident, device rebuilds"


def bench_ensemble(args, torch):
    """64 independent clusters advanced together, one batched launch per engine step."""
    from paper_1602_02832_amd import engine as E
    from paper_1602_02832_amd import workloads as W

    sizes = W.ensemble_sizes(64, 5, 4096, 65536)
    specs = [E.RunSpec(key=k, n=int(n), seed=1000 + k, steps=10**9, theta=0.5, eta=0.01, dt_tree=1.0 / 256,
                       n_crit=256) for k, n in enumerate(sizes)]
    total_n = int(sizes.sum())
    eng = E.Engine(precision="mixed", max_clusters=64, max_active=total_n, max_items=1 << 20, max_rows=total_n,
                   resident=not args.host_engine, device_tree=engine_device_tree(args),
                   tree_n_max=int(sizes.max()), lanes=args.lanes or None, device_loop=args.device_loop)
    t0 = time.perf_counter()
    for sp in specs:
        eng.add(eng.new_cluster(sp))
    log(f"ensemble: 64 clusters, {total_n} particles, set up in {time.perf_counter() - t0:.1f} s")
    # plan tuning chosen on the clusters themselves (untimed; the clusters advance), unless given
    if args.tuning:
        tuning, scores = parse_tuning(args.tuning), {}
        eng.set_tuning(*tuning)
    else:
        tuning, scores = eng.autotune()
    log(f"ensemble: autotuned (gather_cost, target_items) = {tuning}; ms per 1e9 interactions "
        f"{ {str(k): round(v, 3) for k, v in scores.items()} }")
    def engine_steps(count):
        # a device-loop call takes up to loop_steps engine steps; the last call is cut to the count
        e0 = eng.engine_steps
        while eng.engine_steps - e0 < count:
            if eng.device_loop:
                eng.loop_steps = min(32, count - (eng.engine_steps - e0))
            eng.step()
        return eng.engine_steps - e0

    engine_steps(args.warmup)
    eng.step_ms.clear()
    eng.pairs = eng.equiv_pairs = 0
    eng.wall = 0.0
    eng.phase = {k: 0.0 for k in eng.phase}
    eng.subphase.clear()
    eng.set_timing(True)
    torch.cuda.synchronize()
    tw = time.perf_counter()
    n_steps = engine_steps(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - tw
    kms, nl, kp = eng.kernel_timing()
    lat = np.array(eng.step_ms)
    value = eng.pairs / wall
    # force launches inside the device loop's graphs carry no events: no kernel time there
    achieved = FLOPS_PER_PAIR * kp / (kms * 1e-3) / 1e12 if nl else None
    log(f"ensemble: {value:.4g} pairs/s, {1e3 * wall / n_steps:.3f} ms/engine step over {n_steps} engine steps, "
        f"phases {eng.phase}")
    res = {
        "metric": METRIC_ENSEMBLE, "value": value, "unit": "interactions/s", "n_gpus": 1, "steps": n_steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * wall / n_steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": "ensemble64", "clusters": 64, "n_range": [4096, 65536], "n_total": total_n,
                   "engine": engine_name(args), "lanes": eng.n_lanes, "device_loop": eng.device_loop,
                   "theta": 0.5, "eps": "4/N", "dt_tree": 1.0 / 256, "eta": 0.01, "n_crit": 256, "precision": "mixed"},
        "p50_step_ms": float(np.percentile(lat, 50)), "p99_step_ms": float(np.percentile(lat, 99)),
        "equivalent_interactions_per_s": eng.equiv_pairs / wall,
        "phase_s": eng.phase, "host_subphase_s": dict(eng.subphase),
        "autotuned": {"gather_cost": tuning[0], "target_items": tuning[1],
                      "engine_ms_per_1e9_interactions": {str(k): v for k, v in scores.items()}},
        "roofline": None if achieved is None else {
            "bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS, "peak_nonpacked": PEAK_NONPACKED_TFLOPS,
            "frac_nonpacked": achieved / PEAK_NONPACKED_TFLOPS, "traffic": None,
            "kernel": "force_kernel<PrecMixed,false,false,false>", "avg_launch_ms": kms / max(nl, 1)},
    }
    eng.close()
    return res


def bench_served(args, torch):
    """Continuous batching of cluster runs: capacity first, then Poisson arrivals at 80% of it."""
    from paper_1602_02832_amd import engine as E
    from paper_1602_02832_amd import workloads as W

    n_req = args.requests
    sizes = W.ensemble_sizes(n_req, 8, 1024, 262144)
    specs = [E.RunSpec(key=r, n=int(sizes[r]), seed=2000 + r, steps=256, theta=0.5, eta=0.01, dt_tree=1.0 / 256,
                       n_crit=256) for r in range(n_req)]
    budget = int(args.hbm_gb * 2**30)
    cap_active = 1 << 23

    def serve(reqs):
        eng = E.Engine(precision="mixed", max_clusters=args.max_resident, max_active=cap_active, max_items=1 << 20,
                       max_rows=cap_active, resident=not args.host_engine, device_tree=engine_device_tree(args),
                       tree_n_max=int(sizes.max()), lanes=args.lanes or None)
        if args.tuning:
            eng.set_tuning(*parse_tuning(args.tuning))
        srv = E.Server(eng, hbm_budget=budget, max_resident=args.max_resident)
        t = time.perf_counter()
        done = srv.run(reqs)
        span = time.perf_counter() - t
        out = dict(span=span, done=done, step_ms=list(eng.step_ms), pairs=eng.pairs, phase=dict(eng.phase),
                   max_used=srv.max_used, max_waiting=srv.max_waiting, lanes=eng.n_lanes,
                   refused=len(srv.refused))
        srv.close()
        eng.close()
        return out

    n_cap = min(n_req, 2 * args.max_resident)
    cap_run = serve([E.Request(spec=specs[r], arrival=0.0) for r in range(n_cap)])
    capacity = n_cap / cap_run["span"]
    log(f"served: capacity {capacity:.3g} runs/s (closed loop, {n_cap} runs in {cap_run['span']:.1f} s)")
    rate = 0.8 * capacity
    arr = E.poisson_arrivals(n_req, rate, 7)
    run = serve([E.Request(spec=specs[r], arrival=float(arr[r])) for r in range(n_req)])
    done = run["done"]
    lat = np.array(run["step_ms"])
    resp = np.array([r.finished - r.arrival for r in done])
    queue = np.array([r.admitted - r.arrival for r in done])
    log(f"served: {len(done)} runs in {run['span']:.1f} s; engine step p50 {np.percentile(lat, 50):.2f} ms "
        f"p99 {np.percentile(lat, 99):.2f} ms; phases {run['phase']}")
    res = {
        "metric": METRIC_SERVED, "value": float(np.percentile(lat, 99)), "unit": "ms", "n_gpus": 1,
        "steps": len(lat), "warmup": 0, "ms_per_step": float(lat.mean()), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": "served", "requests": n_req, "n_range": [1024, 262144], "block_steps_per_run": 256,
                   "theta": 0.5, "eps": "4/N", "dt_tree": 1.0 / 256, "eta": 0.01, "n_crit": 256,
                   "arrival_rate_per_s": rate, "load": 0.8, "max_resident": args.max_resident,
                   "hbm_budget_gb": args.hbm_gb, "precision": "mixed",
                   "engine": engine_name(args), "lanes": run["lanes"],
                   "tuning": list(parse_tuning(args.tuning)) if args.tuning else "library default"},
        "p50_step_ms": float(np.percentile(lat, 50)), "p99_step_ms": float(np.percentile(lat, 99)),
        "capacity_runs_per_s": capacity, "throughput_runs_per_s": len(done) / run["span"],
        "interactions_per_s": run["pairs"] / run["span"],
        "request_latency_s": {"p50": float(np.percentile(resp, 50)), "p99": float(np.percentile(resp, 99))},
        "queue_delay_s": {"p50": float(np.percentile(queue, 50)), "p99": float(np.percentile(queue, 99))},
        "max_hbm_used_gb": run["max_used"] / 2**30, "max_waiting": run["max_waiting"], "phase_s": run["phase"],
        "refused": run["refused"],
    }
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=8)
    ap.add_argument("--workload", default="plummer1m_salpeter")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-direct", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-all-active", action="store_true")
    ap.add_argument("--no-resident", action="store_true", help="skip the device-resident integration leg")
    ap.add_argument("--no-tree-build", action="store_true", help="skip the device tree-build leg")
    ap.add_argument("--tree-build-only", action="store_true",
                    help="only time step 1 (device builder and host builder) on the workload's initial state")
    ap.add_argument("--host-engine", action="store_true",
                    help="ensemble/served: drive the clusters from the host (scheduler and corrector on the CPU)")
    ap.add_argument("--host-rebuild", action="store_true",
                    help="ensemble/served, resident engine: rebuild trees through the host instead of the device")
    ap.add_argument("--n", type=int, default=0, help="override N (testing only; not the benchmark)")
    ap.add_argument("--n-crit", type=int, default=0, help="override the group size bound n_crit (sweeps)")
    ap.add_argument("--dump-steps", default="", help="write per-step (n_active, pairs, items, ms) JSON here")
    ap.add_argument("--requests", type=int, default=200, help="served workload: number of cluster runs")
    ap.add_argument("--max-resident", type=int, default=32, help="served workload: batch slots")
    ap.add_argument("--tuning", default="",
                    help="plan tuning 'gather_cost,target_items': every cluster of the engine workloads "
                         "(ensemble: instead of the autotune; default for served: the library's), and the tree "
                         "legs of the default workload")
    ap.add_argument("--lanes", type=int, default=0,
                    help="resident engine workloads: cluster lanes stepped out of phase (0: the engine's "
                         "default, one)")
    ap.add_argument("--hbm-gb", type=float, default=64.0, help="served workload: device-memory budget")
    ap.add_argument("--device-loop", action="store_true",
                    help="ensemble workload: run the resident engine as a batched device loop")
    ap.add_argument("--no-engine-records", action="store_true",
                    help="default workload: skip the short ensemble64 and served records")
    ap.add_argument("--graph-leg", action="store_true",
                    help="default workload: also replay the window through ht_step_graph (logged only)")
    ap.add_argument("--placement", type=int, default=None,
                    help="default workload: work-item stretches over the XCDs (0: one per XCD, 1: off; "
                         "default: the library's)")
    ap.add_argument("--predict", choices=("fused", "eager"), default="fused",
                    help="default workload: prediction mode of the tree legs (eager: one pass per step, then the gather)")
    ap.add_argument("--union-width", type=int, default=None, help="default workload: groups per union run (--lists union)")
    ap.add_argument("--lists", choices=("csr", "runs", "union"), default="csr",
                    help="default workload: interaction-list form of the tree legs (the graph leg takes CSR)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (scale for the byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU; WORLD_SIZE > 1 is not supported", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1602_02832_amd import binding as B
    from paper_1602_02832_amd import driver
    from paper_1602_02832_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.calibrate_copy:
        return calibrate_copy(torch, args.calibrate_copy)
    if args.workload == "ensemble64":
        print(json.dumps(bench_ensemble(args, torch)), flush=True)
        return
    if args.workload == "served":
        print(json.dumps(bench_served(args, torch)), flush=True)
        return
    cfg = W.config(args.workload)
    if args.n:
        cfg = W.config(args.workload, n=args.n, eps=4.0 / args.n)
    if args.n_crit:
        cfg = dataclasses.replace(cfg, n_crit=args.n_crit)
    log(f"workload {cfg.name}: N={cfg.n} theta={cfg.theta} eps={cfg.eps:.3g} dt_tree={cfg.dt_tree} "
        f"eta={cfg.eta} n_crit={cfg.n_crit}")
    x, v, m = W.make_initial_conditions(cfg)
    if args.tree_build_only:
        tb = bench_tree_build(torch, B, x, v, m, cfg)
        print(json.dumps({"workload": cfg.name, "tree_build": tb}), flush=True)
        return
    t0 = time.perf_counter()
    # The start-up runs the eagerly-predicting kernel (bit-identical predicted
    # values, another instantiation) so that in a kernel trace every launch of
    # the fused kernel belongs to the measured replay.
    sim = driver.Simulation(x, v, m, eps2=cfg.eps2, dt_tree=cfg.dt_tree, eta=cfg.eta, theta=cfg.theta,
                            n_crit=cfg.n_crit, n_leaf=cfg.n_leaf, precision="mixed", predict_mode="eager")
    log(f"initial tree + force: {time.perf_counter() - t0:.1f} s; groups {sim.tree.n_group}, nodes "
        f"{sim.tree.n_node}, list entries {sim.tree.n_entries}")
    # start-up: everything before the all-particle step at t = dt_tree
    t_start = time.perf_counter()
    last = t_start
    while sim.next_time() < cfg.dt_tree:
        sim.step()
        if time.perf_counter() - last > 10:
            last = time.perf_counter()
            log(f"start-up t={sim.t:.6g} block steps {sim.n_block_steps}")
    t_host_startup = time.perf_counter() - t_start
    steps_startup, psteps_startup = sim.n_block_steps, sim.n_particle_steps
    rec_all = Recorded(sim)
    t_all = sim.next_time()
    sim.step()   # all particles active, then the rebuild
    rec_all.steps.append((t_all, np.arange(sim.n, dtype=np.int32), None))
    log(f"start-up done: {sim.n_block_steps} block steps, {sim.n_particle_steps} particle steps in "
        f"{time.perf_counter() - t_start:.1f} s")
    # the same start-up span integrated three ways with the fused kernel (what a
    # run uses; the recording run above predicts eagerly only to keep the fused
    # kernel's launches in a trace to the measured replay): host-driven, and
    # resident on the device with the tree time rebuilt through the host or on
    # the device
    integ = None
    if not args.no_resident:
        def integrate(resident, device_tree=False, device_loop=False):
            """t = 0 up to the all-particle step at t = dt_tree, then that step and
            the rebuild there."""
            rs = driver.Simulation(x, v, m, eps2=cfg.eps2, dt_tree=cfg.dt_tree, eta=cfg.eta, theta=cfg.theta,
                                   n_crit=cfg.n_crit, n_leaf=cfg.n_leaf, precision="mixed", predict_mode="fused",
                                   resident=resident, device_tree=device_tree, device_loop=device_loop)
            torch.cuda.synchronize()
            t0_ = time.perf_counter()
            if device_loop:
                rs.run(cfg.dt_tree - math.ldexp(1.0, -41))   # every block time before dt_tree
            else:
                while rs.next_time() < cfg.dt_tree:
                    rs.step()
            torch.cuda.synchronize()
            span = time.perf_counter() - t0_
            steps = (rs.n_block_steps, rs.n_particle_steps)
            tree0 = rs.timers["tree"]
            tb = time.perf_counter()
            if device_loop:
                rs.run(cfg.dt_tree)        # the all-particle step, then the rebuild
            else:
                rs.step()
            torch.cuda.synchronize()
            tail = time.perf_counter() - tb
            rebuild = rs.timers["tree"] - tree0
            rs.sync_state()
            state = (rs.x.copy(), rs.ids.copy())
            rs.close()
            return span, steps, tail, rebuild, state
        t_host, st_host, tail_hd, reb_hd, s_hd = integrate(False)
        t_res, st_res, tail_host, reb_host, s_host = integrate(True)
        _, st_dev, tail_dev, reb_dev, s_dev = integrate(True, device_tree=True)
        t_loop, st_loop, tail_loop, _, s_loop = integrate(True, device_tree=True, device_loop=True)
        same = st_host == st_res == st_dev == st_loop == (steps_startup, psteps_startup)
        same_state = all(bool(np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]))
                         for a, b in ((s_hd, s_host), (s_hd, s_dev), (s_hd, s_loop)))
        integ = {"span": f"t = 0 to the all-particle step at t = {cfg.dt_tree} ({steps_startup} block steps, "
                         f"{psteps_startup} particle steps), fused kernel",
                 "host_driven_s": t_host, "resident_s": t_res, "device_loop_s": t_loop, "same_steps": same,
                 "block_steps_per_s": {"host_driven": steps_startup / t_host, "resident": steps_startup / t_res,
                                       "device_loop": steps_startup / t_loop},
                 "particle_steps_per_s": {"host_driven": psteps_startup / t_host,
                                          "resident": psteps_startup / t_res,
                                          "device_loop": psteps_startup / t_loop},
                 "all_particle_step_and_rebuild_s": {"host_driven": tail_hd, "resident_host_builder": tail_host,
                                                     "resident_device_builder": tail_dev},
                 "rebuild_s": {"host_driven": reb_hd, "resident_host_builder": reb_host,
                               "resident_device_builder": reb_dev},
                 "same_state_after_rebuild": same_state}
        log(f"integration start-up (fused): host-driven {t_host:.2f} s, resident {t_res:.2f} s "
            f"({steps_startup / t_res:.0f} block steps/s), device loop {t_loop:.3f} s "
            f"({steps_startup / t_loop:.0f} block steps/s), same steps {same}; rebuild at t={cfg.dt_tree}: host-driven "
            f"{reb_hd * 1e3:.1f} ms, resident via host {reb_host * 1e3:.1f} ms, on the device "
            f"{reb_dev * 1e3:.1f} ms, same state {same_state}")
    rec = Recorded(sim)
    need = args.warmup + args.steps
    while len(rec.steps) < need:
        tn, act = sim.step()
        if math.fmod(tn, cfg.dt_tree) == 0.0:
            raise RuntimeError("a tree rebuild fell inside the measured window")
        rec.add(sim, tn, act)
    n_act = np.array([a.size for _, a, _ in rec.steps[args.warmup:]])
    log(f"recorded {need} block steps: active per step min {n_act.min()} median {int(np.median(n_act))} "
        f"max {n_act.max()}, t {rec.steps[0][0]:.8g} .. {rec.steps[-1][0]:.8g}")
    sim.close()

    stream = torch.cuda.Stream()
    sh = stream.cuda_stream
    # --tuning applies to the tree legs' contexts too (gather cost, target items)
    ctx_tuning = parse_tuning(args.tuning) if args.tuning else None

    def leg(precision, direct=False):
        """The recorded steps three times, each from a fresh copy of the
        snapshot: with kernel timing (kernel time, pairs, items), with one
        event per step (step latency), and clean (throughput)."""
        lists = "csr" if direct else args.lists
        pm = "fused" if direct else args.predict
        ctx = make_ctx(B, rec.snap, rec.n, precision, cfg.eps2, sh, pm, lists=lists, placement=args.placement,
                       union_width=args.union_width, tuning=ctx_tuning)
        r = replay(torch, B, rec, ctx, stream, args.warmup, args.steps, direct=direct, mode="kernel")
        r["placement"] = ctx.placement()
        r["kernel_wall_s"] = r.pop("wall_s")
        ctx.close()
        ctx = make_ctx(B, rec.snap, rec.n, precision, cfg.eps2, sh, pm, lists=lists, placement=args.placement,
                       union_width=args.union_width, tuning=ctx_tuning)
        lt = replay(torch, B, rec, ctx, stream, args.warmup, args.steps, direct=direct, mode="latency")
        r["lat_ms"], r["latency_wall_s"] = lt["lat_ms"], lt["wall_s"]
        ctx.close()
        ctx = make_ctx(B, rec.snap, rec.n, precision, cfg.eps2, sh, pm, lists=lists, placement=args.placement,
                       union_width=args.union_width, tuning=ctx_tuning)
        r["wall_s"] = replay(torch, B, rec, ctx, stream, args.warmup, args.steps, direct=direct)["wall_s"]
        ctx.close()
        return r

    # ---- mixed tree (the headline)
    mixed = leg("mixed")
    log(f"mixed tree: {mixed['pairs'] / mixed['wall_s']:.4g} pairs/s, {1e3 * mixed['wall_s'] / args.steps:.3f} "
        f"ms/step ({1e3 * mixed['latency_wall_s'] / args.steps:.3f} with step events, "
        f"{1e3 * mixed['kernel_wall_s'] / args.steps:.3f} with kernel timing), kernel "
        f"{mixed['kernel_ms']:.3f} ms over {mixed['launches']} launches; step latency p50 "
        f"{np.percentile(mixed['lat_ms'], 50):.4f} ms")
    if args.graph_leg:   # the same steps through the captured step graphs (ht_step_graph): log only
        ctx = make_ctx(B, rec.snap, rec.n, "mixed", cfg.eps2, sh)
        graph_wall = replay(torch, B, rec, ctx, stream, args.warmup, args.steps, graph=True)["wall_s"]
        ctx.close()
        log(f"mixed tree, graph replays: {mixed['pairs'] / graph_wall:.4g} pairs/s, "
            f"{1e3 * graph_wall / args.steps:.3f} ms/step")
    # ---- direct N^2 on the same steps
    direct = None
    if not args.no_direct:
        direct = leg("mixed", direct=True)
        log(f"mixed direct: {direct['pairs'] / direct['wall_s']:.4g} pairs/s, "
            f"{1e3 * direct['wall_s'] / args.steps:.3f} ms/step")
    # ---- FP64 tree
    fp64 = None
    if not args.no_fp64:
        fp64 = leg("fp64")
        log(f"fp64 tree: {fp64['pairs'] / fp64['wall_s']:.4g} pairs/s, {1e3 * fp64['wall_s'] / args.steps:.3f} ms/step")
    # ---- the all-particle step at t = dt_tree
    all_active = None
    if not args.no_all_active:
        ctx = make_ctx(B, rec_all.snap, rec_all.n, "mixed", cfg.eps2, sh, lists=args.lists, placement=args.placement,
                       union_width=args.union_width)
        ids = np.arange(rec_all.n, dtype=np.int32)
        acc = torch.empty((rec_all.n, 3), dtype=torch.float64, device="cuda")
        jrk = torch.empty_like(acc)
        pot = torch.empty(rec_all.n, dtype=torch.float64, device="cuda")
        ctx.predict(t_all)
        ctx.force_async(ids, acc, jrk, pot)   # warm-up
        torch.cuda.synchronize()
        ctx.set_timing(True)
        reps = 3
        tw = time.perf_counter()
        for _ in range(reps):
            ctx.force_async(ids, acc, jrk, pot)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - tw) / reps
        kms, nl, kp = ctx.kernel_timing()
        ctx.set_timing(False)
        pairs_all = kp / nl
        all_active = dict(t=t_all, n_active=rec_all.n, pairs=int(pairs_all), ms=1e3 * wall,
                          kernel_ms=kms / nl, interactions_per_s=pairs_all / wall,
                          equivalent_interactions_per_s=rec_all.n * (rec_all.n - 1) / wall)
        log(f"all-particle step: {1e3 * wall:.2f} ms, {pairs_all / wall:.4g} pairs/s, kernel {kms / nl:.2f} ms")
        ctx.close()

    # ---- step 1 on the device (htd_build) against the host builder, same state
    tree_build = None
    if not args.no_tree_build:
        tree_build = bench_tree_build(torch, B, x, v, m, cfg)
        log(f"tree build: device {tree_build['device_ms']:.2f} ms (phases {tree_build['device_phases_ms']}), "
            f"host builder {tree_build['host_builder_ms']:.1f} ms on {tree_build['host_threads']} threads")

    # ---- CPU baseline (oracle on a bounded sample)
    cpu = None
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle list force for about {args.cpu_seconds:.0f} s")
        cpu, cpu_extra = cpu_baseline(W, cfg, rec, args.warmup, args.cpu_seconds)
        log(f"cpu baseline: {cpu['value']:.4g} interactions/s on {cpu['cores']} threads; direct "
            f"{cpu_extra['direct_interactions_per_s']:.4g}; tree build {cpu_extra['tree_build_s']}")

    K = args.steps
    if args.dump_steps:
        dump = {"mixed": [list(r) + [float(t)] for r, t in zip(mixed["per_step"], mixed["lat_ms"])],
                "tile_pairs": tile_mix(rec, args.warmup)}
        if direct is not None:
            dump["direct"] = [list(r) + [float(t)] for r, t in zip(direct["per_step"], direct["lat_ms"])]
        if fp64 is not None:
            dump["fp64"] = [list(r) + [float(t)] for r, t in zip(fp64["per_step"], fp64["lat_ms"])]
        with open(args.dump_steps, "w") as f:
            json.dump(dump, f)
    value = mixed["pairs"] / mixed["wall_s"]
    eq_pairs = int(sum(a.size for _, a, _ in rec.steps[args.warmup:]) * (rec.n - 1))
    lat = mixed["lat_ms"]
    kernel_avg_ms = mixed["kernel_ms"] / max(mixed["launches"], 1)
    achieved = FLOPS_PER_PAIR * mixed["kernel_pairs"] / (mixed["kernel_ms"] * 1e-3) / 1e12
    alg_bytes = algorithmic_bytes(rec, args.warmup)
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * mixed["wall_s"] / K,
        "latency_replay_ms_per_step": 1e3 * mixed["latency_wall_s"] / K,
        "kernel_replay_ms_per_step": 1e3 * mixed["kernel_wall_s"] / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": cfg.name, "n": cfg.n, "theta": cfg.theta, "eps": cfg.eps, "dt_tree": cfg.dt_tree,
                   "eta": cfg.eta, "n_crit": cfg.n_crit, "n_leaf": cfg.n_leaf,
                   "masses": f"salpeter 1:{cfg.mass_ratio:g}" if cfg.mass_seed is not None else "equal",
                   "window": f"{K} block steps after the rebuild at t={cfg.dt_tree}", "precision": "mixed",
                   "predict": args.predict, "lists": args.lists,
                   "union_width": (args.union_width or 4) if args.lists == "union" else None,
                   "placement": {"runs": mixed["placement"][0], "xcds": mixed["placement"][1]}},
        "p50_step_ms": float(np.percentile(lat, 50)),
        "p99_step_ms": float(np.percentile(lat, 99)),
        "active_per_step": {"min": int(n_act.min()), "median": float(np.median(n_act)), "max": int(n_act.max()),
                            "mean": float(n_act.mean())},
        "equivalent_interactions_per_s": eq_pairs / mixed["wall_s"],
        # eq. (1): the direct scheme's flops for the same active sets, at 57 per pair, over the tree's time
        "equivalent_tflops_at_57": FLOPS_PER_PAIR * eq_pairs / mixed["wall_s"] / 1e12,
        "raw_tflops_at_57": FLOPS_PER_PAIR * value / 1e12,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "peak_nonpacked": PEAK_NONPACKED_TFLOPS,
                     "frac_nonpacked": achieved / PEAK_NONPACKED_TFLOPS,
                     "traffic": measured_traffic(K, args.warmup),
                     "traffic_unit": "bytes/launch", "algorithmic_bytes": alg_bytes,
                     "kernel": "force_kernel<PrecMixed,false,false,false>", "avg_launch_ms": kernel_avg_ms,
                     "pairs_per_launch": mixed["kernel_pairs"] / max(mixed["launches"], 1)},
        # the same launches against HBM: the sparse steps that dominate the window are bound by the
        # bytes their gathers fetch (algorithmic bytes per launch, and the measured traffic's rate)
        "roofline_gather": {"bound": "hbm", "achieved": alg_bytes / (kernel_avg_ms * 1e-3) / 1e9,
                            "peak": PEAK_HBM_GBS, "unit": "GB/s",
                            "frac": alg_bytes / (kernel_avg_ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                            "traffic_rate": (None if measured_traffic(K, args.warmup) is None else
                                             measured_traffic(K, args.warmup) / (kernel_avg_ms * 1e-3) / 1e9)},
    }
    if direct is not None:
        result["direct_interactions_per_s"] = direct["pairs"] / direct["wall_s"]
        result["direct_ms_per_step"] = 1e3 * direct["wall_s"] / K
        result["speedup_vs_direct"] = direct["wall_s"] / mixed["wall_s"]
    if fp64 is not None:
        result["fp64_interactions_per_s"] = fp64["pairs"] / fp64["wall_s"]
        result["fp64_ms_per_step"] = 1e3 * fp64["wall_s"] / K
        result["fp64_p99_step_ms"] = float(np.percentile(fp64["lat_ms"], 99))
    if all_active is not None:
        result["all_active_step"] = all_active
    if integ is not None:
        result["integration"] = integ
    if tree_build is not None:
        result["tree_build"] = tree_build
    if cpu is not None:
        result["cpu_baseline"] = cpu
        result["cpu_oracle_other"] = cpu_extra
    # the batched ensemble and the served stream, short forms (their own --workload runs are the long ones)
    if not args.no_engine_records:
        sub = argparse.Namespace(**vars(args))
        sub.steps, sub.warmup, sub.tuning, sub.device_loop = 32, 8, "12,512", True
        ens = bench_ensemble(sub, torch)
        result["ensemble64"] = {k: ens[k] for k in ("metric", "value", "unit", "ms_per_step", "p50_step_ms",
                                                    "p99_step_ms", "equivalent_interactions_per_s", "steps",
                                                    "warmup", "config")}
        log(f"ensemble64 record: {ens['value']:.4g} interactions/s, {ens['ms_per_step']:.3f} ms per engine step")
        sub = argparse.Namespace(**vars(args))
        sub.requests, sub.tuning = 64, ""
        srv = bench_served(sub, torch)
        result["served"] = {k: srv[k] for k in ("metric", "value", "unit", "p50_step_ms", "p99_step_ms",
                                                "interactions_per_s", "capacity_runs_per_s", "throughput_runs_per_s",
                                                "request_latency_s", "queue_delay_s", "max_hbm_used_gb", "refused",
                                                "config")}
        log(f"served record: p50 {srv['p50_step_ms']:.3f} ms, p99 {srv['p99_step_ms']:.3f} ms per engine step, "
            f"{srv['interactions_per_s']:.4g} interactions/s")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
