"""Batched engine and continuous-batching server on the GPU.

Work plans are made per cluster, so every cluster must come out bit-identical
whether it runs alone or in a batch with others.  The batched forces are also
checked against the FP64 oracle directly: the batched launch on set states,
and engine steps (host-driven, resident, and inside the served stream) whose
active particles' new accelerations, jerks and potentials are the step's
forces, recomputed by the oracle from the state before the step."""
import numpy as np
import pytest
from paper_1602_02832_amd import binding as B
from paper_1602_02832_amd import engine as E
from paper_1602_02832_amd import workloads as W
from parity_util import assert_close, oracle_list_force

pytestmark = pytest.mark.gpu

FIELDS = ("x", "v", "a", "j", "t0", "dt", "pot")


def say(msg):
    print(msg, flush=True)


def snapshot(c):
    """A cluster's state in its current particle order, and its tree."""
    sim = c.sim
    sim.sync_state()
    return dict(t0=sim.t0.copy(), dt=sim.dt.copy(), x=sim.x.copy(), v=sim.v.copy(), a=sim.a.copy(),
                j=sim.j.copy(), m=sim.m.copy(), tree=sim.tree, t_tree=sim.t_tree, eps2=sim.eps2,
                dt_tree=sim.dt_tree)


def oracle_checked_step(eng, oracle, tag, step=None):
    """One engine step (``step``, default eng.step); every stepping cluster
    whose block time is not a tree time (a rebuild reorders the state) has the
    new a, jerk and pot of its active particles compared with the oracle's
    list force on the state before the step.  Returns (clusters checked, the
    step's finished clusters)."""
    eng.drain()
    before = {id(c): snapshot(c) for c in eng.clusters if not c.done}
    finished = (step or eng.step)()
    eng.drain()
    checked = 0
    for c in eng.clusters:
        b = before.get(id(c))
        if b is None:
            continue
        t = float(np.min(b["t0"] + b["dt"]))
        if np.fmod(t, b["dt_tree"]) == 0.0:
            continue
        sim = c.sim
        sim.sync_state()
        act = np.flatnonzero(sim.t0 != b["t0"]).astype(np.int32)
        assert act.size > 0 and np.all(sim.t0[act] == t)
        assert np.array_equal(act, np.flatnonzero(b["t0"] + b["dt"] == t))
        want = oracle_list_force(oracle, t, act, b["t0"], b["m"], b["x"], b["v"], b["a"], b["j"], b["tree"],
                                 b["eps2"], t_tree=b["t_tree"])
        assert_close(f"{tag}: cluster {c.spec.key} t={t} ({act.size} active)", "mixed",
                     (sim.a[act], sim.j[act], sim.pot[act]), want)
        checked += 1
    return checked, finished


def state(sim):
    sim.sync_state()      # resident clusters keep their state on the device
    order = np.argsort(sim.ids)
    return {f: getattr(sim, f)[order].copy() for f in FIELDS}


def run_engine(specs, **kw):
    """Run every cluster to its spec.steps block steps (rebuilds may make a
    cluster sit out engine steps; its own sequence of steps never changes)."""
    eng = E.Engine(max_clusters=16, max_active=1 << 16, max_items=1 << 16, max_rows=1 << 16, **kw)
    clusters = [eng.new_cluster(s) for s in specs]
    for c in clusters:
        eng.add(c)
    while not all(c.done for c in clusters):
        eng.step()
    eng.drain()
    out = [state(c.sim) for c in clusters]
    stats = (eng.pairs, eng.engine_steps, [c.steps_done for c in clusters])
    eng.close()
    return out, stats


def test_batch_update_and_force_equal_per_context(oracle):
    import torch
    say("ht_batch update + force vs per-context calls")
    s = torch.cuda.Stream()
    batch = B.Batch(stream=s.cuda_stream, max_clusters=8, max_items=1 << 15, max_active=1 << 15, max_rows=1 << 15)
    ctx_b, ctx_a, rows_l, act_l, states = [], [], [], [], []
    for k, n in enumerate((700, 2000, 64)):
        x, v, m = W.plummer(n, 90 + k)
        z = np.zeros((n, 3))
        tr = B.HostTree(x, v, z, z, m, 1, 64, 0.5)
        x, v, m = x[tr.perm], v[tr.perm], m[tr.perm]
        t0, a, j = W.random_block_state(n, 95 + k, 0.125)
        states.append((t0, m, x, v, a, j, tr))
        pair = []
        for _ in range(2):
            c = B.Context(n_max=n, node_max=2 * n, group_max=n, list_max=2 * tr.n_entries + 64, active_max=n,
                          eps2=1e-4, precision="mixed", stream=s.cuda_stream)
            c.set_j_particles(t0, m, x, v, a, j)
            c.set_nodes(0.0, tr.node_m, tr.node_x, tr.node_v, tr.node_a, tr.node_j)
            c.set_interaction_lists(tr.group_first, tr.list_off, tr.entries)
            pair.append(c)
        ctx_b.append(pair[0])
        ctx_a.append(pair[1])
        rng = np.random.default_rng(k)
        idx = np.sort(rng.choice(n, n // 3, replace=False)).astype(np.int32)
        rows_l.append(B.make_rows(idx, np.full(idx.size, 0.125), m[idx], x[idx] + 1e-3, v[idx], a[idx] * 0.5,
                                  j[idx] * 0.5))
        act_l.append(np.sort(rng.choice(n, max(1, n // 2), replace=False)).astype(np.int32))
    batch.update_async(ctx_b, rows_l)
    outs = []
    for c, a in zip(ctx_b, act_l):
        c.predict(0.15625)
        outs.append(tuple(torch.empty(sh, dtype=torch.float64, device="cuda") for sh in ((a.size, 3), (a.size, 3), (a.size,))))
    batch.force_async(ctx_b, act_l, [o[0] for o in outs], [o[1] for o in outs], [o[2] for o in outs])
    batch.sync()
    for c, r, a, o in zip(ctx_a, rows_l, act_l, outs):
        c.set_j_particles(r["t0"], r["m"], r["x"], r["v"], r["a"], r["jerk"], idx=r["idx"])
        c.predict(0.15625)
        want = c.force(a)
        for p, q in zip(want, o):
            assert np.array_equal(p, q.cpu().numpy())
    # the batched update and force against the FP64 oracle on the updated state
    for k, (st, r, a, o) in enumerate(zip(states, rows_l, act_l, outs)):
        t0, m, x, v, acc0, j0, tr = (u.copy() if isinstance(u, np.ndarray) else u for u in st)
        idx = r["idx"]
        t0[idx], m[idx], x[idx], v[idx], acc0[idx], j0[idx] = r["t0"], r["m"], r["x"], r["v"], r["a"], r["jerk"]
        want = oracle_list_force(oracle, 0.15625, a, t0, m, x, v, acc0, j0, tr, 1e-4)
        assert_close(f"batched update + force, cluster {k}", "mixed", tuple(q.cpu().numpy() for q in o), want)
    with pytest.raises(B.HTError):
        batch.update_async([ctx_b[0], ctx_b[0]], [rows_l[0], rows_l[0]])


@pytest.mark.parametrize("resident", [True, False], ids=["resident", "host"])
def test_engine_steps_match_oracle(oracle, resident):
    """Engine steps over a mix of clusters (one batched force launch per step)
    checked cluster by cluster against the oracle, through a tree rebuild."""
    say(f"engine steps vs oracle, resident={resident}")
    specs = [E.RunSpec(key=k, n=n, seed=900 + k, steps=10**6, n_crit=64, mass_seed=(950 + k) if k % 2 else None)
             for k, n in enumerate((500, 1800, 3300, 900))]
    eng = E.Engine(max_clusters=8, max_active=1 << 15, max_items=1 << 15, max_rows=1 << 15, rebuild_workers=0,
                   resident=resident)
    for sp in specs:
        eng.add(eng.new_cluster(sp))
    checked = 0
    rebuilt = False
    for k in range(400):
        t_tree = [c.sim.t_tree for c in eng.clusters]
        if k % 3 == 0:
            checked += oracle_checked_step(eng, oracle, f"engine step {k}")[0]
        else:
            eng.step()
        rebuilt |= any(c.sim.t_tree != t for c, t in zip(eng.clusters, t_tree))
        if checked >= 40 and rebuilt and k % 3 == 0:
            break
    eng.close()
    say(f"engine steps vs oracle: {checked} cluster steps checked in {k + 1} engine steps")
    assert checked >= 40 and rebuilt, (checked, rebuilt)


def test_engine_cluster_alone_equals_in_mix():
    say("engine: three clusters alone vs together")
    specs = [E.RunSpec(key=k, n=n, seed=300 + k, steps=40, n_crit=64) for k, n in enumerate((600, 1500, 3000))]
    together, (pairs, nsteps, done) = run_engine(specs)
    assert nsteps >= 40 and pairs > 0 and done == [40, 40, 40]
    for k, s in enumerate(specs):
        alone, _ = run_engine([s], rebuild_workers=0)
        for f in FIELDS:
            assert np.array_equal(alone[0][f], together[k][f]), (k, f)


def test_server_admission_respects_budget_and_results_match(oracle):
    say("server: admission under a small device-memory budget")
    specs = [E.RunSpec(key=k, n=n, seed=400 + k, steps=12, n_crit=64) for k, n in enumerate((800, 1200, 900, 2000, 700))]
    eng = E.Engine(max_clusters=8, max_active=1 << 16, max_items=1 << 16, max_rows=1 << 16)
    sizes = {s.key: eng.new_cluster(s).reserve for s in specs}
    budget = sizes[3] + sizes[1]                   # room for about two runs at a time
    srv = E.Server(eng, hbm_budget=budget, max_resident=8, keep_finished=True)
    reqs = [E.Request(spec=s, arrival=0.0) for s in specs]
    # every fourth served engine step is checked against the oracle
    srv_checked, plain_step = [0, 0], eng.step

    def step():
        srv_checked[1] += 1
        if srv_checked[1] % 4:
            return plain_step()
        n, fin = oracle_checked_step(eng, oracle, f"served engine step {srv_checked[1]}", step=plain_step)
        srv_checked[0] += n
        return fin

    eng.step = step
    done = srv.run(reqs)
    assert len(done) == len(specs)
    assert srv.max_waiting >= 2                    # admission actually held requests back
    assert srv.max_used <= budget
    assert all(r.finished >= r.admitted >= r.arrival for r in done)
    mixed = {r.spec.key: state(r.cluster.sim) for r in done}
    assert srv_checked[0] >= 4
    for r in done:
        r.cluster.close()
    eng.close()
    for s in specs[:3]:
        alone, _ = run_engine([s])
        for f in FIELDS:
            assert np.array_equal(alone[0][f], mixed[s.key][f]), (s.key, f)


def test_server_charges_what_resident_clusters_hold():
    """Resident clusters with device rebuilds: the reservation charged for a
    cluster (ht_cluster_admit: its context workspace plus ht_state_bytes) is
    what its activation takes from torch's allocator, the shared tree
    builder's arrays are held against the same budget, and a request larger
    than the whole budget is refused instead of admitted into an empty pool."""
    import torch
    say("server: charged bytes of resident clusters, tree builder, oversized request")
    small = [E.RunSpec(key=k, n=n, seed=1300 + k, steps=10, n_crit=64) for k, n in enumerate((900, 1500, 700, 1200))]
    eng = E.Engine(max_clusters=8, max_active=1 << 15, max_items=1 << 15, max_rows=1 << 15, rebuild_workers=0,
                   resident=True, device_tree=True, tree_n_max=1500)
    def requested():   # bytes asked of torch's allocator by live tensors (before its block rounding)
        return torch.cuda.memory_stats()["requested_bytes.all.current"]

    for sp in small:                       # charge = bytes taken; the builder warms up to these sizes
        c = eng.new_cluster(sp)
        torch.cuda.synchronize()
        before = requested()
        eng.add(c)
        taken = requested() - before
        assert taken == c.reserve, (sp.n, taken, c.reserve)
        assert c.footprint() == c.reserve
        eng.remove(c)
        c.close()
    tree0 = eng.tree.device_bytes()
    reserves = sorted(eng.new_cluster(sp).reserve for sp in small)
    budget = tree0 + reserves[-1] + reserves[-2]
    n_big = 20000
    while eng.new_cluster(E.RunSpec(key=99, n=n_big, seed=1399, steps=10, n_crit=64)).reserve <= budget:
        n_big *= 2
    big = E.RunSpec(key=99, n=n_big, seed=1399, steps=10, n_crit=64)
    srv = E.Server(eng, hbm_budget=budget, max_resident=8, keep_finished=False)
    reqs = [E.Request(spec=s, arrival=0.0) for s in small[:2]] + [E.Request(spec=big, arrival=0.0)] + \
        [E.Request(spec=s, arrival=0.0) for s in small[2:]]
    done = srv.run(reqs)
    assert [r.spec.key for r in srv.refused] == [99]
    assert sorted(r.spec.key for r in done) == [0, 1, 2, 3]
    assert srv.max_used <= budget + (eng.tree.device_bytes() - tree0)
    assert srv.used == eng.tree.device_bytes()          # only the builder is held at the end
    srv.close()
    eng.close()


def test_engine_matches_single_cluster_simulation():
    """The engine path (pinned row updates, results written to pinned memory,
    the flat batched corrector) gives the same bits as stepping the cluster's
    own Simulation (host-array force, per-cluster corrector)."""
    from paper_1602_02832_amd import driver
    say("engine vs Simulation.step on the same cluster")
    spec = E.RunSpec(key=0, n=1500, seed=510, steps=30, n_crit=64)
    eng = E.Engine(max_clusters=4, max_active=1 << 14, max_items=1 << 15, max_rows=1 << 14, rebuild_workers=0)
    c = eng.new_cluster(spec)
    eng.add(c)
    while not c.done:
        eng.step()
    got = state(c.sim)
    eng.close()
    x, v, m = W.plummer(spec.n, spec.seed)
    eps = 4.0 / spec.n
    sim = driver.Simulation(x, v, m, eps2=eps * eps, dt_tree=spec.dt_tree, eta=spec.eta, theta=spec.theta,
                            n_crit=spec.n_crit, precision="mixed")
    for _ in range(spec.steps):
        sim.step()
    want = state(sim)
    sim.close()
    for f in FIELDS:
        assert np.array_equal(got[f], want[f]), f


def test_resident_engine_equals_host_engine():
    """The engine with every cluster's state on the device (batched scheduler
    and corrector launches) gives the bits of the host-driven engine, through
    tree rebuilds, alone and in a mix."""
    say("engine: resident vs host-driven, three clusters")
    specs = [E.RunSpec(key=k, n=n, seed=600 + k, steps=60, n_crit=64) for k, n in enumerate((700, 2500, 5000))]
    host, _ = run_engine(specs)
    dev, (pairs, nsteps, done) = run_engine(specs, resident=True)
    assert done == [60, 60, 60] and pairs > 0
    for k in range(len(specs)):
        for f in FIELDS:
            assert np.array_equal(host[k][f], dev[k][f]), (k, f)
    alone, _ = run_engine([specs[1]], resident=True, rebuild_workers=0)
    for f in FIELDS:
        assert np.array_equal(alone[0][f], dev[1][f]), f
    # rebuilds on the device, one builder shared by the clusters (the largest
    # cluster does not fit it and rebuilds through the host)
    say("engine: resident with device rebuilds")
    dtree, (_, _, done) = run_engine(specs, resident=True, device_tree=True, tree_n_max=2500)
    assert done == [60, 60, 60]
    for k in range(len(specs)):
        for f in FIELDS:
            assert np.array_equal(host[k][f], dtree[k][f]), (k, f)


def test_resident_engine_lanes_give_the_same_bits():
    """Clusters split into lanes (streams and batches of their own, stepped out
    of phase) give the bits of one lane, also with device rebuilds on the
    builder the lanes share."""
    say("engine: one lane vs three lanes")
    specs = [E.RunSpec(key=k, n=n, seed=700 + k, steps=50, n_crit=64)
             for k, n in enumerate((600, 1700, 900, 2400, 1200))]
    one, (_, _, done1) = run_engine(specs, resident=True, lanes=1)
    three, (_, _, done3) = run_engine(specs, resident=True, lanes=3, device_tree=True, tree_n_max=2500)
    assert done1 == done3 == [50] * 5
    for k in range(len(specs)):
        for f in FIELDS:
            assert np.array_equal(one[k][f], three[k][f]), (k, f)
    with pytest.raises(ValueError):
        E.Engine(lanes=2)              # lanes need the resident engine


@pytest.mark.parametrize("resident", [True, False], ids=["resident", "host"])
def test_engine_many_clusters_alone_equals_in_batch(resident):
    """Ten clusters in one batch give each cluster the bits it gets alone."""
    say(f"engine: ten clusters, resident={resident}")
    sizes = (300, 420, 510, 640, 380, 700, 450, 560, 330, 610)
    specs = [E.RunSpec(key=k, n=n, seed=800 + k, steps=25, n_crit=32) for k, n in enumerate(sizes)]
    together, (_, _, done) = run_engine(specs, resident=resident)
    assert done == [25] * len(specs)
    for k in (0, 3, 9):
        alone, _ = run_engine([specs[k]], resident=resident)
        for f in FIELDS:
            assert np.array_equal(alone[0][f], together[k][f]), (k, f)


def test_batched_device_loop_equals_resident_engine():
    """The batched device loop (ht_batch_dev_run: scheduler, device planner,
    one force and one corrector launch for all clusters per engine step,
    graphs of 32 engine steps, no host round trip) gives every cluster the
    bits of the step-by-step resident engine, through tree rebuilds on the
    device, alone and in a mix, for calls of 7, 32 and 45 engine steps."""
    say("engine: batched device loop vs resident engine")
    specs = [E.RunSpec(key=k, n=n, seed=1100 + k, steps=70, n_crit=64) for k, n in enumerate((700, 2500, 1200, 4000))]
    kw = dict(resident=True, device_tree=True, tree_n_max=4000)
    ref, (_, _, done) = run_engine(specs, **kw)
    assert done == [70] * 4
    for loop_steps in (7, 32, 45):
        got, (pairs, _, done) = run_engine(specs, device_loop=True, loop_steps=loop_steps, **kw)
        assert done == [70] * 4 and pairs > 0
        for k in range(len(specs)):
            for f in FIELDS:
                assert np.array_equal(ref[k][f], got[k][f]), (loop_steps, k, f)
    alone, _ = run_engine([specs[2]], device_loop=True, loop_steps=32, **kw)
    for f in FIELDS:
        assert np.array_equal(alone[0][f], ref[2][f]), f


def test_batched_device_loop_steps_match_oracle(oracle):
    """Single engine steps of the batched device loop (host rebuilds, so the
    tree's node data are at hand) against the oracle's list force."""
    say("engine: batched device loop steps vs oracle")
    specs = [E.RunSpec(key=k, n=n, seed=1200 + k, steps=10**6, n_crit=64, mass_seed=(1250 + k) if k % 2 else None)
             for k, n in enumerate((600, 2100, 900))]
    eng = E.Engine(max_clusters=8, max_active=1 << 15, max_items=1 << 15, max_rows=1 << 15, rebuild_workers=0,
                   resident=True, device_loop=True, loop_steps=1)
    for sp in specs:
        eng.add(eng.new_cluster(sp))
    checked = 0
    for k in range(60):
        if k % 4 == 0:
            checked += oracle_checked_step(eng, oracle, f"device-loop engine step {k}")[0]
        else:
            eng.step()
    eng.close()
    assert checked >= 30, checked
