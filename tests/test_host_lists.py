"""The product host builder (libhtree_host.so) against the oracle: keys,
order, node moments, groups and interaction lists must be bit-identical.
The two share no code; both follow the tree/group/list rules of Section 2
step 1 as read in the oracle's header."""
import numpy as np
import pytest

from paper_1602_02832_amd import binding as B
from paper_1602_02832_amd import workloads as W

FIELDS = ["perm", "keys", "node_m", "node_x", "node_v", "node_a", "node_j", "node_level", "node_begin",
          "node_end", "group_first", "list_off", "entries"]


def assert_same_tree(oracle, x, v, a, j, m, n_leaf, n_crit, theta):
    ref = oracle.Tree(x, v, a, j, m, n_leaf, n_crit, theta)
    got = B.HostTree(x, v, a, j, m, n_leaf, n_crit, theta)
    assert (got.n_node, got.n_group, got.n_entries) == (ref.n_node, ref.n_group, ref.n_entries)
    for f in FIELDS:
        g, r = getattr(got, f), getattr(ref, f)
        assert g.dtype == r.dtype and g.shape == r.shape, f
        assert np.array_equal(g, r), f
    return got


def test_hilbert_keys_match_oracle(oracle):
    rng = np.random.default_rng(1)
    q = rng.integers(0, 1 << 21, (1_000_000, 3)).astype(np.uint32)
    q[:8] = [[0, 0, 0], [(1 << 21) - 1] * 3, [1, 0, 0], [0, 1, 0], [0, 0, 1], [7, 7, 7], [1 << 20] * 3, [5, 1 << 20, 9]]
    assert np.array_equal(B.hilbert_keys(q), oracle.hilbert_keys(q))


@pytest.mark.parametrize("cfg", ["plummer2k", "plummer16k"])
def test_lists_bit_exact_on_workloads(oracle, cfg):
    c = W.config(cfg)
    x, v, m = W.make_initial_conditions(c)
    rng = np.random.default_rng(c.seed + 100)
    a, j = rng.normal(size=(2, c.n, 3))
    t = assert_same_tree(oracle, x, v, a, j, m, c.n_leaf, c.n_crit, c.theta)
    assert t.n_group > 10 and t.n_node > c.n // 4


def _degenerate():
    rng = np.random.default_rng(7)
    out = []
    out.append(("n1", rng.normal(size=(1, 3)), 1, 4, 0.5))
    out.append(("n2", rng.normal(size=(2, 3)), 1, 1, 0.5))
    x = rng.normal(size=(40, 3))
    x[5] = x[6] = x[30]
    out.append(("coincident", x, 1, 4, 0.5))
    out.append(("all_same", np.ones((17, 3)), 1, 4, 0.5))
    out.append(("theta0", rng.normal(size=(300, 3)), 1, 16, 0.0))
    out.append(("theta_large", rng.normal(size=(300, 3)), 1, 16, 50.0))
    out.append(("ncrit1", rng.normal(size=(200, 3)), 1, 1, 0.6))
    out.append(("ncrit_all", rng.normal(size=(200, 3)), 1, 10000, 0.6))
    out.append(("leaf4", rng.normal(size=(500, 3)), 4, 32, 0.5))
    out.append(("flat", np.column_stack([rng.normal(size=(256, 2)), np.zeros(256)]), 1, 16, 0.5))
    out.append(("line", np.column_stack([rng.normal(size=256), np.zeros(256), np.zeros(256)]), 1, 16, 0.5))
    out.append(("tiny_scale", rng.normal(size=(256, 3)) * 1e-200, 1, 16, 0.5))
    return out


@pytest.mark.parametrize("name,x,n_leaf,n_crit,theta", _degenerate(), ids=[d[0] for d in _degenerate()])
def test_lists_bit_exact_degenerate(oracle, name, x, n_leaf, n_crit, theta):
    n = x.shape[0]
    rng = np.random.default_rng(n)
    v, a, j = rng.normal(size=(3, n, 3))
    m = rng.uniform(0.5, 1.5, n) / n
    assert_same_tree(oracle, x, v, a, j, m, n_leaf, n_crit, theta)


@pytest.mark.parametrize("seed", range(6))
def test_lists_bit_exact_random_small(oracle, seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(3, 3000))
    x = rng.standard_cauchy(size=(n, 3)) * 0.1
    v, a, j = rng.normal(size=(3, n, 3))
    m = rng.uniform(0.1, 1.0, n)
    assert_same_tree(oracle, x, v, a, j, m, int(rng.integers(1, 5)), int(rng.integers(1, 200)),
                     float(rng.uniform(0.2, 1.0)))


def test_lists_bit_exact_after_integration(oracle):
    """Rebuilds during an oracle tree/Hermite run see evolved, unsorted-looking
    states; the product builder must reproduce every one."""
    c = W.config("plummer2k")
    x, v, m = W.make_initial_conditions(c)
    states = []

    def hook(sim, rec):
        if np.fmod(rec["t"], c.dt_tree) == 0.0:
            states.append(None)

    sim = oracle.TreeHermite(x, v, m, eps2=c.eps2, dt_tree=c.dt_tree, eta=c.eta, theta=c.theta, n_crit=c.n_crit)
    for _ in range(3):
        t_next = sim.t + c.dt_tree
        while sim.next_time() <= t_next:
            sim.step()
        got = B.HostTree(sim.x, sim.v, sim.a, sim.j, sim.m, c.n_leaf, c.n_crit, c.theta)
        # the oracle has just rebuilt from this same (already sorted) state
        assert np.array_equal(got.perm, np.arange(c.n))
        for f in ("node_m", "node_x", "node_v", "node_a", "node_j", "group_first", "list_off", "entries"):
            assert np.array_equal(getattr(got, f), getattr(sim.tree, f)), f


def test_host_corrector_matches_oracle(oracle):
    """Product host corrector + block step vs the oracle's, same inputs."""
    rng = np.random.default_rng(3)
    n = 500
    t1 = 3.0 / 64
    dt_old = 2.0 ** -rng.integers(6, 10, n)
    t0 = t1 - dt_old
    x, v, a, j = rng.normal(size=(4, n, 3))
    a1 = a + rng.normal(scale=1e-2, size=(n, 3))
    j1 = j + rng.normal(scale=1e-2, size=(n, 3))
    ids = np.arange(n, dtype=np.int32)
    xp, vp = oracle.predict(t1, t0, x, v, a, j)
    x1, v1, dta = oracle.correct(t1, t0, xp, vp, a, j, a1, j1, 0.01)
    want_dt = np.array([oracle.block_step(dta[k], t1, 1 / 64, dt_old[k]) for k in range(n)])
    X, V, A, J, T0, DT = x.copy(), v.copy(), a.copy(), j.copy(), t0.copy(), dt_old.copy()
    B.correct(ids, t1, 0.01, 1 / 64, T0, DT, X, V, A, J, a1, j1)
    assert np.allclose(X, x1, rtol=1e-14, atol=1e-14) and np.allclose(V, v1, rtol=1e-13, atol=1e-13)
    assert np.array_equal(DT, want_dt) and np.all(T0 == t1)
    assert np.array_equal(A, a1) and np.array_equal(J, j1)


def test_next_block_selects_minimum():
    rng = np.random.default_rng(4)
    n = 100000
    dt = 2.0 ** -rng.integers(3, 12, n)
    t0 = np.floor(rng.uniform(0, 1, n) / dt) * dt
    tn, act = B.next_block(t0, dt)
    want = np.flatnonzero(t0 + dt == (t0 + dt).min())
    assert tn == (t0 + dt).min() and np.array_equal(act, want)


@pytest.mark.parametrize("level", [0, 3, 7, 12, 20, 33])
def test_host_block_steps_match_oracle_at_many_block_times(oracle, level):
    """The host quantiser (largest power of two dividing t1, from its bits) gives
    the oracle's block step (halving until t1 is a multiple) at block times with
    many different binary valuations."""
    rng = np.random.default_rng(40 + level)
    n = 400
    k = rng.integers(1, 1 << 12, n) | 1                    # odd multiples
    t1 = float(np.ldexp(k[0], -level)) if level else 5.0
    dt_old = np.ldexp(1.0, -rng.integers(max(level, 1), min(max(level, 1) + 10, 39), n))   # steps stay >= 2^-40
    t0 = t1 - dt_old
    x, v, a, j = rng.normal(size=(4, n, 3))
    a1 = a + rng.normal(scale=10.0 ** rng.uniform(-6, 1), size=(n, 3))
    j1 = j + rng.normal(scale=10.0 ** rng.uniform(-6, 1), size=(n, 3))
    xp, vp = oracle.predict(t1, t0, x, v, a, j)
    _, _, dta = oracle.correct(t1, t0, xp, vp, a, j, a1, j1, 0.02)
    want = np.array([oracle.block_step(dta[q], t1, 1.0, dt_old[q]) for q in range(n)])
    T0, DT = t0.copy(), dt_old.copy()
    B.correct(np.arange(n, dtype=np.int32), t1, 0.02, 1.0, T0, DT, x.copy(), v.copy(), a.copy(), j.copy(), a1, j1)
    assert np.array_equal(DT, want)


def _clusters(sizes, seed):
    rng = np.random.default_rng(seed)
    out = []
    for n in sizes:
        dt = np.ldexp(1.0, -rng.integers(3, 9, n))
        t0 = np.floor(rng.uniform(0, 1, n) / dt) * dt
        x, v, a, j = rng.normal(size=(4, n, 3))
        m = rng.uniform(0.5, 1.5, n) / n
        out.append(dict(n=n, t0=t0, dt=dt, x=x, v=v, a=a, j=j, m=m, pot=np.zeros(n), act=np.empty(n, np.int32)))
    return out


def _structs(cls):
    return (B.HtbCluster * len(cls))(*[B.cluster_struct(c["n"], 0.01, 1.0 / 8, c["t0"], c["dt"], c["x"], c["v"],
                                                        c["a"], c["j"], c["m"], c["pot"], c["act"]) for c in cls])


SIZES = (1, 3, 50, 8191, 8192, 8193, 20000, 40000)


def test_host_wrappers_refuse_mismatched_arrays():
    """The host corrector and scheduler work in place on the caller's arrays:
    the binding refuses the wrong dtype, a non-contiguous view, mismatched
    lengths, a too-short output and ids outside the arrays (the library would
    read or write past them), and leaves the arrays untouched."""
    n = 16
    rng = np.random.default_rng(5)
    t0, dt = np.zeros(n), np.full(n, 1.0 / 64)
    x, v, a, j = rng.normal(size=(4, n, 3))
    keep = [u.copy() for u in (t0, dt, x, v, a, j)]
    ids = np.arange(4, dtype=np.int32)
    a1, j1 = rng.normal(size=(2, 4, 3))
    bad = [
        dict(ids=np.array([0, n], dtype=np.int32)),                   # id past the arrays
        dict(ids=np.array([-1], dtype=np.int32), a1=a1[:1], j1=j1[:1]),
        dict(dt=dt[:-1]),                                             # short dt
        dict(x=x.astype(np.float32)),                                 # float32
        dict(v=np.asfortranarray(v)),                                 # not C-contiguous
        dict(a1=a1[:3]),                                              # one acc row short
    ]
    for b in bad:
        args = dict(ids=ids, t0=t0, dt=dt, x=x, v=v, a=a, j=j, a1=a1, j1=j1)
        args.update(b)
        with pytest.raises(ValueError):
            B.correct(args["ids"], 1.0 / 64, 0.01, 1.0 / 8, args["t0"], args["dt"], args["x"], args["v"], args["a"],
                      args["j"], args["a1"], args["j1"])
    for w, g in zip(keep, (t0, dt, x, v, a, j)):
        assert np.array_equal(w, g)
    with pytest.raises(ValueError):
        B.next_block(t0, dt.astype(np.float32))
    with pytest.raises(ValueError):
        B.next_block(t0, dt, out=np.empty(n - 1, np.int32))
    tn, act = B.next_block(t0, dt)
    assert tn == 1.0 / 64 and np.array_equal(act, np.arange(n))


def test_next_block_many_matches_definition():
    """Batched next block (chunked across threads) vs the definition, per cluster:
    t_next = min(t0 + dt), the due particles in ascending order."""
    cls = _clusters(SIZES, 5)
    S = _structs(cls)
    B.next_block_many(S)
    for k, c in enumerate(cls):
        t = c["t0"] + c["dt"]
        want = np.flatnonzero(t == t.min())
        assert S[k].t_next == t.min()
        assert S[k].n_active == want.size and np.array_equal(c["act"][:want.size], want)


def test_correct_many_matches_per_cluster_corrector():
    """Batched corrector (one loop over all clusters' particles) vs the
    single-cluster corrector: same bits, rows of the corrected particles, and
    rebuild flags at tree times."""
    cls = _clusters(SIZES, 6)
    ref = [{f: (c[f].copy() if isinstance(c[f], np.ndarray) else c[f]) for f in c} for c in cls]
    S = _structs(cls)
    B.next_block_many(S)
    rng = np.random.default_rng(7)
    n_act = np.array([S[k].n_active for k in range(len(cls))], dtype=np.int64)
    off = np.zeros(len(cls), np.int64)
    np.cumsum(n_act[:-1], out=off[1:])
    total = int(n_act.sum())
    acc = rng.normal(size=(total, 3))
    jerk = rng.normal(size=(total, 3))
    pot = rng.normal(size=total)
    rows = np.zeros(total, B.HT_ROW)
    rebuild = np.zeros(len(cls), np.int32)
    B.correct_many(S, off, acc, jerk, pot, off, rows, rebuild)
    for k, (c, r) in enumerate(zip(cls, ref)):
        ids = c["act"][:n_act[k]].copy()
        o, e = off[k], off[k] + n_act[k]
        B.correct(ids, S[k].t_next, 0.01, 1.0 / 8, r["t0"], r["dt"], r["x"], r["v"], r["a"], r["j"], acc[o:e],
                  jerk[o:e])
        for f in ("t0", "dt", "x", "v", "a", "j"):
            assert np.array_equal(c[f], r[f]), (k, f)
        assert np.array_equal(c["pot"][ids], pot[o:e])
        at_tree_time = S[k].t_next % (1.0 / 8) == 0.0
        assert rebuild[k] == at_tree_time
        if not at_tree_time:
            w = rows[o:e]
            assert np.array_equal(w["idx"], ids) and np.array_equal(w["x"], r["x"][ids])
            assert np.array_equal(w["t0"], r["t0"][ids]) and np.array_equal(w["m"], r["m"][ids])
            assert np.array_equal(w["jerk"], r["j"][ids])
