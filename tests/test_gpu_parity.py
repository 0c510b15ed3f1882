"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle.

The oracle integrates; at each block step the j-memory state it used (its
particles, its nodes, lists rebuilt by the product builder and checked
bit-identical to the oracle's) is loaded into GPU contexts, predicted and
summed, and compared element by element with the oracle's forces.

Tolerances (per particle, relative to that particle's own magnitude):
  FP64 form   acc, jerk, pot <= 1e-12
  mixed form  acc <= 2e-6, jerk <= 1e-5, pot <= 1e-6
"""
import numpy as np
import pytest
from paper_1602_02832_amd import binding as B
from paper_1602_02832_amd import workloads as W

from parity_util import TOL, assert_close, errors, oracle_list_force, rel_rows, say  # noqa: F401

pytestmark = pytest.mark.gpu


def make_ctx(prec, n, node_max, group_max, list_max, eps2, mode="fused"):
    return B.Context(n_max=n, node_max=node_max, group_max=group_max, list_max=list_max, active_max=n, eps2=eps2,
                     precision=prec, predict_mode=mode)


class Replayer:
    """Loads an oracle run's j-memory into GPU contexts and checks each step."""

    def __init__(self, oracle, sim, precs, modes=("fused",), list_max=None):
        self.O, self.sim = oracle, sim
        n = sim.n
        lm = list_max or max(4 * sim.tree.n_entries, 4096)
        self.ctxs = {(p, md): make_ctx(p, n, 4 * n + 64, n, lm, sim.eps2, md) for p in precs for md in modes}
        self.tree_seen = None
        self.pending = None
        self.worst = {k: (0.0, 0.0, 0.0) for k in self.ctxs}
        self.steps = 0
        self.sync_tree()

    def sync_tree(self):
        sim = self.sim
        if sim.tree is self.tree_seen:
            return
        got = B.HostTree(sim.x, sim.v, sim.a, sim.j, sim.m, sim.n_leaf, sim.n_crit, sim.theta)
        assert np.array_equal(got.perm, np.arange(sim.n))
        for f in ("node_m", "node_x", "node_v", "node_a", "node_j", "group_first", "list_off", "entries"):
            assert np.array_equal(getattr(got, f), getattr(sim.tree, f)), f"product {f} differs at t={sim.t}"
        for c in self.ctxs.values():
            c.set_j_particles(sim.t0, sim.m, sim.x, sim.v, sim.a, sim.j)
            c.set_nodes(sim.t_tree, got.node_m, got.node_x, got.node_v, got.node_a, got.node_j)
            c.set_interaction_lists(got.group_first, got.list_off, got.entries)
        self.tree_seen = sim.tree
        self.pending = None

    def hook(self, sim, rec):
        want = (rec["acc"], rec["jerk"], rec["pot"])
        # the j-memory update of step 6: the particles the oracle corrected since
        # the last step (a full upload follows every rebuild)
        upd = self.pending
        self.pending = rec["active"].copy()
        for (p, md), c in self.ctxs.items():
            if upd is None:
                c.set_j_particles(sim.t0, sim.m, sim.x, sim.v, sim.a, sim.j)
            else:
                c.set_j_particles(sim.t0[upd], sim.m[upd], sim.x[upd], sim.v[upd], sim.a[upd], sim.j[upd], idx=upd)
            c.predict(rec["t"])
            got = c.force(rec["active"])
            e = assert_close(f"t={rec['t']} n_active={rec['active'].size}", p, got, want)
            self.worst[(p, md)] = tuple(max(a, b) for a, b in zip(self.worst[(p, md)], e))
        self.steps += 1

    def run(self, t_end):
        while self.sim.next_time() <= t_end:
            self.sim.step()
            self.sync_tree()
        return self


# ------------------------------------------------------------------------------------------ predictor
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_predictor_matches_oracle(oracle, prec):
    say(f"predictor {prec}")
    n = 5000
    x, v, m = W.plummer(n, 31)
    t_now = 37.0 / 256
    t0, a, j = W.random_block_state(n, 32, t_now)
    if prec == "mixed":   # the mixed form stores a and jerk in FP32
        a, j = a.astype(np.float32).astype(np.float64), j.astype(np.float32).astype(np.float64)
    c = make_ctx(prec, n, 16, 1, 16, 1e-4)
    c.set_j_particles(t0, m, x, v, a, j)
    c.set_nodes(0.0, np.zeros(0), *(np.zeros((0, 3)) for _ in range(4)))
    c.predict(t_now)
    xp, vp = c.get_predicted(np.arange(n, dtype=np.int32))
    wx, wv = oracle.predict(t_now, t0, x, v, a, j)
    assert np.max(np.abs(xp - wx)) <= 1e-15 * np.max(np.abs(wx)) * 4
    assert np.max(np.abs(vp - wv)) <= 1e-15 * np.max(np.abs(wv)) * 4


# ------------------------------------------------------------------------------------------ C1, every step
def test_parity_plummer2k_every_block_step(oracle):
    c = W.config("plummer2k")
    say(f"plummer2k every block step to t={c.t_end}")
    x, v, m = W.make_initial_conditions(c)
    rp = {}

    def hook(sim, rec):
        rp["r"].hook(sim, rec)

    sim = oracle.TreeHermite(x, v, m, eps2=c.eps2, dt_tree=c.dt_tree, eta=c.eta, theta=c.theta, n_crit=c.n_crit,
                             on_step=hook)
    rp["r"] = Replayer(oracle, sim, ("fp64", "mixed"), modes=("fused", "eager"))
    rp["r"].run(c.t_end)
    say(f"steps {rp['r'].steps} worst {rp['r'].worst}")
    assert rp["r"].steps > 100 and sim.t == c.t_end


# ------------------------------------------------------------------------------------------ C2, every step
def test_parity_plummer16k_every_block_step(oracle):
    """C2 over its whole span (t <= 1/4: 64 tree intervals, about 6200 block
    steps): every block step of the oracle's run replayed in both forms."""
    c = W.config("plummer16k")
    say(f"plummer16k every block step to t={c.t_end}")
    x, v, m = W.make_initial_conditions(c)
    rp = {}

    def hook(sim, rec):
        rp["r"].hook(sim, rec)

    sim = oracle.TreeHermite(x, v, m, eps2=c.eps2, dt_tree=c.dt_tree, eta=c.eta, theta=c.theta, n_crit=c.n_crit,
                             on_step=hook)
    rp["r"] = Replayer(oracle, sim, ("fp64", "mixed"))
    rp["r"].run(c.t_end)
    say(f"steps {rp['r'].steps} worst {rp['r'].worst}")
    assert sim.t == c.t_end and rp["r"].steps > 6000


# ------------------------------------------------------------------------------------------ direct
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_direct_matches_oracle(oracle, prec):
    say(f"direct {prec}")
    n = 3000
    x, v, m = W.plummer(n, 41)
    m = W.salpeter_masses(n, 42)
    t0, a, j = W.random_block_state(n, 43, 0.25)
    c = make_ctx(prec, n, 16, 1, 16, 1e-5)
    c.set_j_particles(t0, m, x, v, a, j)
    c.set_nodes(0.0, np.zeros(0), *(np.zeros((0, 3)) for _ in range(4)))
    c.predict(0.25)
    if prec == "mixed":
        a, j = a.astype(np.float32).astype(np.float64), j.astype(np.float32).astype(np.float64)
        m32 = m.astype(np.float32).astype(np.float64)
    else:
        m32 = m
    xp, vp = oracle.predict(0.25, t0, x, v, a, j)
    for ids in (np.arange(n), np.array([0]), np.arange(5, 3000, 7), np.arange(1, 258), np.array([n - 1])):
        ids = ids.astype(np.int32)
        got = c.force_direct(ids)
        want = oracle.force_direct(ids, xp, vp, m32, 1e-5)
        assert_close(f"direct n_active={ids.size}", prec, got, want)


# ------------------------------------------------------------------------------------------ tiles and edges
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_ragged_tiles_and_sparse_sets(oracle, prec):
    """Active sets whose per-group counts hit every tile size and its edges."""
    say(f"ragged tiles {prec}")
    n = 6000
    x, v, m = W.plummer(n, 51)
    z = np.zeros((n, 3))
    tr = oracle.Tree(x, v, z, z, m, 1, 700, 0.6)
    x, v, m = x[tr.perm], v[tr.perm], m[tr.perm]
    t0, a, j = W.random_block_state(n, 52, 5.0 / 128)
    ptr = B.HostTree(x, v, z, z, m, 1, 700, 0.6)
    assert np.array_equal(ptr.entries, tr.entries)
    c = make_ctx(prec, n, 2 * n, n, 2 * tr.n_entries, 1e-4)
    c.set_j_particles(t0, m, x, v, a, j)
    c.set_nodes(0.0, ptr.node_m, ptr.node_x, ptr.node_v, ptr.node_a, ptr.node_j)
    c.set_interaction_lists(ptr.group_first, ptr.list_off, ptr.entries)
    c.predict(5.0 / 128)
    if prec == "mixed":
        a, j = a.astype(np.float32).astype(np.float64), j.astype(np.float32).astype(np.float64)
        mj = np.concatenate([m, ptr.node_m]).astype(np.float32).astype(np.float64)
        na = ptr.node_a.astype(np.float32).astype(np.float64)
        nj = ptr.node_j.astype(np.float32).astype(np.float64)
    else:
        mj = np.concatenate([m, ptr.node_m])
        na, nj = ptr.node_a, ptr.node_j
    xp, vp = oracle.predict(5.0 / 128, t0, x, v, a, j)
    nxp, nvp = oracle.predict(5.0 / 128, 0.0, ptr.node_x, ptr.node_v, na, nj)
    XP, VP = np.vstack([xp, nxp]), np.vstack([vp, nvp])
    gf = ptr.group_first
    rng = np.random.default_rng(9)
    counts = [1, 2, 3, 5, 15, 17, 31, 33, 63, 64, 65, 127, 129, 255, 256, 257, 511, 513]
    sel = []
    for g in range(ptr.n_group):
        size = gf[g + 1] - gf[g]
        k = min(size, counts[g % len(counts)])
        sel.append(np.sort(rng.choice(np.arange(gf[g], gf[g + 1]), k, replace=False)))
    for ids in (np.concatenate(sel), np.arange(n), np.array([17]), np.arange(0, n, 97)):
        ids = ids.astype(np.int32)
        got = c.force(ids)
        want = oracle.force_list(ids, XP, VP, mj, 1e-4, gf, ptr.list_off, ptr.entries)
        assert_close(f"ragged n_active={ids.size}", prec, got, want)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_tiny_systems(oracle, prec):
    """N = 1 (no partner), N = 2 (exact two-body) and coincident particles."""
    say(f"tiny systems {prec}")
    for name, x in (("n1", np.array([[0.1, 0.2, 0.3]])), ("n2", np.array([[0.0, 0.0, 0.0], [0.5, 0.25, -0.125]])),
                    ("coincident", np.array([[0.0, 0, 0], [0.0, 0, 0], [1.0, 0, 0], [1.0, 0, 0], [0.5, 0.5, 0.5]]))):
        n = x.shape[0]
        v = np.arange(3 * n, dtype=np.float64).reshape(n, 3) * 0.125
        m = np.full(n, 0.5)
        z = np.zeros((n, 3))
        ptr = B.HostTree(x, v, z, z, m, 1, 2, 0.5)
        xs, vs = x[ptr.perm], v[ptr.perm]
        c = make_ctx(prec, n, 8 * n + 64, n, 64, 0.01)
        c.set_j_particles(0.0, m, xs, vs, z, z)
        c.set_nodes(0.0, ptr.node_m, ptr.node_x, ptr.node_v, ptr.node_a, ptr.node_j)
        c.set_interaction_lists(ptr.group_first, ptr.list_off, ptr.entries)
        c.predict(0.0)
        ids = np.arange(n, dtype=np.int32)
        got = c.force(ids)
        XP = np.vstack([xs, ptr.node_x])
        VP = np.vstack([vs, ptr.node_v])
        want = oracle.force_list(ids, XP, VP, np.concatenate([m, ptr.node_m]), 0.01, ptr.group_first, ptr.list_off,
                                 ptr.entries)
        if name == "n1":
            for g in got:
                assert np.all(g == 0.0)
        else:
            assert_close(name, prec, got, want)
        assert all(np.all(np.isfinite(g)) for g in got)


def test_zero_softening_two_body(oracle):
    say("eps = 0 two body")
    x = np.array([[-0.25, 0, 0], [0.25, 0, 0]])
    v = np.array([[0, -0.5, 0], [0, 0.5, 0.0]])
    m = np.array([0.5, 0.5])
    z = np.zeros((2, 3))
    for prec in ("fp64", "mixed"):
        c = make_ctx(prec, 2, 64, 2, 64, 0.0)
        c.set_j_particles(0.0, m, x, v, z, z)
        c.set_nodes(0.0, np.zeros(0), *(np.zeros((0, 3)) for _ in range(4)))
        c.set_interaction_lists([0, 2], [0, 2], [0, 1])
        c.predict(0.0)
        acc, jerk, pot = c.force(np.array([0, 1], dtype=np.int32))
        assert np.allclose(acc, [[2.0, 0, 0], [-2.0, 0, 0]], rtol=1e-6)
        assert np.allclose(pot, [-1.0, -1.0], rtol=1e-6)


def test_api_errors():
    say("api errors")
    n = 64
    x, v, m = W.plummer(n, 3)
    z = np.zeros((n, 3))
    c = make_ctx("fp64", n, 4 * n, n, 8192, 1e-4)
    with pytest.raises(B.HTError) as e:
        c.predict(0.0)
    assert e.value.code == -4
    c.set_j_particles(0.0, m, x, v, z, z)
    with pytest.raises(B.HTError) as e:
        c.force(np.array([0], dtype=np.int32))
    assert e.value.code == -4
    ptr = B.HostTree(x, v, z, z, m, 1, 8, 0.5)
    c.set_j_particles(0.0, m[ptr.perm], x[ptr.perm], v[ptr.perm], z, z)
    c.set_nodes(0.0, ptr.node_m, ptr.node_x, ptr.node_v, ptr.node_a, ptr.node_j)
    bad = ptr.entries.copy()
    bad[3] = n + ptr.n_node
    with pytest.raises(B.HTError) as e:
        c.set_interaction_lists(ptr.group_first, ptr.list_off, bad)
    assert e.value.code == -2
    c.set_interaction_lists(ptr.group_first, ptr.list_off, ptr.entries)
    with pytest.raises(B.HTError) as e:
        c.force(np.array([0], dtype=np.int32))   # not predicted yet
    assert e.value.code == -4
    c.predict(0.0)
    for ids, code in (([3, 2], -1), ([1, 1], -1), ([n], -1), ([-1], -1)):
        with pytest.raises(B.HTError) as e:
            c.force(np.array(ids, dtype=np.int32))
        assert e.value.code == code
    acc, jerk, pot = c.force(np.zeros(0, dtype=np.int32))
    assert acc.shape == (0, 3)
    with pytest.raises(B.HTError) as e:
        c.set_j_particles(0.0, m[:2], x[:2], v[:2], z[:2], z[:2], idx=np.array([5, 5], dtype=np.int32))
    assert e.value.code == -1
    with pytest.raises(B.HTError) as e:
        c.set_interaction_lists(ptr.group_first[::-1].copy(), ptr.list_off, ptr.entries)
    assert e.value.code == -1


def test_capacities_and_list_checks(oracle):
    """Sizes beyond the context's capacities are refused with HT_ERANGE
    (particles, nodes, groups, list entries) and malformed lists with
    HT_EINVAL (offsets not starting at 0 or decreasing, groups not covering
    0..N), all before anything is copied: the lists set before the refusals
    stay in force and the forces still match the oracle.  Arrays of
    mismatched lengths are refused by the binding before the call."""
    say("capacities and list checks")
    n = 300
    x, v, m = W.plummer(n, 5)
    z = np.zeros((n, 3))
    ptr = B.HostTree(x, v, z, z, m, 1, 24, 0.5)
    x, v, m = x[ptr.perm], v[ptr.perm], m[ptr.perm]
    t0, a, j = W.random_block_state(n, 6, 0.125)
    G, M, L = ptr.n_group, ptr.n_node, ptr.n_entries
    assert G >= 2
    c = make_ctx("fp64", n, M, G, L, 1e-4)
    xn, vn, mn = np.vstack([x, x[:1]]), np.vstack([v, v[:1]]), np.concatenate([m, m[:1]])
    codes = []

    def refused(call, *args):
        with pytest.raises(B.HTError) as e:
            call(*args)
        codes.append(e.value.code)

    refused(c.set_j_particles, 0.0, mn, xn, vn, np.zeros((n + 1, 3)), np.zeros((n + 1, 3)))   # n_max + 1
    c.set_j_particles(t0, m, x, v, a, j)
    nm = np.concatenate([ptr.node_m, ptr.node_m[:1]])
    n3 = [np.vstack([u, u[:1]]) for u in (ptr.node_x, ptr.node_v, ptr.node_a, ptr.node_j)]
    refused(c.set_nodes, 0.0, nm, *n3)                                                          # node_max + 1
    c.set_nodes(0.0, ptr.node_m, ptr.node_x, ptr.node_v, ptr.node_a, ptr.node_j)
    gf, lo, en = ptr.group_first, ptr.list_off, ptr.entries
    c.set_interaction_lists(gf, lo, en)
    # one group split in two: G + 1 groups (each keeps a valid list)
    g0 = int(np.argmax(np.diff(gf) >= 2))
    gf2 = np.insert(gf, g0 + 1, gf[g0] + 1)
    lo2 = np.insert(lo, g0 + 1, lo[g0 + 1])
    refused(c.set_interaction_lists, gf2, lo2, en)                                             # group_max + 1
    lo3 = lo.copy()
    lo3[-1] += 1
    refused(c.set_interaction_lists, gf, lo3, np.concatenate([en, en[:1]]))                    # list_max + 1
    assert codes == [-2, -2, -2, -2], codes
    codes.clear()
    lo4 = lo.copy()
    lo4[0] = 1
    refused(c.set_interaction_lists, gf, lo4, en)                                              # offsets from 1
    lo5 = lo.copy()
    lo5[1], lo5[2] = lo[2], lo[1]
    refused(c.set_interaction_lists, gf, lo5, en)                                              # decreasing
    gf6 = gf.copy()
    gf6[-1] = n - 1
    refused(c.set_interaction_lists, gf6, lo, en)                                              # not up to N
    assert codes == [-1, -1, -1], codes
    with pytest.raises(ValueError):
        c.set_interaction_lists(gf, lo[:-1], en)
    with pytest.raises(ValueError):
        c.set_interaction_lists(gf, lo, en[:-1])
    # the lists set before the refusals are still in force
    c.predict(0.125)
    ids = np.arange(0, n, 3, dtype=np.int32)
    got = c.force(ids)
    want = oracle_list_force(oracle, 0.125, ids, t0, m, x, v, a, j, ptr, 1e-4)
    assert_close("after refusals", "fp64", got, want)


def test_binding_refuses_mismatched_tensors():
    """Device tensors handed to the binding are checked before the call (the
    library reads counts the tensors must hold): too few elements, the wrong
    dtype, a non-contiguous view or host memory raise ValueError and nothing
    runs; the same call with proper tensors goes through."""
    import torch
    say("binding tensor checks")
    n = 128
    x, v, m = W.plummer(n, 9)
    z = np.zeros((n, 3))
    c = make_ctx("fp64", n, 0, 1, 1, 1e-4)
    c.set_j_particles(0.0, m, x, v, z, z)
    c.set_nodes(0.0, np.zeros(0), *(np.zeros((0, 3)) for _ in range(4)))
    c.predict(0.0)
    ids = np.arange(0, n, 2, dtype=np.int32)
    k = ids.size
    f64 = dict(dtype=torch.float64, device="cuda")
    good = (torch.empty((k, 3), **f64), torch.empty((k, 3), **f64), torch.empty(k, **f64))
    bad_outs = [
        (torch.empty((k - 1, 3), **f64), good[1], good[2]),                 # too short
        (good[0], good[1].float(), good[2]),                                 # float32
        (good[0], torch.empty((3, 2 * k), **f64).t()[:k], good[2]),          # non-contiguous
        (good[0], good[1], torch.empty(k, dtype=torch.float64)),             # host memory
    ]
    for outs in bad_outs:
        with pytest.raises(ValueError):
            c.force_direct_async(ids, *outs)
        with pytest.raises(ValueError):
            c.step_async(None, 0.0, ids, *outs)
    dev = lambda u, dt=torch.float64: torch.from_numpy(np.ascontiguousarray(u)).to(device="cuda", dtype=dt)  # noqa: E731
    rows = (dev(np.arange(4), torch.int32), dev(np.zeros(4)), dev(m[:4]), dev(x[:4]), dev(v[:4]), dev(z[:4]),
            dev(z[:4]))
    with pytest.raises(ValueError):
        c.set_j_particles_async(5, *rows)                                    # 5 rows from 4-row tensors
    with pytest.raises(ValueError):
        c.set_j_particles_async(4, rows[0].long(), *rows[1:])                # int64 indices
    with pytest.raises(ValueError):
        c.set_j_particles(0.0, m[:4], x[:4], v[:4], z[:4], z[:4], idx=np.arange(3, dtype=np.int32))
    c.set_j_particles_async(4, *rows)
    c.predict(0.0)
    c.force_direct_async(ids, *good)
    c.sync()
    want = c.force_direct(ids)
    for p_, q_ in zip(good, want):
        assert np.array_equal(p_.cpu().numpy(), q_)


@pytest.mark.parametrize("path", ["async", "step", "graph"])
def test_device_rows_out_of_range_are_dropped_and_reported(path):
    """Update rows whose particle indices sit in device memory are checked by
    the kernel that writes them: rows naming an index outside [0, N) are
    dropped, the others are written, and the next synchronising call returns
    HT_ERANGE once.  The bad indices used here (N and N + M - 1, node
    records) lie inside the records array, so even an unchecked write could
    not leave the allocation."""
    import torch
    say(f"device update rows out of range ({path})")
    n = 500
    x, v, m = W.plummer(n, 7)
    z = np.zeros((n, 3))
    ptr = B.HostTree(x, v, z, z, m, 1, 32, 0.5)
    x, v, m = x[ptr.perm], v[ptr.perm], m[ptr.perm]
    t0, a, j = W.random_block_state(n, 8, 0.25)
    ctxs = []
    for _ in range(2):
        c = make_ctx("mixed", n, 2 * n, n, 2 * ptr.n_entries, 1e-4)
        c.set_j_particles(t0, m, x, v, a, j)
        c.set_nodes(0.0, ptr.node_m, ptr.node_x, ptr.node_v, ptr.node_a, ptr.node_j)
        c.set_interaction_lists(ptr.group_first, ptr.list_off, ptr.entries)
        ctxs.append(c)
    got_ctx, ref_ctx = ctxs
    idx = np.array([3, n, 10, n + ptr.n_node - 1], dtype=np.int32)
    good = np.array([0, 2])
    ut0 = np.full(4, 0.25)
    ux = x[np.minimum(idx, n - 1)] + 1e-3
    dev = lambda u: torch.from_numpy(np.ascontiguousarray(u)).cuda()  # noqa: E731
    upd = (4, dev(idx), dev(ut0), dev(m[:4]), dev(ux), dev(v[:4]), dev(a[:4]), dev(j[:4]))
    act = np.array([0, 3, 10, 77], dtype=np.int32)
    out = tuple(torch.empty(sh, dtype=torch.float64, device="cuda") for sh in ((4, 3), (4, 3), (4,)))
    t = 0.28125
    if path == "async":
        got_ctx.set_j_particles_async(*upd)
        got_ctx.predict(t)
    elif path == "step":
        got_ctx.step_async(upd, t, act, *out)
    else:
        got_ctx.step_graph(upd, t, act, *out)
    with pytest.raises(B.HTError) as e:
        got_ctx.sync()
    assert e.value.code == -2
    got_ctx.sync()                     # reported once
    ref_ctx.set_j_particles(ut0[good], m[:4][good], ux[good], v[:4][good], a[:4][good], j[:4][good],
                            idx=idx[good])
    ref_ctx.predict(t)
    probe = np.array([0, 3, 10, n - 1, n, n + ptr.n_node - 1], dtype=np.int32)
    for p_got, p_ref in zip(got_ctx.get_predicted(probe), ref_ctx.get_predicted(probe)):
        assert np.array_equal(p_got, p_ref)
    if path != "async":
        want = ref_ctx.force(act)
        for g, w in zip(out, want):
            assert np.array_equal(g.cpu().numpy(), w)


# ------------------------------------------------------------------------------------------ batch
def test_batch_equals_alone(oracle):
    """Several clusters in one launch give bit-identical results to each alone."""
    import torch
    say("batched launch vs alone")
    s = torch.cuda.Stream()
    sizes = [300, 1000, 2500, 64]
    ctxs, acts, state = [], [], []
    for k, n in enumerate(sizes):
        x, v, m = W.plummer(n, 60 + k)
        m = W.salpeter_masses(n, 65 + k)
        z = np.zeros((n, 3))
        ptr = B.HostTree(x, v, z, z, m, 1, 64, 0.5)
        x, v, m = x[ptr.perm], v[ptr.perm], m[ptr.perm]
        t0, a, j = W.random_block_state(n, 70 + k, 0.125)
        state.append((t0, m, x, v, a, j, ptr))
        c = B.Context(n_max=n, node_max=2 * n, group_max=n, list_max=2 * ptr.n_entries + 64, active_max=n,
                      eps2=1e-4, precision="mixed", stream=s.cuda_stream)
        c.set_j_particles(t0, m, x, v, a, j)
        c.set_nodes(0.0, ptr.node_m, ptr.node_x, ptr.node_v, ptr.node_a, ptr.node_j)
        c.set_interaction_lists(ptr.group_first, ptr.list_off, ptr.entries)
        c.predict(0.125)
        ctxs.append(c)
        acts.append(np.sort(np.random.default_rng(k).choice(n, max(1, n // (k + 2)), replace=False)).astype(np.int32))
    alone = [c.force(a) for c, a in zip(ctxs, acts)]
    outs = [(torch.empty((a.size, 3), dtype=torch.float64, device="cuda"),
             torch.empty((a.size, 3), dtype=torch.float64, device="cuda"),
             torch.empty(a.size, dtype=torch.float64, device="cuda")) for a in acts]
    keep = B.force_batch_async(ctxs, acts, [o[0] for o in outs], [o[1] for o in outs], [o[2] for o in outs])
    ctxs[0].sync()
    del keep
    for (a1, j1, p1), (a2, j2, p2) in zip(alone, outs):
        assert np.array_equal(a1, a2.cpu().numpy())
        assert np.array_equal(j1, j2.cpu().numpy())
        assert np.array_equal(p1, p2.cpu().numpy())
    # each cluster's batched result against the FP64 oracle (unrounded inputs)
    for k, ((t0, m, x, v, a, j, ptr), act, out) in enumerate(zip(state, acts, outs)):
        want = oracle_list_force(oracle, 0.125, act, t0, m, x, v, a, j, ptr, 1e-4)
        assert_close(f"batched cluster {k} (n={sizes[k]}, {act.size} active)", "mixed",
                     tuple(o.cpu().numpy() for o in out), want)


def test_step_async_equals_separate_calls(oracle):
    """ht_step_async (update + predict + force in one call) gives the same bits
    as the three separate calls, and matches the oracle."""
    import torch
    say("step_async vs separate calls")
    n = 4000
    x, v, m = W.plummer(n, 81)
    z = np.zeros((n, 3))
    ptr = B.HostTree(x, v, z, z, m, 1, 128, 0.5)
    x, v, m = x[ptr.perm], v[ptr.perm], m[ptr.perm]
    t0, a, j = W.random_block_state(n, 82, 0.25)
    ctxs = []
    for _ in range(2):
        c = make_ctx("mixed", n, 2 * n, n, 2 * ptr.n_entries, 1e-4)
        c.set_j_particles(t0, m, x, v, a, j)
        c.set_nodes(0.0, ptr.node_m, ptr.node_x, ptr.node_v, ptr.node_a, ptr.node_j)
        c.set_interaction_lists(ptr.group_first, ptr.list_off, ptr.entries)
        ctxs.append(c)
    rng = np.random.default_rng(83)
    upd_ids = np.sort(rng.choice(n, 300, replace=False)).astype(np.int32)
    nt0 = np.full(300, 0.25)
    nx = x[upd_ids] + 1e-3
    dev = lambda u: torch.from_numpy(np.ascontiguousarray(u)).cuda()  # noqa: E731
    upd = (300, dev(upd_ids), dev(nt0), dev(m[upd_ids]), dev(nx), dev(v[upd_ids]), dev(a[upd_ids]), dev(j[upd_ids]))
    act = np.sort(rng.choice(n, 700, replace=False)).astype(np.int32)
    outs = [tuple(torch.empty(s, dtype=torch.float64, device="cuda") for s in ((700, 3), (700, 3), (700,)))
            for _ in range(2)]
    ctxs[0].step_async(upd, 0.3125, act, *outs[0])
    ctxs[0].sync()
    ctxs[1].set_j_particles_async(*upd)
    ctxs[1].predict(0.3125)
    ctxs[1].force_async(act, *outs[1])
    ctxs[1].sync()
    for p, q in zip(outs[0], outs[1]):
        assert torch.equal(p, q)
    # against the oracle on the updated state
    t0u, xu = t0.copy(), x.copy()
    t0u[upd_ids] = 0.25
    xu[upd_ids] = nx
    f32 = lambda u: u.astype(np.float32).astype(np.float64)  # noqa: E731
    xp, vp = oracle.predict(0.3125, t0u, xu, v, f32(a), f32(j))
    nxp, nvp = oracle.predict(0.3125, 0.0, ptr.node_x, ptr.node_v, f32(ptr.node_a), f32(ptr.node_j))
    want = oracle.force_list(act, np.vstack([xp, nxp]), np.vstack([vp, nvp]), f32(np.concatenate([m, ptr.node_m])),
                             1e-4, ptr.group_first, ptr.list_off, ptr.entries)
    assert_close("step_async", "mixed", tuple(o.cpu().numpy() for o in outs[0]), want)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_step_graph_replays_equal_step_async(prec):
    """ht_step_graph replays the captured step graphs (two, alternating) with a
    new plan, update and active set every step; every replay must give the
    bits of ht_step_async on the same sequence, with eager work and
    synchronisations between replays, and sets from one particle to all of
    them (many split tiles, none, a reduce launch that has nothing to do)."""
    import torch
    say(f"step_graph replays vs step_async ({prec})")
    n = 6000
    x, v, m = W.plummer(n, 91)
    z = np.zeros((n, 3))
    ptr = B.HostTree(x, v, z, z, m, 1, 128, 0.5)
    x, v, m = x[ptr.perm], v[ptr.perm], m[ptr.perm]
    t0, a, j = W.random_block_state(n, 92, 0.25)
    ctxs = []
    for _ in range(2):
        c = make_ctx(prec, n, 2 * n, n, 2 * ptr.n_entries, 1e-4)
        c.set_j_particles(t0, m, x, v, a, j)
        c.set_nodes(0.0, ptr.node_m, ptr.node_x, ptr.node_v, ptr.node_a, ptr.node_j)
        c.set_interaction_lists(ptr.group_first, ptr.list_off, ptr.entries)
        ctxs.append(c)
    rng = np.random.default_rng(93)
    dev = lambda u: torch.from_numpy(np.ascontiguousarray(u)).cuda()  # noqa: E731
    sizes = [1, 700, 3, n, 40, 2, 1500, 5, n // 2, 1, 90, 260]
    t = 0.25
    prev = None
    for step, k in enumerate(sizes):
        t += 1.0 / 64
        act = np.sort(rng.choice(n, k, replace=False)).astype(np.int32)
        outs = [tuple(torch.full(s, float("nan"), dtype=torch.float64, device="cuda") for s in ((k, 3), (k, 3), (k,)))
                for _ in range(2)]
        ctxs[0].step_async(prev, t, act, *outs[0])
        ctxs[1].step_graph(prev, t, act, *outs[1])
        if step % 3 == 0:
            torch.cuda.synchronize()
            scratch = torch.randn(1 << 20, device="cuda").sum()   # eager work between replays
            del scratch
        ctxs[0].sync()
        ctxs[1].sync()
        for p, q in zip(outs[0], outs[1]):
            assert torch.equal(p, q), (step, k)
        # this step's active particles, moved a little, are the next step's update
        nu = act.size
        upd_x = x[act] + 1e-4 * (step + 1)
        prev = (nu, dev(act), dev(np.full(nu, t)), dev(m[act]), dev(upd_x), dev(v[act]), dev(a[act]), dev(j[act]))
    with pytest.raises(B.HTError):
        eager = make_ctx(prec, n, 2 * n, n, 2 * ptr.n_entries, 1e-4, mode="eager")
        eager.set_j_particles(t0, m, x, v, a, j)
        eager.set_nodes(0.0, ptr.node_m, ptr.node_x, ptr.node_v, ptr.node_a, ptr.node_j)
        eager.set_interaction_lists(ptr.group_first, ptr.list_off, ptr.entries)
        out = tuple(torch.empty(s, dtype=torch.float64, device="cuda") for s in ((1, 3), (1, 3), (1,)))
        eager.step_graph(None, t, np.array([0], np.int32), *out)


# ------------------------------------------------------------------------------------------ run-length lists
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_run_length_lists_equal_csr(oracle, prec):
    """Run-length lists with per-group node copies (ht_set_list_form RUNS): the
    same work items over the same records in the same order, so every output
    equals the CSR form's bit for bit, for active sets that hit every tile size
    (round boundaries inside runs, runs longer than a round, single-entry
    runs), through a j-memory update and prediction in one call; and the
    oracle agrees."""
    import torch
    say(f"run-length lists vs CSR ({prec})")
    n = 7000
    x, v, m = W.plummer(n, 61)
    m = W.salpeter_masses(n, 62)
    z = np.zeros((n, 3))
    ptr = B.HostTree(x, v, z, z, m, 1, 300, 0.5)
    x, v, m = x[ptr.perm], v[ptr.perm], m[ptr.perm]
    t0, a, j = W.random_block_state(n, 63, 0.25)
    ctxs = {}
    for form in ("csr", "runs"):
        c = make_ctx(prec, n, 2 * n, n, 2 * ptr.n_entries, 1e-4)
        c.set_list_form(form)
        c.set_j_particles(t0, m, x, v, a, j)
        c.set_nodes(0.0, ptr.node_m, ptr.node_x, ptr.node_v, ptr.node_a, ptr.node_j)
        c.set_interaction_lists(ptr.group_first, ptr.list_off, ptr.entries)
        ctxs[form] = c
    gf = ptr.group_first
    # the mixed form stores a, jerk and m in FP32: the oracle gets them so
    r = (lambda u: u.astype(np.float32).astype(np.float64)) if prec == "mixed" else (lambda u: u)
    rng = np.random.default_rng(64)
    counts = [1, 2, 3, 7, 9, 17, 33, 64, 65, 129, 257]
    sel = [np.sort(rng.choice(np.arange(gf[g], gf[g + 1]), min(gf[g + 1] - gf[g], counts[g % len(counts)]),
                              replace=False)) for g in range(ptr.n_group)]
    dev = lambda u: torch.from_numpy(np.ascontiguousarray(u)).cuda()  # noqa: E731
    t = 0.25
    for step, ids in enumerate((np.concatenate(sel), np.arange(n), np.array([5]), np.arange(0, n, 13))):
        ids = ids.astype(np.int32)
        got = {}
        for form, c in ctxs.items():
            c.predict(t)
            got[form] = c.force(ids)
        for p_, q_ in zip(got["csr"], got["runs"]):
            assert np.array_equal(p_, q_), (prec, step)
        xp, vp = oracle.predict(t, t0, x, v, r(a), r(j))
        nxp, nvp = oracle.predict(t, 0.0, ptr.node_x, ptr.node_v, r(ptr.node_a), r(ptr.node_j))
        want = oracle.force_list(ids, np.vstack([xp, nxp]), np.vstack([vp, nvp]), r(np.concatenate([m, ptr.node_m])),
                                 1e-4, gf, ptr.list_off, ptr.entries)
        assert_close(f"runs step {step}", prec, got["runs"], want)
    # an update and the force in one call (ht_step_async)
    upd_ids = np.sort(rng.choice(n, 500, replace=False)).astype(np.int32)
    upd = (500, dev(upd_ids), dev(np.full(500, 0.25)), dev(m[upd_ids]), dev(x[upd_ids] + 1e-4), dev(v[upd_ids]),
           dev(a[upd_ids]), dev(j[upd_ids]))
    act = np.sort(rng.choice(n, 900, replace=False)).astype(np.int32)
    outs = {f: tuple(torch.empty(sh, dtype=torch.float64, device="cuda") for sh in ((900, 3), (900, 3), (900,)))
            for f in ctxs}
    for form, c in ctxs.items():
        c.step_async(upd, 0.28125, act, *outs[form])
        c.sync()
    for p_, q_ in zip(outs["csr"], outs["runs"]):
        assert torch.equal(p_, q_)
    with pytest.raises(B.HTError):
        B.force_batch_async([ctxs["runs"]], [act], [outs["runs"][0]], [outs["runs"][1]], [outs["runs"][2]])


# ------------------------------------------------------------------------------------------ placement over XCDs
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_placement_does_not_change_results(oracle, prec):
    """ht_set_placement only reorders and places the work items: the outputs
    with one stretch per XCD (and with 3 and 16 stretches) equal the unplaced
    plan's bit for bit, for active sets that hit every tile size, a single
    active particle (one long list split over many items) and all particles;
    the oracle agrees."""
    say(f"placement ({prec})")
    n = 6000
    x, v, m = W.plummer(n, 71)
    z = np.zeros((n, 3))
    ptr = B.HostTree(x, v, z, z, m, 1, 300, 0.5)
    x, v, m = x[ptr.perm], v[ptr.perm], m[ptr.perm]
    t0, a, j = W.random_block_state(n, 72, 0.125)
    ctxs = []
    for runs in (1, 0, 3, 16):
        c = make_ctx(prec, n, 2 * n, n, 2 * ptr.n_entries, 1e-4)
        c.set_placement(runs)
        c.set_j_particles(t0, m, x, v, a, j)
        c.set_nodes(0.0, ptr.node_m, ptr.node_x, ptr.node_v, ptr.node_a, ptr.node_j)
        c.set_interaction_lists(ptr.group_first, ptr.list_off, ptr.entries)
        c.predict(0.125)
        ctxs.append(c)
    runs_used, xcds = ctxs[1].placement()
    say(f"  device XCDs {xcds}, runs in use {runs_used}")
    assert runs_used == xcds >= 1 and ctxs[0].placement()[0] == 1 and ctxs[3].placement()[0] == 16
    with pytest.raises(B.HTError):
        ctxs[0].set_placement(17)
    gf = ptr.group_first
    r = (lambda u: u.astype(np.float32).astype(np.float64)) if prec == "mixed" else (lambda u: u)
    xp, vp = oracle.predict(0.125, t0, x, v, r(a), r(j))
    nxp, nvp = oracle.predict(0.125, 0.0, ptr.node_x, ptr.node_v, r(ptr.node_a), r(ptr.node_j))
    XP, VP, MJ = np.vstack([xp, nxp]), np.vstack([vp, nvp]), r(np.concatenate([m, ptr.node_m]))
    rng = np.random.default_rng(73)
    counts = [1, 2, 3, 5, 9, 17, 33, 65, 129, 257]
    sel = [np.sort(rng.choice(np.arange(gf[g], gf[g + 1]), min(gf[g + 1] - gf[g], counts[g % len(counts)]),
                              replace=False)) for g in range(ptr.n_group)]
    for ids in (np.concatenate(sel), np.array([4321]), np.arange(n), np.arange(0, n, 7)):
        ids = ids.astype(np.int32)
        got = [c.force(ids) for c in ctxs]
        for g in got[1:]:
            for p_, q_ in zip(got[0], g):
                assert np.array_equal(p_, q_), (prec, ids.size)
        want = oracle.force_list(ids, XP, VP, MJ, 1e-4, gf, ptr.list_off, ptr.entries)
        assert_close(f"placement n_active={ids.size}", prec, got[1], want)


# ------------------------------------------------------------------------------------------ union tiles
@pytest.mark.parametrize("prec,width", [("fp64", 4), ("mixed", 2), ("mixed", 4), ("mixed", 8)])
def test_union_tiles_match_oracle(oracle, prec, width):
    """Union tiles (HT_LISTS_UNION): runs of `width` consecutive groups share
    tiles over the union of their lists, each pair counted only where the
    entry is in the i-particle's own list.  Every particle still sums exactly
    its own list: checked against the oracle (and against the CSR form, to
    rounding) for one active particle in every group (union tiles chosen
    everywhere), a few per group, every tile size, all particles (per-group
    tiles chosen), a single particle, and through ht_step_async with j-memory
    updates; ε = 0 takes the masked self pair."""
    import torch
    say(f"union tiles ({prec}, width {width})")
    n = 7000
    x, v, m = W.plummer(n, 81)
    m = W.salpeter_masses(n, 82)
    z = np.zeros((n, 3))
    ptr = B.HostTree(x, v, z, z, m, 1, 120, 0.5)
    x, v, m = x[ptr.perm], v[ptr.perm], m[ptr.perm]
    t0, a, j = W.random_block_state(n, 83, 0.25)
    ctxs = {}
    for form in ("csr", "union"):
        c = make_ctx(prec, n, 2 * n, n, 2 * ptr.n_entries, 1e-4)
        c.set_list_form(form)
        if form == "union":
            c.set_union_width(width)
        c.set_j_particles(t0, m, x, v, a, j)
        c.set_nodes(0.0, ptr.node_m, ptr.node_x, ptr.node_v, ptr.node_a, ptr.node_j)
        c.set_interaction_lists(ptr.group_first, ptr.list_off, ptr.entries)
        ctxs[form] = c
    gf = ptr.group_first
    r = (lambda u: u.astype(np.float32).astype(np.float64)) if prec == "mixed" else (lambda u: u)
    rng = np.random.default_rng(84)
    one = np.array([rng.integers(gf[g], gf[g + 1]) for g in range(ptr.n_group)])
    counts = [1, 2, 3, 5, 9, 17, 33, 65, 129]
    few = np.concatenate([np.sort(rng.choice(np.arange(gf[g], gf[g + 1]), min(gf[g + 1] - gf[g], counts[g % 9]),
                                             replace=False)) for g in range(ptr.n_group)])
    t = 0.25
    tol = {"fp64": 1e-12, "mixed": 2e-6}[prec]
    for step, ids in enumerate((one, few, np.arange(n), np.array([4321]))):
        ids = ids.astype(np.int32)
        got = {}
        for form, c in ctxs.items():
            c.predict(t)
            got[form] = c.force(ids)
        xp, vp = oracle.predict(t, t0, x, v, r(a), r(j))
        nxp, nvp = oracle.predict(t, 0.0, ptr.node_x, ptr.node_v, r(ptr.node_a), r(ptr.node_j))
        want = oracle.force_list(ids, np.vstack([xp, nxp]), np.vstack([vp, nvp]), r(np.concatenate([m, ptr.node_m])),
                                 1e-4, gf, ptr.list_off, ptr.entries)
        assert_close(f"union step {step}", prec, got["union"], want)
        ea = errors(got["union"], got["csr"])
        assert ea[0] <= tol, (step, ea)
    # an update and the force in one call (ht_step_async)
    dev = lambda u: torch.from_numpy(np.ascontiguousarray(u)).cuda()  # noqa: E731
    upd_ids = np.sort(rng.choice(n, 600, replace=False)).astype(np.int32)
    upd = (600, dev(upd_ids), dev(np.full(600, 0.25)), dev(m[upd_ids]), dev(x[upd_ids] + 1e-4), dev(v[upd_ids]),
           dev(a[upd_ids]), dev(j[upd_ids]))
    act = one.astype(np.int32)
    outs = {f: tuple(torch.empty(sh, dtype=torch.float64, device="cuda") for sh in ((act.size, 3), (act.size, 3),
                                                                                  (act.size,))) for f in ctxs}
    for form, c in ctxs.items():
        c.step_async(upd, 0.28125, act, *outs[form])
        c.sync()
    got = tuple(o.cpu().numpy() for o in outs["union"])
    x2 = x.copy()
    x2[upd_ids] += 1e-4
    t02 = t0.copy()
    t02[upd_ids] = 0.25
    xp, vp = oracle.predict(0.28125, t02, x2, v, r(a), r(j))
    nxp, nvp = oracle.predict(0.28125, 0.0, ptr.node_x, ptr.node_v, r(ptr.node_a), r(ptr.node_j))
    want = oracle.force_list(act, np.vstack([xp, nxp]), np.vstack([vp, nvp]), r(np.concatenate([m, ptr.node_m])),
                             1e-4, gf, ptr.list_off, ptr.entries)
    assert_close("union step_async", prec, got, want)
    with pytest.raises(B.HTError):
        ctxs["union"].set_union_width(9)
    with pytest.raises(B.HTError):
        B.force_batch_async([ctxs["union"]], [act], [outs["union"][0]], [outs["union"][1]], [outs["union"][2]])


def test_union_tiles_zero_softening(oracle):
    """ε = 0: the self pair is masked by index inside union tiles too."""
    say("union tiles, eps = 0")
    n = 3000
    x, v, m = W.plummer(n, 91)
    z = np.zeros((n, 3))
    ptr = B.HostTree(x, v, z, z, m, 1, 64, 0.5)
    x, v, m = x[ptr.perm], v[ptr.perm], m[ptr.perm]
    t0, a, j = W.random_block_state(n, 92, 0.125)
    c = make_ctx("fp64", n, 2 * n, n, 2 * ptr.n_entries, 0.0)
    c.set_list_form("union")
    c.set_j_particles(t0, m, x, v, a, j)
    c.set_nodes(0.0, ptr.node_m, ptr.node_x, ptr.node_v, ptr.node_a, ptr.node_j)
    c.set_interaction_lists(ptr.group_first, ptr.list_off, ptr.entries)
    c.predict(0.125)
    gf = ptr.group_first
    ids = np.array([gf[g] for g in range(ptr.n_group)], dtype=np.int32)
    got = c.force(ids)
    want = oracle_list_force(oracle, 0.125, ids, t0, m, x, v, a, j, ptr, 0.0)
    assert_close("union eps=0", "fp64", got, want)
