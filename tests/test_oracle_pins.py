"""Pins for the FP64 CPU oracle: checks against closed forms, invariants, brute
force on tiny inputs and the paper's printed numbers.  Nothing here compares
the oracle with itself by retyping its formulas."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from paper_1602_02832_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------- helpers
def kepler_relative(t, a=1.0, e=0.5, GM=1.0):
    """Relative orbit of a Keplerian ellipse starting at pericentre (Kepler's equation)."""
    n = math.sqrt(GM / a**3)
    M = n * t
    E = M if e < 0.8 else math.pi
    for _ in range(60):
        dE = (E - e * math.sin(E) - M) / (1.0 - e * math.cos(E))
        E -= dE
        if abs(dE) < 1e-16:
            break
    b = a * math.sqrt(1.0 - e * e)
    Edot = n / (1.0 - e * math.cos(E))
    r = np.array([a * (math.cos(E) - e), b * math.sin(E), 0.0])
    w = np.array([-a * math.sin(E) * Edot, b * math.cos(E) * Edot, 0.0])
    return r, w


def kepler_run(O, eta, periods=1.0, dt_tree=1.0 / 16):
    e = 0.5
    r0, w0 = kepler_relative(0.0, e=e)
    m = np.array([0.5, 0.5])
    x = np.array([-0.5 * r0, 0.5 * r0])
    v = np.array([-0.5 * w0, 0.5 * w0])
    sim = O.TreeHermite(x, v, m, eps2=0.0, dt_tree=dt_tree, eta=eta, mode="direct")
    t_end = 2.0 * math.pi * periods
    err = 0.0
    steps = 0
    while sim.next_time() <= t_end:
        tn, _ = sim.step()
        steps += 1
        xp, _ = O.predict(tn, sim.t0, sim.x, sim.v, sim.a, sim.j)
        order = np.argsort(sim.ids)
        xp = xp[order]
        rel = xp[1] - xp[0]
        r_exact, _ = kepler_relative(tn, e=e)
        err = max(err, float(np.linalg.norm(rel - r_exact)))
    return err, steps, sim


def numpy_root_box(x):
    lo = x.min(0)
    ext = float((x.max(0) - lo).max())
    if ext == 0.0:
        return lo, 1.0
    _, e = np.frexp(ext)
    return lo, float(np.ldexp(1.0, int(e)))


# ----------------------------------------------------------------------------- Kepler
def test_kepler_closed_form(oracle):
    """Two equal masses, eps = 0, e = 0.5: Hermite orbit vs Kepler's equation."""
    err, steps, _ = kepler_run(oracle, eta=0.01)
    assert steps > 100
    assert err < 2e-5, err


def test_kepler_fourth_order(oracle):
    """Aarseth dt scales as sqrt(eta): eta/4 halves every block step, so a
    4th-order scheme's error must fall by about 2^4."""
    e1, s1, _ = kepler_run(oracle, eta=0.01, dt_tree=1.0)
    e2, s2, _ = kepler_run(oracle, eta=0.0025, dt_tree=1.0)
    assert 1.9 < s2 / s1 < 2.1
    ratio = e1 / e2
    assert 10.0 < ratio < 24.0, (e1, e2, ratio)


def test_kepler_energy(oracle):
    """Energy of the two-body orbit (closed form -G m1 m2 / 2a = -1/8) is kept."""
    _, _, sim = kepler_run(oracle, eta=0.01, periods=0.5)
    xp, vp = oracle.predict(sim.t, sim.t0, sim.x, sim.v, sim.a, sim.j)
    K, Wp = oracle.energy(xp, vp, sim.m, 0.0)
    assert abs((K + Wp) - (-0.125)) < 1e-6


# ----------------------------------------------------------------------------- direct sums
@pytest.fixture(scope="module")
def small_cluster():
    x, v, m = W.plummer(512, 7)
    m = W.salpeter_masses(512, 8)
    return x, v, m


def test_direct_momentum_and_jerk_sums(oracle, small_cluster):
    """Newton's third law: sum m a = 0 and sum m jerk = 0 up to rounding."""
    x, v, m = small_cluster
    ids = np.arange(len(m), dtype=np.int32)
    acc, jerk, pot = oracle.force_direct(ids, x, v, m, 1e-4)
    for q in (acc, jerk):
        s = np.abs((m[:, None] * q).sum(0)).max()
        scale = (m * np.linalg.norm(q, axis=1)).sum()
        assert s < 1e-13 * scale


def test_direct_potential_equals_twice_W(oracle, small_cluster):
    x, v, m = small_cluster
    ids = np.arange(len(m), dtype=np.int32)
    eps2 = 1e-4
    _, _, pot = oracle.force_direct(ids, x, v, m, eps2)
    _, Wp = oracle.energy(x, v, m, eps2)
    assert abs((m * pot).sum() - 2.0 * Wp) < 1e-13 * abs(Wp)


def test_jerk_is_time_derivative_of_acceleration(oracle, small_cluster):
    """With a = jerk = 0 in the predictor every particle moves on x + v t; the
    jerk must equal d a / dt there (central difference, Richardson)."""
    x, v, m = small_cluster
    n = 64
    x, v, m = x[:n], v[:n], m[:n]
    ids = np.arange(n, dtype=np.int32)
    eps2 = 1e-3
    z = np.zeros((n, 3))
    _, jerk, _ = oracle.force_direct(ids, x, v, m, eps2)

    def acc_at(t):
        xp, vp = oracle.predict(t, 0.0, x, v, z, z)
        return oracle.force_direct(ids, xp, vp, m, eps2)[0]

    h = 1.25e-4     # Richardson error falls 16x per halving of h down to here
    D1 = (acc_at(h) - acc_at(-h)) / (2 * h)
    D2 = (acc_at(h / 2) - acc_at(-h / 2)) / h
    R = (4.0 * D2 - D1) / 3.0
    rel = np.linalg.norm(R - jerk, axis=1) / np.linalg.norm(jerk, axis=1)
    assert rel.max() < 1e-8, rel.max()


# ----------------------------------------------------------------------------- Hilbert keys
def _face_neighbours(pts):
    d = np.abs(np.diff(pts.astype(np.int64), axis=0)).sum(1)
    return np.all(d == 1)


def test_hilbert_corner_cube_bijection_and_adjacency(oracle):
    """Points of the cube [0, 16)^3 at the origin fill the first 16^3 keys
    exactly once, and consecutive keys are face neighbours."""
    s = 16
    g = np.stack(np.meshgrid(np.arange(s), np.arange(s), np.arange(s), indexing="ij"), -1).reshape(-1, 3)
    k = oracle.hilbert_keys(g)
    assert np.array_equal(np.sort(k), np.arange(s**3, dtype=np.uint64))
    order = np.argsort(k)
    assert _face_neighbours(g[order])


def test_hilbert_aligned_cells_are_contiguous(oracle):
    """Any aligned cube of side 2^b is one key interval of length 8^b
    (so a cell at any level is a key prefix), traversed by face steps."""
    rng = np.random.default_rng(3)
    for b in (1, 2, 3):
        for _ in range(20):
            base = rng.integers(0, (1 << 21) >> b, 3) << b
            s = 1 << b
            g = np.stack(np.meshgrid(*(np.arange(s) + base[d] for d in range(3)), indexing="ij"), -1).reshape(-1, 3)
            k = np.sort(oracle.hilbert_keys(g))
            assert int(k[-1] - k[0]) == s**3 - 1
            assert int(k[0]) % (s**3) == 0
            assert _face_neighbours(g[np.argsort(oracle.hilbert_keys(g))])


def test_hilbert_global_adjacency_random_runs(oracle):
    """Walk the curve at the finest level: for random points p, the point with
    key k(p)+1 is found among p's 6 face neighbours."""
    rng = np.random.default_rng(5)
    p = rng.integers(1, (1 << 21) - 1, (2000, 3)).astype(np.uint32)
    k = oracle.hilbert_keys(p)
    nb = np.concatenate([p + off for off in np.array(
        [[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], dtype=np.int64).astype(np.uint32)])
    knb = oracle.hilbert_keys(nb).reshape(6, -1)
    assert np.all(np.any(knb == (k + np.uint64(1))[None, :], axis=0))


# ----------------------------------------------------------------------------- tree and node moments
def _tiny_inputs():
    rng = np.random.default_rng(11)
    out = []
    for n in (1, 2, 3, 8, 64):
        out.append(("random%d" % n, rng.normal(size=(n, 3)), rng.uniform(0.1, 1.0, n)))
    x = rng.normal(size=(12, 3))
    x[3] = x[7] = x[9]         # coincident points (same finest cell)
    out.append(("coincident", x, rng.uniform(0.1, 1.0, 12)))
    xx = np.zeros((5, 3))
    out.append(("all_same", xx, np.full(5, 0.2)))
    return out


@pytest.mark.parametrize("name,x,m", _tiny_inputs(), ids=[c[0] for c in _tiny_inputs()])
def test_node_moments_brute_force(oracle, name, x, m):
    rng = np.random.default_rng(2)
    n = len(m)
    v, a, j = rng.normal(size=(3, n, 3))
    tr = oracle.Tree(x, v, a, j, m, 1, 4, 0.5)
    lo, side = numpy_root_box(x)
    assert np.array_equal(lo, tr.lo) and side == tr.side
    q = np.clip(np.floor((x - lo) * (2.0**21 / side)), 0, 2**21 - 1).astype(np.int64)
    for nd in range(tr.n_node):
        L = int(tr.node_level[nd])
        b, e = tr.node_begin[nd], tr.node_end[nd]
        cube = q[tr.perm[b]] >> (21 - L)
        members = np.flatnonzero(np.all((q >> (21 - L)) == cube, axis=1))
        assert np.array_equal(np.sort(members), np.sort(tr.perm[b:e])), (name, nd)
        M = math.fsum(m[members])
        assert abs(tr.node_m[nd] - M) <= 1e-15 * M
        for arr, got in ((x, tr.node_x), (v, tr.node_v), (a, tr.node_a), (j, tr.node_j)):
            for d in range(3):
                want = math.fsum(m[members] * arr[members, d]) / M
                scale = math.fsum(np.abs(m[members] * arr[members, d])) / M
                assert abs(got[nd, d] - want) <= 1e-14 * max(scale, 1e-300), (name, nd, d)


@pytest.fixture(scope="module")
def tree2k(oracle):
    x, v, m = W.plummer(2048, 1)
    rng = np.random.default_rng(9)
    a, j = rng.normal(size=(2, 2048, 3))
    tr = oracle.Tree(x, v, a, j, m, 1, 64, 0.5)
    return x, v, a, j, m, tr


def test_keys_sorted_and_perm_stable(oracle, tree2k):
    x, v, a, j, m, tr = tree2k
    assert np.all(np.diff(tr.keys.astype(np.float64)) >= 0)
    assert np.array_equal(np.sort(tr.perm), np.arange(tr.n))
    same = tr.keys[1:] == tr.keys[:-1]
    assert np.all(tr.perm[1:][same] > tr.perm[:-1][same])


def test_groups_cover_and_sizes(oracle, tree2k):
    x, v, a, j, m, tr = tree2k
    gf = tr.group_first
    assert gf[0] == 0 and gf[-1] == tr.n and np.all(np.diff(gf) > 0)
    assert np.diff(gf).max() <= tr.n_crit


def _cube_ids(x, lo, side, level):
    """Integer id of every particle's cube at a tree level, from the root cube
    alone (no keys, no tree): the level-L cube holds the points whose integer
    coordinates agree in their top L of 21 bits."""
    q = np.clip(np.floor((x - lo) * (2.0**21 / side)), 0, 2**21 - 1).astype(np.int64) >> (21 - level)
    return (q[:, 0] << 42) | (q[:, 1] << 21) | q[:, 2]


def _group_rule_inputs():
    rng = np.random.default_rng(21)
    x2k, _, _ = W.plummer(2048, 1)
    out = [("plummer2k", x2k, 1, 64)]
    # n_crit equal to the size of an actual cell, so that a cell of exactly
    # n_crit particles exists and must be a group (<= versus < tells here)
    lo, side = numpy_root_box(x2k)
    for level, pick in ((3, 0), (4, 1), (5, 2)):
        ids = _cube_ids(x2k, lo, side, level)
        _, cnt = np.unique(ids, return_counts=True)
        cand = np.sort(cnt[(cnt >= 8) & (cnt <= 400)])
        out.append((f"plummer2k_ncrit_cell_L{level}", x2k, 1, int(cand[len(cand) * (pick + 1) // 4])))
    # a pile of coincident points larger than n_crit: a group that cannot split
    xc = rng.normal(size=(300, 3))
    xc[:40] = xc[40]
    out.append(("coincident_pile", xc, 1, 8))
    out.append(("coincident_pile_leaf3", xc, 3, 8))
    out.append(("leaf_above_ncrit", rng.normal(size=(500, 3)), 6, 4))
    return out


@pytest.mark.parametrize("name,x,n_leaf,n_crit", _group_rule_inputs(), ids=[c[0] for c in _group_rule_inputs()])
def test_groups_follow_the_barnes_rule(oracle, name, x, n_leaf, n_crit):
    """Groups (Section 2, the modified tree algorithm after Barnes 1990) are
    the first cells on each path from the root that hold at most n_crit
    particles or cannot be split, checked on cells found by brute force from
    the integer coordinates: every group's members are exactly one cell's; every
    strictly larger cell containing it holds more than n_crit particles and can
    be split (so it is not a group); and a group holds more than n_crit
    particles only when it cannot split (at most n_leaf particles, or points
    that share the finest cell)."""
    n = x.shape[0]
    z = np.zeros_like(x)
    tr = oracle.Tree(x, z, z, z, np.full(n, 1.0 / n), n_leaf, n_crit, 0.5)
    lo, side = numpy_root_box(x)
    assert np.array_equal(lo, tr.lo) and side == tr.side
    levels = [_cube_ids(x, lo, side, L) for L in range(22)]
    counts = []
    for ids in levels:
        u, inv, cnt = np.unique(ids, return_inverse=True, return_counts=True)
        counts.append(cnt[inv])           # size of every particle's cell at this level
    gf = tr.group_first
    assert gf[0] == 0 and gf[-1] == n and np.all(np.diff(gf) > 0)
    sizes = np.diff(gf)
    for g in range(tr.n_group):
        members = tr.perm[gf[g]:gf[g + 1]]
        k0, size = members[0], members.size
        chain = [L for L in range(22)
                 if counts[L][k0] == size and np.all(levels[L][members] == levels[L][k0])]
        assert chain, (name, g, "not a cell")
        assert chain == list(range(chain[0], chain[-1] + 1))
        for L in range(chain[0]):         # every strictly larger cell on the path
            c = counts[L][k0]
            assert c > size and c > n_crit and c > n_leaf, (name, g, L, c)
        if size > n_crit:
            assert size <= n_leaf or chain[-1] == 21, (name, g, size)
    if name.startswith("plummer2k_ncrit_cell"):
        assert np.any(sizes == n_crit), (name, n_crit)
    if name.startswith("coincident_pile"):
        assert np.any(sizes >= 41)


def _mac_accepts(tr, nd, blo, bhi):
    X = tr.node_x[nd]
    gap = np.maximum(np.maximum(blo - X, X - bhi), 0.0)
    d2 = (gap[0] * gap[0] + gap[1] * gap[1]) + gap[2] * gap[2]
    s = tr.side * 2.0 ** (-int(tr.node_level[nd]))
    return s * s < (tr.theta * tr.theta) * d2


def test_lists_are_the_unique_barnes_hut_cover(oracle, tree2k):
    """Each group's list is a disjoint cover of all particles; emitted nodes pass
    the opening test and no non-overlapping ancestor does; directly listed
    particles outside the group have no accepting non-overlapping ancestor;
    entries appear in pre-order (increasing first particle)."""
    x, v, a, j, m, tr = tree2k
    n = tr.n
    xs = x[tr.perm]
    nb, ne = tr.node_begin, tr.node_end
    for g in range(tr.n_group):
        gb, ge = tr.group_first[g], tr.group_first[g + 1]
        lst = tr.list_of(g)
        parts = lst[lst < n]
        nodes = lst[lst >= n] - n
        cover = np.zeros(n, np.int64)
        np.add.at(cover, parts, 1)
        for nd in nodes:
            cover[nb[nd]:ne[nd]] += 1
        assert np.all(cover == 1), g
        starts = np.where(lst < n, lst, nb[np.clip(lst - n, 0, None)])
        assert np.all(np.diff(starts) > 0)
        blo, bhi = xs[gb:ge].min(0), xs[gb:ge].max(0)
        overlap = (nb < ge) & (gb < ne)
        acc = np.array([(not overlap[k]) and _mac_accepts(tr, k, blo, bhi) for k in range(tr.n_node)])
        for nd in nodes:
            assert acc[nd] and not overlap[nd]
            anc = (nb <= nb[nd]) & (ne >= ne[nd]) & (tr.node_level < tr.node_level[nd])
            assert not np.any(acc & anc)
        outside = parts[(parts < gb) | (parts >= ge)]
        for k in outside:
            cont = (nb <= k) & (k < ne)
            assert not np.any(acc & cont)


def _bottom_up_mass_inputs():
    rng = np.random.default_rng(21)
    x, _, _ = W.plummer(4096, 5)
    out = [("plummer4k", x, 1)]
    out.append(("plummer4k_leaf3", x, 3))
    xc = rng.normal(size=(600, 3))
    xc[100:160] = xc[100]          # 60 coincident particles: a level-21 leaf
    out.append(("coincident", xc, 1))
    return out


@pytest.mark.parametrize("name,x,n_leaf", _bottom_up_mass_inputs(), ids=[c[0] for c in _bottom_up_mass_inputs()])
def test_node_mass_is_children_summed_in_key_order(oracle, name, x, n_leaf):
    """The node-moment reading, bit for bit, from the oracle's outputs alone: a
    split node's mass is 0 + its children's masses added left to right in key
    order (a child node's mass, or a single particle's), and a leaf node's is
    0 + its particles' masses in order.  Random masses make the order visible
    in the last bits (a sequential sum over each node's own particles differs
    for most nodes)."""
    rng = np.random.default_rng(4)
    n = len(x)
    m = rng.uniform(0.5, 1.5, n) / n
    v, a, j = rng.normal(size=(3, n, 3))
    tr = oracle.Tree(x, v, a, j, m, n_leaf, 64, 0.5)
    ms = m[tr.perm]
    at = {(int(tr.node_level[q]), int(tr.node_begin[q])): q for q in range(tr.n_node)}
    differs = 0
    for q in range(tr.n_node):
        L, b, e = int(tr.node_level[q]), int(tr.node_begin[q]), int(tr.node_end[q])
        s = 0.0
        if e - b > n_leaf and L < 21:      # split: children in key order
            k = b
            while k < e:
                c = at.get((L + 1, k))
                if c is not None:
                    s = s + float(tr.node_m[c])
                    k = int(tr.node_end[c])
                else:
                    s = s + (0.0 + float(ms[k]))
                    k += 1
        else:
            for k in range(b, e):
                s = s + float(ms[k])
        assert tr.node_m[q] == s, (name, q, L, b, e)
        seq = 0.0
        for k in range(b, e):
            seq = seq + float(ms[k])
        differs += seq != s
    assert tr.n_node > 100
    if name.startswith("plummer"):
        assert differs > tr.n_node // 10   # the check tells the two readings apart


def test_node_prediction_is_mass_weighted_mean(oracle, tree2k):
    """A node predicted from its moments equals the mass-weighted mean of its
    members predicted from the same time (the predictor is linear)."""
    x, v, a, j, m, tr = tree2k
    t = 3.0 / 128
    xs, vs, as_, js, ms = x[tr.perm], v[tr.perm], a[tr.perm], j[tr.perm], m[tr.perm]
    xp, vp = oracle.predict(t, 0.0, xs, vs, as_, js)
    nxp, nvp = oracle.predict(t, 0.0, tr.node_x, tr.node_v, tr.node_a, tr.node_j)
    for nd in range(0, tr.n_node, 7):
        b, e = tr.node_begin[nd], tr.node_end[nd]
        w = ms[b:e] / ms[b:e].sum()
        assert np.allclose(nxp[nd], (w[:, None] * xp[b:e]).sum(0), rtol=0, atol=1e-13)
        assert np.allclose(nvp[nd], (w[:, None] * vp[b:e]).sum(0), rtol=0, atol=1e-13)


# ----------------------------------------------------------------------------- tree vs direct
def test_theta_zero_is_direct_bitwise(oracle):
    """theta -> 0 opens every node: each list is 0..N-1 in order and the list
    force is bit-identical to the direct sum."""
    x, v, m = W.plummer(300, 4)
    z = np.zeros_like(x)
    tr = oracle.Tree(x, v, z, z, m, 1, 16, 0.0)
    for g in range(tr.n_group):
        assert np.array_equal(tr.list_of(g), np.arange(300, dtype=np.int32))
    xs, vs, ms = x[tr.perm], v[tr.perm], m[tr.perm]
    ids = np.arange(300, dtype=np.int32)
    A = oracle.force_list(ids, xs, vs, ms, 1e-4, tr.group_first, tr.list_off, tr.entries)
    B = oracle.force_direct(ids, xs, vs, ms, 1e-4)
    for p, q in zip(A, B):
        assert np.array_equal(p, q)


def test_tree_force_approaches_direct(oracle):
    """Monopole tree error is small and shrinks with theta."""
    x, v, m = W.plummer(4096, 6)
    z = np.zeros_like(x)
    errs = []
    for th in (0.75, 0.5, 0.3):
        tr = oracle.Tree(x, v, z, z, m, 1, 64, th)
        xs, vs, ms = x[tr.perm], v[tr.perm], m[tr.perm]
        jx = np.vstack([xs, tr.node_x])
        jv = np.vstack([vs, tr.node_v])
        jm = np.concatenate([ms, tr.node_m])
        ids = np.arange(0, 4096, 8, dtype=np.int32)
        A = oracle.force_list(ids, jx, jv, jm, 1e-4, tr.group_first, tr.list_off, tr.entries)
        B = oracle.force_direct(ids, xs, vs, ms, 1e-4)
        rel = np.linalg.norm(A[0] - B[0], axis=1) / np.linalg.norm(B[0], axis=1)
        errs.append(np.median(rel))
    assert errs[0] < 1e-2 and errs[2] < errs[1] < errs[0], errs


# ----------------------------------------------------------------------------- predictor
def test_predictor_exact_on_cubic_orbits(oracle):
    """The predictor is the Taylor series to the jerk: on a cubic trajectory
    (constant jerk) it is exact, so x and v match the cubic evaluated in
    rational arithmetic to rounding, for individual t0 and any t - t0."""
    rng = np.random.default_rng(29)
    n = 40
    X0, V0, A0, J0 = rng.normal(size=(4, n, 3))
    t0 = rng.integers(0, 64, n) / 64.0
    t = 1.25
    xp, vp = oracle.predict(t, t0, X0, V0, A0, J0)
    F = Fraction
    for i in range(n):
        d = F(t) - F(float(t0[i]))
        for k in range(3):
            x = F(X0[i, k]) + F(V0[i, k]) * d + F(A0[i, k]) * d**2 / 2 + F(J0[i, k]) * d**3 / 6
            v = F(V0[i, k]) + F(A0[i, k]) * d + F(J0[i, k]) * d**2 / 2
            scale_x = abs(F(X0[i, k])) + abs(F(V0[i, k]) * d) + abs(F(A0[i, k]) * d**2 / 2) + abs(F(J0[i, k]) * d**3 / 6)
            scale_v = abs(F(V0[i, k])) + abs(F(A0[i, k]) * d) + abs(F(J0[i, k]) * d**2 / 2)
            assert abs(xp[i, k] - float(x)) <= 8e-16 * float(scale_x), (i, k)
            assert abs(vp[i, k] - float(v)) <= 8e-16 * float(scale_v), (i, k)


# ----------------------------------------------------------------------------- corrector / timestep
def test_corrector_exact_on_quintic_orbit(oracle):
    """For a(t) cubic the Hermite interpolant is exact: the corrected x, v
    equal the quintic x(t) evaluated exactly (rational arithmetic)."""
    rng = np.random.default_rng(13)
    D = 1.0 / 8
    X0, V0, A0, J0, C2, C3 = rng.normal(size=(6, 3))
    F = Fraction

    def exact(c, d):
        t = F(D)
        x = F(X0[d]) + F(V0[d]) * t + F(A0[d]) * t**2 / 2 + F(J0[d]) * t**3 / 6 + F(C2[d]) * t**4 / 24 + F(C3[d]) * t**5 / 120
        vv = F(V0[d]) + F(A0[d]) * t + F(J0[d]) * t**2 / 2 + F(C2[d]) * t**3 / 6 + F(C3[d]) * t**4 / 24
        aa = F(A0[d]) + F(J0[d]) * t + F(C2[d]) * t**2 / 2 + F(C3[d]) * t**3 / 6
        jj = F(J0[d]) + F(C2[d]) * t + F(C3[d]) * t**2 / 2
        return float(x), float(vv), float(aa), float(jj)

    ex = np.array([exact(None, d) for d in range(3)])
    a1, j1 = ex[:, 2], ex[:, 3]
    xp, vp = oracle.predict(D, 0.0, X0[None], V0[None], A0[None], J0[None])
    x1, v1, dta = oracle.correct(D, 0.0, xp, vp, A0[None], J0[None], a1[None], j1[None], 0.01)
    assert np.allclose(x1[0], ex[:, 0], rtol=1e-13, atol=1e-13)
    assert np.allclose(v1[0], ex[:, 1], rtol=1e-12, atol=1e-12)
    # Aarseth step from the known derivatives at t1: a'' = C2 + C3 D, a''' = C3
    a2 = C2 + C3 * D
    want = math.sqrt(0.01 * (np.linalg.norm(a1) * np.linalg.norm(a2) + np.linalg.norm(j1) ** 2)
                     / (np.linalg.norm(j1) * np.linalg.norm(C3) + np.linalg.norm(a2) ** 2))
    assert abs(dta[0] - want) < 1e-9 * want


@pytest.mark.parametrize("dt,t1,dt_tree,dt_old,want", [
    (0.3, 0.0, 1 / 8, 0.0, 1 / 8),          # capped by the tree interval
    (0.05, 0.0, 1 / 8, 0.0, 1 / 32),        # largest power of two below dt
    (0.05, 3 / 32, 1 / 8, 0.0, 1 / 32),     # t1 commensurate with 1/32
    (0.05, 1 / 64, 1 / 8, 0.0, 1 / 64),     # t1 only a multiple of 1/64
    (0.05, 5 / 128, 1 / 8, 0.0, 1 / 128),
    (1.0, 1 / 8, 1 / 8, 1 / 64, 1 / 32),    # at most doubling
    (1 / 32, 0.0, 1 / 8, 0.0, 1 / 32),      # exact power of two kept
    (2.0**-45, 0.0, 1.0, 0.0, 0.0),         # below the 2^-40 floor
])
def test_block_step_table(oracle, dt, t1, dt_tree, dt_old, want):
    assert oracle.block_step(dt, t1, dt_tree, dt_old) == want


def test_block_step_properties(oracle):
    rng = np.random.default_rng(17)
    dt_tree = 1.0 / 64
    for _ in range(2000):
        dt = 10 ** rng.uniform(-7, 0)
        t1 = rng.integers(0, 2**20) * 2.0**-24
        old = 2.0 ** -rng.integers(6, 24) if rng.uniform() < 0.8 else 0.0
        h = oracle.block_step(dt, t1, dt_tree, old)
        assert h > 0
        assert np.frexp(h)[0] == 0.5                       # power of two
        cap = min(dt, dt_tree, 2 * old if old > 0 else np.inf)
        assert h <= cap and math.fmod(t1, h) == 0.0
        assert 2 * h > cap or math.fmod(t1, 2 * h) != 0.0  # the largest such


# ----------------------------------------------------------------------------- integrator
def test_tree_hermite_synchronised_rebuilds_and_energy(oracle):
    """Tree run on a small Plummer model: every multiple of dt_tree is an
    all-active step, lists are rebuilt there, energy drifts little."""
    x, v, m = W.plummer(512, 21)
    sim = oracle.TreeHermite(x, v, m, eps2=(1 / 64) ** 2, dt_tree=1 / 64, eta=0.02, theta=0.5, n_crit=32)
    E0 = sim.energy()
    sizes = []
    while sim.next_time() <= 1 / 16:
        tn, act = sim.step()
        if math.fmod(tn, 1 / 64) == 0.0:
            sizes.append(act.size)
    assert sizes == [512] * 4
    assert abs(sim.energy() - E0) < 1e-5 * abs(E0)


# ----------------------------------------------------------------------------- paper numbers
def test_paper_eq3_reproduces_table1():
    """eq. (3) with one card's t_pipe and n_pipe = 56 gives Table 1's T_grape
    (read per card) to a few percent; pins our reading of N_int and n_i."""
    tab = json.load(open(os.path.join(GOLDEN, "table1.json")))
    tp, npipe = tab["eq3"]["t_pipe"], tab["eq3"]["n_pipe"]
    for N, th, nint, ni, tg, *_ in tab["rows"]:
        pred = nint * tp * npipe / ni
        assert abs(pred - tg) / tg < 0.04, (N, th, pred, tg)


def test_paper_peak_matches_57_flop_convention():
    f = json.load(open(os.path.join(GOLDEN, "table1.json")))["flops_per_interaction"]
    peak = f["cards"] * f["pipelines"] * f["clock_hz"] * f["value"] / 1e9
    assert abs(peak - f["peak_gflops"]) / f["peak_gflops"] < 0.01


@pytest.mark.slow
def test_table1_list_length_ballpark(oracle):
    """Mean list length per particle at Table 1's parameters (n_crit = 4000):
    same magnitude as the printed N_int (the paper does not give its opening
    test; ours is stricter, so within a factor 1.6), longer for smaller theta
    by a factor 1.4-2.6, and only slowly growing with N."""
    tab = json.load(open(os.path.join(GOLDEN, "table1.json")))
    ours = {}
    for N in (65536, 262144):
        x, v, m = W.plummer(N, 11)
        z = np.zeros_like(x)
        for th in (0.75, 0.5, 0.3):
            tr = oracle.Tree(x, v, z, z, m, 1, tab["n_crit"], th)
            ours[(N, th)] = float((np.diff(tr.list_off) * np.diff(tr.group_first)).sum() / N)
    for N, th, nint, *_ in tab["rows"]:
        r = ours[(N, th)] / nint
        assert 1 / 1.6 < r < 1.6, (N, th, ours[(N, th)], nint)
    for N in (65536, 262144):
        assert 1.4 < ours[(N, 0.5)] / ours[(N, 0.75)] < 2.6
        assert 1.4 < ours[(N, 0.3)] / ours[(N, 0.5)] < 2.6
    for th in (0.75, 0.5, 0.3):
        assert 1.0 < ours[(262144, th)] / ours[(65536, th)] < 1.5


@pytest.mark.slow
def test_table1_active_per_group_ballpark(oracle):
    """Mean number of active particles per group per block step, n_i (Table 1),
    from the oracle's own integration over one tree interval at Table 1's
    parameters (equal-mass Plummer, N = 65536, n_crit = 4000, eta = 0.01,
    eps = 1/N, dt_tree = 1/64): groups with no active particle in a block step
    do not count.  The paper prints 28.6-29.3 for every theta and N; our value
    is about 1.8 times larger (groups and block steps follow readings the
    paper does not fix), so the pin is the magnitude (within a factor 2) and
    that n_i does not depend on theta (the paper's rows agree within 3%;
    the opening angle changes neither the groups nor, to rounding, the block
    steps)."""
    tab = json.load(open(os.path.join(GOLDEN, "table1.json")))
    N = 65536
    x, v, m = W.plummer(N, 11)
    got = {}
    for th in (0.75, 0.5):
        tally = [0, 0]

        def hook(sim, rec):
            g = np.searchsorted(sim.tree.group_first, rec["active"], side="right") - 1
            tally[0] += rec["active"].size
            tally[1] += np.unique(g).size

        sim = oracle.TreeHermite(x, v, m, eps2=(1.0 / N) ** 2, dt_tree=1.0 / 64, eta=0.01, theta=th,
                                 n_crit=tab["n_crit"], on_step=hook)
        sim.run(1.0 / 64)
        got[th] = tally[0] / tally[1]
    paper = {th: ni for n_, th, _, ni, *_ in tab["rows"] if n_ == N}
    for th, ni in got.items():
        assert 0.5 < ni / paper[th] < 2.0, (th, ni, paper[th])
    assert abs(got[0.75] / got[0.5] - 1.0) < 0.05, got
