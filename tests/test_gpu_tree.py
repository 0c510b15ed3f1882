"""Step 1 on the device (htd_*, include/htree_tree.h) against the oracle's tree.

Index work, so the bar is bit-exact: keys, particle order, node moments (the
sums are specified in particle order with rounded products, so they are
bit-identical too), node levels and ranges, the root cube, groups, list
offsets and list entries.  Inputs cover several tiles of every kernel and a
ragged tail, coincident particles, all particles at one point, flattened and
clustered sets, n_leaf above one, single-particle groups (every list a full
cover), theta = 0 (every list the whole particle set), one group holding all
particles (the per-work-group scratch must grow) and lists that overflow the
first staging allocation.  The full-size case is the 2^20-particle Plummer
model with Salpeter masses at the headline workload's parameters.
"""
import sys

import numpy as np
import pytest

from paper_1602_02832_amd import binding as B
from paper_1602_02832_amd import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("perm", "keys", "node_m", "node_x", "node_v", "node_a", "node_j", "node_level", "node_begin", "node_end",
          "group_first", "list_off", "entries")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def build_both(oracle, tree, x, n_leaf, n_crit, theta, seed=0):
    rng = np.random.default_rng(seed)
    n = len(x)
    v, a, j = (rng.standard_normal((n, 3)) for _ in range(3))
    m = rng.random(n) + 0.05
    ref = oracle.Tree(x, v, a, j, m, n_leaf, n_crit, theta)
    tree.build(dev(x), dev(v), dev(a), dev(j), dev(m), n_leaf, n_crit, theta)
    return ref, tree.get()


def assert_same(ref, got, tag):
    assert (got.n_node, got.n_group, got.n_entries) == (ref.n_node, ref.n_group, ref.n_entries), tag
    for f in FIELDS:
        r, g = getattr(ref, f), getattr(got, f)
        assert r.shape == g.shape, f"{tag}: {f} shape {g.shape} vs {r.shape}"
        if r.dtype.kind == "f":   # bit patterns, so that -0.0 and NaN would count too
            assert np.array_equal(r.view(np.uint64), g.view(np.uint64)), f"{tag}: {f} differs"
        else:
            assert np.array_equal(r, g), f"{tag}: {f} differs"
    assert np.array_equal(ref.lo.view(np.uint64), got.lo.view(np.uint64)) and ref.side == got.side, tag


def small_cases():
    rng = np.random.default_rng(3)
    out = [(f"uniform{n}", rng.random((n, 3))) for n in (1, 2, 3, 5, 17, 64, 300, 2000, 5000)]
    x = rng.random((500, 3))
    x[100:140] = x[100]
    out.append(("coincident40", x))
    out.append(("allsame", np.ones((50, 3))))
    out.append(("flat", rng.standard_normal((3000, 3)) * np.array([1, 1e-3, 1])))
    x = rng.random((400, 3))
    x[:200] *= 1e-7
    out.append(("clustered", x))
    return out


PARAMS = ((1, 8, 0.5), (1, 64, 0.0), (3, 16, 0.75), (2, 1, 0.3), (1, 1_000_000, 0.4))


@pytest.fixture(scope="module")
def tree():
    t = B.DeviceTree(n_max=1 << 20)
    yield t
    t.close()


@pytest.mark.parametrize("name,x", small_cases(), ids=[c[0] for c in small_cases()])
def test_device_tree_matches_oracle_small(oracle, tree, name, x):
    for k, (n_leaf, n_crit, theta) in enumerate(PARAMS):
        tag = f"{name} n={len(x)} n_leaf={n_leaf} n_crit={n_crit} theta={theta}"
        say("case " + tag)
        ref, got = build_both(oracle, tree, x, n_leaf, n_crit, theta, seed=k)
        assert_same(ref, got, tag)


def test_device_tree_one_group_and_full_covers(oracle, tree):
    """One group holding 60000 particles (its cut outgrows the first scratch
    size) and single-particle groups at theta = 0 (every list is all N
    particles, so the staged lists outgrow their first allocation)."""
    rng = np.random.default_rng(11)
    x = rng.random((60000, 3))
    say("case one group n=60000")
    ref, got = build_both(oracle, tree, x, 1, 10_000_000, 0.5)
    assert_same(ref, got, "one group")
    assert got.n_group == 1 and got.n_entries == 60000
    x = rng.random((3000, 3))
    say("case single-particle groups n=3000 theta=0")
    ref, got = build_both(oracle, tree, x, 1, 1, 0.0)
    assert_same(ref, got, "full covers")
    assert got.n_entries == 3000 * 3000


def test_device_tree_plummer_c2(oracle, tree):
    x, _, _ = W.plummer(16384, 2)
    say("case plummer16k theta=0.4 n_crit=256")
    ref, got = build_both(oracle, tree, x, 1, 256, 0.4)
    assert_same(ref, got, "plummer16k")


def test_device_tree_full_size_plummer_salpeter(oracle, tree):
    """The 2^20-particle headline model (theta 0.4, n_crit 2048) against the
    oracle, and the builder reused after a smaller build."""
    x, v, _ = W.plummer(1 << 20, 3)
    m = W.salpeter_masses(1 << 20, 4)
    rng = np.random.default_rng(5)
    a, j = rng.standard_normal((2, 1 << 20, 3))
    say("case plummer1m salpeter theta=0.4 n_crit=2048")
    ref = oracle.Tree(x, v, a, j, m, 1, 2048, 0.4)
    tree.build(dev(x), dev(v), dev(a), dev(j), dev(m), 1, 2048, 0.4)
    assert_same(ref, tree.get(), "plummer1m")
    ms = tree.phase_ms()
    say("device build phases (ms): " + ", ".join(f"{k} {v:.2f}" for k, v in ms.items()))
    # a smaller build on the same object, then the full one again
    tree.build(dev(x[:1000]), dev(v[:1000]), dev(a[:1000]), dev(j[:1000]), dev(m[:1000]), 1, 64, 0.5)
    assert_same(oracle.Tree(x[:1000], v[:1000], a[:1000], j[:1000], m[:1000], 1, 64, 0.5), tree.get(), "1000")
    tree.build(dev(x), dev(v), dev(a), dev(j), dev(m), 1, 2048, 0.4)
    assert_same(ref, tree.get(), "plummer1m again")


def test_device_tree_rejects_bad_arguments(tree):
    import torch
    z = torch.zeros((4, 3), dtype=torch.float64, device="cuda")
    m = torch.ones(4, dtype=torch.float64, device="cuda")
    L = B.device_lib()
    for args in ((0, 1, 1, 0.5), (4, 0, 1, 0.5), (4, 1, 0, 0.5), (4, 1, 1, -1.0), (4, 1, 1, float("nan")),
                 ((1 << 20) + 1, 1, 1, 0.5)):
        n, n_leaf, n_crit, theta = args
        rc = L.htd_build(tree._h, n, z.data_ptr(), z.data_ptr(), z.data_ptr(), z.data_ptr(), m.data_ptr(), n_leaf,
                         n_crit, theta)
        assert rc == -1, args
        assert L.htd_last_error()
