"""The no-allocation direct sum (ht_force_direct_noalloc) against the
context's direct sum (ht_force_direct_async) on the same predicted state,
through the C-ABI: two calls in a row on the library's one scratch array, the
second with a smaller input, so that what the first call left there cannot
leak into the second.  Tolerances as for the oracle comparisons (FP64 1e-12;
mixed acc 2e-6, jerk 1e-5, pot 1e-6, per particle)."""
import numpy as np
import pytest
from paper_1602_02832_amd import binding as B
from paper_1602_02832_amd import workloads as W
from parity_util import assert_close, say

pytestmark = pytest.mark.gpu


def context_direct(prec, t, x, v, m, eps2, act):
    """ht_force_direct on a context whose particles all sit at time t, so the
    predictor hands the positions and velocities through unchanged."""
    n = m.shape[0]
    rng = np.random.default_rng(n)
    a, j = rng.normal(size=(2, n, 3))
    c = B.Context(n_max=n, node_max=0, group_max=1, list_max=1, active_max=n, eps2=eps2, precision=prec)
    c.set_j_particles(np.full(n, t), m, x, v, a, j)
    c.set_nodes(t, np.zeros(0), *(np.zeros((0, 3)) for _ in range(4)))
    c.predict(t)
    out = c.force_direct(act)
    c.close()
    return out


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_direct_equals_context_direct(prec):
    import torch
    stream = torch.cuda.Stream()
    eps2 = 1e-5
    for call, (n, k, splits, seed) in enumerate(((3000, 3000, 8, 1), (1200, 300, 5, 2), (900, 77, 1, 3))):
        say(f"no-alloc direct {prec}: call {call}, n {n}, {k} active, {splits} splits")
        x, v, _ = W.plummer(n, 100 + seed)
        m = W.salpeter_masses(n, 200 + seed)
        act = np.sort(np.random.default_rng(seed).choice(n, k, replace=False)).astype(np.int32)
        want = context_direct(prec, 0.125, x, v, m, eps2, act)
        dev = lambda u: torch.from_numpy(np.ascontiguousarray(u)).cuda()  # noqa: E731
        dx, dv, dm, da = dev(x), dev(v), dev(m), dev(act)
        out = tuple(torch.full(sh, float("nan"), dtype=torch.float64, device="cuda") for sh in ((k, 3), (k, 3), (k,)))
        B.force_direct_noalloc(prec, dx, dv, dm, eps2, da, splits, *out, stream=stream)
        stream.synchronize()
        assert_close(f"no-alloc call {call}", prec, tuple(o.cpu().numpy() for o in out), want)
    # a request beyond the scratch array is refused before any launch
    with pytest.raises(B.HTError) as e:
        B.force_direct_noalloc(prec, dx, dv, dm, eps2, da, 65535, *out, stream=stream)
    assert e.value.code == -2 and "scratch" in str(e.value)
    with pytest.raises(B.HTError) as e:
        B.force_direct_noalloc(prec, dx, dv, dm, eps2, da, 0, *out, stream=stream)
    assert e.value.code == -1
