"""Seeded synthetic inputs: Plummer model in standard units and the Salpeter
mass spectrum (the workload template of Section 3)."""
import math

import numpy as np
import pytest
from scipy import stats

from paper_1602_02832_amd import workloads as W


def test_plummer_is_seeded_and_centred():
    a = W.plummer(1000, 5)
    b = W.plummer(1000, 5)
    c = W.plummer(1000, 6)
    for p, q in zip(a, b):
        assert np.array_equal(p, q)
    assert not np.array_equal(a[0], c[0])
    x, v, m = a
    assert abs(m.sum() - 1.0) < 1e-15
    assert np.abs((m[:, None] * x).sum(0)).max() < 1e-14
    assert np.abs((m[:, None] * v).sum(0)).max() < 1e-14


def test_plummer_standard_units(oracle):
    """Standard units (G = M = -4E = 1): E = -1/4, virial ratio 1/2 and the
    Plummer half-mass radius 1.305 * 3 pi / 16 = 0.769, to finite-N noise."""
    x, v, m = W.plummer(16384, 2)
    K, Wp = oracle.energy(x, v, m, 0.0)
    assert abs((K + Wp) + 0.25) < 0.01
    assert abs(K / abs(Wp) - 0.5) < 0.02
    r = np.sort(np.linalg.norm(x, axis=1))
    rh = 0.5 * (r[8191] + r[8192])
    assert abs(rh - 1.3048 * 3 * math.pi / 16) < 0.02


def test_plummer_speeds_below_escape():
    x, v, m = W.plummer(4096, 9)
    r = np.linalg.norm(x, axis=1)
    a = 3 * math.pi / 16
    vesc = math.sqrt(2.0) * (1 + (r / a) ** 2) ** -0.25 / math.sqrt(a)
    assert np.all(np.linalg.norm(v, axis=1) < vesc * 1.05)


def test_salpeter_matches_analytic_cdf():
    m = W.salpeter_masses(20000, 4, ratio=100.0)
    assert abs(m.sum() - 1.0) < 1e-12
    mm = m / m.min()
    assert mm.max() <= 100.0 + 1e-9
    p = 1.0 - 2.35
    cdf = lambda u: (np.power(np.clip(u, 1, 100), p) - 1.0) / (100.0**p - 1.0)
    # the sample minimum sits within ~1e-4 of the lower cut at this size
    res = stats.kstest(mm, cdf)
    assert res.pvalue > 0.001, res


def test_configs_are_the_stated_workloads():
    c = W.config("plummer1m_salpeter")
    assert c.n == 2**20 and c.theta == 0.4 and c.eps == 4.0 / 2**20 and c.dt_tree == 1 / 512
    assert W.config("plummer16k").n == 16384 and W.config("plummer2k").n == 2048
    s = W.ensemble_sizes(64, 5, 4096, 65536)
    assert s.min() >= 4096 and s.max() <= 65536
