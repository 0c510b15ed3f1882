"""Seeded synthetic inputs shared by the GPU path, the oracle tests and the bench.

This module only draws random numbers and shapes them into initial conditions
and parameter sets.  It holds none of the method's arithmetic (no forces, no
prediction, no tree), so both the HIP path and the CPU oracle may consume what
it produces without sharing any computation.

Workload template (Section 3 of the paper): an equal-mass Plummer model in the
standard units of Heggie & Mathieu (G = M = -4E = 1), Aarseth timestep
criterion, N-dependent softening, opening angle theta, group size n_crit and
tree interval dt_tree.  The concrete configurations below follow that template
at the sizes this project measures.

RNG: numpy Generator(PCG64(seed)).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "plummer",
    "salpeter_masses",
    "SimConfig",
    "CONFIGS",
    "config",
    "make_initial_conditions",
    "random_block_state",
    "ensemble_sizes",
]

# Plummer scale length and velocity scale that put an equal-mass Plummer
# model of total mass 1 into standard units (virial radius 1): the model's
# energy is -3*pi/64 * G M^2 / a, so E = -1/4 needs a = 3*pi/16.
_PLUMMER_A = 3.0 * math.pi / 16.0
_PLUMMER_VSCALE = 1.0 / math.sqrt(_PLUMMER_A)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _isotropic(rng: np.random.Generator, r: np.ndarray) -> np.ndarray:
    n = r.shape[0]
    cos_t = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    sin_t = np.sqrt(1.0 - cos_t * cos_t)
    out = np.empty((n, 3))
    out[:, 0] = r * sin_t * np.cos(phi)
    out[:, 1] = r * sin_t * np.sin(phi)
    out[:, 2] = r * cos_t
    return out


def plummer(n: int, seed: int, mass_cut: float = 0.999):
    """Plummer sphere by the Aarseth, Henon & Wielen (1974) sampling.

    Radii come from the inverse of the cumulative mass profile, truncated at
    the enclosed-mass fraction ``mass_cut`` (0.999; the paper states no cut).
    Speeds come from von Neumann rejection on q^2 (1 - q^2)^(7/2), q = v/v_esc.
    Positions and velocities are scaled analytically to standard units and the
    centre of mass is moved to rest at the origin.  No exact energy rescale is
    applied, so E = -1/4 holds up to finite-N sampling noise.

    Returns (x[n,3], v[n,3], m[n]) with equal masses 1/n.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    rng = _rng(seed)
    X = rng.uniform(0.0, mass_cut, n)
    X = np.maximum(X, 1e-300)
    r = 1.0 / np.sqrt(np.power(X, -2.0 / 3.0) - 1.0)
    x = _isotropic(rng, r)
    # speeds: rejection sampling, vectorised in rounds
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        qq = rng.uniform(0.0, 1.0, todo.size)
        yy = rng.uniform(0.0, 0.1, todo.size)
        ok = yy < qq * qq * np.power(1.0 - qq * qq, 3.5)
        q[todo[ok]] = qq[ok]
        todo = todo[~ok]
    vesc = math.sqrt(2.0) * np.power(1.0 + r * r, -0.25)
    v = _isotropic(rng, q * vesc)
    m = np.full(n, 1.0 / n)
    x *= _PLUMMER_A
    v *= _PLUMMER_VSCALE
    x -= (m[:, None] * x).sum(0) / m.sum()
    v -= (m[:, None] * v).sum(0) / m.sum()
    return x, v, m


def salpeter_masses(n: int, seed: int, ratio: float = 100.0, slope: float = 2.35):
    """Salpeter spectrum dN/dm ~ m^-slope on [m_min, ratio*m_min] by inverse CDF,
    normalised so that the total mass is 1.  Drawn independently of positions."""
    rng = _rng(seed)
    u = rng.uniform(0.0, 1.0, n)
    p = 1.0 - slope
    lo, hi = 1.0, float(ratio)
    m = np.power(lo**p + u * (hi**p - lo**p), 1.0 / p)
    return m / m.sum()


@dataclasses.dataclass(frozen=True)
class SimConfig:
    """Parameters of one tree/Hermite run (template: Section 3)."""

    name: str
    n: int
    seed: int
    theta: float
    eps: float
    dt_tree: float
    eta: float
    t_end: float
    n_crit: int
    n_leaf: int = 1
    mass_seed: int | None = None  # Salpeter masses when set
    mass_ratio: float = 100.0

    @property
    def eps2(self) -> float:
        return self.eps * self.eps


CONFIGS = {
    # small plain case, FP64
    "plummer2k": SimConfig("plummer2k", 2048, 1, 0.5, 1.0 / 256, 1.0 / 128, 0.02, 1.0 / 8, 64),
    # FP64 vs mixed on identical lists
    "plummer16k": SimConfig("plummer16k", 16384, 2, 0.4, 1.0 / 1024, 1.0 / 256, 0.01, 1.0 / 4, 256),
    # the headline case: 2^20 particles, Salpeter masses, 64 block steps after start-up
    "plummer1m_salpeter": SimConfig(
        "plummer1m_salpeter", 1 << 20, 3, 0.4, 4.0 / (1 << 20), 1.0 / 512, 0.01, 1.0 / 512, 2048,
        mass_seed=4,
    ),
}


def config(name: str, **overrides) -> SimConfig:
    c = CONFIGS[name]
    return dataclasses.replace(c, **overrides) if overrides else c


def make_initial_conditions(cfg: SimConfig):
    x, v, m = plummer(cfg.n, cfg.seed)
    if cfg.mass_seed is not None:
        m = salpeter_masses(cfg.n, cfg.mass_seed, cfg.mass_ratio)
        x -= (m[:, None] * x).sum(0) / m.sum()
        v -= (m[:, None] * v).sum(0) / m.sum()
    return x, v, m


def random_block_state(n: int, seed: int, t_now: float, dt_levels=(3, 12)):
    """Synthetic per-particle Hermite state for predictor/force tests at t_now.

    Each particle gets a power-of-two step 2^-k (k uniform in dt_levels) and
    a last-update time t0 = t_now - j*2^-k for j in {0, 1} rounded to a
    multiple of its step, plus accelerations and jerks of unit scale.  Only
    random numbers; the physics is whatever the caller does with them.
    """
    rng = _rng(seed)
    k = rng.integers(dt_levels[0], dt_levels[1] + 1, n)
    dt = np.ldexp(1.0, -k)
    back = rng.integers(0, 2, n)
    t0 = np.floor(t_now / dt) * dt - back * dt
    a = rng.normal(0.0, 1.0, (n, 3))
    jerk = rng.normal(0.0, 4.0, (n, 3))
    return t0, a, jerk


def ensemble_sizes(count: int, seed: int, lo: int, hi: int):
    """Cluster sizes log-uniform in [lo, hi] (batched / served workloads)."""
    rng = _rng(seed)
    u = rng.uniform(math.log(lo), math.log(hi), count)
    return np.floor(np.exp(u)).astype(np.int64)
