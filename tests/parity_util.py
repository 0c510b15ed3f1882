"""Helpers shared by the GPU parity tests: the tolerances, the per-particle
relative error and the oracle's list force on an FP64 j-memory.

Tolerances (per particle, relative to that particle's own magnitude):
  FP64 form   acc, jerk, pot <= 1e-12
  mixed form  acc <= 2e-6, jerk <= 1e-5, pot <= 1e-6
"""
import sys

import numpy as np

TOL = {"fp64": (1e-12, 1e-12, 1e-12), "mixed": (2e-6, 1e-5, 1e-6)}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_rows(got, want):
    got = np.asarray(got).reshape(len(want), -1)
    want = np.asarray(want).reshape(len(want), -1)
    return np.linalg.norm(got - want, axis=1) / np.maximum(np.linalg.norm(want, axis=1), 1e-300)


def errors(got, want):
    return tuple(float(rel_rows(g, w).max()) if len(w) else 0.0 for g, w in zip(got, want))


def assert_close(tag, prec, got, want):
    ea, ej, ep = errors(got, want)
    ta, tj, tp = TOL[prec]
    assert ea <= ta and ej <= tj and ep <= tp, f"{tag} {prec}: acc {ea:.3g} jerk {ej:.3g} pot {ep:.3g}"
    return ea, ej, ep


def oracle_list_force(oracle, t, act, t0, m, x, v, a, j, tree, eps2, t_tree=0.0):
    """The oracle's list force at block time t on the FP64 j-memory: particles
    (t0, m, x, v, a, jerk) and the tree's nodes (valid at t_tree), both
    predicted by the oracle; no input is rounded to the mixed form's storage."""
    xp, vp = oracle.predict(t, t0, x, v, a, j)
    nxp, nvp = oracle.predict(t, t_tree, tree.node_x, tree.node_v, tree.node_a, tree.node_j)
    return oracle.force_list(act, np.vstack([xp, nxp]), np.vstack([vp, nvp]), np.concatenate([m, tree.node_m]),
                             eps2, tree.group_first, tree.list_off, tree.entries)


