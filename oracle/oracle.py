"""ctypes shim over the FP64 CPU oracle (oracle.c) and its Hermite integrator.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It never imports the product
package and the product package never imports it; the two share nothing but
the seeded inputs they are both given.

The integrator follows the tree/Hermite procedure of Section 2 (steps 1-7):
the tree, groups and interaction lists are rebuilt at every multiple of the
tree interval, when all particles are synchronised (the maximum step equals
the tree interval); in between, each block step predicts all particles and
nodes to the block time, sums forces over the active particles' lists,
corrects them and picks new block steps.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)


# -O3 without contraction or fast-math: every result is the IEEE-rounded value of
# the stated operation order, so optimisation level and instruction set change no
# bit.  The default instruction set is portable; native=True builds for the
# machine it runs on (the CPU baseline does, on the host it is timed on).
FLAGS = ["-O3", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-fopenmp"]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", *FLAGS, "-o", _LIB_PATH + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def use_native_build() -> str:
    """Compile oracle.c for this machine's instruction set into a library of
    its own and make it the one this module calls (the same bits: see FLAGS)."""
    global _LIB_PATH, _lib
    path = os.path.join(_HERE, "liboracle_native.so")
    cmd = ["gcc", *FLAGS, "-march=native", "-o", path + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(path + ".tmp", path)
    _LIB_PATH, _lib = path, None
    return path


def build_flags(native: bool = False) -> str:
    return " ".join(FLAGS + (["-march=native"] if native else []))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        L.orc_hilbert_key.restype = ctypes.c_uint64
        L.orc_hilbert_key.argtypes = [ctypes.c_uint32] * 3
        L.orc_hilbert_keys.argtypes = [ctypes.c_int64, _u32p, _u64p]
        L.orc_root_box.argtypes = [ctypes.c_int64, _dp, _dp, _dp]
        L.orc_quantize.argtypes = [ctypes.c_int64, _dp, _dp, ctypes.c_double, _u32p]
        L.orc_tree_build.restype = ctypes.c_void_p
        L.orc_tree_build.argtypes = [ctypes.c_int64, _dp, _dp, _dp, _dp, _dp, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_double]
        L.orc_tree_free.argtypes = [ctypes.c_void_p]
        L.orc_tree_sizes.argtypes = [ctypes.c_void_p, _i64p, _i64p, _i64p, _i64p]
        L.orc_tree_root.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.orc_tree_get.argtypes = [ctypes.c_void_p, _i64p, _u64p, _dp, _dp, _dp, _dp, _dp, _i32p, _i64p,
                                   _i64p, _i64p, _i64p, _i32p]
        L.orc_predict.argtypes = [ctypes.c_int64, ctypes.c_double, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_force_list.argtypes = [ctypes.c_int64, _i32p, _dp, _dp, _dp, ctypes.c_double, ctypes.c_int64,
                                     _i64p, _i64p, _i32p, _dp, _dp, _dp]
        L.orc_force_direct.argtypes = [ctypes.c_int64, _i32p, ctypes.c_int64, _dp, _dp, _dp, ctypes.c_double,
                                       _dp, _dp, _dp]
        L.orc_correct.argtypes = [ctypes.c_int64, ctypes.c_double, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                                  ctypes.c_double, _dp, _dp, _dp]
        L.orc_block_step.restype = ctypes.c_double
        L.orc_block_step.argtypes = [ctypes.c_double] * 4
        L.orc_energy.argtypes = [ctypes.c_int64, _dp, _dp, _dp, ctypes.c_double, _dp, _dp]
        _lib = L
    return _lib


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _p(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


# --------------------------------------------------------------------------- keys / box
def hilbert_key(qx: int, qy: int, qz: int) -> int:
    return int(lib().orc_hilbert_key(qx, qy, qz))


def hilbert_keys(q) -> np.ndarray:
    q = _c(q, np.uint32).reshape(-1, 3)
    out = np.empty(q.shape[0], np.uint64)
    lib().orc_hilbert_keys(q.shape[0], _p(q, ctypes.c_uint32), _p(out, ctypes.c_uint64))
    return out


def root_box(x):
    x = _c(x, np.float64).reshape(-1, 3)
    lo = np.zeros(3)
    side = np.zeros(1)
    lib().orc_root_box(x.shape[0], _p(x, ctypes.c_double), _p(lo, ctypes.c_double), _p(side, ctypes.c_double))
    return lo, float(side[0])


def quantize(x, lo, side):
    x = _c(x, np.float64).reshape(-1, 3)
    lo = _c(lo, np.float64)
    q = np.empty((x.shape[0], 3), np.uint32)
    lib().orc_quantize(x.shape[0], _p(x, ctypes.c_double), _p(lo, ctypes.c_double), side, _p(q, ctypes.c_uint32))
    return q


# --------------------------------------------------------------------------- tree
class Tree:
    """Everything the oracle builds at a tree time, copied into numpy arrays."""

    def __init__(self, x, v, a, jerk, m, n_leaf: int, n_crit: int, theta: float):
        x = _c(x, np.float64).reshape(-1, 3)
        n = x.shape[0]
        v = _c(v, np.float64).reshape(n, 3)
        a = _c(a, np.float64).reshape(n, 3)
        jerk = _c(jerk, np.float64).reshape(n, 3)
        m = _c(m, np.float64).reshape(n)
        L = lib()
        h = L.orc_tree_build(n, _p(x, ctypes.c_double), _p(v, ctypes.c_double), _p(a, ctypes.c_double),
                             _p(jerk, ctypes.c_double), _p(m, ctypes.c_double), n_leaf, n_crit, theta)
        if not h:
            raise ValueError("orc_tree_build rejected its arguments")
        try:
            M, G, L_, C = (ctypes.c_int64() for _ in range(4))
            L.orc_tree_sizes(h, ctypes.byref(M), ctypes.byref(G), ctypes.byref(L_), ctypes.byref(C))
            M, G, Ln = M.value, G.value, L_.value
            self.n, self.n_node, self.n_group, self.n_entries, self.n_cell = n, M, G, Ln, C.value
            self.perm = np.empty(n, np.int64)
            self.keys = np.empty(n, np.uint64)
            self.node_m = np.empty(M)
            self.node_x = np.empty((M, 3))
            self.node_v = np.empty((M, 3))
            self.node_a = np.empty((M, 3))
            self.node_j = np.empty((M, 3))
            self.node_level = np.empty(M, np.int32)
            self.node_begin = np.empty(M, np.int64)
            self.node_end = np.empty(M, np.int64)
            self.group_first = np.empty(G + 1, np.int64)
            self.list_off = np.empty(G + 1, np.int64)
            self.entries = np.empty(Ln, np.int32)
            d = ctypes.c_double
            L.orc_tree_get(h, _p(self.perm, ctypes.c_int64), _p(self.keys, ctypes.c_uint64), _p(self.node_m, d),
                           _p(self.node_x, d), _p(self.node_v, d), _p(self.node_a, d), _p(self.node_j, d),
                           _p(self.node_level, ctypes.c_int32), _p(self.node_begin, ctypes.c_int64),
                           _p(self.node_end, ctypes.c_int64), _p(self.group_first, ctypes.c_int64),
                           _p(self.list_off, ctypes.c_int64), _p(self.entries, ctypes.c_int32))
            lo = np.zeros(3)
            side = np.zeros(1)
            L.orc_tree_root(h, _p(lo, d), _p(side, d))
            self.lo, self.side = lo, float(side[0])
        finally:
            L.orc_tree_free(h)
        self.theta, self.n_crit, self.n_leaf = theta, n_crit, n_leaf

    def list_of(self, g: int) -> np.ndarray:
        return self.entries[self.list_off[g]:self.list_off[g + 1]]


# --------------------------------------------------------------------------- kernels
def predict(t, t0, x, v, a, jerk):
    x = _c(x, np.float64).reshape(-1, 3)
    n = x.shape[0]
    t0 = _c(np.broadcast_to(t0, (n,)), np.float64)
    v, a, jerk = (_c(u, np.float64).reshape(n, 3) for u in (v, a, jerk))
    xp = np.empty((n, 3))
    vp = np.empty((n, 3))
    d = ctypes.c_double
    lib().orc_predict(n, float(t), _p(t0, d), _p(x, d), _p(v, d), _p(a, d), _p(jerk, d), _p(xp, d), _p(vp, d))
    return xp, vp


def force_list(active, xp, vp, m, eps2, group_first, list_off, entries):
    active = _c(active, np.int32)
    xp = _c(xp, np.float64).reshape(-1, 3)
    vp = _c(vp, np.float64).reshape(-1, 3)
    m = _c(m, np.float64)
    gf = _c(group_first, np.int64)
    lo = _c(list_off, np.int64)
    en = _c(entries, np.int32)
    k = active.shape[0]
    acc = np.zeros((k, 3))
    jerk = np.zeros((k, 3))
    pot = np.zeros(k)
    d = ctypes.c_double
    lib().orc_force_list(k, _p(active, ctypes.c_int32), _p(xp, d), _p(vp, d), _p(m, d), float(eps2),
                         gf.shape[0] - 1, _p(gf, ctypes.c_int64), _p(lo, ctypes.c_int64),
                         _p(en, ctypes.c_int32), _p(acc, d), _p(jerk, d), _p(pot, d))
    return acc, jerk, pot


def force_direct(active, xp, vp, m, eps2, n=None):
    active = _c(active, np.int32)
    xp = _c(xp, np.float64).reshape(-1, 3)
    vp = _c(vp, np.float64).reshape(-1, 3)
    m = _c(m, np.float64)
    n = xp.shape[0] if n is None else int(n)
    k = active.shape[0]
    acc = np.zeros((k, 3))
    jerk = np.zeros((k, 3))
    pot = np.zeros(k)
    d = ctypes.c_double
    lib().orc_force_direct(k, _p(active, ctypes.c_int32), n, _p(xp, d), _p(vp, d), _p(m, d), float(eps2),
                           _p(acc, d), _p(jerk, d), _p(pot, d))
    return acc, jerk, pot


def correct(t1, t0, xp, vp, a0, j0, a1, j1, eta):
    xp = _c(xp, np.float64).reshape(-1, 3)
    k = xp.shape[0]
    t0 = _c(np.broadcast_to(t0, (k,)), np.float64)
    vp, a0, j0, a1, j1 = (_c(u, np.float64).reshape(k, 3) for u in (vp, a0, j0, a1, j1))
    x1 = np.empty((k, 3))
    v1 = np.empty((k, 3))
    dta = np.empty(k)
    d = ctypes.c_double
    lib().orc_correct(k, float(t1), _p(t0, d), _p(xp, d), _p(vp, d), _p(a0, d), _p(j0, d), _p(a1, d),
                      _p(j1, d), float(eta), _p(x1, d), _p(v1, d), _p(dta, d))
    return x1, v1, dta


def block_step(dt, t1, dt_tree, dt_old=0.0) -> float:
    return float(lib().orc_block_step(float(dt), float(t1), float(dt_tree), float(dt_old)))


def energy(x, v, m, eps2):
    x = _c(x, np.float64).reshape(-1, 3)
    n = x.shape[0]
    v = _c(v, np.float64).reshape(n, 3)
    m = _c(m, np.float64)
    K = ctypes.c_double()
    W = ctypes.c_double()
    d = ctypes.c_double
    lib().orc_energy(n, _p(x, d), _p(v, d), _p(m, d), float(eps2), ctypes.byref(K), ctypes.byref(W))
    return K.value, W.value


# --------------------------------------------------------------------------- integrator
class TreeHermite:
    """Tree/Hermite block-step integrator (Section 2, steps 1-7), all FP64.

    mode="tree": forces over interaction lists rebuilt at multiples of dt_tree.
    mode="direct": the original Hermite scheme, forces over all particles.

    ``on_step(sim, rec)`` is called after every block step's force with a dict
    holding the j-memory state the force saw (t, active ids, particle and node
    Hermite data, lists) and the forces, so a test can replay the same step
    elsewhere.  Particle arrays are kept in the current tree order; ``ids``
    maps them back to the initial particle numbers.
    """

    def __init__(self, x, v, m, *, eps2, dt_tree, eta, theta=0.5, n_crit=64, n_leaf=1, mode="tree",
                 on_step=None, dt_initial=None):
        if mode not in ("tree", "direct"):
            raise ValueError(mode)
        self.x = _c(x, np.float64).reshape(-1, 3).copy()
        self.n = self.x.shape[0]
        self.v = _c(v, np.float64).reshape(self.n, 3).copy()
        self.m = _c(m, np.float64).reshape(self.n).copy()
        self.eps2, self.dt_tree, self.eta = float(eps2), float(dt_tree), float(eta)
        self.theta, self.n_crit, self.n_leaf, self.mode = float(theta), int(n_crit), int(n_leaf), mode
        self.on_step = on_step
        self.a = np.zeros((self.n, 3))
        self.j = np.zeros((self.n, 3))
        self.t0 = np.zeros(self.n)
        self.dt = np.zeros(self.n)
        self.ids = np.arange(self.n)
        self.t = 0.0
        self.tree = None
        self.t_tree = 0.0
        self.n_block_steps = 0
        self.n_particle_steps = 0
        self.n_interactions = 0
        if mode == "tree":
            self._rebuild()
        everyone = np.arange(self.n, dtype=np.int32)
        acc, jerk, pot = self._force(0.0, everyone, self.x, self.v, None)
        self.a, self.j = acc, jerk
        self.pot = pot
        if mode == "tree":
            self._rebuild()          # same order; nodes now carry a and jerk
        for k in range(self.n):
            if dt_initial is not None:
                raw = dt_initial
            else:
                na, nj = np.linalg.norm(self.a[k]), np.linalg.norm(self.j[k])
                raw = self.eta * na / nj if nj > 0 else self.dt_tree
            h = block_step(raw, 0.0, self.dt_tree, 0.0)
            if h == 0.0:
                raise FloatingPointError("initial block step below 2^-40")
            self.dt[k] = h

    # -- step 1: tree, groups, lists (all particles synchronised at t_tree)
    def _rebuild(self):
        tr = Tree(self.x, self.v, self.a, self.j, self.m, self.n_leaf, self.n_crit, self.theta)
        p = tr.perm
        for name in ("x", "v", "a", "j", "m", "t0", "dt", "ids"):
            setattr(self, name, getattr(self, name)[p].copy())
        if hasattr(self, "pot"):
            self.pot = self.pot[p].copy()
        self.tree = tr
        self.t_tree = self.t

    def _jmem(self, t):
        """Predicted combined memory at t: particles then nodes."""
        xp, vp = predict(t, self.t0, self.x, self.v, self.a, self.j)
        if self.mode == "direct" or self.tree.n_node == 0:
            return xp, vp, self.m
        tr = self.tree
        nxp, nvp = predict(t, np.full(tr.n_node, self.t_tree), tr.node_x, tr.node_v, tr.node_a, tr.node_j)
        return np.vstack([xp, nxp]), np.vstack([vp, nvp]), np.concatenate([self.m, tr.node_m])

    def _force(self, t, active, xp_p, vp_p, full):
        if self.mode == "direct":
            xp, vp, mm = (xp_p, vp_p, self.m) if full is None else full
            return force_direct(active, xp, vp, mm, self.eps2, n=self.n)
        xp, vp, mm = self._jmem(t) if full is None else full
        tr = self.tree
        acc, jerk, pot = force_list(active, xp, vp, mm, self.eps2, tr.group_first, tr.list_off, tr.entries)
        self.n_interactions += int(self.interactions(active))
        return acc, jerk, pot

    def interactions(self, active):
        """Sum of list lengths over the active particles (pairs the list force visits)."""
        tr = self.tree
        g = np.searchsorted(tr.group_first, active, side="right") - 1
        return int((tr.list_off[g + 1] - tr.list_off[g]).sum())

    def next_time(self):
        return float(np.min(self.t0 + self.dt))

    def step(self):
        """One block step (Section 2, steps 2-7)."""
        tn = self.next_time()
        active = np.flatnonzero(self.t0 + self.dt == tn).astype(np.int32)
        full = self._jmem(tn) if self.mode == "tree" else None
        if full is None:
            xp, vp = predict(tn, self.t0, self.x, self.v, self.a, self.j)
            full = (xp, vp, self.m)
        xp, vp = full[0], full[1]
        acc, jerk, pot = self._force(tn, active, None, None, full)
        if self.on_step is not None:
            self.on_step(self, dict(t=tn, active=active, acc=acc, jerk=jerk, pot=pot))
        x1, v1, dta = correct(tn, self.t0[active], xp[active], vp[active], self.a[active], self.j[active],
                              acc, jerk, self.eta)
        for q, k in enumerate(active):
            h = block_step(dta[q], tn, self.dt_tree, self.dt[k])
            if h == 0.0:
                raise FloatingPointError(f"block step below 2^-40 for particle {self.ids[k]} at t={tn}")
            self.dt[k] = h
        self.x[active], self.v[active], self.a[active], self.j[active] = x1, v1, acc, jerk
        self.pot[active] = pot
        self.t0[active] = tn
        self.t = tn
        self.n_block_steps += 1
        self.n_particle_steps += active.size
        if self.mode == "tree" and np.fmod(tn, self.dt_tree) == 0.0:
            if not np.all(self.t0 == tn):
                raise AssertionError("particles not synchronised at a tree time")
            self._rebuild()
        return tn, active

    def run(self, t_end):
        while self.next_time() <= t_end:
            self.step()
        return self

    def energy(self):
        """Total energy at the current time (direct potential), valid when synchronised."""
        xp, vp = predict(self.t, self.t0, self.x, self.v, self.a, self.j)
        K, W = energy(xp, vp, self.m, self.eps2)
        return K + W
