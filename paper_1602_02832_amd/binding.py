"""Thin ctypes binding over the native libraries (argument marshalling only).

``libhtree.so`` (include/htree.h) runs every step of the block-step force
evaluation on the GPU; ``libhtree_host.so`` (include/htree_host.h) builds the
tree, groups and lists and runs the host's Hermite bookkeeping.  Both must
have been built in-tree (``python -m paper_1602_02832_amd.build``): there is
no fallback, a missing library raises.

Names follow the C entry points: ``Context.set_j_particles`` calls
``ht_set_j_particles`` and so on.  Host arrays are numpy; device arrays are
torch CUDA tensors (PyTorch provides device memory and streams only).
"""
from __future__ import annotations

import ctypes
import os
import types

import numpy as np

from . import build as _build

__all__ = ["HTError", "Context", "Batch", "HT_ROW", "make_rows", "HostTree", "DeviceTree", "force_batch_async",
           "hilbert_keys",
           "next_block", "correct", "initial_steps", "device_lib", "host_lib"]

HT_PREC = {"fp64": 0, "mixed": 1}
HT_PREDICT = {"fused": 0, "eager": 1}

_c_i32p = ctypes.POINTER(ctypes.c_int32)
_c_i64p = ctypes.POINTER(ctypes.c_int64)
_c_u32p = ctypes.POINTER(ctypes.c_uint32)
_c_u64p = ctypes.POINTER(ctypes.c_uint64)
_c_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


class HTError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"htree error {code}: {message}")
        self.code = code


class HtdView(ctypes.Structure):
    """htd_view (include/htree_tree.h): device pointers to a device-built tree."""
    _fields_ = [(name, ctypes.c_void_p) for name in
                ("perm", "keys", "x", "v", "a", "jerk", "m", "node_m", "node_x", "node_v", "node_a", "node_j",
                 "group_first", "list_off", "entries")]


class HtbCluster(ctypes.Structure):
    """htb_cluster (include/htree_host.h): one cluster's host arrays."""
    _fields_ = [("n", ctypes.c_int64), ("eta", ctypes.c_double), ("dt_tree", ctypes.c_double),
                ("t0", _c_dp), ("dt", _c_dp), ("x", _c_dp), ("v", _c_dp), ("a", _c_dp), ("jerk", _c_dp),
                ("m", _c_dp), ("pot", _c_dp), ("active", _c_i32p), ("n_active", ctypes.c_int64),
                ("t_next", ctypes.c_double)]


class HtConfig(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("precision", ctypes.c_int32), ("predict_mode", ctypes.c_int32),
                ("n_max", ctypes.c_int32), ("node_max", ctypes.c_int32), ("group_max", ctypes.c_int32),
                ("list_max", ctypes.c_int64), ("active_max", ctypes.c_int32), ("eps2", ctypes.c_double),
                ("stream", ctypes.c_void_p)]


# ht_row (include/htree.h): one corrected particle for a j-memory update
HT_ROW = np.dtype([("idx", np.int32), ("pad", np.int32), ("t0", np.float64), ("m", np.float64),
                   ("x", np.float64, 3), ("v", np.float64, 3), ("a", np.float64, 3), ("jerk", np.float64, 3)],
                  align=True)
assert HT_ROW.itemsize == 120


def make_rows(idx, t0, m, x, v, a, jerk):
    """Pack corrected particles into ht_row records (host)."""
    idx = np.asarray(idx)
    r = np.empty(idx.shape[0], HT_ROW)
    r["idx"] = idx
    r["pad"] = 0
    r["t0"] = t0
    r["m"] = m
    r["x"] = x
    r["v"] = v
    r["a"] = a
    r["jerk"] = jerk
    return r


_dev = None
_host = None


def _load(path):
    if not os.path.exists(path):
        raise RuntimeError(f"{os.path.basename(path)} is not built; run `python -m paper_1602_02832_amd.build`")
    return ctypes.CDLL(path)


def device_lib():
    global _dev
    if _dev is None:
        # PyTorch brings its own HIP runtime.  Load it first so that the device
        # library binds to that same runtime: streams and device pointers from
        # torch are then valid in the library, and the process holds one HIP
        # runtime instead of two.
        import torch  # noqa: F401
        L = _load(_build.DEVICE_LIB)
        i, i64, d = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sig = {
            "ht_workspace_bytes": [ctypes.POINTER(HtConfig), ctypes.POINTER(ctypes.c_size_t)],
            "ht_create": [ctypes.POINTER(_vp), ctypes.POINTER(HtConfig), _vp, ctypes.c_size_t],
            "ht_destroy": [_vp],
            "ht_set_j_particles": [_vp, i, _c_i32p, _c_dp, _c_dp, _c_dp, _c_dp, _c_dp, _c_dp],
            "ht_set_j_particles_async": [_vp, i, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
            "ht_set_nodes": [_vp, i, d, _c_dp, _c_dp, _c_dp, _c_dp, _c_dp],
            "ht_set_interaction_lists": [_vp, i, _c_i64p, _c_i64p, _c_i32p],
            "ht_predict": [_vp, d],
            "ht_force": [_vp, i, _c_i32p, _c_dp, _c_dp, _c_dp],
            "ht_force_async": [_vp, i, _c_i32p, _vp, _vp, _vp],
            "ht_force_direct": [_vp, i, _c_i32p, _c_dp, _c_dp, _c_dp],
            "ht_force_direct_async": [_vp, i, _c_i32p, _vp, _vp, _vp],
            "ht_get_predicted": [_vp, i, _c_i32p, _c_dp, _c_dp],
            "ht_step_async": [_vp, i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, d, i, _vp, _vp, _vp, _vp],
            "ht_step_graph": [_vp, i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, d, i, _vp, _vp, _vp, _vp],
            "ht_state_enable": [_vp],
            "ht_state_set": [_vp, i, _c_dp, _c_dp, _c_dp, _c_dp, _c_dp, _c_dp, _c_dp, _c_dp],
            "ht_state_get": [_vp, _c_dp, _c_dp, _c_dp, _c_dp, _c_dp, _c_dp, _c_dp],
            "ht_dev_next_block": [_vp, ctypes.POINTER(ctypes.c_double), _c_i64p, ctypes.POINTER(_c_i32p)],
            "ht_dev_step": [_vp, d, d],
            "ht_dev_step_direct": [_vp, d, d],
            "ht_dev_run": [_vp, d, d, d, i, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double), _c_i64p],
            "ht_state_rebuild": [_vp, _vp, i, i, d, d, _c_i64p],
            "ht_force_batch_async": [i, ctypes.POINTER(_vp), _c_i32p, ctypes.POINTER(_c_i32p),
                                     ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp)],
            "ht_sync": [_vp],
            "ht_last_stats": [_vp, _c_i64p, _c_i32p],
            "ht_set_timing": [_vp, i],
            "ht_set_tuning": [_vp, d, d],
            "ht_kernel_timing": [_vp, _c_dp, _c_i64p, _c_i64p],
            "ht_last_error": [],
            "ht_predict_many": [i, ctypes.POINTER(_vp), _c_dp],
            "ht_batch_workspace_bytes": [i, i64, i64, i64, ctypes.POINTER(ctypes.c_size_t)],
            "ht_batch_create": [ctypes.POINTER(_vp), i, _vp, i, i64, i64, i64, _vp, ctypes.c_size_t],
            "ht_batch_destroy": [_vp],
            "ht_batch_update_async": [_vp, i, ctypes.POINTER(_vp), _c_i32p, ctypes.POINTER(_vp)],
            "ht_batch_force_async": [_vp, i, ctypes.POINTER(_vp), _c_i32p, ctypes.POINTER(_c_i32p),
                                     ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp)],
            "ht_batch_sync": [_vp],
            "ht_batch_set_timing": [_vp, i],
            "ht_batch_kernel_timing": [_vp, _c_dp, _c_i64p, _c_i64p],
            "ht_batch_last_stats": [_vp, _c_i64p, _c_i32p],
            "ht_force_direct_noalloc": [i, _vp, i, i, _vp, _vp, _vp, d, i, _vp, i, _vp, _vp, _vp],
            "ht_batch_dev_run": [_vp, i, _vp, _vp, _vp, _vp, _vp, i, _vp, _vp, _vp, _vp, _vp,
                                 ctypes.POINTER(ctypes.c_int32)],
            "ht_state_bytes": [ctypes.POINTER(HtConfig), ctypes.POINTER(ctypes.c_size_t)],
            "ht_set_list_form": [_vp, i],
            "ht_set_union_width": [_vp, i],
            "ht_set_placement": [_vp, i],
            "ht_get_placement": [_vp, _c_i32p, _c_i32p],
            "ht_state_enable_ws": [_vp, _vp, ctypes.c_size_t],
            "ht_pool_create": [ctypes.POINTER(_vp), i, ctypes.c_size_t],
            "ht_pool_destroy": [_vp],
            "ht_cluster_admit": [_vp, ctypes.POINTER(HtConfig), i, _c_i64p, ctypes.POINTER(ctypes.c_size_t)],
            "ht_pool_reserve": [_vp, ctypes.c_size_t, _c_i64p],
            "ht_pool_resize": [_vp, i64, ctypes.c_size_t],
            "ht_cluster_release": [_vp, i64],
            "ht_pool_usage": [_vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t), _c_i32p],
            "htd_device_bytes": [_vp, ctypes.POINTER(ctypes.c_size_t)],
            "htd_create": [ctypes.POINTER(_vp), i, _vp, i64],
            "htd_destroy": [_vp],
            "htd_build": [_vp, i64, _vp, _vp, _vp, _vp, _vp, i, i, d],
            "htd_sizes": [_vp, _c_i64p, _c_i64p, _c_i64p, _c_i64p],
            "htd_root": [_vp, _c_dp, _c_dp],
            "htd_get": [_vp, _c_i64p, ctypes.POINTER(ctypes.c_uint64), _c_dp, _c_dp, _c_dp, _c_dp, _c_dp, _c_i32p,
                        _c_i64p, _c_i64p, _c_i64p, _c_i64p, _c_i32p],
            "htd_device_view": [_vp, ctypes.POINTER(HtdView)],
            "htd_phase_ms": [_vp, _c_dp],
            "htd_last_error": [],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_char_p if name in ("ht_last_error", "htd_last_error") else ctypes.c_int
        _ = i64
        _dev = L
    return _dev


def host_lib():
    global _host
    if _host is None:
        L = _load(_build.HOST_LIB)
        i, i64, d = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sig = {
            "htb_build": [ctypes.POINTER(_vp), i64, _c_dp, _c_dp, _c_dp, _c_dp, _c_dp, i, i, d],
            "htb_sizes": [_vp, _c_i64p, _c_i64p, _c_i64p],
            "htb_get": [_vp, _c_i64p, _c_u64p, _c_dp, _c_dp, _c_dp, _c_dp, _c_dp, _c_i32p, _c_i64p, _c_i64p,
                        _c_i64p, _c_i64p, _c_i32p],
            "htb_free": [_vp],
            "htb_hilbert_keys": [i64, _c_u32p, _c_u64p],
            "htb_next_block": [i64, _c_dp, _c_dp, _c_dp, _c_i32p, _c_i64p],
            "htb_correct": [i64, _c_i32p, d, d, d, _c_dp, _c_dp, _c_dp, _c_dp, _c_dp, _c_dp, _c_dp, _c_dp],
            "htb_initial_steps": [i64, d, d, _c_dp, _c_dp, _c_dp],
            "htb_next_block_many": [i, ctypes.POINTER(HtbCluster)],
            "htb_correct_many": [i, ctypes.POINTER(HtbCluster), _c_i64p, _c_dp, _c_dp, _c_dp, _c_i64p, _vp, _c_i32p],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = None if name == "htb_free" else ctypes.c_int
        _host = L
    return _host


_raw_fns = {}


def _raw(name, nargs):
    """The device library's entry point `name` with every argument passed as a
    plain integer (addresses included): for callers that keep handles and
    pointers in numpy arrays."""
    f = _raw_fns.get(name)
    if f is None:
        f = device_lib()[name]
        f.argtypes = [ctypes.c_void_p] * nargs
        f.restype = ctypes.c_int
        _raw_fns[name] = f
    return f


def _raw_host(name, nargs):
    """The host library's entry point `name` with every argument a plain integer."""
    key = ("host", name)
    f = _raw_fns.get(key)
    if f is None:
        f = host_lib()[name]
        f.argtypes = [ctypes.c_void_p] * nargs
        f.restype = ctypes.c_int
        _raw_fns[key] = f
    return f


def _check(rc: int):
    if rc != 0:
        msg = device_lib().ht_last_error()
        raise HTError(rc, msg.decode() if msg else "")


def _arr(a, dtype, shape=None):
    a = np.ascontiguousarray(a, dtype=dtype)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype)) if a is not None else None


_NONE7 = (None,) * 7


_TORCH_DTYPE = {"f64": "torch.float64", "i32": "torch.int32"}


def _dptr(t, kind=None, count=0, what="array"):
    """Device address of a torch tensor (or an int address, or None).  A
    tensor must be a contiguous device tensor of `kind` ("f64", "i32") with
    at least `count` elements, else ValueError: the library reads that many
    from the address.  Int addresses are the caller's own and pass as they are."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{what}: a contiguous device tensor is needed")
    if kind is not None and str(t.dtype) != _TORCH_DTYPE[kind]:
        raise ValueError(f"{what}: dtype {t.dtype}, expected {_TORCH_DTYPE[kind]}")
    if t.numel() < count:
        raise ValueError(f"{what}: {t.numel()} elements, the call reads {count}")
    return t.data_ptr()


def _rows_ptrs(n, tensors):
    """Addresses of update rows (idx, t0, m, x, v, a, jerk) for n rows."""
    kinds = (("i32", 1, "idx"), ("f64", 1, "t0"), ("f64", 1, "m"), ("f64", 3, "x"), ("f64", 3, "v"),
             ("f64", 3, "a"), ("f64", 3, "jerk"))
    return tuple(_dptr(t, k, w * n, what) for t, (k, w, what) in zip(tensors, kinds))


def _out_ptrs(n, d_acc, d_jerk, d_pot):
    """Addresses of the outputs for n active particles."""
    return (_dptr(d_acc, "f64", 3 * n, "acc"), _dptr(d_jerk, "f64", 3 * n, "jerk"), _dptr(d_pot, "f64", n, "pot"))


# --------------------------------------------------------------------------------------------- device
class Context:
    """One cluster's j-memory, lists and work buffers on one GPU (ht_ctx)."""

    def __init__(self, *, n_max, node_max, group_max, list_max, active_max, eps2, precision="fp64",
                 predict_mode="fused", device=0, stream=None, torch_workspace=True):
        L = device_lib()
        self.cfg = HtConfig(device, HT_PREC[precision], HT_PREDICT[predict_mode], int(n_max), int(node_max),
                            int(group_max), int(list_max), int(active_max), float(eps2),
                            None if stream is None else int(stream))
        self.precision = precision
        nbytes = ctypes.c_size_t()
        _check(L.ht_workspace_bytes(ctypes.byref(self.cfg), ctypes.byref(nbytes)))
        self.workspace_bytes = nbytes.value
        self._ws = None
        ws_ptr = None
        if torch_workspace:
            import torch
            self._ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=f"cuda:{device}")
            ws_ptr = self._ws.data_ptr()
        h = _vp()
        _check(L.ht_create(ctypes.byref(h), ctypes.byref(self.cfg), ws_ptr, self.workspace_bytes))
        self._h = h
        self._step_async = L.ht_step_async
        self._n = 0   # particle count of the last full upload (the library writes that many in state_get)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            device_lib().ht_destroy(self._h)
            self._h = None
            self._ws = None
            self._state_ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_j_particles(self, t0, m, x, v, a, jerk, idx=None):
        m = _arr(m, np.float64)
        n = m.shape[0]
        t0 = _arr(np.broadcast_to(t0, (n,)), np.float64)
        x, v, a, jerk = (_arr(u, np.float64, (n, 3)) for u in (x, v, a, jerk))
        idx = None if idx is None else _arr(idx, np.int32)
        if idx is not None and idx.shape != (n,):
            raise ValueError(f"idx {idx.shape}: one index per row ({n})")
        d = ctypes.c_double
        _check(device_lib().ht_set_j_particles(self._h, n, _ptr(idx, ctypes.c_int32), _ptr(t0, d), _ptr(m, d),
                                               _ptr(x, d), _ptr(v, d), _ptr(a, d), _ptr(jerk, d)))
        if idx is None:
            self._n = n

    def set_j_particles_async(self, n, d_idx, d_t0, d_m, d_x, d_v, d_a, d_jerk):
        _check(device_lib().ht_set_j_particles_async(self._h, int(n),
                                                     *_rows_ptrs(int(n), (d_idx, d_t0, d_m, d_x, d_v, d_a, d_jerk))))

    def set_nodes(self, t_tree, m, x, v, a, jerk):
        m = _arr(m, np.float64)
        n = m.shape[0]
        x, v, a, jerk = (_arr(u, np.float64, (n, 3)) for u in (x, v, a, jerk))
        d = ctypes.c_double
        _check(device_lib().ht_set_nodes(self._h, n, float(t_tree), _ptr(m, d), _ptr(x, d), _ptr(v, d), _ptr(a, d),
                                         _ptr(jerk, d)))

    def set_interaction_lists(self, group_first, list_off, entries):
        gf = _arr(group_first, np.int64)
        lo = _arr(list_off, np.int64)
        en = _arr(entries, np.int32)
        # the library reads G + 1 offsets of each kind and list_off[G] entries
        if gf.ndim != 1 or gf.shape[0] < 1 or lo.shape != gf.shape:
            raise ValueError(f"group_first {gf.shape} and list_off {lo.shape} must be one-dimensional, of equal length")
        if en.ndim != 1 or lo[-1] > en.shape[0]:
            raise ValueError(f"list_off ends at {int(lo[-1])} but entries holds {en.shape[0]}")
        _check(device_lib().ht_set_interaction_lists(self._h, gf.shape[0] - 1, _ptr(gf, ctypes.c_int64),
                                                     _ptr(lo, ctypes.c_int64), _ptr(en, ctypes.c_int32)))

    def set_placement(self, runs):
        """ht_set_placement: work items in `runs` stretches, one per XCD (0: the
        device's XCD count, 1: off)."""
        _check(device_lib().ht_set_placement(self._h, int(runs)))

    def placement(self):
        """(runs in use, the device's XCD count)."""
        r, x = ctypes.c_int32(), ctypes.c_int32()
        _check(device_lib().ht_get_placement(self._h, ctypes.byref(r), ctypes.byref(x)))
        return r.value, x.value

    def set_list_form(self, form):
        """ht_set_list_form: "csr" (default), "runs" (run-length lists with the
        groups' node copies) or "union" (union tiles over runs of groups); the
        lists must be set again afterwards."""
        _check(device_lib().ht_set_list_form(self._h, {"csr": 0, "runs": 1, "union": 2}[form]))

    def set_union_width(self, width):
        """ht_set_union_width: groups per run of the union tiles (2..8)."""
        _check(device_lib().ht_set_union_width(self._h, int(width)))

    def predict(self, t):
        _check(device_lib().ht_predict(self._h, float(t)))

    def _force_host(self, fn, active):
        active = _arr(active, np.int32)
        k = active.shape[0]
        acc = np.empty((k, 3))
        jerk = np.empty((k, 3))
        pot = np.empty(k)
        d = ctypes.c_double
        _check(fn(self._h, k, _ptr(active, ctypes.c_int32), _ptr(acc, d), _ptr(jerk, d), _ptr(pot, d)))
        return acc, jerk, pot

    def force(self, active):
        return self._force_host(device_lib().ht_force, active)

    def force_direct(self, active):
        return self._force_host(device_lib().ht_force_direct, active)

    def force_async(self, active, d_acc, d_jerk, d_pot):
        active = _arr(active, np.int32)
        _check(device_lib().ht_force_async(self._h, active.shape[0], _ptr(active, ctypes.c_int32),
                                           *_out_ptrs(active.shape[0], d_acc, d_jerk, d_pot)))

    def force_direct_async(self, active, d_acc, d_jerk, d_pot):
        active = _arr(active, np.int32)
        _check(device_lib().ht_force_direct_async(self._h, active.shape[0], _ptr(active, ctypes.c_int32),
                                                  *_out_ptrs(active.shape[0], d_acc, d_jerk, d_pot)))

    def step_async(self, upd, t, active, d_acc, d_jerk, d_pot):
        """ht_step_async: upd = (n, d_idx, d_t0, d_m, d_x, d_v, d_a, d_jerk) or None
        (device tensors, or addresses when d_idx is an int); active = int32 ids,
        or (count, host address) of int32 ids that the caller keeps alive until
        the call returns; outputs as tensors or addresses.  Called once per
        block step, so the marshalling takes the short way for addresses."""
        if type(active) is tuple:
            n_act, a_ptr = active
        else:
            active = _arr(active, np.int32)
            n_act, a_ptr = active.shape[0], active.ctypes.data
        if upd is None:
            n_upd, ptrs = 0, _NONE7
        else:
            n_upd, ptrs = upd[0], (upd[1:] if type(upd[1]) is int else _rows_ptrs(int(upd[0]), upd[1:]))
        if type(d_acc) is not int:
            d_acc, d_jerk, d_pot = _out_ptrs(n_act, d_acc, d_jerk, d_pot)
        rc = self._step_async(self._h, n_upd, *ptrs, t, n_act, a_ptr, d_acc, d_jerk, d_pot)
        if rc:
            _check(rc)

    def step_graph(self, upd, t, active, d_acc, d_jerk, d_pot):
        """ht_step_graph: as step_async, replayed through the context's HIP graphs."""
        active = _arr(active, np.int32)
        if upd is None:
            n_upd, ptrs = 0, (None,) * 7
        else:
            n_upd, ptrs = int(upd[0]), _rows_ptrs(int(upd[0]), upd[1:])
        _check(device_lib().ht_step_graph(self._h, n_upd, *ptrs, float(t), active.shape[0], active.ctypes.data,
                                          *_out_ptrs(active.shape[0], d_acc, d_jerk, d_pot)))

    # device-resident integration ------------------------------------------------
    def state_enable(self, torch_memory=True):
        """ht_state_enable: the resident FP64 state, by default in a torch
        allocation of ht_state_bytes (ht_state_enable_ws), so that all of the
        context's device memory comes from torch's allocator."""
        if getattr(self, "_state_ws", None) is not None:
            return
        if torch_memory:
            import torch
            nbytes = state_bytes(self.cfg)
            self._state_ws = torch.empty(nbytes, dtype=torch.uint8, device=f"cuda:{self.cfg.device}")
            _check(device_lib().ht_state_enable_ws(self._h, self._state_ws.data_ptr(), nbytes))
        else:
            self._state_ws = False
            _check(device_lib().ht_state_enable(self._h))

    def state_set(self, t0, dt, m, x, v, a, jerk, pot=None):
        """ht_state_set: full FP64 state (and the j-records) from host arrays."""
        n = np.asarray(t0).shape[0]
        d = ctypes.c_double
        arrs = [_arr(t0, np.float64), _arr(dt, np.float64), _arr(m, np.float64), _arr(x, np.float64, (n, 3)),
                _arr(v, np.float64, (n, 3)), _arr(a, np.float64, (n, 3)), _arr(jerk, np.float64, (n, 3))]
        p = None if pot is None else _arr(pot, np.float64)
        if any(u.shape != (n,) for u in arrs[:3] + ([p] if p is not None else [])):
            raise ValueError(f"t0, dt, m (and pot) must hold {n} entries each")
        _check(device_lib().ht_state_set(self._h, n, *[_ptr(u, d) for u in arrs], _ptr(p, d)))
        self._n = n

    def state_get(self, n=None):
        """ht_state_get: (t0, dt, x, v, a, jerk, pot) host copies of the device state
        (its N entries; n, if given, must be N)."""
        if n is None:
            n = self._n
        if n != self._n:
            raise ValueError(f"the state holds {self._n} particles, not {n}")
        t0, dt, pot = np.empty(n), np.empty(n), np.empty(n)
        x, v, a, j = (np.empty((n, 3)) for _ in range(4))
        d = ctypes.c_double
        _check(device_lib().ht_state_get(self._h, *[_ptr(u, d) for u in (t0, dt, x, v, a, j, pot)]))
        return t0, dt, x, v, a, j, pot

    def dev_next_block(self):
        """ht_dev_next_block: (t_next, active ids) of the next block step, from the
        device state (the ids are a copy)."""
        t = ctypes.c_double()
        k = ctypes.c_int64()
        p = _c_i32p()
        _check(device_lib().ht_dev_next_block(self._h, ctypes.byref(t), ctypes.byref(k), ctypes.byref(p)))
        act = np.ctypeslib.as_array(p, shape=(k.value,)).copy() if k.value else np.empty(0, np.int32)
        return t.value, act

    def dev_step(self, eta, dt_tree):
        """ht_dev_step: force, corrector and j-record update of the last next block, on the device."""
        _check(device_lib().ht_dev_step(self._h, float(eta), float(dt_tree)))

    def dev_run(self, eta, dt_tree, t_stop, max_steps):
        """ht_dev_run: up to max_steps block steps on the device, stopping at t_stop;
        returns (steps, block time of the last step, particle steps)."""
        k, t, p = ctypes.c_int32(), ctypes.c_double(), ctypes.c_int64()
        _check(device_lib().ht_dev_run(self._h, float(eta), float(dt_tree), float(t_stop), int(max_steps),
                                       ctypes.byref(k), ctypes.byref(t), ctypes.byref(p)))
        return k.value, t.value, p.value

    def dev_step_direct(self, eta, dt_tree):
        """ht_dev_step_direct: as dev_step with the force over all particles (the direct scheme)."""
        _check(device_lib().ht_dev_step_direct(self._h, float(eta), float(dt_tree)))

    def state_rebuild(self, tree, n, n_leaf, n_crit, theta, t_tree, out=None):
        """ht_state_rebuild: step 1 on the device for the resident state with the
        DeviceTree `tree`; returns perm (perm[new] = old), in `out` if given
        (int64, n entries; pinned memory makes the copy faster)."""
        if n != self._n:
            raise ValueError(f"the state holds {self._n} particles, not {n}")
        perm = np.empty(n, np.int64) if out is None else out
        if perm.dtype != np.int64 or perm.shape != (n,) or not perm.flags.c_contiguous:
            raise ValueError("out must be a contiguous int64 array of n entries")
        _check(device_lib().ht_state_rebuild(self._h, tree._h, int(n_leaf), int(n_crit), float(theta),
                                             float(t_tree), _ptr(perm, ctypes.c_int64)))
        return perm

    def get_predicted(self, idx):
        idx = _arr(idx, np.int32)
        n = idx.shape[0]
        xp = np.empty((n, 3))
        vp = np.empty((n, 3))
        d = ctypes.c_double
        _check(device_lib().ht_get_predicted(self._h, n, _ptr(idx, ctypes.c_int32), _ptr(xp, d), _ptr(vp, d)))
        return xp, vp

    def sync(self):
        _check(device_lib().ht_sync(self._h))

    def set_tuning(self, gather_cost=12.0, target_items=2048.0):
        _check(device_lib().ht_set_tuning(self._h, float(gather_cost), float(target_items)))

    def set_timing(self, enable=True):
        _check(device_lib().ht_set_timing(self._h, 1 if enable else 0))

    def kernel_timing(self):
        """(force kernel ms, launches, pairs) since timing was enabled or last read."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        p = ctypes.c_int64()
        _check(device_lib().ht_kernel_timing(self._h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(p)))
        return ms.value, n.value, p.value

    def last_stats(self):
        p = ctypes.c_int64()
        w = ctypes.c_int32()
        _check(device_lib().ht_last_stats(self._h, ctypes.byref(p), ctypes.byref(w)))
        return p.value, w.value


def predict_many(ctxs, t):
    n = len(ctxs)
    t = _arr(t, np.float64)
    H = (_vp * n)(*[c.handle for c in ctxs])
    _check(device_lib().ht_predict_many(n, H, _ptr(t, ctypes.c_double)))


def predict_many_raw(n, handles, t):
    """ht_predict_many with the handle and time arrays given by address."""
    _check(_raw("ht_predict_many", 3)(n, handles, t))


def force_batch_async(ctxs, actives, d_accs, d_jerks, d_pots):
    """ht_force_batch_async over several contexts sharing one stream."""
    n = len(ctxs)
    acts = [_arr(a, np.int32) for a in actives]
    H = (_vp * n)(*[c.handle for c in ctxs])
    N = (ctypes.c_int32 * n)(*[a.shape[0] for a in acts])
    P = (_c_i32p * n)(*[_ptr(a, ctypes.c_int32) for a in acts])
    outs = [_out_ptrs(a.shape[0], *o) for a, o in zip(acts, zip(d_accs, d_jerks, d_pots))]
    A = (_vp * n)(*[o[0] for o in outs])
    J = (_vp * n)(*[o[1] for o in outs])
    Q = (_vp * n)(*[o[2] for o in outs])
    _check(device_lib().ht_force_batch_async(n, H, N, P, A, J, Q))
    return acts  # keep host arrays alive until the caller syncs


def state_bytes(cfg) -> int:
    """ht_state_bytes: device bytes of a resident state for this HtConfig."""
    out = ctypes.c_size_t()
    _check(device_lib().ht_state_bytes(ctypes.byref(cfg), ctypes.byref(out)))
    return int(out.value)


class Pool:
    """Admission by device footprint (ht_pool): a budget of device bytes and
    the reservations held against it.  admit() returns a reservation id, or
    None when the cluster does not fit beside what is held now; it raises
    HTError with code -2 when the cluster exceeds the whole budget."""

    def __init__(self, budget_bytes, device=0):
        self._h = _vp()
        _check(device_lib().ht_pool_create(ctypes.byref(self._h), int(device), int(budget_bytes)))
        self.budget = int(budget_bytes)

    def admit(self, cfg, resident):
        rid, nbytes = ctypes.c_int64(), ctypes.c_size_t()
        rc = device_lib().ht_cluster_admit(self._h, ctypes.byref(cfg), int(bool(resident)), ctypes.byref(rid),
                                           ctypes.byref(nbytes))
        if rc == -3:
            return None, int(nbytes.value)
        _check(rc)
        return int(rid.value), int(nbytes.value)

    def reserve(self, nbytes):
        rid = ctypes.c_int64()
        rc = device_lib().ht_pool_reserve(self._h, int(nbytes), ctypes.byref(rid))
        if rc == -3:
            return None
        _check(rc)
        return int(rid.value)

    def resize(self, rid, nbytes):
        """True when the pool is within its budget afterwards (the size is recorded either way)."""
        rc = device_lib().ht_pool_resize(self._h, int(rid), int(nbytes))
        if rc == -3:
            return False
        _check(rc)
        return True

    def release(self, rid):
        _check(device_lib().ht_cluster_release(self._h, int(rid)))

    def usage(self):
        used, budget, n = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_int32()
        _check(device_lib().ht_pool_usage(self._h, ctypes.byref(used), ctypes.byref(budget), ctypes.byref(n)))
        return int(used.value), int(budget.value), int(n.value)

    def close(self):
        if getattr(self, "_h", None):
            device_lib().ht_pool_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def force_direct_noalloc(precision, d_x, d_v, d_m, eps2, d_active, j_splits, d_acc, d_jerk, d_pot, n=None,
                         n_active=None, stream=None, device=0):
    """ht_force_direct_noalloc: the direct sum on caller-owned device arrays
    (torch tensors or addresses), partial sums in the library's fixed scratch
    array; asynchronous on `stream` (a torch stream, a hipStream_t address or
    None for the null stream)."""
    n = int(d_m.shape[0]) if n is None else int(n)
    n_active = int(d_active.shape[0]) if n_active is None else int(n_active)
    st = getattr(stream, "cuda_stream", stream)
    _check(device_lib().ht_force_direct_noalloc(int(device), st, HT_PREC[precision], n,
                                                _dptr(d_x, "f64", 3 * n, "x"), _dptr(d_v, "f64", 3 * n, "v"),
                                                _dptr(d_m, "f64", n, "m"), float(eps2), n_active,
                                                _dptr(d_active, "i32", n_active, "active"), int(j_splits),
                                                *_out_ptrs(n_active, d_acc, d_jerk, d_pot)))


class Batch:
    """Batched engine object (ht_batch): one update copy + one scatter and one
    plan copy + one force launch per engine step for all member contexts."""

    def __init__(self, *, stream, max_clusters, max_items, max_active, max_rows, device=0, torch_workspace=True):
        L = device_lib()
        nbytes = ctypes.c_size_t()
        _check(L.ht_batch_workspace_bytes(int(max_clusters), int(max_items), int(max_active), int(max_rows),
                                          ctypes.byref(nbytes)))
        self.workspace_bytes = nbytes.value
        self._ws = None
        ws_ptr = None
        if torch_workspace:
            import torch
            self._ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=f"cuda:{device}")
            ws_ptr = self._ws.data_ptr()
        h = _vp()
        _check(L.ht_batch_create(ctypes.byref(h), int(device), int(stream), int(max_clusters), int(max_items),
                                 int(max_active), int(max_rows), ws_ptr, self.workspace_bytes))
        self._h = h
        self._keep = None

    def close(self):
        if getattr(self, "_h", None):
            device_lib().ht_batch_destroy(self._h)
            self._h = None
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def update_async(self, ctxs, rows_list):
        n = len(ctxs)
        rows_list = [np.ascontiguousarray(r, dtype=HT_ROW) for r in rows_list]
        H = (_vp * n)(*[c.handle for c in ctxs])
        N = (ctypes.c_int32 * n)(*[r.shape[0] for r in rows_list])
        R = (_vp * n)(*[r.ctypes.data if r.shape[0] else None for r in rows_list])
        _check(device_lib().ht_batch_update_async(self._h, n, H, N, R))
        self._keep = rows_list   # pinned copy is taken before return; kept for clarity

    def update_async_raw(self, n, handles, n_rows, rows, pinned=False):
        """ht_batch_update_async (pinned: ht_batch_update_pinned_async) with
        every array given by address (handles and row pointers: arrays of n
        addresses; n_rows: n int32)."""
        name = "ht_batch_update_pinned_async" if pinned else "ht_batch_update_async"
        _check(_raw(name, 5)(self._h.value, n, handles, n_rows, rows))

    def force_async_raw(self, n, handles, n_active, ids, d_accs, d_jerks, d_pots):
        """ht_batch_force_async with every array given by address (n_active: n
        int32; the others arrays of n addresses)."""
        _check(_raw("ht_batch_force_async", 8)(self._h.value, n, handles, n_active, ids, d_accs, d_jerks, d_pots))

    def dev_next_block_raw(self, n, handles, t_next, n_active, active):
        """ht_batch_dev_next_block with every array given by address (t_next: n
        float64, n_active: n int64, active: n addresses, all written)."""
        _check(_raw("ht_batch_dev_next_block", 6)(self._h.value, n, handles, t_next, n_active, active))

    def dev_step_raw(self, n, handles, eta, dt_tree):
        """ht_batch_dev_step with every array given by address (eta, dt_tree: n float64)."""
        _check(_raw("ht_batch_dev_step", 5)(self._h.value, n, handles, eta, dt_tree))

    def dev_run(self, handles, eta, dt_tree, t_stop, max_steps, engine_steps):
        """ht_batch_dev_run over the contexts with these handles (uint64 array):
        returns (steps, t_last, particle_steps, pairs, engine-step ms)."""
        n = int(handles.shape[0])
        handles = np.ascontiguousarray(handles, dtype=np.uint64)
        eta, dt_tree, t_stop = (np.ascontiguousarray(u, dtype=np.float64) for u in (eta, dt_tree, t_stop))
        max_steps = np.ascontiguousarray(max_steps, dtype=np.int32)
        steps = np.empty(n, np.int32)
        t_last = np.empty(n)
        psteps = np.empty(n, np.int64)
        pairs = np.empty(n, np.int64)
        step_ms = np.empty(int(engine_steps))
        n_ms = ctypes.c_int32()
        _check(device_lib().ht_batch_dev_run(self._h, n, handles.ctypes.data, eta.ctypes.data, dt_tree.ctypes.data,
                                             t_stop.ctypes.data, max_steps.ctypes.data, int(engine_steps),
                                             steps.ctypes.data, t_last.ctypes.data, psteps.ctypes.data,
                                             pairs.ctypes.data, step_ms.ctypes.data, ctypes.byref(n_ms)))
        return steps, t_last, psteps, pairs, step_ms[:n_ms.value].copy()

    def force_async(self, ctxs, actives, d_accs, d_jerks, d_pots):
        n = len(ctxs)
        acts = [_arr(a, np.int32) for a in actives]
        H = (_vp * n)(*[c.handle for c in ctxs])
        N = (ctypes.c_int32 * n)(*[a.shape[0] for a in acts])
        P = (_c_i32p * n)(*[_ptr(a, ctypes.c_int32) for a in acts])
        outs = [_out_ptrs(a.shape[0], *o) for a, o in zip(acts, zip(d_accs, d_jerks, d_pots))]
        A = (_vp * n)(*[o[0] for o in outs])
        J = (_vp * n)(*[o[1] for o in outs])
        Q = (_vp * n)(*[o[2] for o in outs])
        _check(device_lib().ht_batch_force_async(self._h, n, H, N, P, A, J, Q))

    def sync(self):
        _check(device_lib().ht_batch_sync(self._h))

    def set_timing(self, enable=True):
        _check(device_lib().ht_batch_set_timing(self._h, 1 if enable else 0))

    def kernel_timing(self):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        p = ctypes.c_int64()
        _check(device_lib().ht_batch_kernel_timing(self._h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(p)))
        return ms.value, n.value, p.value

    def last_stats(self):
        p = ctypes.c_int64()
        w = ctypes.c_int32()
        _check(device_lib().ht_batch_last_stats(self._h, ctypes.byref(p), ctypes.byref(w)))
        return p.value, w.value


# ----------------------------------------------------------------------------------------------- host
class HostTree:
    """Tree, node moments, groups and lists (htb_build), copied into numpy arrays."""

    def __init__(self, x, v, a, jerk, m, n_leaf: int, n_crit: int, theta: float):
        L = host_lib()
        x = _arr(x, np.float64, (-1, 3))
        n = x.shape[0]
        v, a, jerk = (_arr(u, np.float64, (n, 3)) for u in (v, a, jerk))
        m = _arr(m, np.float64, (n,))
        d = ctypes.c_double
        h = _vp()
        rc = L.htb_build(ctypes.byref(h), n, _ptr(x, d), _ptr(v, d), _ptr(a, d), _ptr(jerk, d), _ptr(m, d),
                         int(n_leaf), int(n_crit), float(theta))
        if rc != 0:
            raise HTError(rc, "htb_build failed")
        try:
            M, G, E = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
            L.htb_sizes(h, ctypes.byref(M), ctypes.byref(G), ctypes.byref(E))
            M, G, E = M.value, G.value, E.value
            self.n, self.n_node, self.n_group, self.n_entries = n, M, G, E
            self.perm = np.empty(n, np.int64)
            self.keys = np.empty(n, np.uint64)
            self.node_m = np.empty(M)
            self.node_x, self.node_v, self.node_a, self.node_j = (np.empty((M, 3)) for _ in range(4))
            self.node_level = np.empty(M, np.int32)
            self.node_begin = np.empty(M, np.int64)
            self.node_end = np.empty(M, np.int64)
            self.group_first = np.empty(G + 1, np.int64)
            self.list_off = np.empty(G + 1, np.int64)
            self.entries = np.empty(E, np.int32)
            L.htb_get(h, _ptr(self.perm, ctypes.c_int64), _ptr(self.keys, ctypes.c_uint64), _ptr(self.node_m, d),
                      _ptr(self.node_x, d), _ptr(self.node_v, d), _ptr(self.node_a, d), _ptr(self.node_j, d),
                      _ptr(self.node_level, ctypes.c_int32), _ptr(self.node_begin, ctypes.c_int64),
                      _ptr(self.node_end, ctypes.c_int64), _ptr(self.group_first, ctypes.c_int64),
                      _ptr(self.list_off, ctypes.c_int64), _ptr(self.entries, ctypes.c_int32))
        finally:
            L.htb_free(h)

    def list_of(self, g):
        return self.entries[self.list_off[g]:self.list_off[g + 1]]


def _check_tree(rc: int):
    if rc != 0:
        msg = device_lib().htd_last_error()
        raise HTError(rc, msg.decode() if msg else "")


class DeviceTree:
    """Step 1 on the device (htd_*): keys, particle order, octree, node moments,
    groups and lists from particles already in device memory.  `build` takes
    contiguous float64 device tensors; `get` copies the results into numpy
    arrays with the same names as HostTree's."""

    PHASES = ("keys", "sort", "cells", "moments", "lists", "csr", "total")

    def __init__(self, n_max: int, device: int = 0, stream=None):
        self._h = _vp()
        _check_tree(device_lib().htd_create(ctypes.byref(self._h), int(device), None if stream is None else int(stream),
                                            int(n_max)))
        self.n = 0

    def build(self, x, v, a, jerk, m, n_leaf: int, n_crit: int, theta: float):
        n = int(m.shape[0])
        for t, shape in ((x, (n, 3)), (v, (n, 3)), (a, (n, 3)), (jerk, (n, 3)), (m, (n,))):
            if tuple(t.shape) != shape or not t.is_cuda or not t.is_contiguous() or str(t.dtype) != "torch.float64":
                raise ValueError("DeviceTree.build takes contiguous float64 device tensors of matching shapes")
        _check_tree(device_lib().htd_build(self._h, n, _dptr(x), _dptr(v), _dptr(a), _dptr(jerk), _dptr(m),
                                           int(n_leaf), int(n_crit), float(theta)))
        self.n = n
        return self.sizes()

    def sizes(self):
        M, G, E, C = (ctypes.c_int64() for _ in range(4))
        _check_tree(device_lib().htd_sizes(self._h, ctypes.byref(M), ctypes.byref(G), ctypes.byref(E),
                                           ctypes.byref(C)))
        return M.value, G.value, E.value, C.value

    def root(self):
        lo = np.zeros(3)
        side = np.zeros(1)
        _check_tree(device_lib().htd_root(self._h, _ptr(lo, ctypes.c_double), _ptr(side, ctypes.c_double)))
        return lo, float(side[0])

    def get(self):
        M, G, E, C = self.sizes()
        n = self.n
        r = types.SimpleNamespace(n=n, n_node=M, n_group=G, n_entries=E, n_cell=C)
        r.perm = np.empty(n, np.int64)
        r.keys = np.empty(n, np.uint64)
        r.node_m = np.empty(M)
        r.node_x, r.node_v, r.node_a, r.node_j = (np.empty((M, 3)) for _ in range(4))
        r.node_level = np.empty(M, np.int32)
        r.node_begin = np.empty(M, np.int64)
        r.node_end = np.empty(M, np.int64)
        r.group_first = np.empty(G + 1, np.int64)
        r.list_off = np.empty(G + 1, np.int64)
        r.entries = np.empty(E, np.int32)
        d, i64 = ctypes.c_double, ctypes.c_int64
        _check_tree(device_lib().htd_get(self._h, _ptr(r.perm, i64), _ptr(r.keys, ctypes.c_uint64), _ptr(r.node_m, d),
                                         _ptr(r.node_x, d), _ptr(r.node_v, d), _ptr(r.node_a, d), _ptr(r.node_j, d),
                                         _ptr(r.node_level, ctypes.c_int32), _ptr(r.node_begin, i64),
                                         _ptr(r.node_end, i64), _ptr(r.group_first, i64), _ptr(r.list_off, i64),
                                         _ptr(r.entries, ctypes.c_int32)))
        r.lo, r.side = self.root()
        return r

    def view(self):
        v = HtdView()
        _check_tree(device_lib().htd_device_view(self._h, ctypes.byref(v)))
        return v

    def phase_ms(self):
        ms = np.zeros(7)
        _check_tree(device_lib().htd_phase_ms(self._h, _ptr(ms, ctypes.c_double)))
        return dict(zip(self.PHASES, ms.tolist()))

    def device_bytes(self):
        """Device bytes the builder holds now (htd_device_bytes)."""
        out = ctypes.c_size_t()
        _check_tree(device_lib().htd_device_bytes(self._h, ctypes.byref(out)))
        return int(out.value)

    def close(self):
        if self._h:
            device_lib().htd_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def hilbert_keys(q):
    q = _arr(q, np.uint32, (-1, 3))
    out = np.empty(q.shape[0], np.uint64)
    rc = host_lib().htb_hilbert_keys(q.shape[0], _ptr(q, ctypes.c_uint32), _ptr(out, ctypes.c_uint64))
    if rc:
        raise HTError(rc, "htb_hilbert_keys failed")
    return out


def _host_f64(arr, shape, what):
    """A C-contiguous float64 host array of the given shape, or ValueError (the
    host library reads and writes these in place)."""
    if not isinstance(arr, np.ndarray) or arr.dtype != np.float64 or not arr.flags.c_contiguous or arr.shape != shape:
        raise ValueError(f"{what}: a C-contiguous float64 array of shape {shape} is needed")
    return arr


def next_block(t0, dt, out=None):
    """(t_next, active ids) of the next block step; t0, dt float64 [n]."""
    n = t0.shape[0]
    _host_f64(t0, (n,), "t0")
    _host_f64(dt, (n,), "dt")
    out = np.empty(n, np.int32) if out is None else out
    if out.dtype != np.int32 or not out.flags.c_contiguous or out.shape[0] < n:
        raise ValueError(f"out: a C-contiguous int32 array of at least {n} entries is needed")
    tn = ctypes.c_double()
    k = ctypes.c_int64()
    d = ctypes.c_double
    rc = host_lib().htb_next_block(n, _ptr(t0, d), _ptr(dt, d), ctypes.byref(tn), _ptr(out, ctypes.c_int32),
                                   ctypes.byref(k))
    if rc:
        raise HTError(rc, "htb_next_block failed")
    return tn.value, out[:k.value]


def correct(ids, t1, eta, dt_tree, t0, dt, x, v, a, jerk, acc1, jerk1):
    """Hermite corrector + block step for particles ids (arrays updated in place)."""
    ids = _arr(ids, np.int32)
    acc1 = _arr(acc1, np.float64, (-1, 3))
    jerk1 = _arr(jerk1, np.float64, (-1, 3))
    n = t0.shape[0]
    for arr, shape, what in ((t0, (n,), "t0"), (dt, (n,), "dt"), (x, (n, 3), "x"), (v, (n, 3), "v"),
                             (a, (n, 3), "a"), (jerk, (n, 3), "jerk")):
        _host_f64(arr, shape, what)
    if acc1.shape != (ids.shape[0], 3) or jerk1.shape != (ids.shape[0], 3):
        raise ValueError("acc1 and jerk1 need one row per id")
    if ids.size and (ids.min() < 0 or ids.max() >= n):
        raise ValueError(f"ids outside [0, {n})")
    d = ctypes.c_double
    rc = host_lib().htb_correct(ids.shape[0], _ptr(ids, ctypes.c_int32), float(t1), float(eta), float(dt_tree),
                                _ptr(t0, d), _ptr(dt, d), _ptr(x, d), _ptr(v, d), _ptr(a, d), _ptr(jerk, d),
                                _ptr(acc1, d), _ptr(jerk1, d))
    if rc == -2:
        raise FloatingPointError("block step below 2^-40")
    if rc:
        raise HTError(rc, "htb_correct failed")


def cluster_struct(n, eta, dt_tree, t0, dt, x, v, a, jerk, m, pot, active):
    """HtbCluster pointing at the given arrays (which must stay alive and in place)."""
    for arr, shape, what in ((t0, (n,), "t0"), (dt, (n,), "dt"), (x, (n, 3), "x"), (v, (n, 3), "v"),
                             (a, (n, 3), "a"), (jerk, (n, 3), "jerk"), (m, (n,), "m"), (pot, (n,), "pot")):
        _host_f64(arr, shape, what)
    if active.dtype != np.int32 or not active.flags.c_contiguous or active.shape[0] < n:
        raise ValueError(f"active: a C-contiguous int32 array of at least {n} entries is needed")
    d = ctypes.c_double
    return HtbCluster(int(n), float(eta), float(dt_tree), _ptr(t0, d), _ptr(dt, d), _ptr(x, d), _ptr(v, d), _ptr(a, d),
                      _ptr(jerk, d), _ptr(m, d), _ptr(pot, d), _ptr(active, ctypes.c_int32), 0, 0.0)


def next_block_many(structs):
    rc = host_lib().htb_next_block_many(len(structs), structs)
    if rc:
        raise HTError(rc, "htb_next_block_many failed")


def next_block_many_raw(n, clusters):
    """htb_next_block_many over n htb_cluster records at address `clusters`."""
    rc = _raw_host("htb_next_block_many", 2)(n, clusters)
    if rc:
        raise HTError(rc, "htb_next_block_many failed")


def correct_many_raw(n, clusters, off, acc, jerk, pot, row_off, rows, rebuild):
    """htb_correct_many with every array given by address."""
    rc = _raw_host("htb_correct_many", 9)(n, clusters, off, acc, jerk, pot, row_off, rows, rebuild)
    if rc == -2:
        raise FloatingPointError("block step below 2^-40")
    if rc:
        raise HTError(rc, "htb_correct_many failed")


def correct_many(structs, off, acc, jerk, pot, row_off, rows, rebuild):
    d = ctypes.c_double
    rc = host_lib().htb_correct_many(len(structs), structs, _ptr(off, ctypes.c_int64), _ptr(acc, d), _ptr(jerk, d),
                                     _ptr(pot, d), _ptr(row_off, ctypes.c_int64), rows.ctypes.data,
                                     _ptr(rebuild, ctypes.c_int32))
    if rc == -2:
        raise FloatingPointError("block step below 2^-40")
    if rc:
        raise HTError(rc, "htb_correct_many failed")


def initial_steps(eta, dt_tree, a, jerk):
    a = _arr(a, np.float64, (-1, 3))
    jerk = _arr(jerk, np.float64, (-1, 3))
    dt = np.empty(a.shape[0])
    d = ctypes.c_double
    rc = host_lib().htb_initial_steps(a.shape[0], float(eta), float(dt_tree), _ptr(a, d), _ptr(jerk, d), _ptr(dt, d))
    if rc == -2:
        raise FloatingPointError("initial block step below 2^-40")
    if rc:
        raise HTError(rc, "htb_initial_steps failed")
    return dt
