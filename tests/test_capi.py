"""The C-ABI libraries load and export every entry point their headers
declare; configuration validation needs no GPU."""
import ctypes
import os
import re

import pytest

from paper_1602_02832_amd import binding as B
from paper_1602_02832_amd import build as build_mod

from conftest import gpu_available

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\s*\*)\s*(\w+)\s*\(", text, flags=re.M)))


@pytest.mark.parametrize("header,lib,least", [("htree.h", "device", 15), ("htree_tree.h", "device", 8),
                                              ("htree_host.h", "host", 8)])
def test_every_declared_symbol_is_exported(header, lib, least):
    names = declared(header)
    assert len(names) >= least
    so = ctypes.CDLL(build_mod.DEVICE_LIB if lib == "device" else build_mod.HOST_LIB)
    for name in names:
        assert hasattr(so, name), name


def test_workspace_size_and_config_validation():
    L = B.device_lib()
    cfg = B.HtConfig(0, 1, 0, 1 << 20, 1 << 20, 4096, 40_000_000, 1 << 20, 1e-11, None)
    n = ctypes.c_size_t()
    assert L.ht_workspace_bytes(ctypes.byref(cfg), ctypes.byref(n)) == 0
    # j-memory records alone are 128 bytes per particle or node
    assert n.value > 128 * (2 << 20) + 4 * 40_000_000
    bad = B.HtConfig(0, 7, 0, 10, 10, 10, 10, 10, 0.0, None)
    assert L.ht_workspace_bytes(ctypes.byref(bad), ctypes.byref(n)) == -1
    assert b"invalid configuration" in L.ht_last_error()
    bad = B.HtConfig(0, 0, 0, 0, 10, 10, 10, 10, 0.0, None)
    assert L.ht_workspace_bytes(ctypes.byref(bad), ctypes.byref(n)) == -1


def test_workspace_holds_one_record_line_per_entry():
    """Every particle and node owns one 128-byte j-memory record (one cache
    line per list-indexed gather), whatever the precision form."""
    L = B.device_lib()
    for prec in (0, 1):
        sizes = []
        for n in (100000, 200000):
            cfg = B.HtConfig(0, prec, 0, n, n, 1000, 1000000, n, 1e-4, None)
            b = ctypes.c_size_t()
            assert L.ht_workspace_bytes(ctypes.byref(cfg), ctypes.byref(b)) == 0
            sizes.append(b.value)
        assert sizes[1] - sizes[0] >= 128 * 200000


@pytest.mark.skipif(gpu_available(), reason="checks the no-device error path")
def test_create_without_device_fails_cleanly():
    L = B.device_lib()
    cfg = B.HtConfig(0, 1, 0, 16, 16, 16, 16, 16, 1e-4, None)
    h = ctypes.c_void_p()
    rc = L.ht_create(ctypes.byref(h), ctypes.byref(cfg), None, 0)
    assert rc == -5 and not h.value
    assert L.ht_last_error()


def test_missing_library_raises(tmp_path, monkeypatch):
    monkeypatch.setattr(build_mod, "DEVICE_LIB", str(tmp_path / "absent.so"))
    monkeypatch.setattr(B, "_dev", None)
    with pytest.raises(RuntimeError, match="not built"):
        B.device_lib()
