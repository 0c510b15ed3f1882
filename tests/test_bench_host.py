"""Host-side parts of bench.py that run without a GPU: the one-GPU contract and
argument parsing."""
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), (["--gpus", "8"], {}), ([], {"WORLD_SIZE": "2"})],
                         ids=["gpus2", "gpus8", "world_size2"])
def test_more_than_one_gpu_exits_with_a_message(argv, env):
    """There is no multi-GPU path: asked for one, bench.py says so and exits
    before it touches a device."""
    e = dict(os.environ, **env)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv], env=e, capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_parse_tuning():
    assert bench.parse_tuning("12,1024") == (12.0, 1024.0)
    assert bench.parse_tuning("8.5, 256") == (8.5, 256.0)
    with pytest.raises(ValueError):
        bench.parse_tuning("12")


def test_traffic_reported_only_for_the_profiled_source_and_window(monkeypatch):
    """roofline.traffic comes from byte counters taken on one kernel source and
    one window: it is reported for exactly that source and (steps, warmup), and
    is null for any other window or once the source differs."""
    here = dict(bench.TRAFFIC, kernel_source_sha256=bench.kernel_source_sha256(), steps=20, warmup=5,
                fetch_bytes_per_launch=1.0e8, write_bytes_per_launch=2.0e5)
    monkeypatch.setattr(bench, "TRAFFIC", here)
    assert bench.measured_traffic(20, 5) == 1.0e8 + 2.0e5
    assert bench.measured_traffic(64, 8) is None
    assert bench.measured_traffic(20, 4) is None
    monkeypatch.setattr(bench, "TRAFFIC", dict(here, kernel_source_sha256="0" * 64))
    assert bench.measured_traffic(20, 5) is None
    monkeypatch.setattr(bench, "TRAFFIC", dict(here, fetch_bytes_per_launch=None))
    assert bench.measured_traffic(20, 5) is None
