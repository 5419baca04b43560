"""CPU checks of bench.py's command-line contract (no device needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=300)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
    assert res.stdout.strip() == ""


def test_traffic_is_null_once_the_sources_change(monkeypatch):
    import bench
    fetch, write, files, digest = bench.TRAFFIC_KIB["k_force_sym"]
    monkeypatch.setitem(bench.TRAFFIC_KIB, "k_force_sym", (fetch, write, files, "0" * 16))
    assert bench.traffic_bytes("k_force_sym") is None
    assert bench.traffic_bytes("k_no_such_kernel") is None
    assert bench.traffic_bytes("split_force") is None  # several kernels: no counter bytes
    monkeypatch.setitem(bench.TRAFFIC_KIB, "k_force_sym", (1.0, 2.0, files, digest))
    got = bench.traffic_bytes("k_force_sym")
    assert got is None or got == (1.0 * 2.0 + 2.0 * 1.0) * 1024.0
