"""Host-side checks of bench.py that need no GPU: it refuses more than one GPU before touching
the device, and reports HBM traffic only while the kernel sources hash as they did when the
counters were taken."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_follows_the_kernel_sources(monkeypatch):
    import bench
    t = bench.measured_traffic(bench.TRAFFIC["workload"])
    want = (bench.TRAFFIC["fetch_kib"] * bench.TRAFFIC["fetch_scale"] +
            bench.TRAFFIC["write_kib"] * bench.TRAFFIC["write_scale"]) * 1024.0
    assert t == want, "the committed counters no longer match the kernel sources"
    assert bench.measured_traffic("edges8_shelf") is None          # counters of another batch
    stale = dict(bench.TRAFFIC, sources=dict(bench.TRAFFIC["sources"], **{"vk_kernels.hip": "0" * 16}))
    monkeypatch.setattr(bench, "TRAFFIC", stale)
    assert bench.measured_traffic(stale["workload"]) is None
