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
    """The counters count while the kernel sources and the build hash as recorded, and read
    null otherwise."""
    import hashlib
    import bench
    pkg = os.path.join(ROOT, "paper_2309_14545_amd")
    now = {}
    for f in bench.TRAFFIC["sources"]:
        with open(os.path.join(pkg, f), "rb") as fh:
            now[f] = hashlib.sha256(fh.read()).hexdigest()[:16]
    fresh = dict(bench.TRAFFIC, sources=now)
    monkeypatch.setattr(bench, "TRAFFIC", fresh)
    want = (fresh["fetch_kib"] * fresh["fetch_scale"] +
            fresh["write_kib"] * fresh["write_scale"]) * 1024.0
    assert bench.measured_traffic(fresh["workload"]) == want
    assert bench.measured_traffic("edges8_shelf") is None          # counters of another batch
    for f in now:
        stale = dict(fresh, sources=dict(now, **{f: "0" * 16}))
        monkeypatch.setattr(bench, "TRAFFIC", stale)
        assert bench.measured_traffic(stale["workload"]) is None
