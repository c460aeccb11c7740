"""Host-side checks of bench.py that need no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_sgs_source_digest_is_stable():
    sys.path.insert(0, ROOT)
    import bench
    d1, d2 = bench.sgs_source_digest(), bench.sgs_source_digest()
    assert d1 == d2 and len(d1) == 16


def test_measured_traffic_follows_the_kernel_sources(monkeypatch):
    """The committed counter record is used only while the half sweep's
    sources are the ones it was taken with; it then reads about the
    algorithmic 432 bytes per update of 524,288 cells."""
    sys.path.insert(0, ROOT)
    import bench
    t = bench.measured_traffic()
    if t is not None:
        assert 0.95 < t / (432 * 524288) < 1.2
    monkeypatch.setattr(bench, "sgs_source_digest", lambda: "0" * 16)
    assert bench.measured_traffic() is None
