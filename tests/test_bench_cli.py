"""bench.py's contract on the host: it measures one GPU, and asking for more
ends with a message and a nonzero status before anything touches a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_counted_traffic_is_null_once_the_sources_change(tmp_path):
    """roofline.traffic comes from a committed counter summary only while the
    kernel sources hash to the value it was taken on."""
    import hashlib
    sys.path.insert(0, ROOT)
    import bench
    src = tmp_path / "k.hip"
    src.write_bytes(b"kernel v1\n")
    sha = hashlib.sha256(b"kernel v1\n").hexdigest()
    summary = tmp_path / "counters.md"
    summary.write_text("text\n```\nsource_sha256=%s\ntraffic_bytes_per_launch.a=1.5e+09\n"
                       "traffic_bytes_per_launch.ab=7\n```\n" % sha)
    key = "traffic_bytes_per_launch.a"
    assert bench._counted_traffic(str(summary), [str(src)], key) == 1.5e9
    assert bench._counted_traffic(str(summary), [str(src)], "traffic_bytes_per_launch.b") is None
    assert bench._counted_traffic(str(tmp_path / "missing.md"), [str(src)], key) is None
    src.write_bytes(b"kernel v2\n")
    assert bench._counted_traffic(str(summary), [str(src)], key) is None
