"""bench.py's host-side contract (CPU): more than one GPU is refused with a
message before any device work, and the stored counter traffic covers the
kernel classes the step roofline sums."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_stored_traffic_covers_every_kernel_class():
    sys.path.insert(0, ROOT)
    import bench
    assert len(bench.TRAFFIC_SOURCES) == 16 and int(bench.TRAFFIC_SOURCES, 16) >= 0
    assert set(bench.TRAFFIC_BYTES) == set(bench.LAUNCHES_PER_STEP) == set(bench.KERNEL_VALUES)
    assert all(v > 0 for k, v in bench.TRAFFIC_BYTES.items() if k != "flux")
    assert bench.TRAFFIC_BYTES["flux"] and all(
        v > 0 and len(b.split("x")) == 2 for b, v in bench.TRAFFIC_BYTES["flux"].items())
