"""Host-side checks of bench.py (CPU): more than one GPU is refused before
any GPU work, and the roofline constants are consistent."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_roofline_constants():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.PEAK_FP64_TFLOPS == 78.6
    # counted flop per interface point, and the calibrated bytes of one launch
    # (state read plus interface results written: at least the algorithmic
    # 0.81 + 3.36 GB of the 2048^2 workload)
    assert 6000 < bench.FLOPS_PER_IFACE_POINT_STAGE1 < 8000
    assert 4.17e9 <= bench.TRAFFIC_BYTES_PER_LAUNCH_STAGE1 < 6e9
