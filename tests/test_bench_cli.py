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
    # counted flop per interface point (about 5.6k since the solver's moment
    # products are evaluated as one-dimensional combinations), and the
    # calibrated bytes of one launch (state read plus interface results
    # written: at least the algorithmic 0.81 + 3.36 GB of the 2048^2 workload)
    assert 5000 < bench.FLOPS_PER_IFACE_POINT_STAGE1 < 8000
    assert 4.17e9 <= bench.TRAFFIC_BYTES_PER_LAUNCH_STAGE1 < 6e9


def test_roofline_constants_come_from_the_committed_profile():
    """bench.py's flop and traffic figures for the stage-1 interface sweep are
    the ones the committed rocprofv3 summary records for that kernel (its
    counter table row: flop / unit, read GB, written GB after calibration)."""
    import re
    sys.path.insert(0, ROOT)
    import bench
    rows = [ln for ln in open(os.path.join(ROOT, "profiles", "k_edges2d_shear2048.md"))
            if ln.startswith("| `k_edges2d<1, double, false>`") and ln.count("|") >= 8]
    assert rows, "counter row of the stage-1 interface sweep"
    cells = [c.strip() for c in rows[0].strip().strip("|").split("|")]
    flop_per_point = int(cells[4])
    read_gb, written_gb = float(cells[5]), float(cells[6])
    assert bench.FLOPS_PER_IFACE_POINT_STAGE1 == flop_per_point
    assert abs(bench.TRAFFIC_BYTES_PER_LAUNCH_STAGE1 - (read_gb + written_gb) * 1e9) <= 2e6
    assert re.search(r"2 \(n\+3\)\^2", open(os.path.join(ROOT, "profiles", "k_edges2d_shear2048.md")).read())


def test_3d_flop_constant_comes_from_the_committed_profile():
    import re
    sys.path.insert(0, ROOT)
    import bench
    txt = open(os.path.join(ROOT, "profiles", "k_edges3d_taylor_green128.md")).read()
    rows = [ln for ln in txt.splitlines() if ln.startswith("| `k_edges3d<true, false>`") and ln.count("|") >= 8]
    assert rows
    cells = [c.strip() for c in rows[0].strip().strip("|").split("|")]
    assert bench.FLOPS_PER_SOLVE_3D_STAGE1 == int(cells[4])
    assert re.search(r"12 interface solves per cell", txt)


def test_fused_roofline_constants_come_from_the_committed_profile():
    """The default stage's dominant kernel (the fused interface sweep and
    update): flop per node update and calibrated bytes per launch as the
    committed rocprofv3 summary records them."""
    sys.path.insert(0, ROOT)
    import bench
    txt = open(os.path.join(ROOT, "profiles", "k_fused2d_shear2048.md")).read()
    rows = [ln for ln in txt.splitlines() if ln.startswith("| `k_fused2d<1, double, false>`") and ln.count("|") >= 8]
    assert rows, "counter row of the stage-1 fused kernel"
    cells = [c.strip() for c in rows[0].strip().strip("|").split("|")]
    assert bench.FLOPS_PER_NODE_FUSED_STAGE1 == int(cells[4])
    read_gb, written_gb = float(cells[5]), float(cells[6])
    assert abs(bench.TRAFFIC_BYTES_PER_LAUNCH_FUSED_STAGE1 - (read_gb + written_gb) * 1e9) <= 2e6
    assert "2 n^2" in txt
