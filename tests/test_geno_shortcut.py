"""The GENO routine decides smooth data (path function saturated, chi = 1)
before any division; tests/geno_shortcut.cpp checks on the host, over seeded
smoothness indicators spanning the double range, that this never changes a
result bit against the full path function and blend (CPU)."""
import json
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def test_smooth_test_keeps_every_bit(tmp_path):
    import pytest
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "geno_shortcut")
    subprocess.run([HIPCC, "-std=c++17", "-O2", "--cuda-host-only", "-x", "hip",
                    os.path.join(HERE, "geno_shortcut.cpp"), "-o", exe], check=True, capture_output=True)
    r = json.loads(subprocess.run([exe], check=True, capture_output=True, text=True).stdout)
    print(r)
    assert r["total"] == 4 * 3 * 4 * 250000
    assert r["saturated"] > r["total"] // 10  # the smooth case is well represented
    assert r["differ"] == 0
