"""The oracle under host AddressSanitizer and UndefinedBehaviorSanitizer
(CPU): small 2D stages and steps (periodic, no-slip walls, characteristic
variables with reflecting walls) and a 1D reflecting run, built with g++ and
run in a subprocess; any sanitizer report fails the test."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.slow
def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "sanitize_oracle"
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", os.path.join(HERE, "sanitize_oracle.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok" in r.stdout
