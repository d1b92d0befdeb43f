"""The library's reverse characteristic reconstructions (gks_adjoint.hpp:
the frame's eigenvectors depend on the line's values, so the adjoint also
flows through them), compiled for the host, against central differences of
the forward reconstructions (gks_device.hpp) along random directions, on
smooth line data where the reconstructions are differentiable (CPU).  The
GPU tests then hold the whole step adjoint to the oracle's tangent."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
G = 1.4


@pytest.fixture(scope="module")
def host_exe(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("charadj") / "char_adjoint_host")
    subprocess.run([HIPCC, "-std=c++17", "-O2", "-ffp-contract=off", "--cuda-host-only", "-x", "hip",
                    os.path.join(HERE, "char_adjoint_host.cpp"), "-o", exe], check=True, capture_output=True)
    return exe


def _line(rng, npts, h=0.05):
    """Smooth conservative states at npts consecutive nodes (local frame) and
    their averaged derivatives."""
    x0 = rng.uniform(0, 1)
    a = rng.uniform(-0.3, 0.3, size=4)
    xs = x0 + h * np.arange(npts)
    rho = 1.0 + 0.2 * np.sin(2 * xs + a[0])
    u = 0.4 * np.cos(3 * xs + a[1])
    v = 0.3 * np.sin(xs + a[2])
    p = 1.0 + 0.2 * np.cos(2 * xs + a[3])
    W = np.array([rho, rho * u, rho * v, p / (G - 1) + 0.5 * rho * (u * u + v * v)])
    dW = np.gradient(W, h, axis=1)
    return W, dW


def _run(exe, lines):
    out = subprocess.run([exe], input="\n".join(lines) + "\n", check=True, capture_output=True, text=True).stdout
    return [tuple(float(v) for v in ln.split()) for ln in out.strip().splitlines()]


def _check(exe, lines):
    """Each case at two difference steps: the GENO weights are strongly curved
    (eps_a = 1e-6), so the central difference's own error, O(eps^2), can
    reach 1e-6 at eps = 1e-6; it falls a hundredfold at eps = 1e-7, where
    round-off is still far below the bar.  A wrong reverse term stays off at
    both."""
    r6 = _run(exe, [ln + " 1e-6" for ln in lines])
    r7 = _run(exe, [ln + " 1e-7" for ln in lines])
    for (an, fd6), (_, fd7) in zip(r6, r7):
        err = min(abs(an - fd6), abs(an - fd7)) / max(1.0, abs(fd7))
        assert err <= 1e-6, (an, fd6, fd7)


@pytest.mark.parametrize("variant", [0, 1])
def test_reverse_char_line_reconstruction(host_exe, variant):
    rng = np.random.default_rng(10 + variant)
    lines = []
    for _ in range(30):
        Q, X = _line(rng, 4)
        rb = rng.standard_normal((4, 4))
        chib = rng.standard_normal()
        dQ, dX = rng.standard_normal((4, 4)), rng.standard_normal((4, 4))
        vals = [G, variant, *Q.ravel(), *X.ravel(), *rb.ravel(), chib, *dQ.ravel(), *dX.ravel()]
        lines.append("L " + " ".join(repr(float(v)) for v in vals))
    _check(host_exe, lines)


@pytest.mark.parametrize("variant", [0, 1])
def test_reverse_char_node_reconstruction(host_exe, variant):
    rng = np.random.default_rng(20 + variant)
    lines = []
    for _ in range(30):
        Q, X = _line(rng, 3)
        db = rng.standard_normal(4)
        dQ, dX = rng.standard_normal((4, 3)), rng.standard_normal((4, 3))
        vals = [G, variant, *Q.ravel(), *X.ravel(), *db, *dQ.ravel(), *dX.ravel()]
        lines.append("N " + " ".join(repr(float(v)) for v in vals))
    _check(host_exe, lines)
