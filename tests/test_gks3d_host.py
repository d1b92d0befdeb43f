"""The library's 3D gas-kinetic solvers (gks3d_device.hpp), compiled for the
host, against the oracle's 3D interface and nodal solvers on seeded states
with every component jumping, random slopes along all three axes, Euler and
Navier-Stokes (CPU).  Catches a wrong closed-form 5x5 slope, moment index or
heat-flux term before any GPU run; the GPU parity tests then check the
kernels around them."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from tests.helpers import settings

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
G = 1.4


def _state(rng):
    rho, p = 0.5 + rng.random(), 0.5 + rng.random()
    u = rng.uniform(-0.8, 0.8, 3)
    return np.array([rho, *(rho * u), p / (G - 1) + 0.5 * rho * (u @ u)])


@pytest.fixture(scope="module")
def host_exe(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("gks3d") / "gks3d_host")
    subprocess.run([HIPCC, "-std=c++17", "-O2", "-ffp-contract=off", "--cuda-host-only", "-x", "hip",
                    os.path.join(HERE, "gks3d_host.cpp"), "-o", exe], check=True, capture_output=True)
    return exe


def _run(exe, lines):
    out = subprocess.run([exe], input="\n".join(lines) + "\n", check=True, capture_output=True, text=True).stdout
    return [np.array([float(v) for v in ln.split()]) for ln in out.strip().splitlines()]


@pytest.mark.parametrize("mu", [0.0, 2e-3])
def test_interface_solver_matches_oracle(oracle, host_exe, mu):
    rng = np.random.default_rng(int(mu * 1e4) + 1)
    pr = 0.72 if mu > 0 else 1.0
    cases, lines = [], []
    for _ in range(40):
        WL, WR = _state(rng), _state(rng)
        sl = [rng.normal(size=5) for _ in range(4)]
        dt = 10 ** rng.uniform(-3, -1.5)
        c1 = rng.choice([0.0, 0.05])
        cases.append((WL, WR, sl, dt, c1))
        vals = [G, mu, pr, c1, 1.0, dt, *WL, *WR, *np.concatenate(sl)]
        lines.append("I " + " ".join(repr(float(v)) for v in vals))
    got = _run(host_exe, lines)
    for (WL, WR, sl, dt, c1), g in zip(cases, got):
        par = oracle.make_par(**settings(dim=3, nx=8, ny=8, nz=8, lx=1.0, mu=mu, prandtl=pr, tau_c1=c1))
        r = oracle.gks_interface(par, 3, WL, WR, sl[0], sl[1], sl[2], dt, Wt2=sl[3])
        for s, key in enumerate(["F", "Ft", "Wl", "Wr", "Wlt", "Wrt"]):
            o = r[key]
            err = np.abs(g[5 * s:5 * s + 5] - o).max() / np.abs(o).max()
            # time derivatives are differences of the dt/2 and dt time
            # integrals over dt^2: their round-off grows like 1/dt (measured
            # worst 1.4e-12 at dt = 1.4e-3, tau ~ dt; values stay below 2e-15)
            tol = 1e-12 * max(1.0, 0.01 / dt) if key.endswith("t") else 1e-12
            assert err < tol, (key, err, dt)


@pytest.mark.parametrize("mu", [0.0, 2e-3])
def test_nodal_solver_matches_oracle(oracle, host_exe, mu):
    rng = np.random.default_rng(int(mu * 1e4) + 7)
    pr = 0.72 if mu > 0 else 1.0
    cases, lines = [], []
    for _ in range(40):
        W = _state(rng)
        d = [rng.normal(size=5) for _ in range(3)]
        cases.append((W, d))
        lines.append("N " + " ".join(repr(float(v)) for v in [G, mu, pr, *W, *np.concatenate(d)]))
    got = _run(host_exe, lines)
    for (W, d), g in zip(cases, got):
        par = oracle.make_par(**settings(dim=3, nx=8, ny=8, nz=8, lx=1.0, mu=mu, prandtl=pr))
        r = oracle.gks_node(par, 3, W, d[0], d[1], d[2])
        for ax, (kf, kt) in enumerate((("F", "Ft"), ("G", "Gt"), ("H", "Ht"))):
            for lab, o, gg in ((kf, r[kf], g[5 * ax:5 * ax + 5]), (kt, r[kt], g[15 + 5 * ax:20 + 5 * ax])):
                err = np.abs(gg - o).max() / max(np.abs(o).max(), 1e-300)
                assert err < 1e-12, (lab, err, gg, o)
