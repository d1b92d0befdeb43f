"""Pins of the oracle's characteristic-variable reconstruction (Sec. 3: Q is a
characteristic component; chi from the U +- c fields) (CPU)."""
import numpy as np
import pytest

import workloads as WL
from tests.helpers import oracle_par, settings

GAMMA = 1.4


def _euler_flux(W, dim):
    """Exact Euler flux along the local normal (component 1 = normal momentum)."""
    rho = W[0]
    u = W[1] / rho
    v = W[2] / rho if dim >= 2 else 0.0
    w = W[3] / rho if dim == 3 else 0.0
    E = W[dim + 1]
    p = (GAMMA - 1.0) * (E - 0.5 * rho * (u * u + v * v + w * w))
    if dim == 3:
        return np.array([rho * u, rho * u * u + p, rho * u * v, rho * u * w, (E + p) * u])
    if dim == 2:
        return np.array([rho * u, rho * u * u + p, rho * u * v, (E + p) * u])
    return np.array([rho * u, rho * u * u + p, (E + p) * u])


def _state(rng, dim):
    rho, u, v, p = rng.uniform(0.3, 2.0), rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0.2, 3.0)
    if dim == 3:
        w = rng.uniform(-1, 1)
        return (np.array([rho, rho * u, rho * v, rho * w, p / (GAMMA - 1) + 0.5 * rho * (u * u + v * v + w * w)]),
                (rho, u, v, p))
    if dim == 2:
        return np.array([rho, rho * u, rho * v, p / (GAMMA - 1) + 0.5 * rho * (u * u + v * v)]), (rho, u, v, p)
    return np.array([rho, rho * u, p / (GAMMA - 1) + 0.5 * rho * u * u]), (rho, u, v, p)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_basis_diagonalises_the_flux_jacobian(oracle, dim):
    """A R = R diag(u - c, u, [u,] u + c) with A the Jacobian of the exact flux
    by central differences, and L R = I."""
    rng = np.random.default_rng(dim)
    n = dim + 2
    for _ in range(20):
        W, (rho, u, v, p) = _state(rng, dim)
        R, L = oracle.char_basis(dim, GAMMA, W)
        A = np.zeros((n, n))
        for b in range(n):
            e = np.zeros(n)
            e[b] = 1e-6 * max(1.0, abs(W[b]))
            A[:, b] = (_euler_flux(W + e, dim) - _euler_flux(W - e, dim)) / (2 * e[b])
        c = np.sqrt(GAMMA * p / rho)
        lam = [u - c] + [u] * dim + [u + c]
        assert np.abs(A @ R - R @ np.diag(lam)).max() <= 1e-7 * np.abs(A).max() * np.abs(R).max()
        assert np.abs(L @ R - np.eye(n)).max() <= 1e-13


def _stage_pair(oracle, s, pr, dt):
    out = []
    for mode in ("conservative", "characteristic"):
        par = oracle_par(oracle, dict(s, recon_vars=mode))
        out.append(oracle.stage2d(par, 1, dt, pr.P, pr.D))
    return out


def test_linear_reconstruction_is_the_same_in_either_variables(oracle):
    """With the linear scheme the reconstruction is linear, so transforming to
    characteristic variables and back changes nothing but round-off."""
    for s, pr in ((settings(dim=2, nx=20, ny=12, lx=1.0, variant="linear"), WL.random_rough2d(20, 12, seed=1)),
                  (settings(dim=2, nx=16, ny=16, lx=10.0, variant="linear"), WL.vortex(16, seed=2))):
        a, b = _stage_pair(oracle, s, pr, 0.2 * pr.h / 3)
        for x, y in zip(a, b):
            assert np.abs(x - y).max() <= 1e-12 * np.abs(x).max()
    s = settings(dim=1, nx=40, lx=1.0, bc="zero_gradient", variant="linear")
    S = WL.sod(40).S
    o = [oracle.stage1d(oracle_par(oracle, dict(s, recon_vars=m)), 1, 1e-3, S)[0]
         for m in ("conservative", "characteristic")]
    assert np.abs(o[0] - o[1]).max() <= 1e-12 * np.abs(o[0]).max()


def test_free_stream_is_preserved(oracle):
    n = 12
    rho, u, v, p = 1.3, 0.4, -0.7, 0.9
    W = np.array([rho, rho * u, rho * v, p / 0.4 + 0.5 * rho * (u * u + v * v)])
    P = np.zeros((12, n, n))
    P[:4] = W[:, None, None]
    D = P.copy()
    par = oracle_par(oracle, settings(dim=2, nx=n, ny=n, lx=1.0, recon_vars="characteristic"))
    oP, oD, _, _ = oracle.stage2d(par, 1, 1e-3, P, D)
    assert np.abs(oP - P).max() <= 1e-13 and np.abs(oD - D).max() <= 1e-13


def test_smooth_data_differences_vanish_with_resolution(oracle):
    """On smooth data both variable sets reconstruct the same function to
    high order: the difference of the stage results falls by well over
    2^3 when the mesh is halved (measured: 1.7e-3 -> 5.1e-5)."""
    diffs = []
    for n in (24, 48):
        pr = WL.vortex(n, seed=0)
        a, b = _stage_pair(oracle, settings(dim=2, nx=n, ny=n, lx=10.0), pr, 0.2 * pr.h / 3)
        diffs.append(max(np.abs(x[:4] - y[:4]).max() / np.abs(x[:4]).max() for x, y in zip(a[:2], b[:2])))
    assert diffs[1] < diffs[0] / 8.0, diffs


def test_conservation_and_chi_range(oracle):
    """Periodic sums are conserved in characteristic mode, and the flux
    weights stay in [0, 1]."""
    pr = WL.riemann2d(20, seed=3)
    s = settings(dim=2, nx=20, ny=20, lx=1.0, recon_vars="characteristic")
    par = oracle_par(oracle, s)
    P, D, _, k = oracle.step2d(par, pr.P, pr.D, 2, cfl=0.4)
    assert k == 2
    for A, B in ((P, pr.P), (D, pr.D)):
        for c in range(4):
            assert abs(A[c].sum() - B[c].sum()) <= 1e-12 * np.abs(B[c]).sum()
    X, Y, _, _ = oracle.intermediates2d(par, 0.2 * pr.h / 3, pr.P, pr.D)
    for E in (X, Y):
        chi = E[:, 8]
        assert chi.min() >= 0.0 and chi.max() <= 1.0 + 1e-15


# ---------------------------------------------------------------------- 3D
def _stage3_pair(oracle, s, pr, dt):
    return [oracle.stage3d(oracle_par(oracle, dict(s, recon_vars=m)), 1, dt, pr.S)
            for m in ("conservative", "characteristic")]


def test_3d_linear_reconstruction_is_the_same_in_either_variables(oracle):
    pr = WL.random_rough3d(6, 5, 4, seed=1)
    s = settings(dim=3, nx=6, ny=5, nz=4, lx=1.0, variant="linear")
    a, b = _stage3_pair(oracle, s, pr, 0.2 * pr.h / 3)
    for x, y in zip(a, b):
        assert np.abs(x - y).max() <= 1e-12 * np.abs(x).max()


def test_3d_free_stream_conservation_and_chi_range(oracle):
    n = 5
    S = np.zeros((4, 20, n, n, n))
    S[:, 0:5] = WL.conservative3d(1.3, 0.4, -0.7, 0.25, 2.0)[None, :, None, None, None]
    par = oracle_par(oracle, settings(dim=3, nx=n, ny=n, nz=n, lx=1.0, recon_vars="characteristic"))
    out, _ = oracle.stage3d(par, 1, 1e-3, S)
    assert np.abs(out - S).max() <= 1e-13
    pr = WL.random_rough3d(6, 5, 4, seed=4)
    par = oracle_par(oracle, settings(dim=3, nx=6, ny=5, nz=4, lx=1.0, recon_vars="characteristic"))
    o, _, k = oracle.step3d(par, pr.S, 2, dt=0.2 * pr.h / 3)
    for g in range(4):
        for c in range(5):
            assert abs(o[g, c].sum() - pr.S[g, c].sum()) <= 1e-13 * np.abs(pr.S[g, c]).sum()
    E, _ = oracle.intermediates3d(par, 0.2 * pr.h / 3, pr.S)
    chi = E[:, :, 10]
    assert chi.min() >= 0.0 and chi.max() <= 1.0 + 1e-15


def test_3d_smooth_data_differences_vanish_with_resolution(oracle):
    """Both variable sets reconstruct smooth 3D data to high order: their
    difference after a stage falls by well over 2^3 when h is halved."""
    diffs = []
    for n in (6, 12):
        pr = WL.random_smooth3d(n, n, n, seed=2, amp=0.2)
        s = settings(dim=3, nx=n, ny=n, nz=n, lx=1.0)
        a, b = _stage3_pair(oracle, s, pr, 0.2 * pr.h / 3)
        diffs.append(np.abs(a[0][:, :5] - b[0][:, :5]).max() / np.abs(a[0][:, :5]).max())
    assert diffs[1] < diffs[0] / 8.0, diffs
