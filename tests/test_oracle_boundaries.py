"""Pins of the oracle's non-periodic boundaries (CPU).

Reading: primary nodes sit half a mesh inside a boundary and dual nodes on
it, so along a bounded axis the dual grid has one more node; reflecting and
no-slip sides continue the solution by its mirror image (normal momentum odd,
no-slip: both momenta odd); zero-gradient sides copy the boundary node with a
zero normal derivative; dual nodes on a wall carry the wall's velocity
condition.  A reflecting problem is then the restriction of a periodic one on
the doubled domain with mirror-symmetric data, which pins the ghost rules
(positions, signs, derivative parities) and the boundary-node bookkeeping
against the periodic scheme."""
import math

import numpy as np
import pytest

import workloads as WL
from tests.helpers import oracle_par, settings

LX, LY = 1.0, 0.75


def _walled(oracle, nx, ny, bx, by, sides, fn=None, **kw):
    h = LX / nx
    assert abs(ny * h - LY) < 1e-14
    fn = fn or WL.mirror_flow(LX, LY, bx, by)
    P, D = WL.sample_bounded(fn, nx, ny, h, bx, by)
    par = oracle_par(oracle, settings(dim=2, nx=nx, ny=ny, lx=LX, ly=LY, sides=sides, **kw))
    return par, P, D


def _doubled(oracle, nx, ny, bx, by, fn, **kw):
    """The periodic problem on the domain doubled across every bounded axis."""
    h = LX / nx
    mx, my = nx * (1 + bx), ny * (1 + by)
    P, D = WL.sample_bounded(fn, mx, my, h, 0, 0, x0=-LX * bx, y0=-LY * by)
    par = oracle_par(oracle, settings(dim=2, nx=mx, ny=my, lx=LX * (1 + bx), ly=LY * (1 + by), **kw))
    return par, P, D


def _restrict(A, nx, ny, bx, by, grid):
    """Nodes of the walled domain inside the doubled periodic arrays."""
    if grid == 0:
        return A[:, ny * by:ny * by + ny, nx * bx:nx * bx + nx]
    j0 = ny - 1 if by else 0
    i0 = nx - 1 if bx else 0
    return A[:, j0:j0 + ny + by, i0:i0 + nx + bx]


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1.0))


@pytest.mark.parametrize("bx,by,order", [(1, 0, 6), (0, 1, 6), (1, 1, 6), (1, 1, 8)])
def test_reflecting_equals_mirrored_periodic(oracle, bx, by, order):
    nx, ny = 16, 12
    sides = ["reflecting" if bx else "periodic"] * 2 + ["reflecting" if by else "periodic"] * 2
    fn = WL.mirror_flow(LX, LY, bx, by)
    par, P, D = _walled(oracle, nx, ny, bx, by, sides, fn, flux_order=order)
    assert D.shape == (12, ny + by, nx + bx)
    qar, Q, E = _doubled(oracle, nx, ny, bx, by, fn, flux_order=order)
    dt = 0.2 * (LX / nx) / 3
    a = oracle.stage2d(par, 1, dt, P, D)
    b = oracle.stage2d(qar, 1, dt, Q, E)
    for k in range(4):
        assert _rel(a[k], _restrict(b[k], nx, ny, bx, by, k % 2)) <= 1e-12, k
    oP, oD, t, n = oracle.step2d(par, P, D, 3, cfl=0.5)
    qP, qD, t2, n2 = oracle.step2d(qar, Q, E, 3, cfl=0.5)
    assert n == n2 == 3 and abs(t - t2) <= 1e-14 * t
    assert _rel(oP, _restrict(qP, nx, ny, bx, by, 0)) <= 1e-12
    assert _rel(oD, _restrict(qD, nx, ny, bx, by, 1)) <= 1e-12


@pytest.mark.parametrize("order", [6, 8])
def test_reflecting_1d_equals_mirrored_periodic(oracle, order):
    N = 40
    h = 1.0 / N
    x = (np.arange(2 * N) + 0.5) * h - 1.0

    def state(xx):
        rho = 1.0 + 0.2 * np.cos(math.pi * xx) + 0.05 * np.cos(3 * math.pi * xx)
        U = 0.4 * np.sin(math.pi * xx)
        p = 1.0 + 0.1 * np.cos(2 * math.pi * xx)
        return WL.conservative1d(rho, U, p)

    S2 = np.zeros((1, 6, 2 * N))
    S2[0, :3] = state(x)
    S2[0, 3:] = (state(x + h / 2) - state(x - h / 2)) / h
    S1 = np.ascontiguousarray(S2[:, :, N:])
    p1 = oracle_par(oracle, settings(dim=1, nx=N, lx=1.0, bc="reflecting", flux_order=order))
    p2 = oracle_par(oracle, settings(dim=1, nx=2 * N, lx=2.0, flux_order=order))
    a, _, k1 = oracle.step1d(p1, S1, 5, cfl=0.5)
    b, _, k2 = oracle.step1d(p2, S2, 5, cfl=0.5)
    assert k1 == k2 == 5
    assert _rel(a, b[:, :, N:]) <= 1e-12


def test_reflecting_conserves_primary_sums(oracle):
    """Walls let no mass or energy through: the primary grid's sums of rho
    and rho E are conserved (its boundary faces lie on the walls)."""
    nx, ny = 16, 12
    par, P, D = _walled(oracle, nx, ny, 1, 1, ["reflecting"] * 4)
    oP, oD, _, n = oracle.step2d(par, P, D, 3, cfl=0.5)
    assert n == 3
    for c in (0, 3):
        assert abs(oP[c].sum() - P[c].sum()) <= 1e-13 * np.abs(P[c]).sum(), c


def test_no_slip_equals_reflecting_without_tangential_flow(oracle):
    nx, ny = 16, 12
    fn0 = WL.mirror_flow(LX, LY, 1, 0)

    def fn(X, Y):
        W = fn0(X, 0.0 * Y + 0.1)
        W[3] = W[3] - 0.5 * W[2] ** 2 / W[0]  # drop the tangential kinetic energy
        W[2] = 0.0
        return W

    out = []
    for wall in ("reflecting", "no_slip"):
        par, P, D = _walled(oracle, nx, ny, 1, 0, [wall, wall, "periodic", "periodic"], fn, mu=1e-3, prandtl=0.72)
        out.append(oracle.step2d(par, P, D, 2, cfl=0.5)[:2])
    for a, b in zip(out[0], out[1]):
        assert _rel(a, b) <= 1e-15


@pytest.mark.parametrize("order", [6, 8])
def test_zero_gradient_matches_wider_periodic_while_quiet(oracle, order):
    """With the data uniform within 8 nodes of every side, one step on a
    zero-gradient domain equals the same step on a periodic domain 8 nodes
    wider on each side, restricted (nothing has reached the boundary)."""
    n, m = 24, 8
    h = 1.0 / n
    bump = lambda X, Y: WL.conservative(  # noqa: E731
        1.0 + 0.3 * np.exp(-80 * ((X - 0.5) ** 2 + (Y - 0.5) ** 2)), 0.2, -0.1,
        1.0 + 0.2 * np.exp(-80 * ((X - 0.45) ** 2 + (Y - 0.55) ** 2)))

    def quiet(X, Y):
        W = bump(X, Y)
        far = (X < 8.5 * h) | (X > 1 - 8.5 * h) | (Y < 8.5 * h) | (Y > 1 - 8.5 * h)
        return np.where(far[None], bump(0.0 * X, 0.0 * Y), W)

    P, D = WL.sample_bounded(quiet, n, n, h, 1, 1)
    par = oracle_par(oracle, settings(dim=2, nx=n, ny=n, lx=1.0, bc="zero_gradient", flux_order=order))
    # the same data embedded in a uniform frame of m nodes
    Q = np.zeros((12, n + 2 * m, n + 2 * m))
    Q[0:4] = P[0:4, 0, 0][:, None, None]
    E = Q.copy()
    Q[:, m:m + n, m:m + n] = P
    E[:, m - 1:m + n, m - 1:m + n] = D
    qar = oracle_par(oracle, settings(dim=2, nx=n + 2 * m, ny=n + 2 * m, lx=1.0 + 2 * m * h, flux_order=order))
    dt = 0.2 * h / 3
    a = oracle.step2d(par, P, D, 1, dt=dt)
    b = oracle.step2d(qar, Q, E, 1, dt=dt)
    assert np.abs(a[0] - b[0][:, m:m + n, m:m + n]).max() <= 1e-15
    assert np.abs(a[1] - b[1][:, m - 1:m + n, m - 1:m + n]).max() <= 1e-15


def test_stokes_first_problem(oracle):
    """Fluid sliding at V0 along a resting no-slip wall (low Mach, mu > 0):
    near the wall the tangential velocity approaches the incompressible
    Stokes solution V0 erf(x / (2 sqrt(nu t)))."""
    nx, ny, V0, mu, T = 96, 4, 0.05, 5e-3, 0.04
    h = 1.0 / nx

    def fn(X, Y):
        V = np.where((X <= 0.0) | (X >= 1.0), 0.0, V0)
        return WL.conservative(1.0 + 0 * X, 0.0, V, 1.0)

    P, D = WL.sample_bounded(fn, nx, ny, h, 1, 0, jumps=True)
    par = oracle_par(oracle, settings(dim=2, nx=nx, ny=ny, lx=1.0, ly=ny * h, mu=mu, prandtl=0.72,
                                      sides=["no_slip", "no_slip", "periodic", "periodic"]))
    oP, oD, t, n = oracle.step2d(par, P, D, 100000, cfl=0.5, t_end=T)
    assert abs(t - T) < 1e-14
    x = (np.arange(nx) + 0.5) * h
    V = oP[2, 0] / oP[0, 0]
    exact = V0 * np.array([math.erf(v / (2 * math.sqrt(mu * T))) for v in x])
    near = x < 0.15
    err = np.abs(V[near] - exact[near]).max() / V0
    print(f"Stokes first problem: max |V - V0 erf| / V0 = {err:.3e} near the wall ({n} steps)")
    assert err < 0.02
    assert np.all(oD[1:3, :, 0] == 0.0) and np.all(oD[1:3, :, nx] == 0.0)


def test_periodic_side_needs_periodic_partner(oracle):
    with pytest.raises(ValueError):
        oracle_par(oracle, settings(dim=2, nx=8, ny=8, lx=1.0,
                                    sides=["periodic", "reflecting", "periodic", "periodic"]))
