"""Pins of the oracle's forward-mode step derivative (orc_step2d_tangent),
the reference of the GPU adjoint: its value part is the plain step, and its
tangent matches central differences of the plain step on smooth data (CPU)."""
import numpy as np

import workloads as WL
from tests.helpers import oracle_par, settings


def _setup(oracle, n=16, seed=21, **kw):
    s = settings(dim=2, nx=n, ny=n, lx=1.0, **kw)
    pr = WL.random_smooth2d(n, n, seed=seed)
    return oracle_par(oracle, s), pr, 0.2 * pr.h / 3.0


def test_tangent_value_part_is_the_step(oracle):
    par, pr, dt = _setup(oracle)
    v = np.random.default_rng(0).standard_normal((2,) + pr.P.shape)
    oP, oD, _, _ = oracle.step2d_tangent(par, dt, pr.P, pr.D, v[0], v[1])
    P, D, _, k = oracle.step2d(par, pr.P, pr.D, 1, dt=dt)
    assert k == 1
    assert np.array_equal(oP, P) and np.array_equal(oD, D)


def _fd_check(oracle, par, pr, dt, seed, eps):
    """Largest per-plane max |FD - Jv| / max |Jv| for central differences of
    the oracle's plain step with step eps along a random direction v."""
    rng = np.random.default_rng(seed)
    S = np.stack([pr.P, pr.D])
    v = rng.standard_normal(S.shape) * np.abs(S).max(axis=(2, 3), keepdims=True)
    _, _, dP, dD = oracle.step2d_tangent(par, dt, S[0], S[1], v[0], v[1])
    Jv = np.stack([dP, dD])

    def f(X):
        P, D, _, _ = oracle.step2d(par, X[0], X[1], 1, dt=dt)
        return np.stack([P, D])
    fd = (f(S + eps * v) - f(S - eps * v)) / (2 * eps)
    num = np.abs(fd - Jv).max(axis=(2, 3))
    den = np.abs(Jv).max(axis=(2, 3))
    return float((num / den).max())


# The linear-flux scheme with a collision time free of |p_l - p_r| is an
# analytic map: central differences converge as eps^2 to the tangent.
def test_tangent_analytic_euler(oracle):
    par, pr, dt = _setup(oracle, variant="linear", tau_c1=0.05, tau_c2=0.0)
    assert _fd_check(oracle, par, pr, dt, 1, 1e-5) < 1e-8


def test_tangent_analytic_ns(oracle):
    par, pr, dt = _setup(oracle, variant="linear", tau_c2=0.0, mu=1e-3, prandtl=0.72, seed=22)
    assert _fd_check(oracle, par, pr, dt, 2, 1e-5) < 1e-8


def test_tangent_geno_second_order_convergence(oracle):
    """GENO weights are smooth away from their switching points but strongly
    curved (eps_a = 1e-6): the FD error must still fall as eps^2."""
    par, pr, dt = _setup(oracle, tau_c1=0.05, tau_c2=0.0, seed=24)
    e6 = _fd_check(oracle, par, pr, dt, 4, 1e-6)
    e7 = _fd_check(oracle, par, pr, dt, 4, 1e-7)
    assert e7 < 1e-5 and e6 / e7 > 30.0, (e6, e7)


def test_tangent_default_scheme_small_eps(oracle):
    """Default collision time tau_c2 dt |p_l - p_r| / (p_l + p_r): on smooth
    data p_l - p_r is tiny, so the kink of |.| is close and only small
    steps stay on one side of it."""
    par, pr, dt = _setup(oracle)
    assert _fd_check(oracle, par, pr, dt, 5, 1e-8) < 1e-6
    par, pr, dt = _setup(oracle, variant="6-2", grad_carried=1, seed=23)
    assert _fd_check(oracle, par, pr, dt, 3, 1e-8) < 1e-6


def _bounded_fd_check(oracle, par, P, D, dt, seed, eps):
    """As _fd_check for a problem with bounded axes (the dual state is larger)."""
    rng = np.random.default_rng(seed)
    vP = rng.standard_normal(P.shape) * np.abs(P).max(axis=(1, 2), keepdims=True)
    vD = rng.standard_normal(D.shape) * np.abs(D).max(axis=(1, 2), keepdims=True)
    _, _, dP, dD = oracle.step2d_tangent(par, dt, P, D, vP, vD)

    def f(X, Y):
        return oracle.step2d(par, X, Y, 1, dt=dt)[:2]
    a, b = f(P + eps * vP, D + eps * vD), f(P - eps * vP, D - eps * vD)
    worst = 0.0
    for g, Jv in ((0, dP), (1, dD)):
        fd = (a[g] - b[g]) / (2 * eps)
        num = np.abs(fd - Jv).max(axis=(1, 2))
        den = np.abs(Jv).max(axis=(1, 2))
        worst = max(worst, float((num / np.maximum(den, 1e-300)).max()))
    return worst


def test_tangent_bounded_sides(oracle):
    """Walls and zero-gradient sides (ghost values mirrored, copied or zeroed;
    wall conditions on the dual boundary nodes): on the analytic
    linear-flux map central differences converge to the tangent as eps^2,
    and the value part is the plain step."""
    cases = [
        (["reflecting", "reflecting", "no_slip", "no_slip"], 14, 9),
        (["zero_gradient", "zero_gradient", "reflecting", "zero_gradient"], 11, 12),
        (["periodic", "periodic", "no_slip", "reflecting"], 12, 10),
    ]
    for sides, nx, ny in cases:
        bx, by = int(sides[0] != "periodic"), int(sides[2] != "periodic")
        h = 1.0 / nx
        P, D = WL.sample_bounded(WL.mirror_flow(1.0, ny * h, bx, by), nx, ny, h, bx, by)
        s = settings(dim=2, nx=nx, ny=ny, lx=1.0, sides=sides, variant="linear", tau_c1=0.05, tau_c2=0.0,
                     mu=1e-3, prandtl=0.72)
        par = oracle_par(oracle, s)
        dt = 0.2 * h / 3.0
        assert D.shape == (12, ny + by, nx + bx)
        v = np.zeros_like(P), np.zeros_like(D)
        oP, oD, dP, dD = oracle.step2d_tangent(par, dt, P, D, *v)
        sP, sD, _, k = oracle.step2d(par, P, D, 1, dt=dt)
        assert k == 1 and np.array_equal(oP, sP) and np.array_equal(oD, sD)
        assert not dP.any() and not dD.any()
        e5 = _bounded_fd_check(oracle, par, P, D, dt, 7, 1e-5)
        e4 = _bounded_fd_check(oracle, par, P, D, dt, 7, 1e-4)
        assert e5 < 1e-8 and e4 / e5 > 30.0, (sides, e4, e5)
