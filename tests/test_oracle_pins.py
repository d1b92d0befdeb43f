"""Pins of the oracle's building blocks against what the paper and the
mathematics fix, computed here by independent means (brute-force linear
solves, quadrature, closed forms, limits).  CPU only."""
import math

import numpy as np
import pytest
from scipy import integrate

from tests.helpers import settings

G = 1.4


@pytest.fixture(scope="module")
def par(oracle):
    return oracle.make_par(**settings(dim=2, nx=8, ny=8, lx=1.0))


def _par(oracle, **kw):
    return oracle.make_par(**settings(**{**dict(dim=2, nx=8, ny=8, lx=1.0), **kw}))


# ------------------------------------------------- compact flux, Sec. 2.1-2.2
def _brute_flux_coeffs(h=1.0):
    """Degree-4 polynomial F(x) whose averages over the node cells of j, j+1
    and over the interval [x_{i-1}, x_i] for i = j, j+1, j+2 are given
    (the five conditions of Eq. fd-conservative-flux-recons); returns the
    weights of F(x_{j+1/2}) on (F_{j-1/2}, F_{j+1/2}, F_{j+3/2}, F_j, F_{j+1})."""
    # node j at x = 0, interface j+1/2 at h/2; the interval [x_{i-1}, x_i]
    # between nodes i-1 and i carries the interface flux F_{i-1/2}
    cells = [(-h, 0.0), (0.0, h), (h, 2 * h)]
    nodes = [(-0.5 * h, 0.5 * h), (0.5 * h, 1.5 * h)]
    A = np.zeros((5, 5))
    for r, (a, b) in enumerate(cells + nodes):
        for k in range(5):
            A[r, k] = (b ** (k + 1) - a ** (k + 1)) / ((k + 1) * (b - a))
    ev = np.array([(0.5 * h) ** k for k in range(5)])
    return np.linalg.solve(A.T, ev)  # weights w with F(x_{j+1/2}) = w . data


def test_linear_compact_flux_is_the_five_condition_solution(oracle):
    p = _par(oracle, variant="linear")
    w = _brute_flux_coeffs()
    rng = np.random.default_rng(0)
    for _ in range(20):
        Fm, Fc, Fp, N0, N1 = rng.normal(size=5)
        want = w @ np.array([Fm, Fc, Fp, N0, N1])
        assert abs(oracle.compact_flux(p, Fm, Fc, Fp, N0, N1, 0.3) - want) < 1e-13


def test_compact_flux_truncation_constant(oracle):
    """F-bar_{j+1/2} = F(x_{j+1/2}) + h^6 F^(6)/8960 + O(h^8) (Sec. 2.1)."""
    p = _par(oracle, variant="linear")
    for h in (0.2, 0.1, 0.05):
        # F(x) = sin(x + 0.3): node values are cell averages, interface values interval averages
        F = lambda x: math.sin(x + 0.3)  # noqa: E731
        avg = lambda a, b: (math.cos(a + 0.3) - math.cos(b + 0.3)) / (b - a)  # noqa: E731
        Fm, Fc, Fp = avg(-h, 0), avg(0, h), avg(h, 2 * h)
        N0, N1 = avg(-0.5 * h, 0.5 * h), avg(0.5 * h, 1.5 * h)
        err = oracle.compact_flux(p, Fm, Fc, Fp, N0, N1, 1.0) - F(0.5 * h)
        lead = h ** 6 * (-math.sin(0.5 * h + 0.3)) / 8960.0
        assert abs(err - lead) < 0.02 * abs(lead), (h, err, lead)


def test_64_low_order_term_is_fourth_order(oracle):
    """(6-4) with chi = 0: (8 F_{j+1/2} - F_j - F_{j+1})/6 reproduces F(x_{j+1/2})
    for cubics (the 1/6 of reading D1); without it the result is 6x off."""
    p = _par(oracle, variant="6-4")
    for coef in np.random.default_rng(1).normal(size=(5, 4)):
        P = np.polynomial.Polynomial(coef)
        I = P.integ()
        avg = lambda a, b: (I(b) - I(a)) / (b - a)  # noqa: E731
        h = 0.37
        val = oracle.compact_flux(p, avg(-h, 0), avg(0, h), avg(h, 2 * h), avg(-h / 2, h / 2), avg(h / 2, 1.5 * h), 0.0)
        assert abs(val - P(h / 2)) < 1e-12


def test_62_and_blend(oracle):
    p62 = _par(oracle, variant="6-2")
    pl = _par(oracle, variant="linear")
    a = (0.3, 1.1, -0.4, 0.8, 0.9)
    Fb = oracle.compact_flux(pl, *a, 0.0)
    assert oracle.compact_flux(p62, *a, 0.0) == pytest.approx(1.1, abs=1e-15)
    assert oracle.compact_flux(p62, *a, 1.0) == pytest.approx(Fb, abs=1e-15)
    assert oracle.compact_flux(p62, *a, 0.25) == pytest.approx(0.75 * 1.1 + 0.25 * Fb, abs=1e-15)


def _brute_wide_flux_coeffs(h=1.0):
    """The seven-condition solve for flux_order 8: the conditions of
    _brute_flux_coeffs plus the averages over the node cells of j-1 and j+2
    (a degree-6 polynomial).  Weights on (F_{j-1/2}, F_{j+1/2}, F_{j+3/2},
    F_{j-1}, F_j, F_{j+1}, F_{j+2})."""
    cells = [(-h, 0.0), (0.0, h), (h, 2 * h)]
    nodes = [(-1.5 * h, -0.5 * h), (-0.5 * h, 0.5 * h), (0.5 * h, 1.5 * h), (1.5 * h, 2.5 * h)]
    A = np.zeros((7, 7))
    for r, (a, b) in enumerate(cells + nodes):
        for k in range(7):
            A[r, k] = (b ** (k + 1) - a ** (k + 1)) / ((k + 1) * (b - a))
    ev = np.array([(0.5 * h) ** k for k in range(7)])
    return np.linalg.solve(A.T, ev)


def test_wide_linear_flux_is_the_seven_condition_solution(oracle):
    p = _par(oracle, variant="linear", flux_order=8)
    w = _brute_wide_flux_coeffs()
    rng = np.random.default_rng(2)
    for _ in range(20):
        Fm, Fc, Fp, Nm, N0, N1, Np2 = rng.normal(size=7)
        want = w @ np.array([Fm, Fc, Fp, Nm, N0, N1, Np2])
        got = oracle.compact_flux(p, Fm, Fc, Fp, N0, N1, 0.3, Nm=Nm, Np2=Np2)
        assert abs(got - want) < 1e-13


def test_wide_flux_truncation_constant(oracle):
    """Order 8: exact for polynomials of degree 7 (symmetry about the
    interface), leading error -h^8 F^(8) / 161280 (from the moments of the
    seven-condition solve)."""
    p = _par(oracle, variant="linear", flux_order=8)
    w = _brute_wide_flux_coeffs()
    cells = [(-1.0, 0.0), (0.0, 1.0), (1.0, 2.0), (-1.5, -0.5), (-0.5, 0.5), (0.5, 1.5), (1.5, 2.5)]
    mom = lambda k: np.array([(b ** (k + 1) - a ** (k + 1)) / ((k + 1) * (b - a)) for a, b in cells])  # noqa: E731
    assert abs(w @ mom(7) - 0.5 ** 7) < 1e-12
    assert abs((w @ mom(8) - 0.5 ** 8) / math.factorial(8) + 1.0 / 161280.0) < 1e-15
    for h in (0.4, 0.2, 0.1):
        F = lambda x: math.sin(x + 0.3)  # noqa: E731
        avg = lambda a, b: (math.cos(a + 0.3) - math.cos(b + 0.3)) / (b - a)  # noqa: E731
        Fm, Fc, Fp = avg(-h, 0), avg(0, h), avg(h, 2 * h)
        Nm, N0, N1, Np2 = avg(-1.5 * h, -0.5 * h), avg(-0.5 * h, 0.5 * h), avg(0.5 * h, 1.5 * h), avg(1.5 * h, 2.5 * h)
        err = oracle.compact_flux(p, Fm, Fc, Fp, N0, N1, 1.0, Nm=Nm, Np2=Np2) - F(0.5 * h)
        lead = -h ** 8 * math.sin(0.5 * h + 0.3) / 161280.0
        assert abs(err - lead) < 0.05 * abs(lead), (h, err, lead)


def test_wide_flux_keeps_the_low_order_blend(oracle):
    """flux_order changes only the linear flux F-bar: (6-4) and (6-2) blend it
    with the same low-order fluxes and chi."""
    a = (0.3, 1.1, -0.4, 0.8, 0.9)
    Fb = oracle.compact_flux(_par(oracle, variant="linear", flux_order=8), *a, 0.0, Nm=0.2, Np2=-0.7)
    lo = {"6-4": (8 * 1.1 - 0.8 - 0.9) / 6, "6-2": 1.1}
    for v, L in lo.items():
        q = _par(oracle, variant=v, flux_order=8)
        assert oracle.compact_flux(q, *a, 0.25, Nm=0.2, Np2=-0.7) == pytest.approx(0.75 * L + 0.25 * Fb, abs=1e-15)
    with pytest.raises(ValueError):
        _par(oracle, flux_order=7)


# --------------------------------------------------- reconstruction, Sec. 3
def _poly_data(P, h, centers):
    """Nodal values and interval-averaged derivatives of polynomial P."""
    Q = np.array([P(c) for c in centers])
    X = np.array([(P(c + h / 2) - P(c - h / 2)) / h for c in centers])
    return Q, X


@pytest.mark.parametrize("deg", [0, 1, 2, 3, 4, 5, 6])
def test_interface_high_order_exact_to_degree_6(oracle, deg):
    p = _par(oracle, variant="linear")
    h = 0.3
    P = np.polynomial.Polynomial(np.random.default_rng(deg).normal(size=deg + 1))
    Q, X = _poly_data(P, h, [-h, 0, h, 2 * h])
    vl, dl, cl, vr, dr, cr = oracle.recon_interface(p, Q, X, h)
    x = h / 2
    assert vl == pytest.approx(P(x), abs=1e-12) and vr == pytest.approx(P(x), abs=1e-12)
    assert dl == pytest.approx(P.deriv()(x), abs=1e-11) and dr == pytest.approx(P.deriv()(x), abs=1e-11)


def test_interface_high_order_error_at_degree_7(oracle):
    p = _par(oracle, variant="linear")
    h = 0.3
    P = np.polynomial.Polynomial([0] * 7 + [1.0])
    Q, X = _poly_data(P, h, [-h, 0, h, 2 * h])
    vl, dl, _, vr, dr, _ = oracle.recon_interface(p, Q, X, h)
    assert abs(vl - P(h / 2)) > 1e-9 and abs(vr - P(h / 2)) > 1e-9  # degree 7 is where exactness ends


@pytest.mark.parametrize("deg", [0, 1, 2, 3, 4, 5, 6])
def test_node_derivative_exact(oracle, deg):
    """P^5_x (Eq. 6th-compact-recons) is exact up to degree 6."""
    p = _par(oracle, variant="linear")
    h = 0.25
    P = np.polynomial.Polynomial(np.random.default_rng(10 + deg).normal(size=deg + 1))
    Q, X = _poly_data(P, h, [-h, 0, h])
    assert oracle.recon_node(p, Q, X, h) == pytest.approx(P.deriv()(0.0), abs=1e-11)


def test_node_derivative_degree_7_and_8(oracle):
    """Exactness ends at degree 7; the stencil is antisymmetric about the node,
    so the even monomial x^8 (zero derivative at the node) is again exact."""
    p = _par(oracle, variant="linear")
    h = 0.25
    P7 = np.polynomial.Polynomial([0] * 7 + [1.0])
    Q, X = _poly_data(P7, h, [-h, 0, h])
    assert abs(oracle.recon_node(p, Q, X, h) - 0.0) > 1e-6
    P8 = np.polynomial.Polynomial([0] * 8 + [1.0])
    Q, X = _poly_data(P8, h, [-h, 0, h])
    assert oracle.recon_node(p, Q, X, h) == pytest.approx(0.0, abs=1e-15)


@pytest.mark.parametrize("deg", [0, 1, 2])
def test_geno_sub_stencils_exact_for_quadratics(oracle, deg):
    """For quadratic data every sub-stencil polynomial of App. C equals the data,
    so the nonlinear GENO result is exact whatever the weights; and every
    smoothness indicator measures the same quadratic on the same cell, so
    IS_1 = IS_2 = IS_3 and the path function is 1."""
    p = _par(oracle, variant="6-4")
    h = 0.2
    for seed in range(5):
        P = np.polynomial.Polynomial(np.random.default_rng(100 * deg + seed).normal(size=deg + 1))
        Q, X = _poly_data(P, h, [-h, 0, h, 2 * h])
        vl, dl, cl, vr, dr, cr = oracle.recon_interface(p, Q, X, h)
        assert vl == pytest.approx(P(h / 2), abs=1e-13) and vr == pytest.approx(P(h / 2), abs=1e-13)
        assert dl == pytest.approx(P.deriv()(h / 2), abs=1e-12)
        assert dr == pytest.approx(P.deriv()(h / 2), abs=1e-12)
        assert cl == pytest.approx(1.0, abs=1e-12) and cr == pytest.approx(1.0, abs=1e-12)
        Qn, Xn = _poly_data(P, h, [-h, 0, h])
        assert oracle.recon_node(p, Qn, Xn, h) == pytest.approx(P.deriv()(0.0), abs=1e-12)


def _substencil_quadratic(points, h):
    """Brute force: quadratic through the given constraints.  points: list of
    ('v', x, value) point values or ('d', x, value) interval-averaged
    derivatives over [x - h/2, x + h/2]."""
    A, b = [], []
    for kind, x, val in points:
        if kind == "v":
            A.append([1, x, x * x])
        else:
            A.append([0, 1, 2 * x])  # (q(x+h/2) - q(x-h/2))/h of a quadratic
        b.append(val)
    return np.polynomial.Polynomial(np.linalg.solve(np.array(A, float), np.array(b, float)))


def _jiang_shu(q, a, b, h):
    d1, d2 = q.deriv(), q.deriv(2)
    i1 = integrate.quad(lambda x: d1(x) ** 2, a, b)[0]
    i2 = integrate.quad(lambda x: d2(x) ** 2, a, b)[0]
    return h * i1 + h ** 3 * i2


def test_geno_low_order_weights_at_a_discontinuity(oracle):
    """Left state at j+1/2 with a jump between j+1 and j+2: the path function
    drops to ~0 and the value is the WENO-type blend of the sub-stencil
    quadratics (built here by brute force, with Jiang-Shu indicators by
    quadrature), weights d_k/(IS_k+eps_a)^2 with d = (1, 8, 1) (App. C1 order,
    reading D5)."""
    p = _par(oracle, variant="6-4")
    h = 0.1
    xs = [-h, 0.0, h, 2 * h]
    Q = [1.0, 1.02, 1.05, 3.0]
    X = [0.15, 0.2, 0.3, 0.0]
    subs = [
        _substencil_quadratic([("v", xs[0], Q[0]), ("v", xs[1], Q[1]), ("d", xs[0], X[0])], h),
        _substencil_quadratic([("v", xs[0], Q[0]), ("v", xs[1], Q[1]), ("v", xs[2], Q[2])], h),
        _substencil_quadratic([("v", xs[1], Q[1]), ("v", xs[2], Q[2]), ("v", xs[3], Q[3])], h),
    ]
    IS = [_jiang_shu(q, -h / 2, h / 2, h) for q in subs]
    d = [1.0, 8.0, 1.0]
    w = np.array([d[k] / (IS[k] + 1e-6) ** 2 for k in range(3)])
    w /= w.sum()
    PL = sum(w[k] * subs[k](h / 2) for k in range(3))
    PLx = sum(w[k] * subs[k].deriv()(h / 2) for k in range(3))
    vl, dl, cl, *_ = oracle.recon_interface(p, Q, X, h)
    assert cl < 1e-6
    assert vl == pytest.approx(PL, rel=1e-6) and dl == pytest.approx(PLx, rel=1e-5)


def test_geno_node_discontinuity_picks_smooth_side(oracle):
    p = _par(oracle, variant="6-4")
    h = 0.1
    # smooth on the left (linear, slope 1), jump to the right of node j
    Q = [0.9, 1.0, 5.0]
    X = [1.0, 1.0, 0.0]
    assert oracle.recon_node(p, Q, X, h) == pytest.approx(1.0, rel=1e-3)


def test_geno_blend_limits(oracle):
    p = _par(oracle)
    q = [1.0, 2.0, 3.0]
    dq = [0.1, 0.2, 0.3]
    d = [1.0, 8.0, 1.0]
    v, der, chi = oracle.geno_blend(p, [0.5, 0.5, 0.5], 0, d, q, dq, 7.0, 0.7)
    assert chi == pytest.approx(1.0, abs=1e-15) and v == pytest.approx(7.0) and der == pytest.approx(0.7)
    # one sub-stencil perfectly flat, the others rough: chi -> 0, weight -> that sub-stencil
    v, der, chi = oracle.geno_blend(p, [0.0, 1.0, 1.0], 0, d, q, dq, 7.0, 0.7)
    assert chi < 1e-12 and v == pytest.approx(1.0, rel=1e-9) and der == pytest.approx(0.1, rel=1e-9)
    # path function: tanh(C alpha)/tanh(C) with alpha = 2 aH/(aH + aL), r = 3, eps = 1e-15
    IS = np.array([0.2, 0.5, 0.3])
    tau = 0.5 * abs(IS[1] + IS[2] - 2 * IS[0])
    aH = 1 + (tau / (IS.max() + 1e-15)) ** 3
    aL = 1 + (tau / (IS.min() + 1e-15)) ** 3
    chi_want = math.tanh(20 * 2 * aH / (aH + aL)) / math.tanh(20)
    v, der, chi = oracle.geno_blend(p, IS, 0, d, q, dq, 7.0, 0.7)
    assert chi == pytest.approx(chi_want, rel=1e-14)


# --------------------------------------------------- Maxwellian, App. A
@pytest.mark.parametrize("U,lam", [(0.3, 0.7), (-1.2, 2.0), (0.0, 0.5), (2.5, 1.3)])
def test_maxwell_moments_by_quadrature(oracle, U, lam):
    K = 3.0
    for half in (0, 1, -1):
        mu, mv, mx = oracle.maxwell(U, 0.4, lam, K, half, 2)
        lo, hi = {0: (-np.inf, np.inf), 1: (0, np.inf), -1: (-np.inf, 0)}[half]
        for n in range(7):
            f = lambda u: u ** n * math.sqrt(lam / math.pi) * math.exp(-lam * (u - U) ** 2)  # noqa: E731
            want = integrate.quad(f, lo, hi, epsabs=1e-13, epsrel=1e-12)[0]
            assert mu[n] == pytest.approx(want, rel=1e-9, abs=1e-12), (half, n)
    for n in range(7):
        f = lambda v: v ** n * math.sqrt(lam / math.pi) * math.exp(-lam * (v - 0.4) ** 2)  # noqa: E731
        assert mv[n] == pytest.approx(integrate.quad(f, -np.inf, np.inf, epsabs=1e-13)[0], rel=1e-9, abs=1e-12)
    # internal degrees of freedom: K independent Gaussian components
    g2 = integrate.quad(lambda x: x * x * math.sqrt(lam / math.pi) * math.exp(-lam * x * x), -np.inf, np.inf)[0]
    g4 = integrate.quad(lambda x: x ** 4 * math.sqrt(lam / math.pi) * math.exp(-lam * x * x), -np.inf, np.inf)[0]
    assert mx[1] == pytest.approx(K * g2, rel=1e-12)
    assert mx[2] == pytest.approx(K * g4 + K * (K - 1) * g2 * g2, rel=1e-12)


def _moment_system_by_quadrature(W, s, dim):
    """<psi (s.psi)> rho for the Maxwellian of W, by 2D/1D quadrature in (u, v)
    and the Gaussian moments of xi."""
    rho = W[0]
    U = W[1] / rho
    V = W[2] / rho if dim == 2 else 0.0
    p = (G - 1) * (W[-1] - 0.5 * rho * (U * U + V * V))
    lam = rho / (2 * p)
    K = (4 - 2 * G) / (G - 1) if dim == 2 else (3 - G) / (G - 1)
    xi2 = K / (2 * lam)
    xi4 = K * (K + 2) / (4 * lam * lam)
    out = []
    if dim == 2:
        def gauss(u, v):
            return lam / math.pi * math.exp(-lam * ((u - U) ** 2 + (v - V) ** 2))

        def sp(u, v, x2):  # s . psi, with xi^2 -> x2 (linear in x2)
            return s[0] + s[1] * u + s[2] * v + 0.5 * s[3] * (u * u + v * v + x2)
        psis = [lambda u, v: 1.0, lambda u, v: u, lambda u, v: v, None]
        for i in range(4):
            if i < 3:
                f = lambda u, v, i=i: psis[i](u, v) * sp(u, v, xi2) * gauss(u, v)  # noqa: E731
            else:
                # psi_4 (s.psi) = 1/2 (e + x2)(c + s3/2 x2) with e = u^2+v^2: average over xi
                def f(u, v):
                    e = u * u + v * v
                    c = s[0] + s[1] * u + s[2] * v + 0.5 * s[3] * e
                    return 0.5 * (e * c + e * 0.5 * s[3] * xi2 + c * xi2 + 0.5 * s[3] * xi4) * gauss(u, v)
            val = integrate.dblquad(lambda v, u: f(u, v), U - 12 / math.sqrt(lam), U + 12 / math.sqrt(lam),
                                    V - 12 / math.sqrt(lam), V + 12 / math.sqrt(lam), epsabs=1e-11, epsrel=1e-11)[0]
            out.append(rho * val)
    return np.array(out)


def test_slope_solves_the_moment_system(oracle):
    W = np.array([1.2, 0.3, -0.5, 3.1])
    D = np.array([0.4, -0.2, 0.7, 1.5])
    s = oracle.slope(W, D, 2, G)
    assert np.allclose(_moment_system_by_quadrature(W, s, 2), D, rtol=1e-8, atol=1e-9)


def test_slope_matches_closed_form(oracle):
    """Closed-form micro slope of the BGK-NS literature, derived independently."""
    rng = np.random.default_rng(3)
    for _ in range(10):
        rho, U, V, p = 0.5 + rng.random(), rng.normal(), rng.normal(), 0.5 + rng.random()
        W = np.array([rho, rho * U, rho * V, p / (G - 1) + 0.5 * rho * (U * U + V * V)])
        D = rng.normal(size=4)
        lam = rho / (2 * p)
        K = (4 - 2 * G) / (G - 1)
        d = D / rho
        e = U * U + V * V + (K + 2) / (2 * lam)
        B = 2 * d[3] - e * d[0]
        A = d[1] - U * d[0]
        Cc = d[2] - V * d[0]
        a4 = 4 * lam * lam / (K + 2) * (B - 2 * U * A - 2 * V * Cc)
        a3 = 2 * lam * Cc - V * a4
        a2 = 2 * lam * A - U * a4
        a1 = d[0] - U * a2 - V * a3 - 0.5 * a4 * e
        assert np.allclose(oracle.slope(W, D, 2, G), [a1, a2, a3, a4], rtol=1e-10, atol=1e-12)


# --------------------------------------------------- BGK time integrals
@pytest.mark.parametrize("T,tau", [(0.1, 0.01), (0.02, 0.05), (1e-3, 1e-4)])
def test_time_coefficients_by_quadrature(oracle, T, tau):
    """Integrals over [0, T] of the time factors of the BGK integral solution
    (Eq. integral_f with a linear-in-space-time equilibrium)."""
    fs = [lambda t: 1 - math.exp(-t / tau),
          lambda t: (t + tau) * math.exp(-t / tau) - tau,
          lambda t: t - tau + tau * math.exp(-t / tau),
          lambda t: math.exp(-t / tau),
          lambda t: -(t + tau) * math.exp(-t / tau)]
    q = oracle.qcoef(T, tau)
    for k in range(5):
        want = integrate.quad(fs[k], 0, T, epsabs=1e-16, epsrel=1e-13)[0]
        assert q[k] == pytest.approx(want, rel=1e-10, abs=1e-18)


# --------------------------------------------------- gas-kinetic solver
def _euler_flux(W):
    rho, m, n, E = W
    U, V = m / rho, n / rho
    p = (G - 1) * (E - 0.5 * rho * (U * U + V * V))
    return np.array([m, m * U + p, m * V, U * (E + p)]), np.array([n, n * U, n * V + p, V * (E + p)])


def _jac(fun, W, eps=1e-6):
    J = np.zeros((4, 4))
    for k in range(4):
        d = np.zeros(4)
        d[k] = eps * max(1.0, abs(W[k]))
        J[:, k] = (fun(W + d) - fun(W - d)) / (2 * d[k])
    return J


def test_uniform_interface_is_exact_euler_flux(oracle):
    W = np.array([1.3, 0.4, -0.2, 2.9])
    z = np.zeros(4)
    for dt in (0.01, 1e-4):
        r = oracle.gks_interface(_par(oracle), 2, W, W, z, z, z, dt)
        F, _ = _euler_flux(W)
        assert np.allclose(r["F"], F, rtol=1e-14, atol=1e-14)
        assert np.allclose(r["Ft"], 0, atol=1e-12)
        assert np.allclose(r["Wl"], W, rtol=1e-14) and np.allclose(r["Wr"], W, rtol=1e-14)
        assert np.allclose(r["Wlt"], 0, atol=1e-12)


def test_node_euler_flux_and_time_derivative(oracle):
    """Euler node: F = exact Euler flux; F_t = F'(W) W_t with
    W_t = -(F'(W) W_x + G'(W) W_y) (finite-difference Jacobians of the
    closed-form Euler fluxes)."""
    rng = np.random.default_rng(7)
    for _ in range(5):
        rho, U, V, p = 0.7 + rng.random(), rng.normal(0, 0.5), rng.normal(0, 0.5), 0.7 + rng.random()
        W = np.array([rho, rho * U, rho * V, p / (G - 1) + 0.5 * rho * (U * U + V * V)])
        Wx, Wy = rng.normal(size=4), rng.normal(size=4)
        r = oracle.gks_node(_par(oracle), 2, W, Wx, Wy)
        F, Gf = _euler_flux(W)
        A = _jac(lambda w: _euler_flux(w)[0], W)
        B = _jac(lambda w: _euler_flux(w)[1], W)
        Wt = -(A @ Wx + B @ Wy)
        assert np.allclose(r["F"], F, rtol=1e-13) and np.allclose(r["G"], Gf, rtol=1e-13)
        assert np.allclose(r["Ft"], A @ Wt, rtol=1e-7, atol=1e-8)
        assert np.allclose(r["Gt"], B @ Wt, rtol=1e-7, atol=1e-8)


def test_node_navier_stokes_shear_and_heat_flux(oracle):
    """Chapman-Enskog node with tau = mu/p: simple shear gives the stress
    -mu dU/dy; a temperature gradient at rest gives the Fourier flux
    -mu c_p / Pr dT/dx (R = 1, c_p = gamma/(gamma-1)) once the Prandtl fix is
    applied."""
    mu, Pr = 2e-3, 0.72
    p = _par(oracle, mu=mu, prandtl=Pr)
    rho, pr = 1.1, 0.9
    # shear: U = U(y)
    W = np.array([rho, rho * 0.3, 0.0, pr / (G - 1) + 0.5 * rho * 0.09])
    Uy = 0.8
    Wy = np.array([0.0, rho * Uy, 0.0, rho * 0.3 * Uy])
    r = oracle.gks_node(p, 2, W, np.zeros(4), Wy)
    Fe, Ge = _euler_flux(W)
    assert r["G"][1] - Ge[1] == pytest.approx(-mu * Uy, rel=1e-12)
    # heat: U = V = 0, uniform p, rho varying in x  ->  T = p/rho
    W = np.array([rho, 0.0, 0.0, pr / (G - 1)])
    rx = 0.3
    Wx = np.array([rx, 0.0, 0.0, 0.0])
    r = oracle.gks_node(p, 2, W, Wx, np.zeros(4))
    Tx = -pr / rho ** 2 * rx
    cp = G / (G - 1)
    assert r["F"][0] == pytest.approx(0.0, abs=1e-15)
    assert r["F"][3] == pytest.approx(-mu * cp / Pr * Tx, rel=1e-12)


@pytest.mark.parametrize("mu", [0.0, 1e-3])
def test_continuous_interface_equals_nodal_form(oracle, mu):
    """With identical, continuous left/right data the interface solution
    collapses to the smooth form g[1 - tau((a.psi)u + (b.psi)v + A.psi)] + t A g
    of the nodal solver (same tau)."""
    p = _par(oracle, mu=mu, prandtl=0.72 if mu else 1.0)
    W = np.array([1.1, 0.2, 0.35, 2.6])
    Wn, Wt = np.array([0.1, -0.3, 0.2, 0.5]), np.array([-0.2, 0.1, 0.05, -0.4])
    r = oracle.gks_interface(p, 2, W, W, Wn, Wn, Wt, 0.01)
    nd = oracle.gks_node(p, 2, W, Wn, Wt)
    assert np.allclose(r["F"], nd["F"], rtol=1e-12, atol=1e-13)
    assert np.allclose(r["Ft"], nd["Ft"], rtol=1e-10, atol=1e-11)


def test_1d_interface_and_node(oracle):
    p = _par(oracle, dim=1, nx=8)
    rho, U, pr = 1.2, 0.4, 0.8
    W = np.array([rho, rho * U, pr / (G - 1) + 0.5 * rho * U * U])
    r = oracle.gks_interface(p, 1, W, W, np.zeros(3), np.zeros(3), None, 0.01)
    assert np.allclose(r["F"], [rho * U, rho * U * U + pr, U * (W[2] + pr)], rtol=1e-14)
    Wx = np.array([0.3, -0.1, 0.2])
    f1 = lambda w: np.array([w[1], w[1] ** 2 / w[0] + (G - 1) * (w[2] - 0.5 * w[1] ** 2 / w[0]),  # noqa: E731
                             w[1] / w[0] * (w[2] + (G - 1) * (w[2] - 0.5 * w[1] ** 2 / w[0]))])
    J = np.zeros((3, 3))
    for k in range(3):
        d = np.zeros(3)
        d[k] = 1e-6
        J[:, k] = (f1(W + d) - f1(W - d)) / 2e-6
    nd = oracle.gks_node(p, 1, W, Wx)
    assert np.allclose(nd["F"], f1(W), rtol=1e-13)
    assert np.allclose(nd["Ft"], J @ (-(J @ Wx)), rtol=1e-7, atol=1e-9)


# ---------------------------------------------------------------- S2O4
def test_s2o4_on_linear_ode(oracle):
    """W' = lam W with L = lam W, L_t = lam^2 W: one step reproduces
    1 + z + z^2/2 + z^3/6 + z^4/24 (Eq. eq-nodal-update with L-tilde = L, D8)."""
    for lam, dt in ((-1.3, 0.2), (0.7, 0.1), (-5.0, 0.05)):
        W = 1.7
        ws, acc = oracle.s2o4_scalar(1, dt, W, lam * W, lam * lam * W)
        wn, _ = oracle.s2o4_scalar(2, dt, ws, lam * ws, lam * lam * ws, acc)
        z = lam * dt
        assert wn == pytest.approx(W * (1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24), rel=1e-14)
