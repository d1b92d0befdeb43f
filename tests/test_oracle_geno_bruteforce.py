"""Pin of the oracle's GENO reconstruction on non-smooth data, built here by
brute force from the definitions of Sec. 3 and App. C.  CPU only.

For every interface state (App. C1 left, App. C2 right) and every node
derivative (App. C3), the reference below:

* solves for the high-order polynomial of Eq. 7th-compact-recons /
  Eq. 6th-compact-recons from its interpolation conditions (point values at
  nodes, interval-averaged derivatives (P(x + h/2) - P(x - h/2)) / h over node
  cells), by a linear solve;
* solves for each quadratic sub-stencil polynomial from its three conditions;
* takes the smoothness indicators h int (q')^2 + h^3 int (q'')^2 over the
  cell of the node the state belongs to by Gauss-Legendre quadrature;
* forms IS^L, IS^H, IS^tau, alpha, the path function chi and the low-order
  weights d_k / (IS_k + eps_a)^2 as Eqs. GENO-nonlinear, GENO-IS-linear and
  GENO-1d-IS-HL state them, with the readings of the oracle: r = 3,
  eps = 1e-15, weight 8 on the central three-point sub-stencil, which at a
  node is also the IS^tau reference; at an interface the reference is the
  compact one-sided sub-stencil;
* blends value and derivative with the same weights.

Data with jumps and kinks put chi anywhere in [0, 1], so the low-order part,
its weights and the path function all enter the result; the comparison is at
1e-12.
"""
import math

import numpy as np
import pytest

from tests.helpers import settings

R_EXP, EPS, EPS_A, C = 3, 1e-15, 1e-6, 20.0


def _fit(conds, deg):
    """Polynomial of degree `deg` from conditions ('v', x, value) or
    ('d', x, averaged derivative over [x - h/2, x + h/2]), h carried in each."""
    A, b = [], []
    for kind, x, val, h in conds:
        if kind == "v":
            A.append([x ** k for k in range(deg + 1)])
        else:
            A.append([((x + h / 2) ** k - (x - h / 2) ** k) / h for k in range(deg + 1)])
        b.append(val)
    return np.polynomial.Polynomial(np.linalg.solve(np.array(A, float), np.array(b, float)))


def _indicator(q, a, b, h):
    x, w = np.polynomial.legendre.leggauss(12)
    x = 0.5 * (b - a) * x + 0.5 * (b + a)
    w = 0.5 * (b - a) * w
    d1, d2 = q.deriv(), q.deriv(2)
    return h * np.sum(w * d1(x) ** 2) + h ** 3 * np.sum(w * d2(x) ** 2)


def _geno(IS, ref, d, vals, ders, PH, PHx):
    others = [k for k in range(3) if k != ref]
    tau = abs(0.5 * (IS[others[0]] + IS[others[1]]) - IS[ref])
    aH = 1 + (tau / (max(IS) + EPS)) ** R_EXP
    aL = 1 + (tau / (min(IS) + EPS)) ** R_EXP
    chi = math.tanh(C * 2 * aH / (aH + aL)) / math.tanh(C)
    wt = np.array([d[k] / (IS[k] + EPS_A) ** 2 for k in range(3)])
    wt /= wt.sum()
    PL, PLx = float(np.dot(wt, vals)), float(np.dot(wt, ders))
    return chi * PH + (1 - chi) * PL, chi * PHx + (1 - chi) * PLx, chi


def brute_interface(Q, X, h):
    """Left and right states at j+1/2 from nodes j-1..j+2 (node j at x = 0)."""
    xs = [-h, 0.0, h, 2 * h]
    xi = h / 2
    Pl = _fit([("v", xs[i], Q[i], h) for i in range(4)] + [("d", xs[k], X[k], h) for k in range(3)], 6)
    Pr = _fit([("v", xs[i], Q[i], h) for i in range(4)] + [("d", xs[k], X[k], h) for k in range(1, 4)], 6)
    Px = _fit([("v", xs[i], Q[i], h) for i in range(4)] + [("d", xs[k], X[k], h) for k in (1, 2)], 5).deriv()
    out = []
    for side in ("l", "r"):
        if side == "l":  # App. C1: cell of node j
            subs = [[("v", xs[0], Q[0], h), ("v", xs[1], Q[1], h), ("d", xs[0], X[0], h)],
                    [("v", xs[0], Q[0], h), ("v", xs[1], Q[1], h), ("v", xs[2], Q[2], h)],
                    [("v", xs[1], Q[1], h), ("v", xs[2], Q[2], h), ("v", xs[3], Q[3], h)]]
            cell, PH = (-h / 2, h / 2), Pl(xi)
        else:  # App. C2 (mirror image): cell of node j+1
            subs = [[("v", xs[3], Q[3], h), ("v", xs[2], Q[2], h), ("d", xs[3], X[3], h)],
                    [("v", xs[3], Q[3], h), ("v", xs[2], Q[2], h), ("v", xs[1], Q[1], h)],
                    [("v", xs[2], Q[2], h), ("v", xs[1], Q[1], h), ("v", xs[0], Q[0], h)]]
            cell, PH = (h / 2, 3 * h / 2), Pr(xi)
        qs = [_fit(s, 2) for s in subs]
        IS = [_indicator(q, cell[0], cell[1], h) for q in qs]
        out.append(_geno(IS, 0, [1.0, 8.0, 1.0], [q(xi) for q in qs], [q.deriv()(xi) for q in qs], PH, Px(xi)))
    return out


def brute_node(Q, X, h):
    """Derivative at node j from nodes j-1..j+1 (node j at x = 0)."""
    xs = [-h, 0.0, h]
    P = _fit([("v", xs[i], Q[i], h) for i in range(3)] + [("d", xs[i], X[i], h) for i in range(3)], 5)
    subs = [[("v", xs[0], Q[0], h), ("v", xs[1], Q[1], h), ("v", xs[2], Q[2], h)],   # central
            [("v", xs[0], Q[0], h), ("v", xs[1], Q[1], h), ("d", xs[0], X[0], h)],
            [("v", xs[1], Q[1], h), ("v", xs[2], Q[2], h), ("d", xs[2], X[2], h)]]
    qs = [_fit(s, 2) for s in subs]
    IS = [_indicator(q, -h / 2, h / 2, h) for q in qs]
    return _geno(IS, 0, [8.0, 1.0, 1.0], [q(0.0) for q in qs], [q.deriv()(0.0) for q in qs], Q[1], P.deriv()(0.0))


def _cases(n_nodes, seed):
    """Smooth background plus a jump or a kink at a random place in the stencil,
    of random size (some nearly smooth)."""
    rng = np.random.default_rng(seed)
    h = 0.1
    out = []
    for _ in range(150):
        a, b = rng.normal(size=2)
        x = np.arange(n_nodes) * h
        base = 1.0 + a * x + b * x * x
        dbase = a + b * (2 * x)  # averaged derivative of the quadratic background
        jump = 10.0 ** rng.uniform(-4, 0.5) * rng.choice([-1, 1])
        at = rng.integers(0, n_nodes - 1)  # jump between node `at` and `at` + 1
        kind = rng.choice(["jump", "kink"])
        Q = base.copy()
        X = dbase.copy()
        if kind == "jump":
            Q[at + 1:] += jump
        else:
            Q[at + 1:] += jump * (x[at + 1:] - x[at] - h / 2)
            X[at + 1:] += jump
            X[at] += jump / 2  # the kink sits at the middle of the cell edge
        out.append((Q, X, h))
    return out


def test_interface_geno_on_jumps_and_kinks(oracle):
    p = oracle.make_par(**settings(dim=2, nx=8, ny=8, lx=1.0, variant="6-4"))
    chis = []
    for Q, X, h in _cases(4, 0):
        (vl, dl, cl), (vr, dr, cr) = brute_interface(Q, X, h)
        ovl, odl, ocl, ovr, odr, ocr = oracle.recon_interface(p, Q, X, h)
        sv = max(abs(q) for q in Q)
        sd = max(abs(q) for q in X) + max(abs(Q[i + 1] - Q[i]) for i in range(3)) / h
        assert abs(ovl - vl) <= 1e-12 * sv and abs(ovr - vr) <= 1e-12 * sv, (Q, X)
        assert abs(odl - dl) <= 1e-12 * sd and abs(odr - dr) <= 1e-12 * sd, (Q, X)
        assert abs(ocl - cl) <= 1e-12 and abs(ocr - cr) <= 1e-12, (Q, X)
        chis += [cl, cr]
    chis = np.array(chis)
    # the cases cover the whole range of the path function
    assert (chis < 0.01).sum() > 5 and ((chis > 0.05) & (chis < 0.95)).sum() > 5 and (chis > 0.999).sum() > 5


def test_node_geno_on_jumps_and_kinks(oracle):
    p = oracle.make_par(**settings(dim=2, nx=8, ny=8, lx=1.0, variant="6-4"))
    for Q, X, h in _cases(3, 1):
        _, d, _ = brute_node(Q, X, h)
        od = oracle.recon_node(p, Q, X, h)
        sd = max(abs(q) for q in X) + max(abs(Q[i + 1] - Q[i]) for i in range(2)) / h
        assert abs(od - d) <= 1e-12 * sd, (Q, X, od, d)


def test_node_geno_path_function_spans_its_range():
    chis = np.array([brute_node(Q, X, h)[2] for Q, X, h in _cases(3, 1)])
    assert (chis < 0.01).sum() > 5 and ((chis > 0.05) & (chis < 0.95)).sum() > 3 and (chis > 0.999).sum() > 5


@pytest.mark.parametrize("ref", [1, 2])
def test_node_pin_is_sharp(oracle, ref):
    """Another IS^tau reference (one of the one-sided sub-stencils) changes the
    node derivative by far more than the tolerance on these cases."""
    p = oracle.make_par(**settings(dim=2, nx=8, ny=8, lx=1.0, variant="6-4"))
    worst = 0.0
    for Q, X, h in _cases(3, 1):
        xs = [-h, 0.0, h]
        P = _fit([("v", xs[i], Q[i], h) for i in range(3)] + [("d", xs[i], X[i], h) for i in range(3)], 5)
        subs = [[("v", xs[0], Q[0], h), ("v", xs[1], Q[1], h), ("v", xs[2], Q[2], h)],
                [("v", xs[0], Q[0], h), ("v", xs[1], Q[1], h), ("d", xs[0], X[0], h)],
                [("v", xs[1], Q[1], h), ("v", xs[2], Q[2], h), ("d", xs[2], X[2], h)]]
        qs = [_fit(s, 2) for s in subs]
        IS = [_indicator(q, -h / 2, h / 2, h) for q in qs]
        _, d, _ = _geno(IS, ref, [8.0, 1.0, 1.0], [0, 0, 0], [q.deriv()(0.0) for q in qs], Q[1], P.deriv()(0.0))
        sd = max(abs(q) for q in X) + max(abs(Q[i + 1] - Q[i]) for i in range(2)) / h
        worst = max(worst, abs(oracle.recon_node(p, Q, X, h) - d) / sd)
    assert worst > 1e-6
