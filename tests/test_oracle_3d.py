"""Pins of the oracle's 3D scheme (the four-grid lattice of the dual-grid
layout carried to three dimensions, readings D32/D33).  CPU only.

* a uniform state is preserved exactly, and the uniform interface and node
  solvers give the exact 3D Euler fluxes;
* the sums of all five conservative components are conserved on each of the
  four grids;
* a state that does not vary along one axis, with no velocity along it, is a
  2D problem in the other two: the values after a stage on the primary grid
  and on the dual grid that is even along both remaining axes equal the 2D
  oracle's on its primary and dual grids (the 3D Maxwellian with K = 2 and
  the w direction at rest has the moments of the 2D one with K = 3), for each
  of the three axes, inviscid and viscous;
* a stage commutes with every permutation of the axes and with periodic
  shifts;
* the smooth 3D advection test (the Sec. 5.1 test with U = V = W = 1 and
  rho = 1 + 0.2 sin(pi (x + y + z))) converges at the design order 6.
"""
import itertools

import numpy as np
import pytest

import workloads as WL
from tests.helpers import settings


def _p3(oracle, nx, ny=None, nz=None, lx=1.0, **kw):
    return oracle.make_par(**settings(dim=3, nx=nx, ny=ny or nx, nz=nz or nx, lx=lx, **kw))


def _euler3(W, gamma=1.4):
    rho, m, E = W[0], W[1:4], W[4]
    u = m / rho
    p = (gamma - 1) * (E - 0.5 * rho * (u @ u))
    fl = []
    for a in range(3):
        f = np.zeros(5)
        f[0] = m[a]
        f[1:4] = m * u[a]
        f[1 + a] += p
        f[4] = u[a] * (E + p)
        fl.append(f)
    return fl


def test_free_stream_is_preserved_exactly(oracle):
    n = 5
    S = np.zeros((4, 20, n, n, n))
    S[:, 0:5] = WL.conservative3d(1.3, 0.4, -0.7, 0.25, 2.0)[None, :, None, None, None]
    par = _p3(oracle, n)
    out, t, k = oracle.step3d(par, S, 2, dt=0.01)
    assert np.abs(out - S).max() < 1e-14


def test_uniform_solvers_give_the_euler_fluxes(oracle):
    W = WL.conservative3d(1.2, 0.3, -0.4, 0.5, 0.9)
    z = np.zeros(5)
    par = _p3(oracle, 4)
    F = _euler3(W)
    r = oracle.gks_interface(par, 3, W, W, z, z, z, 0.01, Wt2=z)
    assert np.allclose(r["F"], F[0], rtol=1e-14, atol=1e-14)
    nd = oracle.gks_node(par, 3, W, z, z, z)
    for a, k in enumerate("FGH"):
        assert np.allclose(nd[k], F[a], rtol=1e-14, atol=1e-14), k
        assert np.abs(nd[k + "t"]).max() < 1e-14


@pytest.mark.parametrize("case", ["rough", "smooth"])
def test_conservation_on_all_four_grids(oracle, case):
    pr = WL.random_rough3d(6, 5, 4, seed=1) if case == "rough" else WL.random_smooth3d(6, 5, 4, seed=2)
    par = _p3(oracle, pr.nx, pr.ny, pr.nz, lx=pr.lx)
    out, t, k = oracle.step3d(par, pr.S, 2, dt=0.2 * pr.h / 3)
    for g in range(4):
        for c in range(5):
            scale = np.abs(pr.S[g, c]).sum()
            assert abs(out[g, c].sum() - pr.S[g, c].sum()) <= 1e-13 * scale, (g, c)


def _embed(P2, D2, axis, n_axis, rng):
    """3D state constant along `axis` from a 2D state whose axes (x2, y2) are
    the remaining 3D axes in increasing order.  The two grids with no 2D
    counterpart get random values constant along `axis`, at rest along it."""
    p, q = [a for a in range(3) if a != axis]
    comp = [0, 1 + p, 1 + q, 4]          # 2D component -> 3D component
    fld = [0, 1 + p, 1 + q]              # 2D field (W, W_x2, W_y2) -> 3D field
    ny2, nx2 = P2.shape[1:]
    shape = [0, 0, 0]
    shape[p], shape[q], shape[axis] = nx2, ny2, n_axis
    nz, ny, nx = shape[2], shape[1], shape[0]
    S = np.zeros((4, 20, nz, ny, nx))

    def place(A2):  # (ny2, nx2) -> (nz, ny, nx), constant along axis
        A = A2.T  # indices (x2, y2)
        idx = [None, None, None]
        idx[p], idx[q] = slice(None), slice(None)
        A = np.expand_dims(A, axis)  # axes ordered (x, y, z) with `axis` inserted
        A = np.broadcast_to(A, (nx, ny, nz))
        return np.transpose(A, (2, 1, 0))

    even = {frozenset(): 0, frozenset({0, 1}): 1, frozenset({0, 2}): 2, frozenset({1, 2}): 3}
    gP, gD = 0, even[frozenset({p, q})]
    for g, A2 in ((gP, P2), (gD, D2)):
        for f2 in range(3):
            for c2 in range(4):
                S[g, 5 * fld[f2] + comp[c2]] = place(A2[4 * f2 + c2])
    for g in range(4):
        if g in (gP, gD):
            continue
        rho = rng.uniform(0.8, 1.2, (ny2, nx2))
        u = rng.uniform(-0.3, 0.3, (2, ny2, nx2))
        pr = rng.uniform(0.8, 1.2, (ny2, nx2))
        W = WL.conservative(rho, u[0], u[1], pr)
        for c2 in range(4):
            S[g, comp[c2]] = place(W[c2])
            S[g, 5 * (1 + p) + comp[c2]] = place(rng.normal(0, 0.3, (ny2, nx2)))
            S[g, 5 * (1 + q) + comp[c2]] = place(rng.normal(0, 0.3, (ny2, nx2)))
    return np.ascontiguousarray(S), gP, gD, comp, p, q


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("mu", [0.0, 2e-3])
def test_reduces_to_2d(oracle, axis, mu):
    pr2 = WL.random_rough2d(6, 5, seed=3)
    rng = np.random.default_rng(4)
    S, gP, gD, comp, p, q = _embed(pr2.P, pr2.D, axis, 4, rng)
    kw = dict(mu=mu, prandtl=0.72) if mu > 0 else {}
    par2 = oracle.make_par(**settings(dim=2, nx=6, ny=5, lx=pr2.lx, **kw))
    n3 = [0, 0, 0]
    n3[p], n3[q], n3[axis] = 6, 5, 4
    par3 = _p3(oracle, n3[0], n3[1], n3[2], lx=pr2.h * n3[0], **kw)
    dt = 0.01
    o2P, o2D, a2P, a2D = oracle.stage2d(par2, 1, dt, pr2.P, pr2.D)
    o3, a3 = oracle.stage3d(par3, 1, dt, S)
    for g3, o2, a2 in ((gP, o2P, a2P), (gD, o2D, a2D)):
        for c2 in range(4):
            for out3, out2 in ((o3, o2), (a3, a2)):
                ref = out2[c2].T  # (x2, y2)
                got = np.transpose(out3[g3, comp[c2]], (2, 1, 0))  # (x, y, z)
                got = np.moveaxis(got, axis, -1)  # (x2, y2, along axis)
                scale = np.abs(ref).max()
                err = np.abs(got - ref[:, :, None]).max()
                assert err <= 1e-12 * scale, (g3, c2, err)
        # no momentum along the constant axis appears
        assert np.abs(o3[g3, 1 + axis]).max() < 1e-13


def _permute(S, pa):
    """Relabel axes: new axis b is old axis pa[b] (grids, momenta, gradient
    fields and array axes follow)."""
    inv = {a: b for b, a in enumerate(pa)}
    evens = [set(), {0, 1}, {0, 2}, {1, 2}]
    order = [2 - pa[2 - m] for m in range(3)]
    out = np.empty((4, 20) + np.transpose(S[0, 0], order).shape)
    for g in range(4):
        ng = evens.index({inv[a] for a in evens[g]})
        for f in range(4):
            nf = 0 if f == 0 else 1 + inv[f - 1]
            for c in range(5):
                nc = c if c in (0, 4) else 1 + inv[c - 1]
                out[ng, 5 * nf + nc] = np.transpose(S[g, 5 * f + c], order)
    return out


@pytest.mark.parametrize("pa", [(1, 2, 0), (1, 0, 2), (2, 1, 0)])
def test_axis_permutation_symmetry(oracle, pa):
    pr = WL.random_rough3d(5, 4, 6, seed=5)
    n = (pr.nx, pr.ny, pr.nz)
    par = _p3(oracle, *n, lx=pr.lx)
    npar = _p3(oracle, *(n[pa[b]] for b in range(3)), lx=pr.h * n[pa[0]])
    a = oracle.stage3d(par, 1, 0.02, pr.S)
    b = oracle.stage3d(npar, 1, 0.02, _permute(pr.S, pa))
    for k in range(2):
        pa_k = _permute(a[k], pa)
        assert np.allclose(pa_k, b[k], rtol=1e-12, atol=1e-12 * np.abs(b[k]).max()), k


def test_shift_equivariance(oracle):
    pr = WL.random_rough3d(5, 4, 3, seed=6)
    par = _p3(oracle, 5, 4, 3, lx=pr.lx)
    r = lambda S: np.ascontiguousarray(np.roll(S, (1, -1, 2), axis=(-3, -2, -1)))  # noqa: E731
    a = oracle.stage3d(par, 1, 0.02, pr.S)
    b = oracle.stage3d(par, 1, 0.02, r(pr.S))
    for k in range(2):
        assert np.array_equal(r(a[k]), b[k])


def test_3d_accuracy_order(oracle):
    """Design order on the smooth 3D advection test (N = 5, 10 on [0, 2]^3,
    dt = 0.1 h (h / 0.4) / max(|U| + c) as in the 2D test, t = 0.25):
    measured orders 6.7 (L1) and 6.5 (Linf) over all four grids."""
    errs = []
    T = 0.25
    for N in (5, 10):
        h = 2.0 / N
        pr = WL.advection3d(N)
        par = _p3(oracle, N, lx=2.0, variant="6-2")
        dt = 0.1 * h * (h / 0.4) / (1 + np.sqrt(1.4 / 0.8))
        nst = int(np.ceil(T / dt))
        S, t, k = oracle.step3d(par, pr.S, nst, dt=T / nst)
        e = np.abs(S[:, 0] - WL.advection3d_exact(N, T)[:, 0])
        errs.append((e.mean(), e.max()))
    (a, b), (c, d) = errs
    assert np.log2(a / c) > 5.5 and np.log2(b / d) > 5.5, errs


def test_sampled_stage_equals_whole_grid(oracle):
    """The sampled 3D stage (used at sizes too large for a whole sweep) gives
    the whole-grid stage's values at its nodes, bit for bit (order 6 and 8)."""
    pr = WL.random_rough3d(6, 5, 7, seed=9)
    rng = np.random.default_rng(3)
    ns = 30
    grid, kk, jj, ii = (rng.integers(0, 4, ns), rng.integers(0, 7, ns), rng.integers(0, 5, ns),
                        rng.integers(0, 6, ns))
    for order in (6, 8):
        par = _p3(oracle, 6, 5, 7, lx=pr.lx, flux_order=order, mu=1e-3, prandtl=0.72)
        o1, a1 = oracle.stage3d(par, 1, 0.01, pr.S)
        s1, sa = oracle.stage3d_sample(par, 1, 0.01, pr.S, grid, kk, jj, ii)
        o2 = oracle.stage3d(par, 2, 0.01, o1, a1)
        s2, _ = oracle.stage3d_sample(par, 2, 0.01, o1, grid, kk, jj, ii, acc=a1)
        for q in range(ns):
            at = (grid[q], slice(None), kk[q], jj[q], ii[q])
            assert np.array_equal(s1[q], o1[at]) and np.array_equal(sa[q], a1[at]) and np.array_equal(s2[q], o2[at])
