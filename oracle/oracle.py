"""ctypes front end of the FD-CGKS oracle (``fdcgks_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py``.  It never imports the product package
and the product package never imports it.

Arrays cross the boundary as contiguous float64 numpy arrays.  3D state:
(4, 20, nz, ny, nx), the four grids of the 3D lattice.  2D state: one
array per grid holding W[0..3], Wx[0..3], Wy[0..3]: (12, ny, nx) for the
primary grid, (12, ny + by, nx + bx) for the dual grid, with bx (by) = 1 when
the x (y) sides are not periodic (the boundary lines carry dual nodes).  1D
state: (lines, 6, N) holding W[0..2], Wx[0..2] per line.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fdcgks_oracle.cpp")
LIB = os.path.join(HERE, "liboracle_fdcgks.so")


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (FP contraction off so the arithmetic is the
    written one, OpenMP over grid rows)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


class Par(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("bc", C.c_int32),
        ("dual_1d", C.c_int32), ("variant", C.c_int32), ("r", C.c_int32), ("grad_carried", C.c_int32),
        ("recon_char", C.c_int32), ("flux_order", C.c_int32), ("side", C.c_int32 * 4),
        ("x0", C.c_double), ("lx", C.c_double), ("y0", C.c_double), ("ly", C.c_double),
        ("gamma", C.c_double), ("mu", C.c_double), ("prandtl", C.c_double),
        ("C", C.c_double), ("eps", C.c_double), ("eps_a", C.c_double),
        ("d_central", C.c_double), ("d_side", C.c_double),
        ("tau_c1", C.c_double), ("tau_c2", C.c_double),
        ("z0", C.c_double), ("lz", C.c_double), ("nz", C.c_int32), ("pad_", C.c_int32),
    ]


VARIANTS = {"6-4": 0, "6-2": 1, "linear": 2}
BCS = {"periodic": 0, "zero_gradient": 1, "reflecting": 2, "no_slip": 3}


def make_par(*, dim=2, nx=16, ny=16, nz=1, x0=0.0, lx=1.0, y0=0.0, ly=None, z0=0.0, lz=None, bc="periodic", dual_1d=0,
             gamma=1.4, mu=0.0, prandtl=1.0, variant="6-4", geno_C=20.0, geno_r=3,
             geno_eps=1e-15, geno_eps_a=1e-6, d_central=8.0, d_side=1.0, tau_c1=0.0,
             tau_c2=1.0, grad_carried=0, recon_vars="conservative", sides=None, flux_order=6, **_ignored) -> Par:
    """Problem description with the oracle's own field layout.  Defaults are the
    readings of the paper (C = 20, r = 3, eps = 1e-15, eps_a = 1e-6, d = 8/1,
    tau = 0 * dt + dt |dp|/(p_l+p_r) for Euler: D11 as amended).  2D sides
    (x-low, x-high, y-low, y-high) default to `bc` on every side.  flux_order
    6 is the compact flux of Sec. 2.1; 8 the wider stencil over nodes
    j-1..j+2 (a reading: the paper mentions it without formulas).  3D
    problems (dim 3) are periodic on all sides, with nz nodes along z."""
    p = Par()
    p.dim, p.nx, p.ny = dim, nx, (ny if dim >= 2 else 1)
    p.nz = nz if dim == 3 else 1
    if dim == 3 and (bc != "periodic" or sides is not None):
        raise ValueError("3D problems are periodic")
    p.bc = BCS[bc] if isinstance(bc, str) else int(bc)
    sd = [p.bc] * 4 if sides is None else [BCS[b] if isinstance(b, str) else int(b) for b in sides]
    if dim == 2:
        for ax in range(2):
            if (sd[2 * ax] == 0) != (sd[2 * ax + 1] == 0):
                raise ValueError("a periodic side needs a periodic opposite side")
    p.side[:] = sd
    p.dual_1d = int(dual_1d)
    p.variant = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    p.r = int(geno_r)
    p.x0, p.lx, p.y0 = x0, lx, y0
    p.ly = lx * p.ny / nx if ly is None else ly
    p.z0 = z0
    p.lz = lx * p.nz / nx if lz is None else lz
    p.gamma, p.mu, p.prandtl = gamma, mu, prandtl
    p.C, p.eps, p.eps_a, p.d_central, p.d_side = geno_C, geno_eps, geno_eps_a, d_central, d_side
    p.tau_c1, p.tau_c2 = tau_c1, tau_c2
    p.grad_carried = int(grad_carried)
    if int(flux_order) not in (6, 8):
        raise ValueError("flux_order is 6 or 8")
    p.flux_order = int(flux_order)
    p.recon_char = {"conservative": 0, "characteristic": 1}[recon_vars] if isinstance(recon_vars, str) \
        else int(recon_vars)
    return p


_lib = None
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        P = C.POINTER(Par)
        d, i = C.c_double, C.c_int
        sig = {
            "orc_abi_version": (i, []),
            "orc_recon_interface": (None, [P, _dp, _dp, d, _dp]),
            "orc_recon_node": (d, [P, _dp, _dp, d]),
            "orc_char_basis": (None, [C.c_int, d, _dp, _dp, _dp]),
            "orc_geno_blend": (None, [P, _dp, i, _dp, _dp, _dp, d, d, _dp]),
            "orc_maxwell": (None, [d, d, d, d, i, i, _dp]),
            "orc_slope": (None, [_dp, _dp, i, d, _dp]),
            "orc_qcoef": (None, [d, d, _dp]),
            "orc_gks_interface": (None, [P, i, _dp, _dp, _dp, _dp, _dp, _dp, d, _dp]),
            "orc_gks_node": (None, [P, i, _dp, _dp, _dp, _dp, _dp]),
            "orc_compact_flux": (d, [P, d, d, d, d, d, d, d, d]),
            "orc_s2o4_scalar": (None, [i, d, d, d, d, d, _dp]),
            "orc_stage2d": (None, [P, i, d, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]),
            "orc_dt2d": (d, [P, _dp, _dp, d]),
            "orc_step2d": (i, [P, _dp, _dp, i, d, d, d, _dp]),
            "orc_intermediates2d": (None, [P, d, _dp, _dp, _dp, _dp, _dp, _dp]),
            "orc_stage2d_sample": (None, [P, i, d, _dp, _dp, _dp, _dp, i, _ip, _ip, _ip, _dp]),
            "orc_step2d_tangent": (None, [P, d, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]),
            "orc_stage3d": (None, [P, i, d, _dp, _dp, _dp, _dp]),
            "orc_dt3d": (d, [P, _dp, d]),
            "orc_step3d": (i, [P, _dp, i, d, d, d, _dp]),
            "orc_intermediates3d": (None, [P, d, _dp, _dp, _dp]),
            "orc_stage3d_sample": (None, [P, i, d, _dp, _dp, i, _ip, _ip, _ip, _ip, _dp]),
            "orc_stage1d": (None, [P, i, d, _dp, _dp, _dp, _dp]),
            "orc_dt1d": (d, [P, _dp, d]),
            "orc_step1d": (i, [P, _dp, i, d, d, d, _dp]),
            "orc_intermediates1d": (None, [P, d, _dp, _dp, _dp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _arr(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if n is not None:
        assert a.size == n
    return a


# ---------------------------------------------------------------- unit level
def recon_interface(par, Q, X, h):
    """(v_l, d_l, chi_l, v_r, d_r, chi_r) at j+1/2 from Q_{j-1..j+2}, Q_{x,j-1..j+2}."""
    out = np.zeros(6)
    lib().orc_recon_interface(C.byref(par), _p(_arr(Q, 4)), _p(_arr(X, 4)), h, _p(out))
    return out


def recon_node(par, Q, X, h):
    return lib().orc_recon_node(C.byref(par), _p(_arr(Q, 3)), _p(_arr(X, 3)), h)


def char_basis(dim, gamma, W):
    """(R, L) (n x n, n = dim + 2) at the local-frame conservative state W."""
    R = np.zeros(25)
    L = np.zeros(25)
    lib().orc_char_basis(dim, gamma, _p(_arr(W, dim + 2)), _p(R), _p(L))
    n = dim + 2
    return R.reshape(5, 5)[:n, :n], L.reshape(5, 5)[:n, :n]


def geno_blend(par, IS, ref, d, q, dq, PH, PHx):
    out = np.zeros(3)
    lib().orc_geno_blend(C.byref(par), _p(_arr(IS, 3)), ref, _p(_arr(d, 3)), _p(_arr(q, 3)),
                         _p(_arr(dq, 3)), PH, PHx, _p(out))
    return out  # value, derivative, chi


def maxwell(U, V, lam, K, half, dim):
    out = np.zeros(23)
    lib().orc_maxwell(U, V, lam, K, half, dim, _p(out))
    return out[:10], out[10:20], out[20:23]


def slope(W, D, dim, gamma):
    s = np.zeros(dim + 2)
    lib().orc_slope(_p(_arr(W, dim + 2)), _p(_arr(D, dim + 2)), dim, gamma, _p(s))
    return s


def qcoef(T, tau):
    q = np.zeros(5)
    lib().orc_qcoef(T, tau, _p(q))
    return q


def gks_interface(par, dim, WL, WR, WnL, WnR, Wt, dt, Wt2=None):
    """Interface solver in the local frame; Wt, Wt2: tangential slopes along
    the v and (3D) w axes."""
    n = dim + 2
    out = np.zeros(9 * n + 1)
    wt = _arr(Wt if Wt is not None else np.zeros(n), n)
    wt2 = _arr(Wt2 if Wt2 is not None else np.zeros(n), n)
    lib().orc_gks_interface(C.byref(par), dim, _p(_arr(WL, n)), _p(_arr(WR, n)), _p(_arr(WnL, n)),
                            _p(_arr(WnR, n)), _p(wt), _p(wt2), dt, _p(out))
    keys = ["F", "Ft", "We", "Wet", "Wl", "Wr", "Wlt", "Wrt"]
    r = {k: out[i * n:(i + 1) * n].copy() for i, k in enumerate(keys)}
    r["tau"] = out[8 * n]
    r["W0"] = out[8 * n + 1:9 * n + 1].copy()
    return r


def gks_node(par, dim, W, Wx, Wy=None, Wz=None):
    n = dim + 2
    out = np.zeros(6 * n)
    wy = _arr(Wy if Wy is not None else np.zeros(n), n)
    wz = _arr(Wz if Wz is not None else np.zeros(n), n)
    lib().orc_gks_node(C.byref(par), dim, _p(_arr(W, n)), _p(_arr(Wx, n)), _p(wy), _p(wz), _p(out))
    return {"F": out[:n], "Ft": out[n:2 * n], "G": out[2 * n:3 * n], "Gt": out[3 * n:4 * n],
            "H": out[4 * n:5 * n], "Ht": out[5 * n:]}


def compact_flux(par, Fm, Fc, Fp, N0, N1, chi, Nm=0.0, Np2=0.0):
    """Interface fluxes Fm, Fc, Fp at j-1/2, j+1/2, j+3/2; nodal fluxes N0, N1
    at j, j+1 (and Nm, Np2 at j-1, j+2, read by flux_order 8)."""
    return lib().orc_compact_flux(C.byref(par), Fm, Fc, Fp, Nm, N0, N1, Np2, chi)


def s2o4_scalar(stage, dt, W, L, Lt, acc=0.0):
    out = np.zeros(2)
    lib().orc_s2o4_scalar(stage, dt, W, L, Lt, acc, _p(out))
    return out


# ---------------------------------------------------------------------- 2D
def stage2d(par, stage, dt, P, D, accP=None, accD=None):
    P, D = _arr(P), _arr(D)
    oP, oD = np.zeros_like(P), np.zeros_like(D)
    aP = np.zeros_like(P) if stage == 1 else None
    aD = np.zeros_like(D) if stage == 1 else None
    lib().orc_stage2d(C.byref(par), stage, dt, _p(P), _p(D), _p(None if accP is None else _arr(accP)),
                      _p(None if accD is None else _arr(accD)), _p(oP), _p(oD), _p(aP), _p(aD))
    return (oP, oD, aP, aD) if stage == 1 else (oP, oD)


def dual_shape(par):
    """(ny, nx) of the dual grid."""
    return par.ny + (par.side[2] != 0), par.nx + (par.side[0] != 0)


def dt2d(par, P, D, cfl):
    return lib().orc_dt2d(C.byref(par), _p(_arr(P)), _p(_arr(D)), cfl)


def step2d(par, P, D, nsteps, dt=0.0, cfl=0.5, t_end=0.0, t=0.0):
    """Advance; returns (P, D, t, steps)."""
    P, D = _arr(P).copy(), _arr(D).copy()
    tt = C.c_double(t)
    k = lib().orc_step2d(C.byref(par), _p(P), _p(D), nsteps, dt, cfl, t_end, C.byref(tt))
    return P, D, tt.value, k


def intermediates2d(par, dt, P, D):
    """Per-interface (X, Y: (2 normals, 25, ny, nx)) and per-node (P, D:
    (16, ny, nx)) intermediates of stage 1."""
    ny, nx = par.ny, par.nx
    X = np.zeros((2, 25, ny, nx)); Y = np.zeros((2, 25, ny, nx))
    NP = np.zeros((16, ny, nx)); ND = np.zeros((16, ny, nx))
    lib().orc_intermediates2d(C.byref(par), dt, _p(_arr(P)), _p(_arr(D)), _p(X), _p(Y), _p(NP), _p(ND))
    return X, Y, NP, ND


def stage2d_sample(par, stage, dt, P, D, grid, jj, ii, accP=None, accD=None):
    """Stage output at the listed nodes only: (ns, 12) state and (ns, 12) accumulators."""
    grid = np.ascontiguousarray(grid, dtype=np.int32)
    jj = np.ascontiguousarray(jj, dtype=np.int32)
    ii = np.ascontiguousarray(ii, dtype=np.int32)
    ns = grid.size
    out = np.zeros((ns, 24))
    ip = lambda a: a.ctypes.data_as(_ip)  # noqa: E731
    lib().orc_stage2d_sample(C.byref(par), stage, dt, _p(_arr(P)), _p(_arr(D)),
                             _p(None if accP is None else _arr(accP)), _p(None if accD is None else _arr(accD)),
                             ns, ip(grid), ip(jj), ip(ii), _p(out))
    return out[:, :12], out[:, 12:]


def step2d_tangent(par, dt, P, D, dP, dD):
    """One step and its derivative along (dP, dD) (forward mode, dual
    numbers through both stages).  D and dD have the dual grid's size, one
    node more along a bounded axis."""
    P, D, dP, dD = _arr(P), _arr(D), _arr(dP), _arr(dD)
    if dP.shape != P.shape or dD.shape != D.shape:
        raise ValueError("the direction must have the state's shape")
    oP, odP = np.zeros_like(P), np.zeros_like(P)
    oD, odD = np.zeros_like(D), np.zeros_like(D)
    lib().orc_step2d_tangent(C.byref(par), dt, _p(P), _p(D), _p(dP), _p(dD), _p(oP), _p(oD), _p(odP), _p(odD))
    return oP, oD, odP, odD


def state_from_samples(par, S):
    """Input state from point samples of the initial field on the
    half-spacing lattice, periodic (Eq. define-averaged-gradient, D31): the
    nodal value is the sample at the node, the averaged derivative the
    difference of the samples at the node's two bounding interfaces over h.
    2D: S (ncomp, 2ny, 2nx), sample (ky, kx) at (x0 + (kx+1)h/2,
    y0 + (ky+1)h/2); returns (P, D).  1D: S (ncomp, 2nx); returns the
    (lines, 6, nx) line state (line 1, the shifted copy, from odd samples)."""
    S = np.asarray(S, dtype=np.float64)
    h = par.lx / par.nx
    if par.dim == 2:
        nc, NY, NX = S.shape
        out = []
        for g in range(2):
            A = np.zeros((12, par.ny, par.nx))
            for j in range(par.ny):
                for i in range(par.nx):
                    kx, ky = 2 * i + g, 2 * j + g
                    for c in range(nc):
                        A[c, j, i] = S[c, ky, kx]
                        A[4 + c, j, i] = (S[c, ky, (kx + 1) % NX] - S[c, ky, (kx - 1) % NX]) / h
                        A[8 + c, j, i] = (S[c, (ky + 1) % NY, kx] - S[c, (ky - 1) % NY, kx]) / h
            out.append(A)
        return out[0], out[1]
    nc, NX = S.shape
    lines = 2 if par.dual_1d else 1
    A = np.zeros((lines, 6, par.nx))
    for ln in range(lines):
        for j in range(par.nx):
            k = 2 * j + ln
            for c in range(nc):
                A[ln, c, j] = S[c, k]
                A[ln, 3 + c, j] = (S[c, (k + 1) % NX] - S[c, (k - 1) % NX]) / h
    return A


# ---------------------------------------------------------------------- 3D
def _s3(par, S):
    S = _arr(S)
    assert S.shape == (4, 20, par.nz, par.ny, par.nx), S.shape
    return S


def stage3d(par, stage, dt, S, acc=None):
    """One stage on the four 3D grids, S (4, 20, nz, ny, nx); stage 1 returns
    (out, acc), stage 2 out."""
    S = _s3(par, S)
    out = np.zeros_like(S)
    a = np.zeros_like(S) if stage == 1 else None
    lib().orc_stage3d(C.byref(par), stage, dt, _p(S), _p(None if acc is None else _s3(par, acc)), _p(out), _p(a))
    return (out, a) if stage == 1 else out


def dt3d(par, S, cfl):
    return lib().orc_dt3d(C.byref(par), _p(_s3(par, S)), cfl)


def step3d(par, S, nsteps, dt=0.0, cfl=0.5, t_end=0.0, t=0.0):
    """Advance; returns (S, t, steps)."""
    S = _s3(par, S).copy()
    tt = C.c_double(t)
    k = lib().orc_step3d(C.byref(par), _p(S), nsteps, dt, cfl, t_end, C.byref(tt))
    return S, tt.value, k


def intermediates3d(par, dt, S):
    """Stage-1 intermediates: interface classes (4, 3 normals, 31, nz, ny, nx)
    and nodal fluxes (4 grids, 30, nz, ny, nx)."""
    shp = (par.nz, par.ny, par.nx)
    E = np.zeros((4, 3, 31) + shp)
    N = np.zeros((4, 30) + shp)
    lib().orc_intermediates3d(C.byref(par), dt, _p(_s3(par, S)), _p(E), _p(N))
    return E, N


def stage3d_sample(par, stage, dt, S, grid, kk, jj, ii, acc=None):
    """Stage output at the listed nodes only: (ns, 20) state and (ns, 20)
    accumulators."""
    ar = [np.ascontiguousarray(a, dtype=np.int32) for a in (grid, kk, jj, ii)]
    ns = ar[0].size
    out = np.zeros((ns, 40))
    ip = lambda a: a.ctypes.data_as(_ip)  # noqa: E731
    lib().orc_stage3d_sample(C.byref(par), stage, dt, _p(_s3(par, S)), _p(None if acc is None else _s3(par, acc)),
                             ns, *(ip(a) for a in ar), _p(out))
    return out[:, :20], out[:, 20:]


# ---------------------------------------------------------------------- 1D
def stage1d(par, stage, dt, S, acc=None):
    S = _arr(S)
    out = np.zeros_like(S)
    a = np.zeros_like(S) if stage == 1 else None
    lib().orc_stage1d(C.byref(par), stage, dt, _p(S), _p(None if acc is None else _arr(acc)), _p(out), _p(a))
    return (out, a) if stage == 1 else out


def dt1d(par, S, cfl):
    return lib().orc_dt1d(C.byref(par), _p(_arr(S)), cfl)


def step1d(par, S, nsteps, dt=0.0, cfl=0.5, t_end=0.0, t=0.0):
    S = _arr(S).copy()
    tt = C.c_double(t)
    k = lib().orc_step1d(C.byref(par), _p(S), nsteps, dt, cfl, t_end, C.byref(tt))
    return S, tt.value, k


def intermediates1d(par, dt, S):
    """Interfaces j+1/2 for j = -2..N: (19, N+3); nodes j = -1..N: (6, N+2)."""
    N = par.nx
    E = np.zeros((19, N + 3)); Nn = np.zeros((6, N + 2))
    lib().orc_intermediates1d(C.byref(par), dt, _p(_arr(S)), _p(E), _p(Nn))
    return E, Nn
