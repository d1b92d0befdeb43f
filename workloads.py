"""Seeded synthetic inputs shaped like the paper's test problems.

This module holds no arithmetic of the method: it only samples analytic
initial conditions and turns samples into the scheme's input state (nodal
conservative values and interval-averaged derivatives).  Both the oracle tests
and the HIP path take their inputs from here; nothing else is shared.

Conventions
-----------
Mesh size h.  Samples live on the half-spacing lattice: point (I, J) at
(x0 + I h/2, y0 + J h/2).  Primary node P[j][i] is lattice (2i+1, 2j+1), dual
node D[j][i] is (2i+2, 2j+2) (periodic wrap).  The interval-averaged
derivative of a node is the difference of the exact values at its two bounding
interfaces divided by h (the Gauss form of the averaged gradient); for initial
data with jumps placed on interfaces the derivative is set to zero.

2D state per grid: float64 array (12, ny, nx) = W[0..3], Wx[0..3], Wy[0..3],
W = (rho, rho U, rho V, rho E).  1D state per line: (6, N) = W[0..2], Wx[0..2].

3D: point (I, J, L) of the lattice at (x0 + I h/2, y0 + J h/2, z0 + L h/2).
Four grids: primary P (odd, odd, odd) and the face-offset duals Dxy (even,
even, odd), Dxz (even, odd, even), Dyz (odd, even, even); stored node i along
an axis is lattice coordinate 2i+1 where the grid is odd and 2i+2 where it is
even (periodic wrap).  State: (4, 20, nz, ny, nx) = per grid W[0..4],
Wx[0..4], Wy[0..4], Wz[0..4], W = (rho, rho U, rho V, rho W, rho E).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GAMMA = 1.4


def conservative(rho, U, V, p, gamma=GAMMA):
    rho, U, V, p = np.broadcast_arrays(*(np.asarray(a, dtype=np.float64) for a in (rho, U, V, p)))
    return np.stack([rho, rho * U, rho * V, p / (gamma - 1.0) + 0.5 * rho * (U * U + V * V)])


def conservative1d(rho, U, p, gamma=GAMMA):
    rho, U, p = np.broadcast_arrays(*(np.asarray(a, dtype=np.float64) for a in (rho, U, p)))
    return np.stack([rho, rho * U, p / (gamma - 1.0) + 0.5 * rho * U * U])


# --------------------------------------------------------------------- 2D
def state_from_samples(S, h):
    """S: (4, 2ny, 2nx) conservative samples on the half lattice -> (P, D)."""
    _, JJ, II = S.shape
    ny, nx = JJ // 2, II // 2
    j = np.arange(ny)[:, None]
    i = np.arange(nx)[None, :]

    def at(J, I):
        return S[:, J % JJ, I % II]

    P = np.empty((12, ny, nx))
    D = np.empty((12, ny, nx))
    P[0:4] = at(2 * j + 1, 2 * i + 1)
    P[4:8] = (at(2 * j + 1, 2 * i + 2) - at(2 * j + 1, 2 * i)) / h
    P[8:12] = (at(2 * j + 2, 2 * i + 1) - at(2 * j, 2 * i + 1)) / h
    D[0:4] = at(2 * j + 2, 2 * i + 2)
    D[4:8] = (at(2 * j + 2, 2 * i + 3) - at(2 * j + 2, 2 * i + 1)) / h
    D[8:12] = (at(2 * j + 3, 2 * i + 2) - at(2 * j + 1, 2 * i + 2)) / h
    return np.ascontiguousarray(P), np.ascontiguousarray(D)


def lattice(nx, ny, x0, y0, h):
    I = np.arange(2 * nx)
    J = np.arange(2 * ny)
    X = x0 + I[None, :] * h / 2
    Y = y0 + J[:, None] * h / 2
    return np.broadcast_arrays(X, Y)


@dataclass
class Problem2D:
    name: str
    nx: int
    ny: int
    x0: float
    lx: float
    y0: float
    ly: float
    P: np.ndarray
    D: np.ndarray
    params: dict = field(default_factory=dict)

    @property
    def h(self):
        return self.lx / self.nx


def advection2d(n, lx=2.0):
    """Smooth density wave rho = 1 + 0.2 sin(pi (x+y)), U = V = p = 1 on
    [0, 2]^2 (Sec. 5.1 accuracy test)."""
    h = lx / n
    X, Y = lattice(n, n, 0.0, 0.0, h)
    S = conservative(1.0 + 0.2 * np.sin(np.pi * (X + Y)), 1.0, 1.0, 1.0)
    P, D = state_from_samples(S, h)
    return Problem2D("advection2d", n, n, 0.0, lx, 0.0, lx, P, D, {"gamma": GAMMA, "mu": 0.0})


def advection2d_exact(n, t, lx=2.0):
    h = lx / n
    X, Y = lattice(n, n, 0.0, 0.0, h)
    S = conservative(1.0 + 0.2 * np.sin(np.pi * (X + Y - 2 * t)), 1.0, 1.0, 1.0)
    return state_from_samples(S, h)


def vortex(n, seed=0, L=10.0, beta=5.0, gamma=GAMMA):
    """Isentropic vortex (strength beta) in a (1,1,1,1) free stream on a
    periodic [0, L]^2, centre L/2 plus a seeded offset in [-0.5, 0.5]^2."""
    rng = np.random.default_rng(seed)
    xc, yc = L / 2 + rng.uniform(-0.5, 0.5, size=2)
    h = L / n
    X, Y = lattice(n, n, 0.0, 0.0, h)
    S = _vortex_samples(X, Y, xc, yc, beta, gamma, L)
    P, D = state_from_samples(S, h)
    return Problem2D("vortex", n, n, 0.0, L, 0.0, L, P, D,
                     {"gamma": gamma, "mu": 0.0, "center": (xc, yc), "beta": beta})


def _vortex_samples(X, Y, xc, yc, beta, gamma, L):
    # nearest periodic image of the centre
    xb = (X - xc + L / 2) % L - L / 2
    yb = (Y - yc + L / 2) % L - L / 2
    r2 = xb * xb + yb * yb
    dT = -(gamma - 1.0) * beta ** 2 / (8.0 * gamma * math.pi ** 2) * np.exp(1.0 - r2)
    du = beta / (2 * math.pi) * np.exp(0.5 * (1.0 - r2))
    T = 1.0 + dT
    rho = T ** (1.0 / (gamma - 1.0))
    return conservative(rho, 1.0 - du * yb, 1.0 + du * xb, rho * T, gamma)


def vortex_exact(prob, t):
    xc, yc = prob.params["center"]
    L = prob.lx
    X, Y = lattice(prob.nx, prob.ny, 0.0, 0.0, prob.h)
    S = _vortex_samples(X, Y, (xc + t) % L, (yc + t) % L, prob.params["beta"], prob.params["gamma"], L)
    return state_from_samples(S, prob.h)


def shear_layer(n, seed=0, k=80.0, delta=0.05, Ma=0.15, gamma=GAMMA, mu=1e-4, prandtl=0.72):
    """Doubly periodic double shear layer on [0,1]^2: U = tanh(k(y-1/4)) below
    y = 1/2, tanh(k(3/4-y)) above; V = delta sin(2 pi (x + phi)), phi seeded;
    rho = 1, p = 1/(gamma Ma^2) (Sec. 5.7 shape; k = 80 <-> thickness 1/80)."""
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0.0, 1.0)
    h = 1.0 / n
    X, Y = lattice(n, n, 0.0, 0.0, h)
    U = np.where(Y <= 0.5, np.tanh(k * (Y - 0.25)), np.tanh(k * (0.75 - Y)))
    V = delta * np.sin(2 * math.pi * (X + phi))
    S = conservative(1.0, U, V, 1.0 / (gamma * Ma * Ma), gamma)
    P, D = state_from_samples(S, h)
    return Problem2D("shear_layer", n, n, 0.0, 1.0, 0.0, 1.0, P, D,
                     {"gamma": gamma, "mu": mu, "prandtl": prandtl, "phi": phi})


def riemann2d(n, seed=0, gamma=GAMMA):
    """Four-quadrant Riemann data on a periodic [0,1]^2 (quadrant states seeded
    from rho in [0.1,1], u, v in [-1,1], p in [0.1,1]); jumps on interfaces,
    zero initial derivatives."""
    rng = np.random.default_rng(seed)
    q = [(rng.uniform(0.1, 1), rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0.1, 1)) for _ in range(4)]
    h = 1.0 / n
    X, Y = lattice(n, n, 0.0, 0.0, h)
    quad = (X >= 0.5).astype(int) + 2 * (Y >= 0.5).astype(int)
    rho = np.choose(quad, [s[0] for s in q])
    U = np.choose(quad, [s[1] for s in q])
    V = np.choose(quad, [s[2] for s in q])
    p = np.choose(quad, [s[3] for s in q])
    S = conservative(rho, U, V, p, gamma)
    P, D = state_from_samples(S, h)
    P[4:] = 0.0
    D[4:] = 0.0
    return Problem2D("riemann2d", n, n, 0.0, 1.0, 0.0, 1.0, P, D, {"gamma": gamma, "mu": 0.0, "states": q})


def random_smooth2d(nx, ny, seed=0, amp=0.1, modes=3, lx=1.0):
    """A seeded smooth periodic flow (sums of low Fourier modes) for parity
    tests on non-square grids."""
    rng = np.random.default_rng(seed)
    h = lx / nx
    X, Y = lattice(nx, ny, 0.0, 0.0, h)
    ly = h * ny

    def field(base):
        f = np.full_like(X, base)
        for _ in range(modes):
            kx, ky = rng.integers(1, 3, size=2)
            ph = rng.uniform(0, 2 * math.pi)
            f = f + amp * rng.uniform(-1, 1) * np.sin(2 * math.pi * (kx * X / lx + ky * Y / ly) + ph)
        return f

    S = conservative(field(1.0), field(0.3), field(-0.2), field(1.0))
    P, D = state_from_samples(S, h)
    return Problem2D("random_smooth2d", nx, ny, 0.0, lx, 0.0, ly, P, D, {"gamma": GAMMA, "mu": 0.0})


def random_rough2d(nx, ny, seed=0, lx=1.0):
    """Seeded noisy data (independent random nodal values and derivatives)
    that drive every GENO branch; for parity tests only."""
    rng = np.random.default_rng(seed)
    P = np.empty((12, ny, nx))
    D = np.empty((12, ny, nx))
    for A in (P, D):
        rho = rng.uniform(0.5, 1.5, size=(ny, nx))
        U = rng.uniform(-0.5, 0.5, size=(ny, nx))
        V = rng.uniform(-0.5, 0.5, size=(ny, nx))
        p = rng.uniform(0.5, 1.5, size=(ny, nx))
        A[0:4] = conservative(rho, U, V, p)
        A[4:12] = rng.normal(0.0, 0.5, size=(8, ny, nx))
    return Problem2D("random_rough2d", nx, ny, 0.0, lx, 0.0, lx * ny / nx, P, D, {"gamma": GAMMA, "mu": 0.0})


# ------------------------------------------------------ bounded 2D axes
def sample_bounded(fn, nx, ny, h, bx, by, x0=0.0, y0=0.0, jumps=False):
    """(P, D) from an analytic conservative field fn(X, Y) -> (4, ...) when
    axes may be bounded (bx, by = 1).  Along a bounded axis the dual grid has
    a node on each boundary line, so the dual state is (12, ny + by, nx + bx)
    with dual node i at lattice 2i (else 2i + 2).  Derivatives are Gauss
    differences of fn across each node's bounding interfaces (zero with
    jumps=True)."""
    def grid(I, J):
        X = x0 + I * h / 2
        Y = y0 + J * h / 2
        X, Y = np.broadcast_arrays(X, Y)
        G = np.zeros((12,) + X.shape)
        G[0:4] = fn(X, Y)
        if not jumps:
            G[4:8] = (fn(X + h / 2, Y) - fn(X - h / 2, Y)) / h
            G[8:12] = (fn(X, Y + h / 2) - fn(X, Y - h / 2)) / h
        return np.ascontiguousarray(G)

    P = grid(2 * np.arange(nx)[None, :] + 1, 2 * np.arange(ny)[:, None] + 1)
    D = grid(2 * np.arange(nx + bx)[None, :] + (0 if bx else 2), 2 * np.arange(ny + by)[:, None] + (0 if by else 2))
    return P, D


def mirror_flow(lx, ly, bx, by, gamma=GAMMA):
    """Smooth field for walls: along a bounded axis rho, p and the tangential
    momentum are even and the normal momentum odd about both boundary lines
    (half-period cosines and sines); along a periodic axis it is periodic."""
    kx = math.pi / lx if bx else 2 * math.pi / lx
    ky = math.pi / ly if by else 2 * math.pi / ly

    def fn(X, Y):
        cx, cy, sx, sy = np.cos(kx * X), np.cos(ky * Y), np.sin(kx * X), np.sin(ky * Y)
        rho = 1.0 + 0.2 * cx * cy + 0.1 * np.cos(2 * kx * X)
        U = 0.3 * sx * (1.0 + 0.2 * cy)
        V = 0.3 * sy * (1.0 + 0.2 * cx)
        p = 1.0 + 0.15 * cx * cy
        return conservative(rho, U, V, p, gamma)
    return fn


def quadrants(states, xs=0.5, ys=0.5, gamma=GAMMA):
    """Piecewise-constant four-quadrant field (states: (rho, U, V, p) of the
    quadrants x < xs / x >= xs, then y < ys / y >= ys); use with jumps=True."""
    def fn(X, Y):
        quad = (X >= xs).astype(int) + 2 * (Y >= ys).astype(int)
        return conservative(*(np.choose(quad, [s[k] for s in states]) for k in range(4)), gamma=gamma)
    return fn


def riemann2d_bounded(n, seed=0, gamma=GAMMA):
    """Four-quadrant Riemann data on [0,1]^2 with every side bounded (states
    as in riemann2d); dual nodes on the boundary lines."""
    rng = np.random.default_rng(seed)
    q = [(rng.uniform(0.1, 1), rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0.1, 1)) for _ in range(4)]
    P, D = sample_bounded(quadrants(q, gamma=gamma), n, n, 1.0 / n, 1, 1, jumps=True)
    return Problem2D("riemann2d_bounded", n, n, 0.0, 1.0, 0.0, 1.0, P, D,
                     {"gamma": gamma, "mu": 0.0, "states": q, "bc": "zero_gradient"})


def viscous_shock_tube(nx, gamma=GAMMA, mu=0.005, prandtl=0.72):
    """Viscous shock tube (Sec. 5, Daru-Tenaud): the lower half [0,1] x [0,0.5]
    of a unit cavity, (rho, U, V, p) = (120, 0, 0, 120/gamma) for x < 0.5 and
    (1.2, 0, 0, 1.2/gamma) beyond, jump on an interface (nx even); adiabatic
    no-slip walls left, right and bottom, a symmetry plane on top; Re = 200
    (mu = 0.005), Pr = 0.72.  ny = nx / 2."""
    ny = nx // 2
    h = 1.0 / nx
    fn = quadrants([(120.0, 0.0, 0.0, 120.0 / gamma), (1.2, 0.0, 0.0, 1.2 / gamma)] * 2, xs=0.5, ys=10.0, gamma=gamma)
    P, D = sample_bounded(fn, nx, ny, h, 1, 1, jumps=True)
    return Problem2D("viscous_shock_tube", nx, ny, 0.0, 1.0, 0.0, 0.5, P, D,
                     {"gamma": gamma, "mu": mu, "prandtl": prandtl,
                      "sides": ("no_slip", "no_slip", "no_slip", "reflecting")})


def batch_sizes(count=64, lo=64, hi=512, seed=0):
    rng = np.random.default_rng(seed)
    return [int(v) for v in rng.integers(lo, hi + 1, size=count)]


def batch_problems(count=64, lo=64, hi=512, seed=0, bounded=False):
    """Batched workload: even members isentropic vortices, odd members
    four-quadrant Riemann problems (periodic, or with zero-gradient sides and
    the dual grid's boundary nodes when bounded), sides seeded in [lo, hi]."""
    out = []
    for b, n in enumerate(batch_sizes(count, lo, hi, seed)):
        if b % 2 == 0:
            out.append(vortex(n, seed=seed * 1000 + b))
        else:
            out.append((riemann2d_bounded if bounded else riemann2d)(n, seed=seed * 1000 + b))
    return out


# --------------------------------------------------------------------- 1D
@dataclass
class Problem1D:
    name: str
    N: int
    x0: float
    lx: float
    S: np.ndarray           # (lines, 6, N)
    bc: str = "periodic"
    params: dict = field(default_factory=dict)

    @property
    def h(self):
        return self.lx / self.N


def line_from_samples(S, h, shifted=False):
    """S: (3, 2N) samples at x0 + I h/2 (periodic) -> (6, N) state of the
    primary line (nodes at odd I) or of the shifted copy (even I)."""
    N = S.shape[1] // 2
    j = np.arange(N)
    c = 2 * j + (2 if shifted else 1)
    out = np.empty((6, N))
    out[0:3] = S[:, c % (2 * N)]
    out[3:6] = (S[:, (c + 1) % (2 * N)] - S[:, (c - 1) % (2 * N)]) / h
    return out


def advection1d(N, seed=0, noise=1e-3, lx=2.0, dual=True):
    """rho = 1 + 0.2 sin(pi x) (+ seeded N(0,1) noise of size `noise` on node
    values only), U = p = 1, periodic [0, 2]; derivatives from the smooth part."""
    rng = np.random.default_rng(seed)
    h = lx / N
    x = np.arange(2 * N) * h / 2
    S = conservative1d(1.0 + 0.2 * np.sin(np.pi * x), 1.0, 1.0)
    lines = [line_from_samples(S, h, False)]
    if dual:
        lines.append(line_from_samples(S, h, True))
    for L in lines:
        if noise:
            d = noise * rng.standard_normal(N)
            L[0] += d
            L[1] += d      # U = 1 kept: rho U moves with rho
            L[2] += 0.5 * d  # p kept: rho E = p/(g-1) + rho/2
    return Problem1D("advection1d", N, 0.0, lx, np.ascontiguousarray(np.stack(lines)), "periodic",
                     {"gamma": GAMMA, "mu": 0.0})


def advection1d_exact(N, t, lx=2.0, shifted=False):
    h = lx / N
    x = np.arange(2 * N) * h / 2
    S = conservative1d(1.0 + 0.2 * np.sin(np.pi * (x - t)), 1.0, 1.0)
    return line_from_samples(S, h, shifted)


def shock_tube(N, left, right, x_jump=0.5, lx=1.0, gamma=GAMMA):
    """Piecewise-constant (rho, u, p) data, jump at an interface, zero
    derivatives, zero-gradient ends.  Nodes at (j + 1/2) h."""
    h = lx / N
    x = (np.arange(N) + 0.5) * h
    L = conservative1d(*left, gamma=gamma)
    R = conservative1d(*right, gamma=gamma)
    W = np.where(x[None, :] < x_jump, L[:, None], R[:, None])
    S = np.zeros((1, 6, N))
    S[0, 0:3] = W
    return Problem1D("shock_tube", N, 0.0, lx, S, "zero_gradient",
                     {"gamma": gamma, "mu": 0.0, "left": left, "right": right, "x_jump": x_jump})


def seeded_shock_tube(N=400, seed=0):
    rng = np.random.default_rng(seed)
    left = (rng.uniform(0.1, 1), rng.uniform(-1, 1), rng.uniform(0.1, 1))
    right = (rng.uniform(0.1, 1), rng.uniform(-1, 1), rng.uniform(0.1, 1))
    return shock_tube(N, left, right)


def blast_wave(N=400, gamma=GAMMA):
    """Woodward-Colella blast waves on [0, 1] (Sec. 5 blast test): p = 1000,
    0.01, 100 on [0, 0.1), [0.1, 0.9), [0.9, 1], rho = 1, u = 0, reflecting
    ends, t = 0.038.  Jumps fall on interfaces for N a multiple of 10."""
    h = 1.0 / N
    x = (np.arange(N) + 0.5) * h
    p = np.where(x < 0.1, 1000.0, np.where(x < 0.9, 0.01, 100.0))
    S = np.zeros((1, 6, N))
    S[0, 0:3] = conservative1d(1.0, 0.0, p, gamma)
    return Problem1D("blast_wave", N, 0.0, 1.0, S, "reflecting", {"gamma": gamma, "mu": 0.0, "t_end": 0.038})


def sod(N=100):
    return shock_tube(N, (1.0, 0.0, 1.0), (0.125, 0.0, 0.1))


def lax(N=100):
    return shock_tube(N, (0.445, 0.698, 3.528), (0.5, 0.0, 0.571))


# --------------------------------------------------------------------- 3D
# grid g is even along axis a where EVEN3[g][a]
EVEN3 = ((0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1))


def conservative3d(rho, U, V, Wv, p, gamma=GAMMA):
    rho, U, V, Wv, p = np.broadcast_arrays(*(np.asarray(a, dtype=np.float64) for a in (rho, U, V, Wv, p)))
    return np.stack([rho, rho * U, rho * V, rho * Wv, p / (gamma - 1.0) + 0.5 * rho * (U * U + V * V + Wv * Wv)])


def lattice3(nx, ny, nz, h, x0=0.0, y0=0.0, z0=0.0):
    """(X, Y, Z), each (2nz, 2ny, 2nx): coordinates of the half-spacing lattice."""
    X = x0 + np.arange(2 * nx)[None, None, :] * h / 2
    Y = y0 + np.arange(2 * ny)[None, :, None] * h / 2
    Z = z0 + np.arange(2 * nz)[:, None, None] * h / 2
    return np.broadcast_arrays(X, Y, Z)


def state3d_from_samples(S, h):
    """S: (5, 2nz, 2ny, 2nx) conservative samples on the half lattice ->
    (4, 20, nz, ny, nx): nodal values and the averaged derivatives (difference
    of the samples at the two bounding interfaces over h) of the four grids."""
    _, LL, JJ, II = S.shape
    n = (II // 2, JJ // 2, LL // 2)
    out = np.empty((4, 20, n[2], n[1], n[0]))
    for g in range(4):
        c = [2 * np.arange(n[a]) + (2 if EVEN3[g][a] else 1) for a in range(3)]
        I, J, L = c[0][None, None, :], c[1][None, :, None], c[2][:, None, None]

        def at(di, dj, dl):
            return S[:, (L + dl) % LL, (J + dj) % JJ, (I + di) % II]

        out[g, 0:5] = at(0, 0, 0)
        out[g, 5:10] = (at(1, 0, 0) - at(-1, 0, 0)) / h
        out[g, 10:15] = (at(0, 1, 0) - at(0, -1, 0)) / h
        out[g, 15:20] = (at(0, 0, 1) - at(0, 0, -1)) / h
    return np.ascontiguousarray(out)


@dataclass
class Problem3D:
    name: str
    nx: int
    ny: int
    nz: int
    lx: float
    S: np.ndarray
    params: dict = field(default_factory=dict)

    @property
    def h(self):
        return self.lx / self.nx

    @property
    def ly(self):
        return self.h * self.ny

    @property
    def lz(self):
        return self.h * self.nz


def advection3d(n, lx=2.0):
    """rho = 1 + 0.2 sin(pi (x+y+z)), U = V = W = p = 1 on [0, 2]^3: the
    accuracy test of Sec. 5.1 carried to 3D."""
    h = lx / n
    X, Y, Z = lattice3(n, n, n, h)
    S = conservative3d(1.0 + 0.2 * np.sin(np.pi * (X + Y + Z)), 1.0, 1.0, 1.0, 1.0)
    return Problem3D("advection3d", n, n, n, lx, state3d_from_samples(S, h), {"gamma": GAMMA, "mu": 0.0})


def advection3d_exact(n, t, lx=2.0):
    h = lx / n
    X, Y, Z = lattice3(n, n, n, h)
    S = conservative3d(1.0 + 0.2 * np.sin(np.pi * (X + Y + Z - 3 * t)), 1.0, 1.0, 1.0, 1.0)
    return state3d_from_samples(S, h)


def random_smooth3d(nx, ny, nz, seed=0, amp=0.1, modes=3, lx=1.0):
    """A seeded smooth periodic 3D flow (sums of low Fourier modes)."""
    rng = np.random.default_rng(seed)
    h = lx / nx
    X, Y, Z = lattice3(nx, ny, nz, h)
    ly, lz = h * ny, h * nz

    def fld(base):
        f = np.full_like(X, base)
        for _ in range(modes):
            kx, ky, kz = rng.integers(1, 3, size=3)
            ph = rng.uniform(0, 2 * math.pi)
            f = f + amp * rng.uniform(-1, 1) * np.sin(2 * math.pi * (kx * X / lx + ky * Y / ly + kz * Z / lz) + ph)
        return f

    S = conservative3d(fld(1.0), fld(0.3), fld(-0.2), fld(0.1), fld(1.0))
    return Problem3D("random_smooth3d", nx, ny, nz, lx, state3d_from_samples(S, h), {"gamma": GAMMA, "mu": 0.0})


def random_rough3d(nx, ny, nz, seed=0, lx=1.0):
    """Seeded noisy 3D data (independent random nodal values and derivatives)
    that drive every GENO branch; for parity tests only."""
    rng = np.random.default_rng(seed)
    S = np.empty((4, 20, nz, ny, nx))
    for g in range(4):
        shp = (nz, ny, nx)
        S[g, 0:5] = conservative3d(rng.uniform(0.5, 1.5, shp), rng.uniform(-0.5, 0.5, shp),
                                   rng.uniform(-0.5, 0.5, shp), rng.uniform(-0.5, 0.5, shp),
                                   rng.uniform(0.5, 1.5, shp))
        S[g, 5:20] = rng.normal(0.0, 0.5, size=(15,) + shp)
    return Problem3D("random_rough3d", nx, ny, nz, lx, S, {"gamma": GAMMA, "mu": 0.0})


def taylor_green3d(n, Ma=0.1, gamma=GAMMA, mu=None, Re=1600.0):
    """Taylor-Green vortex on the periodic [0, 2 pi]^3: U = sin x cos y cos z,
    V = -cos x sin y cos z, W = 0, rho = 1, p = 1/(gamma Ma^2) +
    (cos 2x + cos 2y)(cos 2z + 2)/16 (unit velocity and length scales);
    mu = 1/Re unless given."""
    lx = 2 * math.pi
    h = lx / n
    X, Y, Z = lattice3(n, n, n, h)
    U = np.sin(X) * np.cos(Y) * np.cos(Z)
    V = -np.cos(X) * np.sin(Y) * np.cos(Z)
    p = 1.0 / (gamma * Ma * Ma) + (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0) / 16.0
    S = conservative3d(1.0, U, V, 0.0, p, gamma)
    return Problem3D("taylor_green3d", n, n, n, lx, state3d_from_samples(S, h),
                     {"gamma": gamma, "mu": (1.0 / Re) if mu is None else mu, "Ma": Ma})
