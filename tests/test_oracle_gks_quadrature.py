"""Pin of the oracle's gas-kinetic interface solver at discontinuous data, by
brute force in time and velocity space.  CPU only.

The oracle builds the interface distribution from moment recursions, the
polynomial algebra of its terms and closed-form time integrals.  Here the same
solution is evaluated point by point instead:

* the distribution at the interface is the integral solution of the BGK
  equation (App. A1, Eq. integral_f), evaluated along the particle
  trajectories with a numerical integral over the emission time t', from
  - the equilibrium g(x, y, t) = g0 (1 + (a0.psi) x + (b0.psi) y + (A0.psi) t),
  - the initial distribution f0 = g_s (1 + (a_s.psi) x + (b_s.psi) y
    - tau ((a_s.psi) u + (b_s.psi) v + A_s.psi)) on the side s of the
    interface that the trajectory starts from (left for u > 0, right for u < 0);
* g_l, g_r, g0 are Maxwellians tabulated on Gauss-Legendre grids in (u, v)
  and in |xi| (K internal degrees of freedom, radial measure r^(K-1)),
  normalised numerically; in 3D the tangential directions v and w take
  Gauss-Hermite nodes about the Maxwellian's own V and W instead, which
  integrate its polynomial-times-Gaussian integrands exactly (at most degree 9
  per direction here, 12 nodes);
* the compatibility state W0 is the psi-moment of the left half-space
  Maxwellian plus that of the right one; micro slopes solve the moment systems
  <psi (s.psi) g> = D with matrices integrated on the grid (numpy solve);
  time slopes come from the compatibility condition <psi ((a.psi) u +
  (b.psi) v + A.psi) g> = 0;
* the time integrals over [0, T] of the psi-, u psi- and heat-flux moments
  are taken by Gauss-Legendre in t, and f^n, f_t^n follow from the T = dt/2
  and T = dt values (App. A1), F-hat, W^e from their moments (App. A2);
* the interface values of Eq. W-model use tau_0 = tau, W^{l,r} the
  reconstructed states and W^{l,r}_t = -<psi ((a.psi) u + (b.psi) v) g>.

The readings are the oracle's (collision time, the averaged normal slope of
g0, the one-sided time derivatives, the Prandtl fix); what this pins is the
arithmetic that turns them into F, F_t, W^e, W^e_t, W0 and W-hat at a jump:
the half-space weights, the sign of every term, the time coefficients and
their combination, the xi moments and the slope systems.
"""
import numpy as np
import pytest

from tests.helpers import settings

G = 1.4


def _kdof(dim):
    # K + dim = 2 / (gamma - 1)
    return 2 / (G - 1) - dim


def _gl(a, b, n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


class _Maxwellian:
    """A Maxwellian rho (lam/pi)^((K+D)/2) exp(-lam (|u - U|^2 + xi^2))
    tabulated on a grid covering its mass; half = +1 keeps u > 0, -1 keeps
    u < 0, 0 the whole line.  Arrays broadcast as (u, v, w, r) in 3D,
    (u, v, r) in 2D and (u, r) in 1D; `w` holds quadrature weight times the
    Maxwellian."""

    def __init__(self, W, dim, half=0, n=96):
        self.dim = dim
        rho = W[0]
        U = W[1] / rho
        V = W[2] / rho if dim >= 2 else 0.0
        Wv = W[3] / rho if dim == 3 else 0.0
        p = (G - 1) * (W[-1] - 0.5 * rho * (U * U + V * V + Wv * Wv))
        lam = rho / (2 * p)
        self.rho, self.U, self.V, self.Wv, self.p, self.lam = rho, U, V, Wv, p, lam
        K = _kdof(dim)
        span = 13.0 / np.sqrt(lam)
        lo, hi = U - span, U + span
        if half > 0:
            lo = max(lo, 0.0)
        if half < 0:
            hi = min(hi, 0.0)
        # the full-space normalisation comes from the full line in u
        uf, wuf = _gl(U - span, U + span, n)
        u, wu = (uf, wuf) if half == 0 else _gl(lo, hi, n) if hi > lo else (np.zeros(1), np.zeros(1))
        v, wv = _gl(V - span, V + span, n) if dim == 2 else (np.zeros(1), np.ones(1))
        r, wr = _gl(0.0, span, 40)
        wr = wr * r ** (K - 1)
        gu = np.exp(-lam * (u - U) ** 2) * wu
        guf = np.exp(-lam * (uf - U) ** 2) * wuf
        gv = np.exp(-lam * (v - V) ** 2) * wv if dim == 2 else wv
        gr = np.exp(-lam * r * r) * wr
        norm = guf.sum() * gv.sum() * gr.sum()
        if dim == 3:
            # Gauss-Hermite in v and w: nodes V + x / sqrt(lam), W + x / sqrt(lam)
            # carry the Gaussian itself (gv above is then the plain weight 1)
            x, wx = np.polynomial.hermite.hermgauss(12)
            v, gv = V + x / np.sqrt(lam), wx / wx.sum()
            w = Wv + x / np.sqrt(lam)
            gw = wx / wx.sum()
            self.u, self.v = u[:, None, None, None], v[None, :, None, None]
            self.wv, self.x2 = w[None, None, :, None], (r * r)[None, None, None, :]
            self.w = (rho * gu[:, None, None, None] * gv[None, :, None, None] * gw[None, None, :, None]
                      * gr[None, None, None, :] / norm)
        elif dim == 2:
            self.u, self.v, self.x2 = u[:, None, None], v[None, :, None], (r * r)[None, None, :]
            self.w = rho * gu[:, None, None] * gv[None, :, None] * gr[None, None, :] / norm
        else:
            self.u, self.v, self.x2 = u[:, None], np.zeros(1)[:, None], (r * r)[None, :]
            self.w = rho * gu[:, None] * gr[None, :] / norm
        self.ps = self.psi()
        self.ups = [self.u * ps for ps in self.ps]

    def psi(self):
        if self.dim == 3:
            return [np.ones_like(self.u), self.u, self.v, self.wv,
                    0.5 * (self.u ** 2 + self.v ** 2 + self.wv ** 2 + self.x2)]
        if self.dim == 2:
            return [np.ones_like(self.u), self.u, self.v, 0.5 * (self.u ** 2 + self.v ** 2 + self.x2)]
        return [np.ones_like(self.u), self.u, 0.5 * (self.u ** 2 + self.x2)]

    def lin(self, s):
        """s . psi on the grid"""
        return sum(si * pi for si, pi in zip(s, self.psi()))

    def moments(self, f):
        """<psi f> for a function f tabulated on the grid (times the Maxwellian)"""
        wf = self.w * f
        return np.array([np.sum(wf * ps) for ps in self.ps])

    def slope(self, D):
        """micro slope s with <psi (s.psi) g> = D"""
        ps = self.psi()
        M = np.array([[np.sum(self.w * a * b) for b in ps] for a in ps])
        return np.linalg.solve(M, D)


def _brute_interface(WL, WR, WnL, WnR, Wt, dt, dim, mu=0.0, prandtl=1.0, c1=0.0, c2=1.0, nt=16, mistake=None,
                     Wt2=None):
    """`mistake` plants one plausible error (for the sharpness test only).
    Wt, Wt2: tangential slopes along v and (3D) w."""
    n = dim + 2
    hl, hr = _Maxwellian(WL, dim, +1), _Maxwellian(WR, dim, -1 if mistake != "half_space" else +1)
    fl, fr = _Maxwellian(WL, dim, 0), _Maxwellian(WR, dim, 0)
    W0 = hl.moments(1.0) + hr.moments(1.0)
    g0 = _Maxwellian(W0, dim, 0)
    Wt = np.zeros(n) if Wt is None else np.asarray(Wt, float)
    Wt2 = np.zeros(n) if Wt2 is None else np.asarray(Wt2, float)

    def transport(m, a, b, c):
        tr = m.lin(a) * m.u + m.lin(b) * m.v
        return tr + m.lin(c) * m.wv if dim == 3 else tr

    def slopes(full, Dn):
        a = full.slope(Dn)
        b = full.slope(Wt) if dim >= 2 else np.zeros(n)
        c = full.slope(Wt2) if dim == 3 else np.zeros(n)
        # one-sided Euler time derivative and the time slope from compatibility
        Wtime = -full.moments(transport(full, a, b, c))
        A = full.slope(Wtime)
        return a, b, c, A, Wtime

    aL, bL, cL, AL, WtL = slopes(fl, np.asarray(WnL, float))
    aR, bR, cR, AR, WtR = slopes(fr, np.asarray(WnR, float))
    a0, b0, c0, A0, _ = slopes(g0, 0.5 * (np.asarray(WnL, float) + np.asarray(WnR, float)))
    tau = (mu / g0.p if mu > 0 else c1 * dt) + c2 * dt * abs(hl.p - hr.p) / (hl.p + hr.p)
    assert tau > 0

    for m in (g0, hl, hr):  # 1/2 (u - U0)((u - U0)^2 + (v - V0)^2 + (w - W0)^2 + xi^2)
        du, dv = m.u - g0.U, m.v - g0.V
        c2 = du * du + (dv * dv if dim >= 2 else 0.0) + m.x2
        if dim == 3:
            c2 = c2 + (m.wv - g0.Wv) ** 2
        m.heat = 0.5 * du * c2

    # distribution at the interface at time t, per Maxwellian it multiplies
    def f_at(t):
        tp, wp = _gl(0.0, t, nt)
        e = np.exp(-(t - tp) / tau) * wp / tau
        ca, cb, cc = e.sum(), (e * (t - tp)).sum(), (e * tp).sum()
        # (1/tau) int g(-u (t-t'), -v (t-t'), t') e^{-(t-t')/tau} dt'
        feq = ca - cb * transport(g0, a0, b0, c0) + cc * g0.lin(A0) * (mistake != "no_A0")
        out = [(g0, feq)]
        for h, a, b, c, A in ((hl, aL, bL, cL, AL), (hr, aR, bR, cR, AR)):
            tr = transport(h, a, b, c)
            # e^{-t/tau} f0(-u t, -v t) on the half space the trajectory starts from
            tA = 0.0 if mistake == "no_tauA" else tau * h.lin(A)
            out.append((h, np.exp(-t / tau) * (1.0 - t * tr - tau * tr - tA)))
        return out

    def integrated(T):
        ts, ws = _gl(0.0, T, nt)
        Wb, Fb, qb = np.zeros(n), np.zeros(n), 0.0
        for t, w in zip(ts, ws):
            for m, f in f_at(t):
                wf = m.w * f
                Wb += w * np.array([np.sum(wf * ps) for ps in m.ps])
                Fb += w * np.array([np.sum(wf * ups) for ups in m.ups])
                qb += w * np.sum(wf * m.heat)
        return Wb, Fb, qb

    Wh, Fh, qh = integrated(0.5 * dt)
    Wf, Ff, qf = integrated(dt)
    fit = lambda h, f: ((4 * h - f) / dt, 4 * (f - 2 * h) / dt ** 2)  # noqa: E731
    F, Ftime = fit(Fh, Ff)
    We, Wet = fit(Wh, Wf)
    if mu > 0:
        q, qt = fit(qh, qf)
        F[-1] += (1 / prandtl - 1) * q
        Ftime[-1] += (1 / prandtl - 1) * qt
    E = np.exp(-dt / tau)
    if mistake == "wmodel_weights":
        E = 1 - E
    WL, WR = np.asarray(WL, float), np.asarray(WR, float)
    return {"F": F, "Ft": Ftime, "We": We, "Wet": Wet, "W0": W0, "tau": tau,
            "Wl": (1 - E) * We + E * WL, "Wr": (1 - E) * We + E * WR,
            "Wlt": (1 - E) * Wet + E * WtL, "Wrt": (1 - E) * Wet + E * WtR}


def _state(rng, dim):
    rho, p = 0.5 + rng.random(), 0.5 + rng.random()
    U = rng.uniform(-0.8, 0.8)
    if dim == 1:
        return np.array([rho, rho * U, p / (G - 1) + 0.5 * rho * U * U])
    V = rng.uniform(-0.8, 0.8)
    if dim == 3:
        Wv = rng.uniform(-0.8, 0.8)
        return np.array([rho, rho * U, rho * V, rho * Wv, p / (G - 1) + 0.5 * rho * (U * U + V * V + Wv * Wv)])
    return np.array([rho, rho * U, rho * V, p / (G - 1) + 0.5 * rho * (U * U + V * V)])


def _compare(r, b, keys, tol):
    for k in keys:
        scale = max(np.abs(b[k]).max(), 1e-300)
        err = np.abs(np.asarray(r[k]) - b[k]).max() / scale
        assert err <= tol, (k, err, r[k], b[k])


CASES = [
    # dim, mu, c1, dt, seed
    (2, 0.0, 0.0, 0.02, 1),
    (2, 0.0, 0.0, 0.05, 2),
    (2, 0.0, 0.05, 0.01, 3),
    (2, 2e-3, 0.0, 0.02, 4),
    (1, 0.0, 0.0, 0.02, 5),
    (1, 2e-3, 0.0, 0.01, 6),
    (3, 0.0, 0.0, 0.02, 7),
    (3, 0.0, 0.05, 0.01, 8),
    (3, 2e-3, 0.0, 0.02, 9),
]


@pytest.mark.parametrize("dim,mu,c1,dt,seed", CASES)
def test_interface_solver_at_a_jump_by_quadrature(oracle, dim, mu, c1, dt, seed):
    """Random left and right states (every component jumps), random normal
    slopes on each side and a random tangential slope, tau > 0: the oracle's
    F, F_t, W^e, W^e_t, W0, tau and W-hat^{l,r} (values and time
    derivatives) equal the brute-force evaluation of the integral solution."""
    rng = np.random.default_rng(seed)
    n = dim + 2
    WL, WR = _state(rng, dim), _state(rng, dim)
    WnL, WnR = rng.normal(size=n), rng.normal(size=n)
    Wt = rng.normal(size=n) if dim >= 2 else None
    Wt2 = rng.normal(size=n) if dim == 3 else None
    pr = 0.72 if mu > 0 else 1.0
    par = oracle.make_par(**settings(dim=dim, nx=8, ny=8, nz=8, lx=1.0, mu=mu, prandtl=pr, tau_c1=c1))
    r = oracle.gks_interface(par, dim, WL, WR, WnL, WnR, Wt, dt, Wt2=Wt2)
    b = _brute_interface(WL, WR, WnL, WnR, Wt, dt, dim, mu=mu, prandtl=pr, c1=c1, Wt2=Wt2)
    assert r["tau"] == pytest.approx(b["tau"], rel=1e-12)
    # measured: <= 1.3e-14 on values, <= 1e-13 on time derivatives (the
    # differences of the two time integrals divided by dt^2 amplify quadrature
    # round-off by ~1/dt)
    _compare(r, b, ["W0", "F", "We", "Wl", "Wr"], 1e-13)
    _compare(r, b, ["Ft", "Wet", "Wlt", "Wrt"], 1e-12)


@pytest.mark.parametrize("mistake,keys", [
    ("half_space", ["W0", "F"]),          # right state integrated over u > 0
    ("no_A0", ["Ft", "Wet"]),             # equilibrium time slope dropped
    ("no_tauA", ["F", "We"]),             # tau A term of the initial distribution dropped
    ("wmodel_weights", ["Wl", "Wrt"]),    # Eq. W-model weights exchanged
])
def test_quadrature_pin_is_sharp(oracle, mistake, keys):
    """Each plausible mistake, planted in the brute-force evaluation, moves the
    compared outputs by far more than the tolerances above (so the same
    mistake in the oracle could not pass)."""
    rng = np.random.default_rng(1)
    WL, WR = _state(rng, 2), _state(rng, 2)
    WnL, WnR, Wt = rng.normal(size=4), rng.normal(size=4), rng.normal(size=4)
    dt = 0.02
    par = oracle.make_par(**settings(dim=2, nx=8, ny=8, lx=1.0))
    r = oracle.gks_interface(par, 2, WL, WR, WnL, WnR, Wt, dt)
    b = _brute_interface(WL, WR, WnL, WnR, Wt, dt, 2, mistake=mistake)
    for k in keys:
        err = np.abs(r[k] - b[k]).max() / np.abs(r[k]).max()
        assert err > 1e-6, (mistake, k, err)
