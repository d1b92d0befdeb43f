// Device arithmetic of the 3D gas-kinetic solvers for gfx950: the BGK
// interface solver and the smooth nodal solver of App. A with the collision
// invariants psi = (1, u, v, w, (u^2 + v^2 + w^2 + xi^2)/2), in FP64.
//
// The structure is that of the 2D solver (gks_device.hpp): Maxwellian moments
// from the recursion <c^(n+2)> = U <c^(n+1)> + (n+1)/(2 lambda) <c^n> per
// velocity direction, the closed-form solution of the 5x5 moment system for
// the micro slopes, and the moments of the interface distribution assembled
// term by term.  Everything is inlined so the moment indices are
// compile-time constants.
#pragma once

#include "gks_device.hpp"

namespace fdk3 {

using fdk::Consts;
using fdk::TimeCoef;
using fdk::m_abs;
using fdk::m_erfc;
using fdk::m_exp;
using fdk::m_sqrt;
using fdk::mu_rec;

// Per unit density: mu[n] = <u^n> (full or half line), mv[n] = <v^n>,
// mw[n] = <w^n> (full lines), x2 = <xi^2>, x4 = <xi^4>.
struct Mom3 {
  double mu[7], mv[7], mw[7];
  double x2, x4;
};

// <u^P v^Q w^S xi^(2R) psi>, R in {0, 1}
template <int P, int Q, int S, int R> FDK_HD void muvw(const Mom3& m, double o[5]) {
  const double xr = R == 0 ? 1.0 : m.x2;
  const double xr1 = R == 0 ? m.x2 : m.x4;
  const double vw = m.mv[Q] * m.mw[S];
  const double b = m.mu[P] * vw;
  o[0] = b * xr;
  o[1] = m.mu[P + 1] * vw * xr;
  o[2] = m.mu[P] * m.mv[Q + 1] * m.mw[S] * xr;
  o[3] = m.mu[P] * m.mv[Q] * m.mw[S + 1] * xr;
  o[4] = 0.5 * ((m.mu[P + 2] * vw + m.mu[P] * m.mv[Q + 2] * m.mw[S] + m.mu[P] * m.mv[Q] * m.mw[S + 2]) * xr + b * xr1);
}
// <(s.psi) u^P v^Q w^S psi>.  With g = s.psi = s0 + s1 u + s2 v + s3 w +
// h4 (u^2 + v^2 + w^2 + xi^2), h4 = s4 / 2, a moment of g splits into
// one-dimensional parts:
//   <g u^a v^b w^c> = mv[b] mw[c] cu(a) + mu[a] mw[c] cv(b) + mu[a] mv[b] cw(c),
//   cu(a) = (s0 + h4 x2) mu[a] + s1 mu[a+1] + h4 mu[a+2],
//   cv(b) = s2 mv[b+1] + h4 mv[b+2],  cw(c) = s3 mw[c+1] + h4 mw[c+2],
// and <g u^a v^b w^c xi^2> = x2 <g u^a v^b w^c> + h4 mu[a] mv[b] mw[c] (x4 - x2^2).
template <int P, int Q, int S> FDK_HD void ma(const double s[5], const Mom3& m, double o[5]) {
  const double h4 = 0.5 * s[4];
  const double c0 = s[0] + h4 * m.x2;
  double cu[3], cv[3], cw[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    cu[d] = c0 * m.mu[P + d] + s[1] * m.mu[P + d + 1] + h4 * m.mu[P + d + 2];
    cv[d] = s[2] * m.mv[Q + d + 1] + h4 * m.mv[Q + d + 2];
    cw[d] = s[3] * m.mw[S + d + 1] + h4 * m.mw[S + d + 2];
  }
  // <g u^(P+a) v^(Q+b) w^(S+c)>
  auto G = [&](int a, int b, int c) {
    return m.mv[Q + b] * m.mw[S + c] * cu[a] + m.mu[P + a] * m.mw[S + c] * cv[b] + m.mu[P + a] * m.mv[Q + b] * cw[c];
  };
  o[0] = G(0, 0, 0);
  o[1] = G(1, 0, 0);
  o[2] = G(0, 1, 0);
  o[3] = G(0, 0, 1);
  const double gx = m.x2 * o[0] + h4 * (m.mu[P] * m.mv[Q] * m.mw[S]) * (m.x4 - m.x2 * m.x2);
  o[4] = 0.5 * ((G(2, 0, 0) + G(0, 2, 0)) + (G(0, 0, 2) + gx));
}

struct Prim {
  double rho, irho, U, V, Wv, p, lam, i2l, ip;  // i2l = 1/(2 lambda) = p/rho, ip = 1/p
};
FDK_HD Prim prim(const double* W, double gamma) {
  Prim s;
  s.rho = W[0];
  s.irho = 1.0 / W[0];
  s.U = W[1] * s.irho;
  s.V = W[2] * s.irho;
  s.Wv = W[3] * s.irho;
  s.p = (gamma - 1.0) * (W[4] - 0.5 * s.rho * (s.U * s.U + s.V * s.V + s.Wv * s.Wv));
  s.i2l = s.p * s.irho;
  s.ip = 1.0 / s.p;
  s.lam = 0.5 * s.rho * s.ip;
  return s;
}
// v, w and xi moments (full lines)
FDK_HD void mom_common(const Prim& s, double K, Mom3& m) {
  m.mv[0] = 1.0;
  m.mv[1] = s.V;
  mu_rec(m.mv, s.V, s.i2l);
  m.mw[0] = 1.0;
  m.mw[1] = s.Wv;
  mu_rec(m.mw, s.Wv, s.i2l);
  m.x2 = K * s.i2l;
  m.x4 = m.x2 * (K + 2.0) * s.i2l;
}
FDK_HD void mom_full(const Prim& s, Mom3& m) {
  m.mu[0] = 1.0;
  m.mu[1] = s.U;
  mu_rec(m.mu, s.U, s.i2l);
}
// half line: sgn = +1 (u > 0) or -1 (u < 0)
FDK_HD void mom_half(const Prim& s, double sgn, Mom3& m) {
  const double sl = m_sqrt(s.lam);
  m.mu[0] = 0.5 * m_erfc(-sgn * sl * s.U);
  // 1/(2 sqrt(pi lambda)) = (1/(2 lambda)) sqrt(lambda) / sqrt(pi)
  m.mu[1] = s.U * m.mu[0] + sgn * m_exp(-s.lam * s.U * s.U) * (s.i2l * sl) * 0.56418958354775628695;
  mu_rec(m.mu, s.U, s.i2l);
}

// Micro slope s with <psi (s.psi)> = d (per unit density), closed form of the
// 5x5 moment system: with e = |U|^2 + (K + 3)/(2 lambda),
//   s4 = 4 lambda^2 / (K + 3) (2 d4 - e d0 - 2 U.(d_m - U d0)),
//   s_m = 2 lambda (d_m - U_m d0) - U_m s4 (m = 1, 2, 3),
//   s0 = d0 - U.s_m - e s4 / 2.
// iKd = 1/(K + 3).
FDK_HD void slope(const Prim& q, double K, double iKd, const double* d, double* s) {
  const double e = q.U * q.U + q.V * q.V + q.Wv * q.Wv + (K + 3.0) * q.i2l;
  const double B = 2.0 * d[4] - e * d[0];
  const double A1 = d[1] - q.U * d[0], A2 = d[2] - q.V * d[0], A3 = d[3] - q.Wv * d[0];
  const double tl = 2.0 * q.lam;
  s[4] = tl * tl * iKd * (B - 2.0 * q.U * A1 - 2.0 * q.V * A2 - 2.0 * q.Wv * A3);
  s[3] = tl * A3 - q.Wv * s[4];
  s[2] = tl * A2 - q.V * s[4];
  s[1] = tl * A1 - q.U * s[4];
  s[0] = d[0] - q.U * s[1] - q.V * s[2] - q.Wv * s[3] - 0.5 * s[4] * e;
}

// tr = <psi ((a.psi) u + (b.psi) v + (c.psi) w)>, tru = <u psi (...)>
FDK_HD void transport(const double* a, const double* b, const double* c, const Mom3& m, double* tr, double* tru) {
  double x[5], y[5], z[5];
  ma<1, 0, 0>(a, m, x);
  ma<0, 1, 0>(b, m, y);
  ma<0, 0, 1>(c, m, z);
#pragma unroll
  for (int i = 0; i < 5; ++i) tr[i] = x[i] + y[i] + z[i];
  ma<2, 0, 0>(a, m, x);
  ma<1, 1, 0>(b, m, y);
  ma<1, 0, 1>(c, m, z);
#pragma unroll
  for (int i = 0; i < 5; ++i) tru[i] = x[i] + y[i] + z[i];
}
// <psi> and <u psi> of a (half or full) state
FDK_HD void psi_moms(const Mom3& m, double* p, double* u) {
  p[0] = m.mu[0];
  p[1] = m.mu[1];
  p[2] = m.mu[0] * m.mv[1];
  p[3] = m.mu[0] * m.mw[1];
  p[4] = 0.5 * (m.mu[2] + m.mu[0] * (m.mv[2] + m.mw[2] + m.x2));
  muvw<1, 0, 0, 0>(m, u);
}

// Local frame: the normal velocity is component 1 (u); v and w are the
// tangential velocities, Wt and Wt2 the tangential slopes along their axes.
struct GksIO3 {
  double WL[5], WR[5], nL[5], nR[5], Wt[5], Wt2[5];
  double F[5], Ft[5], Wl[5], Wr[5], Wlt[5], Wrt[5];
};

// Contribution of one side s to the moments of f^n and f_t^n over its half
// line, and its one-sided Euler time derivative Wt (full line).
FDK_HD void side_terms(const Prim& s, const Mom3& h, const double* n, const double* t, const double* t2, double K,
                       double iKd, double tau, const TimeCoef<double>& tc, bool both, double* F, double* Ft,
                       double* We, double* Wet, double* Wt) {
  Mom3 f = h;
  mom_full(s, f);
  double a[5], b[5], c[5], A[5], d[5], tf[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) d[i] = n[i] * s.irho;
  slope(s, K, iKd, d, a);
#pragma unroll
  for (int i = 0; i < 5; ++i) d[i] = t[i] * s.irho;
  slope(s, K, iKd, d, b);
#pragma unroll
  for (int i = 0; i < 5; ++i) d[i] = t2[i] * s.irho;
  slope(s, K, iKd, d, c);
  {
    double x[5], y[5], z[5];
    ma<1, 0, 0>(a, f, x);
    ma<0, 1, 0>(b, f, y);
    ma<0, 0, 1>(c, f, z);
#pragma unroll
    for (int i = 0; i < 5; ++i) tf[i] = x[i] + y[i] + z[i];
  }
#pragma unroll
  for (int i = 0; i < 5; ++i) { d[i] = -tf[i]; Wt[i] = -s.rho * tf[i]; }
  slope(s, K, iKd, d, A);
  double ph[5], uh[5], tp[5], tu[5], Ap[5], Au[5];
  psi_moms(h, ph, uh);
  transport(a, b, c, h, tp, tu);
  ma<0, 0, 0>(A, h, Ap);
  ma<1, 0, 0>(A, h, Au);
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const double nu = uh[i] - tau * Au[i], np = ph[i] - tau * Ap[i];
    Ft[i] += s.rho * (tc.ct[3] * nu + tc.ct[4] * tu[i]);
    Wet[i] += s.rho * (tc.ct[3] * np + tc.ct[4] * tp[i]);
    if (both) {
      F[i] += s.rho * (tc.c[3] * nu + tc.c[4] * tu[i]);
      We[i] += s.rho * (tc.c[3] * np + tc.c[4] * tp[i]);
    }
  }
}

// Interface solver (App. A1-A2): flux, its time derivative and the values of
// Eq. W-model with their time derivatives.  VALUES = false skips F and the
// values (stage 2 uses only time derivatives).
template <bool VALUES> FDK_HD void gks_iface(const Consts& k, double dt, GksIO3& io) {
  const double K = k.K, gam = k.gamma, iKd = k.inv_Kd;
  const bool both = VALUES || k.mu > 0;
  Prim sL = prim(io.WL, gam), sR = prim(io.WR, gam);
  Mom3 hL, hR;
  mom_common(sL, K, hL);
  mom_half(sL, 1.0, hL);
  mom_common(sR, K, hR);
  mom_half(sR, -1.0, hR);
  double W0[5];
  {
    double pL[5], pR[5], u[5];
    psi_moms(hL, pL, u);
    psi_moms(hR, pR, u);
#pragma unroll
    for (int i = 0; i < 5; ++i) W0[i] = sL.rho * pL[i] + sR.rho * pR[i];
  }
  Prim s0 = prim(W0, gam);
  const double tau = (k.mu > 0 ? k.mu * s0.ip : k.tau_c1 * dt) + k.tau_c2 * dt * m_abs(sL.p - sR.p) / (sL.p + sR.p);
  TimeCoef<double> tc = fdk::time_coef(dt, tau);
  double F[5], We[5], Wet[5], WtL[5], WtR[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) { F[i] = 0.0; io.Ft[i] = 0.0; We[i] = 0.0; Wet[i] = 0.0; }
  side_terms(sL, hL, io.nL, io.Wt, io.Wt2, K, iKd, tau, tc, both, F, io.Ft, We, Wet, WtL);
  side_terms(sR, hR, io.nR, io.Wt, io.Wt2, K, iKd, tau, tc, both, F, io.Ft, We, Wet, WtR);
  // equilibrium part: slopes from the averaged normal slope and the two
  // tangential slopes; time slope from compatibility
  {
    Mom3 m0;
    mom_common(s0, K, m0);
    mom_full(s0, m0);
    double a0[5], b0[5], c0[5], A0[5], d[5], t0[5], tu0[5], Ap0[5], Au0[5], p0[5], u0[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) d[i] = 0.5 * (io.nL[i] + io.nR[i]) * s0.irho;
    slope(s0, K, iKd, d, a0);
#pragma unroll
    for (int i = 0; i < 5; ++i) d[i] = io.Wt[i] * s0.irho;
    slope(s0, K, iKd, d, b0);
#pragma unroll
    for (int i = 0; i < 5; ++i) d[i] = io.Wt2[i] * s0.irho;
    slope(s0, K, iKd, d, c0);
    transport(a0, b0, c0, m0, t0, tu0);
#pragma unroll
    for (int i = 0; i < 5; ++i) d[i] = -t0[i];
    slope(s0, K, iKd, d, A0);
    ma<0, 0, 0>(A0, m0, Ap0);
    ma<1, 0, 0>(A0, m0, Au0);
    psi_moms(m0, p0, u0);
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      io.Ft[i] += s0.rho * (tc.ct[0] * u0[i] + tc.ct[1] * tu0[i] + tc.ct[2] * Au0[i]);
      Wet[i] += s0.rho * (tc.ct[0] * p0[i] + tc.ct[1] * t0[i] + tc.ct[2] * Ap0[i]);
      if (both) {
        F[i] += s0.rho * (tc.c[0] * u0[i] + tc.c[1] * tu0[i] + tc.c[2] * Au0[i]);
        We[i] += s0.rho * (tc.c[0] * p0[i] + tc.c[1] * t0[i] + tc.c[2] * Ap0[i]);
      }
    }
  }
  // Prandtl-number correction: (1/Pr - 1) times the heat flux
  // 1/2 <(u-U0)((u-U0)^2 + (v-V0)^2 + (w-W0)^2 + xi^2)>, written with the
  // moments of psi (We) and u psi (F) of the same distribution.
  if (k.mu > 0) {
    const double U = s0.U, V = s0.V, Wv = s0.Wv, f = k.prfix;
    const double q2 = U * U + V * V + Wv * Wv;
    const double a = U * U + 0.5 * q2, b = 0.5 * U * q2;
    const double q = F[4] - U * F[1] - V * F[2] - Wv * F[3] + a * F[0] - U * We[4] + U * V * We[2] +
                     U * Wv * We[3] - b * We[0];
    const double qt = io.Ft[4] - U * io.Ft[1] - V * io.Ft[2] - Wv * io.Ft[3] + a * io.Ft[0] - U * Wet[4] +
                      U * V * Wet[2] + U * Wv * Wet[3] - b * Wet[0];
    F[4] += f * q;
    io.Ft[4] += f * qt;
  }
  const double e = tc.e1, oe = 1.0 - tc.e1;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    io.Wlt[i] = oe * Wet[i] + e * WtL[i];
    io.Wrt[i] = oe * Wet[i] + e * WtR[i];
    if (VALUES) {
      io.F[i] = F[i];
      io.Wl[i] = oe * We[i] + e * io.WL[i];
      io.Wr[i] = oe * We[i] + e * io.WR[i];
    }
  }
}

// Smooth nodal solver: f^n = g [1 - tauN ((a.psi) u + (b.psi) v + (c.psi) w
// + A.psi)], f_t = (A.psi) g.  F[a], Ft[a]: flux along axis a (x, y, z) and
// its time derivative.  VALUES = false: F skipped.
template <bool VALUES>
FDK_HD void gks_node(const Consts& k, const double* W, const double* Wx, const double* Wy, const double* Wz,
                     double F[3][5], double Ft[3][5]) {
  const double K = k.K, iKd = k.inv_Kd;
  const Prim s = prim(W, k.gamma);
  Mom3 m;
  mom_common(s, K, m);
  mom_full(s, m);
  double a[5], b[5], c[5], A[5], d[5], tr[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) d[i] = Wx[i] * s.irho;
  slope(s, K, iKd, d, a);
#pragma unroll
  for (int i = 0; i < 5; ++i) d[i] = Wy[i] * s.irho;
  slope(s, K, iKd, d, b);
#pragma unroll
  for (int i = 0; i < 5; ++i) d[i] = Wz[i] * s.irho;
  slope(s, K, iKd, d, c);
  {
    double x[5], y[5], z[5];
    ma<1, 0, 0>(a, m, x);
    ma<0, 1, 0>(b, m, y);
    ma<0, 0, 1>(c, m, z);
#pragma unroll
    for (int i = 0; i < 5; ++i) tr[i] = x[i] + y[i] + z[i];
  }
#pragma unroll
  for (int i = 0; i < 5; ++i) d[i] = -tr[i];
  slope(s, K, iKd, d, A);
  const double tauN = k.mu > 0 ? k.mu * s.ip : 0.0;
  const bool visc = k.mu > 0;
  double At[3][5];
  ma<1, 0, 0>(A, m, At[0]);
  ma<0, 1, 0>(A, m, At[1]);
  ma<0, 0, 1>(A, m, At[2]);
#pragma unroll
  for (int ax = 0; ax < 3; ++ax)
#pragma unroll
    for (int i = 0; i < 5; ++i) Ft[ax][i] = s.rho * At[ax][i];
  if (VALUES || visc) {
    double f0[3][5];
    muvw<1, 0, 0, 0>(m, f0[0]);
    muvw<0, 1, 0, 0>(m, f0[1]);
    muvw<0, 0, 1, 0>(m, f0[2]);
    if (visc) {
      double x[5], y[5], z[5];
      ma<2, 0, 0>(a, m, x); ma<1, 1, 0>(b, m, y); ma<1, 0, 1>(c, m, z);
#pragma unroll
      for (int i = 0; i < 5; ++i) f0[0][i] -= tauN * (x[i] + y[i] + z[i] + At[0][i]);
      ma<1, 1, 0>(a, m, x); ma<0, 2, 0>(b, m, y); ma<0, 1, 1>(c, m, z);
#pragma unroll
      for (int i = 0; i < 5; ++i) f0[1][i] -= tauN * (x[i] + y[i] + z[i] + At[1][i]);
      ma<1, 0, 1>(a, m, x); ma<0, 1, 1>(b, m, y); ma<0, 0, 2>(c, m, z);
#pragma unroll
      for (int i = 0; i < 5; ++i) f0[2][i] -= tauN * (x[i] + y[i] + z[i] + At[2][i]);
    }
#pragma unroll
    for (int ax = 0; ax < 3; ++ax)
#pragma unroll
      for (int i = 0; i < 5; ++i) F[ax][i] = s.rho * f0[ax][i];
  }
  if (visc) {
    // Prandtl correction with the node's velocity along each axis; the psi
    // moments are W (values) and W_t = -rho tr (time derivatives)
    const double Uv[3] = {s.U, s.V, s.Wv}, f = k.prfix;
    const double q2 = s.U * s.U + s.V * s.V + s.Wv * s.Wv;
    double Wt[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) Wt[i] = -s.rho * tr[i];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const double Un = Uv[ax];
      const double a = Un * Un + 0.5 * q2, b = 0.5 * Un * q2;
      // (u_ax - U_ax)(|c - U|^2 + xi^2) / 2 expanded: momentum moments of the
      // other axes enter as U_ax U_m W_m
      double q = F[ax][4] - Uv[0] * F[ax][1] - Uv[1] * F[ax][2] - Uv[2] * F[ax][3] + a * F[ax][0] - Un * W[4] - b * W[0];
      double qt = Ft[ax][4] - Uv[0] * Ft[ax][1] - Uv[1] * Ft[ax][2] - Uv[2] * Ft[ax][3] + a * Ft[ax][0] - Un * Wt[4] -
                  b * Wt[0];
#pragma unroll
      for (int m2 = 0; m2 < 3; ++m2)
        if (m2 != ax) {
          q += Un * Uv[m2] * W[1 + m2];
          qt += Un * Uv[m2] * Wt[1 + m2];
        }
      F[ax][4] += f * q;
      Ft[ax][4] += f * qt;
    }
  }
}

}  // namespace fdk3
