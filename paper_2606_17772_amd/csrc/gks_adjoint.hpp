// Reverse-mode (adjoint) arithmetic of the 2D gas-kinetic interface and
// nodal solvers and of the GENO reconstructions, FP64.
//
// Every *_b routine takes the inputs of its forward counterpart in
// gks_device.hpp, recomputes the forward intermediates it needs, and, given
// the adjoint of the forward outputs, ADDS the adjoint of the forward inputs
// into the caller's accumulators (suffix b).  Non-smooth points follow the
// forward code: |x| has derivative 0 at 0, max/min route the adjoint to the
// argument the forward selected (ties: the first), tau = 0 takes the
// tau -> 0+ limit.
#pragma once

#include "gks_device.hpp"

namespace fdk {

// The reverse of the kinetic solvers below lets the compiler fuse any
// multiply and add into one FMA (about 11% fewer FP64 instructions in the
// reverse interface and node sweeps).  Its rounding then differs from the forward
// solver's in the last bits, which no result depends on: it makes no branch
// decision (those use the forward solver's own functions).  The GENO and
// reconstruction reverse further down compares smoothness indicators and keeps
// the forward code's contraction.
#pragma clang fp contract(fast)

// Adjoint of the fields of a Prim<double>.
struct PrimB {
  double rho, irho, U, V, p, i2l, lam;
};
FDK_HD PrimB primb_zero() { return PrimB{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0}; }
FDK_HD void mom_zero(Mom<double>& m) {
#pragma unroll
  for (int i = 0; i < 7; ++i) { m.mu[i] = 0.0; m.mv[i] = 0.0; }
  m.x2 = 0.0;
  m.x4 = 0.0;
}

// prim (2D): W -> (rho, irho, U, V, p, i2l, lam).  Adds the adjoint of W.
FDK_HD void prim_b(const double* W, const Prim<double>& s, double gamma, const PrimB& b, double* Wb) {
  const double i2lb = b.i2l - b.lam * s.lam / s.i2l;  // lam = 0.5 / i2l
  const double pb = b.p + i2lb * s.irho;              // i2l = p irho
  double irhob = b.irho + i2lb * s.p;
  const double gm = gamma - 1.0;                       // p = (g-1)(rE - rho (U^2+V^2)/2)
  const double rEb = gm * pb;
  const double rhob = b.rho - gm * 0.5 * (s.U * s.U + s.V * s.V) * pb;
  const double Ub = b.U - gm * s.rho * s.U * pb;
  const double Vb = b.V - gm * s.rho * s.V * pb;
  Wb[1] += Ub * s.irho;                                // U = W1 irho, V = W2 irho
  irhob += Ub * W[1];
  Wb[2] += Vb * s.irho;
  irhob += Vb * W[2];
  Wb[0] += rhob - irhob * s.irho * s.irho;             // irho = 1 / W0, rho = W0
  Wb[3] += rEb;
}

// m[n+2] = U m[n+1] + (n+1) i2l m[n], n = 0..4.  mb is consumed in place.
FDK_HD void mu_rec_b(const double* m, double U, double i2l, double* mb, double& Ub, double& i2lb) {
#pragma unroll
  for (int n = 4; n >= 0; --n) {
    const double g = mb[n + 2];
    mb[n + 1] += U * g;
    Ub += m[n + 1] * g;
    i2lb += double(n + 1) * m[n] * g;
    mb[n] += double(n + 1) * i2l * g;
  }
}

// mv (v moments), x2, x4 of a state.
FDK_HD void mom_common_b(const Prim<double>& s, double K, const Mom<double>& m, const Mom<double>& mb, PrimB& b) {
  const double x2b = mb.x2 + mb.x4 * (K + 2.0) * s.i2l;  // x4 = x2 (K+2) i2l
  b.i2l += mb.x4 * m.x2 * (K + 2.0) + K * x2b;           // x2 = K i2l
  double mvb[7];
#pragma unroll
  for (int i = 0; i < 7; ++i) mvb[i] = mb.mv[i];
  double Vb = 0.0, i2lb = 0.0;
  mu_rec_b(m.mv, s.V, s.i2l, mvb, Vb, i2lb);
  b.V += Vb + mvb[1];
  b.i2l += i2lb;
}

// mu of the full line.
FDK_HD void mom_full_b(const Prim<double>& s, const Mom<double>& m, const Mom<double>& mb, PrimB& b) {
  double mub[7];
#pragma unroll
  for (int i = 0; i < 7; ++i) mub[i] = mb.mu[i];
  double Ub = 0.0, i2lb = 0.0;
  mu_rec_b(m.mu, s.U, s.i2l, mub, Ub, i2lb);
  b.U += Ub + mub[1];
  b.i2l += i2lb;
}

// mu of the half line u > 0 (sgn = +1) or u < 0 (sgn = -1).
FDK_HD void mom_half_b(const Prim<double>& s, double sgn, const Mom<double>& m, const Mom<double>& mb, PrimB& b) {
  double mub[7];
#pragma unroll
  for (int i = 0; i < 7; ++i) mub[i] = mb.mu[i];
  double Ub = 0.0, i2lb = 0.0;
  mu_rec_b(m.mu, s.U, s.i2l, mub, Ub, i2lb);
  const double sl = sqrt(s.lam), z = -sgn * sl * s.U;
  const double ex = exp(-s.lam * s.U * s.U), sq = sqrt(s.i2l);
  const double c = 0.39894228040143267794;
  // mu1 = U mu0 + sgn ex sq c
  Ub += m.mu[0] * mub[1];
  const double mu0b = mub[0] + s.U * mub[1];
  const double exb = sgn * sq * c * mub[1], sqb = sgn * ex * c * mub[1];
  double lamb = -s.U * s.U * ex * exb;
  Ub += -2.0 * s.lam * s.U * ex * exb;
  i2lb += sqb / (2.0 * sq);
  // mu0 = erfc(z) / 2
  const double zb = -0.56418958354775628695 * exp(-z * z) * mu0b;
  Ub += -sgn * sl * zb;
  lamb += -sgn * s.U * zb / (2.0 * sl);
  b.U += Ub;
  b.i2l += i2lb;
  b.lam += lamb;
}

template <int P, int Q, int R>
FDK_HD void muv_b(const Mom<double>& m, const double ob[4], Mom<double>& mb) {
  const double xr = R == 0 ? 1.0 : m.x2;
  const double xr1 = R == 0 ? m.x2 : m.x4;
  const double bv = m.mu[P] * m.mv[Q];
  const double bb = ob[0] * xr + 0.5 * ob[3] * xr1;
  const double xrb = ob[0] * bv + ob[1] * m.mu[P + 1] * m.mv[Q] + ob[2] * m.mu[P] * m.mv[Q + 1] +
                     0.5 * ob[3] * (m.mu[P + 2] * m.mv[Q] + m.mu[P] * m.mv[Q + 2]);
  const double xr1b = 0.5 * ob[3] * bv;
  mb.mu[P + 1] += ob[1] * m.mv[Q] * xr;
  mb.mv[Q] += ob[1] * m.mu[P + 1] * xr;
  mb.mu[P] += ob[2] * m.mv[Q + 1] * xr;
  mb.mv[Q + 1] += ob[2] * m.mu[P] * xr;
  const double t = 0.5 * ob[3] * xr;
  mb.mu[P + 2] += t * m.mv[Q];
  mb.mv[Q] += t * m.mu[P + 2];
  mb.mu[P] += t * m.mv[Q + 2];
  mb.mv[Q + 2] += t * m.mu[P];
  mb.mu[P] += bb * m.mv[Q];
  mb.mv[Q] += bb * m.mu[P];
  if (R == 0) {
    mb.x2 += xr1b;
  } else {
    mb.x2 += xrb;
    mb.x4 += xr1b;
  }
}

// o = <(s.psi) u^P v^Q psi>: reverse of the one-dimensional combinations of
// ma (cu, cv and the xi^2 row; see ma in gks_device.hpp).
template <int P, int Q>
FDK_HD void ma_b(const double s[4], const Mom<double>& m, const double ob[4], double sb[4], Mom<double>& mb) {
  const double h3 = 0.5 * s[3];
  const double c0 = s[0] + h3 * m.x2;
  double u[3], v[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    u[d] = c0 * m.mu[P + d] + s[1] * m.mu[P + d + 1] + h3 * m.mu[P + d + 2];
    v[d] = s[2] * m.mv[Q + d + 1] + h3 * m.mv[Q + d + 2];
  }
  const double o0 = m.mv[Q] * u[0] + m.mu[P] * v[0];
  const double D = m.x4 - m.x2 * m.x2, muv = m.mu[P] * m.mv[Q];
  // o3 = (mv[Q] u2 + mu[P+2] v0 + mv[Q+2] u0 + mu[P] v2 + gx) / 2,  gx = x2 o0 + h3 mu[P] mv[Q] D
  const double t = 0.5 * ob[3];
  double ub[3], vb[3];
  ub[2] = t * m.mv[Q];
  vb[2] = t * m.mu[P];
  mb.mv[Q] += t * u[2];
  mb.mu[P + 2] += t * v[0];
  mb.mv[Q + 2] += t * u[0];
  mb.mu[P] += t * v[2];
  const double o0b = ob[0] + t * m.x2;
  double x2b = t * o0, h3b = t * muv * D;
  const double Db = t * h3 * muv;
  mb.mu[P] += t * h3 * m.mv[Q] * D;
  mb.mv[Q] += t * h3 * m.mu[P] * D;
  mb.x4 += Db;
  x2b -= 2.0 * m.x2 * Db;
  // o2 = mv[Q+1] u0 + mu[P] v1;  o1 = mv[Q] u1 + mu[P+1] v0;  o0 = mv[Q] u0 + mu[P] v0
  ub[0] = ob[2] * m.mv[Q + 1] + o0b * m.mv[Q] + t * m.mv[Q + 2];
  vb[1] = ob[2] * m.mu[P];
  ub[1] = ob[1] * m.mv[Q];
  vb[0] = ob[1] * m.mu[P + 1] + o0b * m.mu[P] + t * m.mu[P + 2];
  mb.mv[Q + 1] += ob[2] * u[0];
  mb.mu[P] += ob[2] * v[1] + o0b * v[0];
  mb.mv[Q] += ob[1] * u[1] + o0b * u[0];
  mb.mu[P + 1] += ob[1] * v[0];
  // u_d = c0 mu[P+d] + s1 mu[P+d+1] + h3 mu[P+d+2];  v_d = s2 mv[Q+d+1] + h3 mv[Q+d+2]
  double c0b = 0.0;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    c0b += ub[d] * m.mu[P + d];
    sb[1] += ub[d] * m.mu[P + d + 1];
    h3b += ub[d] * m.mu[P + d + 2] + vb[d] * m.mv[Q + d + 2];
    sb[2] += vb[d] * m.mv[Q + d + 1];
    mb.mu[P + d] += ub[d] * c0;
    mb.mu[P + d + 1] += ub[d] * s[1];
    mb.mu[P + d + 2] += ub[d] * h3;
    mb.mv[Q + d + 1] += vb[d] * s[2];
    mb.mv[Q + d + 2] += vb[d] * h3;
  }
  // c0 = s0 + h3 x2,  h3 = s3 / 2
  sb[0] += c0b;
  h3b += c0b * m.x2;
  x2b += c0b * h3;
  mb.x2 += x2b;
  sb[3] += 0.5 * h3b;
}

// <psi> and <u psi>
FDK_HD void psi_moms_b(const Mom<double>& m, const double pb[4], const double ub[4], Mom<double>& mb) {
  mb.mu[0] += pb[0] + pb[2] * m.mv[1] + 0.5 * pb[3] * (m.mv[2] + m.x2);
  mb.mu[1] += pb[1];
  mb.mv[1] += pb[2] * m.mu[0];
  mb.mu[2] += 0.5 * pb[3];
  mb.mv[2] += 0.5 * pb[3] * m.mu[0];
  mb.x2 += 0.5 * pb[3] * m.mu[0];
  muv_b<1, 0, 0>(m, ub, mb);
}

// s = slope(q, d) (2D closed form).  s holds the forward result; sb the
// adjoint of s.  Adds the adjoint of d and of q's fields.
FDK_HD void slope_b(const Prim<double>& q, double K, double iKd, const double d[4], const double s[4],
                    const double sb[4], double db[4], PrimB& b) {
  const double e = q.U * q.U + q.V * q.V + (K + 2.0) * q.i2l;
  const double B = 2.0 * d[3] - e * d[0];
  const double A = d[1] - q.U * d[0];
  const double Cc = d[2] - q.V * d[0];
  const double tl = 2.0 * q.lam;
  const double X = B - 2.0 * q.U * A - 2.0 * q.V * Cc;
  double s1b = sb[1], s2b = sb[2], s3b = sb[3];
  // s0 = d0 - U s1 - V s2 - s3 e / 2
  double d0b = sb[0];
  double Ub = -s[1] * sb[0], Vb = -s[2] * sb[0];
  s1b += -q.U * sb[0];
  s2b += -q.V * sb[0];
  s3b += -0.5 * e * sb[0];
  double eb = -0.5 * s[3] * sb[0];
  // s1 = tl A - U s3, s2 = tl Cc - V s3
  double tlb = A * s1b + Cc * s2b;
  double Ab = tl * s1b, Ccb = tl * s2b;
  Ub += -s[3] * s1b;
  Vb += -s[3] * s2b;
  s3b += -q.U * s1b - q.V * s2b;
  // s3 = tl^2 iKd X
  tlb += 2.0 * tl * iKd * X * s3b;
  const double Xb = tl * tl * iKd * s3b;
  const double Bb = Xb;
  Ub += -2.0 * A * Xb;
  Ab += -2.0 * q.U * Xb;
  Vb += -2.0 * Cc * Xb;
  Ccb += -2.0 * q.V * Xb;
  b.lam += 2.0 * tlb;
  db[2] += Ccb;
  Vb += -d[0] * Ccb;
  d0b += -q.V * Ccb;
  db[1] += Ab;
  Ub += -d[0] * Ab;
  d0b += -q.U * Ab;
  db[3] += 2.0 * Bb;
  eb += -d[0] * Bb;
  d0b += -e * Bb;
  Ub += 2.0 * q.U * eb;
  Vb += 2.0 * q.V * eb;
  b.i2l += (K + 2.0) * eb;
  db[0] += d0b;
  b.U += Ub;
  b.V += Vb;
}

// Adjoint of the time coefficients with respect to tau.
FDK_HD double time_coef_b(double dt, double tau, const double cb[5], const double ctb[5], double e1b) {
  const double Eh = tau > 0 ? exp(-0.5 * dt / tau) : 0.0;
  const double Ef = Eh * Eh;
  const double idt = 1.0 / dt, idt2 = 4.0 * idt * idt;
  double taub = 0.0, Ehb = 0.0, Efb = e1b;
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    const double T = half == 0 ? 0.5 * dt : dt, E = half == 0 ? Eh : Ef;
    double qb[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) qb[k] = half == 0 ? 4.0 * idt * cb[k] - 2.0 * idt2 * ctb[k] : -idt * cb[k] + idt2 * ctb[k];
    taub += qb[0] * (-(1.0 - E)) + qb[1] * (4.0 * tau - T - (T + 4.0 * tau) * E) + qb[2] * (-T + 2.0 * tau * (1.0 - E)) +
            qb[3] * (1.0 - E) + qb[4] * (T * E + 4.0 * tau * E - 4.0 * tau);
    const double Eb = qb[0] * tau - qb[1] * tau * (T + 2.0 * tau) - qb[2] * tau * tau - qb[3] * tau +
                      qb[4] * tau * (T + 2.0 * tau);
    if (half == 0) Ehb += Eb; else Efb += Eb;
  }
  Ehb += 2.0 * Eh * Efb;
  if (tau > 0) taub += Ehb * Eh * 0.5 * dt / (tau * tau);
  return taub;
}

// Adjoints of the accumulated moments of f^n and f_t^n and the outputs.
struct AccB {
  double F[4], Ft[4], We[4], Wet[4];
  double cb[5], ctb[5], taub, eb;  // adjoints of the time coefficients, of tau and of exp(-dt/tau)
  double pad;  // odd size in 8-byte words: per-thread copies in LDS spread over the banks
};
// Inputs of one interface solve (or their adjoints), padded like AccB.
struct SolveIO {
  double WL[4], WR[4], nL[4], nR[4], Wt[4];
  double pad;
};

// One side's terms (see side_terms).  Wtb: adjoint of this side's Euler time
// derivative output.  Adds to nb, tb (slopes), sb (state), hb (half moments),
// taub and the adjoints of c[3], c[4], ct[3], ct[4].
FDK_HD void side_terms_b(const Prim<double>& s, const Mom<double>& h, const double* n, const double* t, double K,
                         double iKd, double tau, const TimeCoef<double>& tc, const AccB& ab, const double* Wtb,
                         double* nb, double* tb, PrimB& sb, Mom<double>& hb, double& taub, double cb[5],
                         double ctb[5]) {
  // forward recomputation
  Mom<double> f = h;
  mom_full(s, f);
  double a[4], bs[4], A[4], d[4], dtn[4], dA[4], tf[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) { d[i] = n[i] * s.irho; dtn[i] = t[i] * s.irho; }
  slope<double, 2>(s, K, iKd, d, a);
  slope<double, 2>(s, K, iKd, dtn, bs);
  {
    double x[4], y[4];
    ma<1, 0>(a, f, x);
    ma<0, 1>(bs, f, y);
#pragma unroll
    for (int i = 0; i < 4; ++i) { tf[i] = x[i] + y[i]; dA[i] = -tf[i]; }
  }
  slope<double, 2>(s, K, iKd, dA, A);
  double ph[4], uh[4], tp[4], tu[4], Ap[4], Au[4];
  psi_moms<double, 2>(h, ph, uh);
  transport<double, 2>(a, bs, h, tp, tu);
  tslope<double, 2>(A, h, Ap, Au);
  // accumulation
  double rhob = 0.0, uhb[4], phb[4], tub[4], tpb[4], Aub[4], Apb[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double nu = uh[i] - tau * Au[i], np = ph[i] - tau * Ap[i];
    rhob += ab.Ft[i] * (tc.ct[3] * nu + tc.ct[4] * tu[i]) + ab.Wet[i] * (tc.ct[3] * np + tc.ct[4] * tp[i]) +
            ab.F[i] * (tc.c[3] * nu + tc.c[4] * tu[i]) + ab.We[i] * (tc.c[3] * np + tc.c[4] * tp[i]);
    ctb[3] += s.rho * (ab.Ft[i] * nu + ab.Wet[i] * np);
    ctb[4] += s.rho * (ab.Ft[i] * tu[i] + ab.Wet[i] * tp[i]);
    cb[3] += s.rho * (ab.F[i] * nu + ab.We[i] * np);
    cb[4] += s.rho * (ab.F[i] * tu[i] + ab.We[i] * tp[i]);
    const double nub = s.rho * (tc.ct[3] * ab.Ft[i] + tc.c[3] * ab.F[i]);
    const double npb = s.rho * (tc.ct[3] * ab.Wet[i] + tc.c[3] * ab.We[i]);
    tub[i] = s.rho * (tc.ct[4] * ab.Ft[i] + tc.c[4] * ab.F[i]);
    tpb[i] = s.rho * (tc.ct[4] * ab.Wet[i] + tc.c[4] * ab.We[i]);
    uhb[i] = nub;
    phb[i] = npb;
    Aub[i] = -tau * nub;
    Apb[i] = -tau * npb;
    taub += -Au[i] * nub - Ap[i] * npb;
  }
  double Ab[4] = {0, 0, 0, 0}, abv[4] = {0, 0, 0, 0}, bb[4] = {0, 0, 0, 0};
  ma_b<0, 0>(A, h, Apb, Ab, hb);
  ma_b<1, 0>(A, h, Aub, Ab, hb);
  ma_b<1, 0>(a, h, tpb, abv, hb);
  ma_b<0, 1>(bs, h, tpb, bb, hb);
  ma_b<2, 0>(a, h, tub, abv, hb);
  ma_b<1, 1>(bs, h, tub, bb, hb);
  psi_moms_b(h, phb, uhb, hb);
  double dAb[4] = {0, 0, 0, 0}, tfb[4];
  slope_b(s, K, iKd, dA, A, Ab, dAb, sb);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    tfb[i] = -dAb[i] - s.rho * Wtb[i];  // dA = -tf, Wt = -rho tf
    rhob += -tf[i] * Wtb[i];
  }
  Mom<double> fb;
  mom_zero(fb);
  ma_b<1, 0>(a, f, tfb, abv, fb);
  ma_b<0, 1>(bs, f, tfb, bb, fb);
#pragma unroll
  for (int i = 0; i < 7; ++i) hb.mv[i] += fb.mv[i];
  hb.x2 += fb.x2;
  hb.x4 += fb.x4;
  mom_full_b(s, f, fb, sb);
  double dtb[4] = {0, 0, 0, 0}, db[4] = {0, 0, 0, 0};
  slope_b(s, K, iKd, dtn, bs, bb, dtb, sb);
  slope_b(s, K, iKd, d, a, abv, db, sb);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    tb[i] += dtb[i] * s.irho;
    nb[i] += db[i] * s.irho;
    sb.irho += t[i] * dtb[i] + n[i] * db[i];
  }
  sb.rho += rhob;
}

// Equilibrium part at the interface (see gks_iface).
FDK_HD void equilibrium_b(const Prim<double>& s0, double K, double iKd, const double* nL, const double* nR,
                          const double* Wt, const TimeCoef<double>& tc, const AccB& ab, double* nLb, double* nRb,
                          double* Wtb, PrimB& s0b, double cb[5], double ctb[5]) {
  Mom<double> m0;
  mom_common<double, 2>(s0, K, m0);
  mom_full(s0, m0);
  double a0[4], b0[4], A0[4], d[4], dw[4], dA[4], t0[4], tu0[4], Ap0[4], Au0[4], p0[4], u0[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) { d[i] = 0.5 * (nL[i] + nR[i]) * s0.irho; dw[i] = Wt[i] * s0.irho; }
  slope<double, 2>(s0, K, iKd, d, a0);
  slope<double, 2>(s0, K, iKd, dw, b0);
  transport<double, 2>(a0, b0, m0, t0, tu0);
#pragma unroll
  for (int i = 0; i < 4; ++i) dA[i] = -t0[i];
  slope<double, 2>(s0, K, iKd, dA, A0);
  tslope<double, 2>(A0, m0, Ap0, Au0);
  psi_moms<double, 2>(m0, p0, u0);
  double rhob = 0.0, u0b[4], tu0b[4], Au0b[4], p0b[4], t0b[4], Ap0b[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    rhob += ab.Ft[i] * (tc.ct[0] * u0[i] + tc.ct[1] * tu0[i] + tc.ct[2] * Au0[i]) +
            ab.Wet[i] * (tc.ct[0] * p0[i] + tc.ct[1] * t0[i] + tc.ct[2] * Ap0[i]) +
            ab.F[i] * (tc.c[0] * u0[i] + tc.c[1] * tu0[i] + tc.c[2] * Au0[i]) +
            ab.We[i] * (tc.c[0] * p0[i] + tc.c[1] * t0[i] + tc.c[2] * Ap0[i]);
    ctb[0] += s0.rho * (ab.Ft[i] * u0[i] + ab.Wet[i] * p0[i]);
    ctb[1] += s0.rho * (ab.Ft[i] * tu0[i] + ab.Wet[i] * t0[i]);
    ctb[2] += s0.rho * (ab.Ft[i] * Au0[i] + ab.Wet[i] * Ap0[i]);
    cb[0] += s0.rho * (ab.F[i] * u0[i] + ab.We[i] * p0[i]);
    cb[1] += s0.rho * (ab.F[i] * tu0[i] + ab.We[i] * t0[i]);
    cb[2] += s0.rho * (ab.F[i] * Au0[i] + ab.We[i] * Ap0[i]);
    u0b[i] = s0.rho * (tc.ct[0] * ab.Ft[i] + tc.c[0] * ab.F[i]);
    tu0b[i] = s0.rho * (tc.ct[1] * ab.Ft[i] + tc.c[1] * ab.F[i]);
    Au0b[i] = s0.rho * (tc.ct[2] * ab.Ft[i] + tc.c[2] * ab.F[i]);
    p0b[i] = s0.rho * (tc.ct[0] * ab.Wet[i] + tc.c[0] * ab.We[i]);
    t0b[i] = s0.rho * (tc.ct[1] * ab.Wet[i] + tc.c[1] * ab.We[i]);
    Ap0b[i] = s0.rho * (tc.ct[2] * ab.Wet[i] + tc.c[2] * ab.We[i]);
  }
  Mom<double> m0b;
  mom_zero(m0b);
  psi_moms_b(m0, p0b, u0b, m0b);
  double A0b[4] = {0, 0, 0, 0}, a0b[4] = {0, 0, 0, 0}, b0b[4] = {0, 0, 0, 0};
  ma_b<0, 0>(A0, m0, Ap0b, A0b, m0b);
  ma_b<1, 0>(A0, m0, Au0b, A0b, m0b);
  double dAb[4] = {0, 0, 0, 0};
  slope_b(s0, K, iKd, dA, A0, A0b, dAb, s0b);
#pragma unroll
  for (int i = 0; i < 4; ++i) t0b[i] -= dAb[i];
  ma_b<1, 0>(a0, m0, t0b, a0b, m0b);
  ma_b<0, 1>(b0, m0, t0b, b0b, m0b);
  ma_b<2, 0>(a0, m0, tu0b, a0b, m0b);
  ma_b<1, 1>(b0, m0, tu0b, b0b, m0b);
  double dwb[4] = {0, 0, 0, 0}, db[4] = {0, 0, 0, 0};
  slope_b(s0, K, iKd, dw, b0, b0b, dwb, s0b);
  slope_b(s0, K, iKd, d, a0, a0b, db, s0b);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    Wtb[i] += dwb[i] * s0.irho;
    nLb[i] += 0.5 * db[i] * s0.irho;
    nRb[i] += 0.5 * db[i] * s0.irho;
    s0b.irho += Wt[i] * dwb[i] + 0.5 * (nL[i] + nR[i]) * db[i];
  }
  mom_full_b(s0, m0, m0b, s0b);
  mom_common_b(s0, K, m0, m0b, s0b);
  s0b.rho += rhob;
}

// A value the optimiser may not reuse from an earlier identical computation:
// the adjoint below recomputes cheap forward quantities (primitive states,
// half-line moments, time coefficients) where they are needed instead of
// keeping them in registers through the whole reverse sweep.
FDK_HD double fresh(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" : "+v"(x));
#endif
  return x;
}
// A compiler-only memory barrier between the phases of the solver adjoint:
// values the caller keeps in memory (the LDS-resident inputs and
// accumulators) are reloaded after it instead of being held in registers.
FDK_HD void phase_barrier() {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" ::: "memory");
#endif
}
// Primitive state and half-line moments of one side (sgn = +1: u > 0).
FDK_HD void side_state(const double* W, double gamma, double K, double sgn, Prim<double>& s, Mom<double>& h) {
  double Wf[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) Wf[i] = fresh(W[i]);
  s = prim<double, 2>(Wf, gamma);
  mom_common<double, 2>(s, K, h);
  mom_half(s, sgn, h);
}

// A phase number the compiler cannot see through: the solver adjoint below
// runs its phases as iterations of one loop over it, so that no phase's code
// is peeled, merged or scheduled into another.
FDK_HD int opaque_int(int x) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" : "+s"(x));
#endif
  return x;
}

// A pointer the compiler cannot see through (address arithmetic on it stays
// where it is written).
template <class T> FDK_HD T* opaque_ptr(T* p) {
#if defined(__HIP_DEVICE_COMPILE__)
  asm volatile("" : "+v"(p));
#endif
  return p;
}

// Adjoint of the 2D interface solver with all outputs (gks_iface<double, 2,
// true>).  obload(ob) fills ob with the adjoints of F, Ft, Wl, Wr, Wlt, Wrt;
// it is called once, inside the first phase.  Adds the adjoints of WL, WR, nL,
// nR, Wt into inb (same field names).  in, inb and the moment adjoint ab are
// references to storage the caller chooses (the reverse interface sweep keeps
// them in LDS).
//
// The work runs as seven phases, the iterations of one loop over an opaque
// phase number; only W0, tau, the compatibility state's adjoint and the
// seeds of the two sides' time derivatives (20 doubles) are carried in
// registers from phase to phase, the time-coefficient adjoints in ab, and
// everything else is recomputed in the phase that needs it:
//   0  forward solve (kept: W0, tau), then the reverse of the output blend
//      and of the Prandtl correction;
//   1  reverse of the equilibrium part;
//   2, 3  reverse of the left / right side terms, reduced to the adjoint of
//      that side's W at once;
//   4  reverse of the collision time and time coefficients, giving the
//      adjoint of W0;
//   5, 6  the compatibility state's share of the left / right W adjoint (W0
//      is a sum of half-line moments of the two sides).
// Written as straight-line code, the compiler interleaves the phases and keeps
// recomputed values of one phase alive into the next: about 400 registers
// spill.  As loop iterations each phase holds only its own values.
template <class TIn, class TOb, class TInb>
FDK_HD void gks_iface_b(const Consts& k, double dt, const TIn& in, const TOb& obload, TInb& inb, AccB& ab) {
  const double K = k.K, gam = k.gamma, iKd = k.inv_Kd;
  // carried between phases
  double W0[4], tau = 0.0, WtLb[4], WtRb[4];
  PrimB s0b = primb_zero();
  double* cb = ab.cb;
  double* ctb = ab.ctb;
  double& taub = ab.taub;
  double& eb = ab.eb;
#pragma unroll
  for (int i = 0; i < 5; ++i) { cb[i] = 0.0; ctb[i] = 0.0; }
  taub = 0.0;
  eb = 0.0;
#pragma unroll 1
  for (int ph0 = 0; ph0 < 7; ++ph0) {
    phase_barrier();
    const int ph = opaque_int(ph0);
    if (ph == 0) {
      // ---- forward
      double F[4], Ft[4], We[4], Wet[4], WtL[4], WtR[4];
      {
        Prim<double> sL, sR;
        Mom<double> hL, hR;
        side_state(in.WL, gam, K, 1.0, sL, hL);
        side_state(in.WR, gam, K, -1.0, sR, hR);
        {
          double pL[4], pR[4], u[4];
          psi_moms<double, 2>(hL, pL, u);
          psi_moms<double, 2>(hR, pR, u);
#pragma unroll
          for (int i = 0; i < 4; ++i) W0[i] = sL.rho * pL[i] + sR.rho * pR[i];
        }
        const Prim<double> s0 = prim<double, 2>(W0, gam);
        tau = (k.mu > 0 ? k.mu / s0.p : k.tau_c1 * dt) + k.tau_c2 * dt * m_abs(sL.p - sR.p) / (sL.p + sR.p);
        const TimeCoef<double> tc = time_coef(dt, tau);
#pragma unroll
        for (int i = 0; i < 4; ++i) { F[i] = 0.0; Ft[i] = 0.0; We[i] = 0.0; Wet[i] = 0.0; }
        side_terms<double, 2, true>(sL, hL, in.nL, in.Wt, K, iKd, tau, tc, true, F, Ft, We, Wet, WtL);
        side_terms<double, 2, true>(sR, hR, in.nR, in.Wt, K, iKd, tau, tc, true, F, Ft, We, Wet, WtR);
        Mom<double> m0;
        mom_common<double, 2>(s0, K, m0);
        mom_full(s0, m0);
        double a0[4], b0[4], A0[4], d[4], t0[4], tu0[4], Ap0[4], Au0[4], p0[4], u0[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) d[i] = 0.5 * (in.nL[i] + in.nR[i]) * s0.irho;
        slope<double, 2>(s0, K, iKd, d, a0);
#pragma unroll
        for (int i = 0; i < 4; ++i) d[i] = in.Wt[i] * s0.irho;
        slope<double, 2>(s0, K, iKd, d, b0);
        transport<double, 2>(a0, b0, m0, t0, tu0);
#pragma unroll
        for (int i = 0; i < 4; ++i) d[i] = -t0[i];
        slope<double, 2>(s0, K, iKd, d, A0);
        tslope<double, 2>(A0, m0, Ap0, Au0);
        psi_moms<double, 2>(m0, p0, u0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          Ft[i] += s0.rho * (tc.ct[0] * u0[i] + tc.ct[1] * tu0[i] + tc.ct[2] * Au0[i]);
          Wet[i] += s0.rho * (tc.ct[0] * p0[i] + tc.ct[1] * t0[i] + tc.ct[2] * Ap0[i]);
          F[i] += s0.rho * (tc.c[0] * u0[i] + tc.c[1] * tu0[i] + tc.c[2] * Au0[i]);
          We[i] += s0.rho * (tc.c[0] * p0[i] + tc.c[1] * t0[i] + tc.c[2] * Ap0[i]);
        }
      }
      // ---- reverse: outputs
      GksIO<double, 2> ob;
      obload(ob);
      const double e = time_coef(dt, tau).e1, oe = 1.0 - e;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        ab.Wet[i] = oe * (ob.Wlt[i] + ob.Wrt[i]);
        WtLb[i] = e * ob.Wlt[i];
        WtRb[i] = e * ob.Wrt[i];
        ab.We[i] = oe * (ob.Wl[i] + ob.Wr[i]);
        inb.WL[i] += e * ob.Wl[i];
        inb.WR[i] += e * ob.Wr[i];
        eb += (WtL[i] - Wet[i]) * ob.Wlt[i] + (WtR[i] - Wet[i]) * ob.Wrt[i] + (in.WL[i] - We[i]) * ob.Wl[i] +
              (in.WR[i] - We[i]) * ob.Wr[i];
        ab.F[i] = ob.F[i];
        ab.Ft[i] = ob.Ft[i];
      }
      // ---- reverse: Prandtl correction (F, Ft hold the values before it)
      if (k.mu > 0) {
        const Prim<double> s0 = prim<double, 2>(W0, gam);
        const double U = s0.U, V = s0.V, f = k.prfix;
        const double a = 1.5 * U * U + 0.5 * V * V, bq = 0.5 * U * (U * U + V * V);
        const double qb = f * ab.F[3], qtb = f * ab.Ft[3];
        s0b.U += qb * (-F[1] + 3.0 * U * F[0] - We[3] + V * We[2] - 0.5 * (3.0 * U * U + V * V) * We[0]) +
                 qtb * (-Ft[1] + 3.0 * U * Ft[0] - Wet[3] + V * Wet[2] - 0.5 * (3.0 * U * U + V * V) * Wet[0]);
        s0b.V += qb * (-F[2] + V * F[0] + U * We[2] - U * V * We[0]) +
                 qtb * (-Ft[2] + V * Ft[0] + U * Wet[2] - U * V * Wet[0]);
        ab.F[3] += qb; ab.F[1] += -U * qb; ab.F[2] += -V * qb; ab.F[0] += a * qb;
        ab.We[3] += -U * qb; ab.We[2] += U * V * qb; ab.We[0] += -bq * qb;
        ab.Ft[3] += qtb; ab.Ft[1] += -U * qtb; ab.Ft[2] += -V * qtb; ab.Ft[0] += a * qtb;
        ab.Wet[3] += -U * qtb; ab.Wet[2] += U * V * qtb; ab.Wet[0] += -bq * qtb;
      }
    } else if (ph == 1) {
      // ---- reverse: equilibrium
      const Prim<double> s0 = prim<double, 2>(W0, gam);
      equilibrium_b(s0, K, iKd, in.nL, in.nR, in.Wt, time_coef(dt, tau), ab, inb.nL, inb.nR, inb.Wt, s0b, cb, ctb);
    } else if (ph <= 3) {
      // ---- reverse: one side's terms, reduced to the adjoint of its W
      const int side = ph - 2;
      const double sgn = side == 0 ? 1.0 : -1.0;
      Prim<double> s;
      Mom<double> h, hb;
      side_state(side == 0 ? in.WL : in.WR, gam, K, sgn, s, h);
      mom_zero(hb);
      PrimB sb = primb_zero();
      double wtb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) wtb[i] = side == 0 ? WtLb[i] : WtRb[i];
      side_terms_b(s, h, side == 0 ? in.nL : in.nR, in.Wt, K, iKd, tau, time_coef(dt, tau), ab, wtb,
                   side == 0 ? inb.nL : inb.nR, inb.Wt, sb, hb, taub, cb, ctb);
      mom_half_b(s, sgn, h, hb, sb);
      mom_common_b(s, K, h, hb, sb);
      prim_b(side == 0 ? in.WL : in.WR, s, gam, sb, side == 0 ? inb.WL : inb.WR);
    } else if (ph == 4) {
      // ---- reverse: collision time and time coefficients; the adjoint of W0
      const Prim<double> s0 = prim<double, 2>(W0, gam);
      taub += time_coef_b(dt, tau, cb, ctb, eb);
      if (k.mu > 0) s0b.p += -k.mu / (s0.p * s0.p) * taub;
      const Prim<double> pl = prim<double, 2>(in.WL, gam), pr = prim<double, 2>(in.WR, gam);
      const double dP = pl.p - pr.p, sP = pl.p + pr.p;
      const double g = k.tau_c2 * dt, sg = dP > 0 ? 1.0 : (dP < 0 ? -1.0 : 0.0), ad = m_abs(dP);
      // reuse: cb[0..3] = adjoint of W0, cb[4], ctb[0] = adjoints of the two sides' p
      const double pLb = g * (sg / sP - ad / (sP * sP)) * taub;
      const double pRb = g * (-sg / sP - ad / (sP * sP)) * taub;
      double W0b[4] = {0, 0, 0, 0};
      prim_b(W0, s0, gam, s0b, W0b);
#pragma unroll
      for (int i = 0; i < 4; ++i) cb[i] = W0b[i];
      cb[4] = pLb;
      ctb[0] = pRb;
    } else {
      // ---- reverse: the compatibility state's share of each side's state
      const int side = ph - 5;
      const double sgn = side == 0 ? 1.0 : -1.0;
      Prim<double> s;
      Mom<double> h, hb;
      side_state(side == 0 ? in.WL : in.WR, gam, K, sgn, s, h);
      mom_zero(hb);
      PrimB sb = primb_zero();
      sb.p = side == 0 ? cb[4] : ctb[0];
      const double zero[4] = {0, 0, 0, 0};
      double p[4], u[4], pb[4];
      psi_moms<double, 2>(h, p, u);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        pb[i] = s.rho * cb[i];
        sb.rho += p[i] * cb[i];
      }
      psi_moms_b(h, pb, zero, hb);
      mom_half_b(s, sgn, h, hb, sb);
      mom_common_b(s, K, h, hb, sb);
      prim_b(side == 0 ? in.WL : in.WR, s, gam, sb, side == 0 ? inb.WL : inb.WR);
    }
  }
}

// Adjoint of the 2D nodal solver with all outputs (gks_node<double, 2, true>).
FDK_HD void gks_node_b(const Consts& k, const double* W, const double* Wx, const double* Wy, const double* Fb_in,
                       const double* Ftb_in, const double* Gb_in, const double* Gtb_in, double* Wb, double* Wxb,
                       double* Wyb) {
  const double K = k.K, iKd = k.inv_Kd;
  const Prim<double> s = prim<double, 2>(W, k.gamma);
  Mom<double> m;
  mom_common<double, 2>(s, K, m);
  mom_full(s, m);
  double a[4], b[4], A[4], dx[4], dy[4], dA[4], tr[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) { dx[i] = Wx[i] * s.irho; dy[i] = Wy[i] * s.irho; }
  slope<double, 2>(s, K, iKd, dx, a);
  slope<double, 2>(s, K, iKd, dy, b);
  {
    double x[4], y[4];
    ma<1, 0>(a, m, x);
    ma<0, 1>(b, m, y);
#pragma unroll
    for (int i = 0; i < 4; ++i) { tr[i] = x[i] + y[i]; dA[i] = -tr[i]; }
  }
  slope<double, 2>(s, K, iKd, dA, A);
  const bool visc = k.mu > 0;
  const double tauN = visc ? k.mu / s.p : 0.0;
  double Fu[4], Gv[4], u0[4], v0[4], xa[4], yb[4], xb[4], zb[4];
  ma<1, 0>(A, m, Fu);
  ma<0, 1>(A, m, Gv);
  muv<1, 0, 0>(m, u0);
  muv<0, 1, 0>(m, v0);
  if (visc) {
    ma<2, 0>(a, m, xa);
    ma<1, 1>(b, m, yb);
    ma<1, 1>(a, m, xb);
    ma<0, 2>(b, m, zb);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      u0[i] -= tauN * (xa[i] + yb[i] + Fu[i]);
      v0[i] -= tauN * (xb[i] + zb[i] + Gv[i]);
    }
  }
  double Fv[4], Gvv[4], Ftv[4], Gtv[4];  // values before the Prandtl correction
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    Fv[i] = s.rho * u0[i]; Gvv[i] = s.rho * v0[i]; Ftv[i] = s.rho * Fu[i]; Gtv[i] = s.rho * Gv[i];
  }
  double Fb[4], Ftb[4], Gb[4], Gtb[4], trb[4] = {0, 0, 0, 0};
  PrimB sb = primb_zero();
#pragma unroll
  for (int i = 0; i < 4; ++i) { Fb[i] = Fb_in[i]; Ftb[i] = Ftb_in[i]; Gb[i] = Gb_in[i]; Gtb[i] = Gtb_in[i]; }
  if (visc) {
    const double U = s.U, V = s.V, f = k.prfix;
    const double ax = 1.5 * U * U + 0.5 * V * V, ay = 1.5 * V * V + 0.5 * U * U;
    const double bx = 0.5 * U * (U * U + V * V), by = 0.5 * V * (U * U + V * V);
    double Wt[4], Wtb[4] = {0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < 4; ++i) Wt[i] = -s.rho * tr[i];
    const double qxb = f * Fb[3], qyb = f * Gb[3], qxtb = f * Ftb[3], qytb = f * Gtb[3];
    sb.U += qxb * (-Fv[1] + 3.0 * U * Fv[0] - W[3] + V * W[2] - 0.5 * (3.0 * U * U + V * V) * W[0]) +
            qyb * (-Gvv[1] + U * Gvv[0] + V * W[1] - U * V * W[0]) +
            qxtb * (-Ftv[1] + 3.0 * U * Ftv[0] - Wt[3] + V * Wt[2] - 0.5 * (3.0 * U * U + V * V) * Wt[0]) +
            qytb * (-Gtv[1] + U * Gtv[0] + V * Wt[1] - U * V * Wt[0]);
    sb.V += qxb * (-Fv[2] + V * Fv[0] + U * W[2] - U * V * W[0]) +
            qyb * (-Gvv[2] + 3.0 * V * Gvv[0] - W[3] + U * W[1] - 0.5 * (U * U + 3.0 * V * V) * W[0]) +
            qxtb * (-Ftv[2] + V * Ftv[0] + U * Wt[2] - U * V * Wt[0]) +
            qytb * (-Gtv[2] + 3.0 * V * Gtv[0] - Wt[3] + U * Wt[1] - 0.5 * (U * U + 3.0 * V * V) * Wt[0]);
    Fb[3] += qxb; Fb[1] += -U * qxb; Fb[2] += -V * qxb; Fb[0] += ax * qxb;
    Wb[3] += -U * qxb; Wb[2] += U * V * qxb; Wb[0] += -bx * qxb;
    Gb[3] += qyb; Gb[2] += -V * qyb; Gb[1] += -U * qyb; Gb[0] += ay * qyb;
    Wb[3] += -V * qyb; Wb[1] += U * V * qyb; Wb[0] += -by * qyb;
    Ftb[3] += qxtb; Ftb[1] += -U * qxtb; Ftb[2] += -V * qxtb; Ftb[0] += ax * qxtb;
    Wtb[3] += -U * qxtb; Wtb[2] += U * V * qxtb; Wtb[0] += -bx * qxtb;
    Gtb[3] += qytb; Gtb[2] += -V * qytb; Gtb[1] += -U * qytb; Gtb[0] += ay * qytb;
    Wtb[3] += -V * qytb; Wtb[1] += U * V * qytb; Wtb[0] += -by * qytb;
#pragma unroll
    for (int i = 0; i < 4; ++i) {  // Wt = -rho tr
      trb[i] += -s.rho * Wtb[i];
      sb.rho += -tr[i] * Wtb[i];
    }
  }
  Mom<double> mb;
  mom_zero(mb);
  double u0b[4], v0b[4], Fub[4], Gvb[4], Ab[4] = {0, 0, 0, 0}, abv[4] = {0, 0, 0, 0}, bbv[4] = {0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < 4; ++i) {  // F = rho u0, G = rho v0, Ft = rho Fu, Gt = rho Gv
    u0b[i] = s.rho * Fb[i];
    v0b[i] = s.rho * Gb[i];
    Fub[i] = s.rho * Ftb[i];
    Gvb[i] = s.rho * Gtb[i];
    sb.rho += u0[i] * Fb[i] + v0[i] * Gb[i] + Fu[i] * Ftb[i] + Gv[i] * Gtb[i];
  }
  if (visc) {
    double tauNb = 0.0, xab[4], xbb[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      tauNb += -(xa[i] + yb[i] + Fu[i]) * u0b[i] - (xb[i] + zb[i] + Gv[i]) * v0b[i];
      xab[i] = -tauN * u0b[i];
      xbb[i] = -tauN * v0b[i];
      Fub[i] += xab[i];
      Gvb[i] += xbb[i];
    }
    ma_b<2, 0>(a, m, xab, abv, mb);
    ma_b<1, 1>(b, m, xab, bbv, mb);
    ma_b<1, 1>(a, m, xbb, abv, mb);
    ma_b<0, 2>(b, m, xbb, bbv, mb);
    sb.p += -k.mu / (s.p * s.p) * tauNb;
  }
  muv_b<1, 0, 0>(m, u0b, mb);
  muv_b<0, 1, 0>(m, v0b, mb);
  ma_b<1, 0>(A, m, Fub, Ab, mb);
  ma_b<0, 1>(A, m, Gvb, Ab, mb);
  double dAb[4] = {0, 0, 0, 0};
  slope_b(s, K, iKd, dA, A, Ab, dAb, sb);
#pragma unroll
  for (int i = 0; i < 4; ++i) trb[i] -= dAb[i];
  ma_b<1, 0>(a, m, trb, abv, mb);
  ma_b<0, 1>(b, m, trb, bbv, mb);
  double dxb[4] = {0, 0, 0, 0}, dyb[4] = {0, 0, 0, 0};
  slope_b(s, K, iKd, dy, b, bbv, dyb, sb);
  slope_b(s, K, iKd, dx, a, abv, dxb, sb);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    Wxb[i] += dxb[i] * s.irho;
    Wyb[i] += dyb[i] * s.irho;
    sb.irho += Wx[i] * dxb[i] + Wy[i] * dyb[i];
  }
  mom_full_b(s, m, mb, sb);
  mom_common_b(s, K, m, mb, sb);
  prim_b(W, s, k.gamma, sb, Wb);
}

#pragma clang fp contract(on)

// ------------------------------------------------------------------ GENO
struct GenoIn {
  double IS1, IS2, IS3, q1, q2, q3, dq1, dq2, dq3, PH, PHx;
};

// Adjoint of geno() for outputs v, d, chi with adjoints vb, db, chib.
FDK_HD void geno_b(const Consts& k, const GenoIn& g, double d1, double d2, double d3, double vb, double db,
                   double chib, GenoIn& gb) {
  const double X = (g.IS2 + g.IS3) - 2.0 * g.IS1;
  const double tau = 0.5 * fabs(X);
  const double in23 = g.IS3 > g.IS2 ? g.IS3 : g.IS2;
  const int iH = in23 > g.IS1 ? (g.IS3 > g.IS2 ? 3 : 2) : 1;
  const double ISH = in23 > g.IS1 ? in23 : g.IS1;
  const double ln23 = g.IS3 < g.IS2 ? g.IS3 : g.IS2;
  const int iL = ln23 < g.IS1 ? (g.IS3 < g.IS2 ? 3 : 2) : 1;
  const double ISL = ln23 < g.IS1 ? ln23 : g.IS1;
  const double eH = ISH + k.eps, eL = ISL + k.eps;
  const double inv = 1.0 / (eH * eL);
  const double xH = tau * eL * inv, xL = tau * eH * inv;
  const double aH = 1.0 + ipow(xH, k.r), aL = 1.0 + ipow(xL, k.r);
  const double alpha = 2.0 * aH / (aH + aL);
  const double th = g_tanh(k.C * alpha);
  const double chi = th * k.inv_tanhC;
  if (th == 1.0 && chi == 1.0) {  // as in the forward: v = PH, d = PHx, d chi / d alpha = 0
    gb.PH += vb;
    gb.PHx += db;
    return;
  }
  const double t1 = sqr(g.IS1 + k.eps_a), t2 = sqr(g.IS2 + k.eps_a), t3 = sqr(g.IS3 + k.eps_a);
  const double w1 = d1 * t2 * t3, w2 = d2 * t1 * t3, w3 = d3 * t1 * t2;
  const double is = 1.0 / (w1 + w2 + w3);
  const double N = w1 * g.q1 + w2 * g.q2 + w3 * g.q3, Nx = w1 * g.dq1 + w2 * g.dq2 + w3 * g.dq3;
  const double PL = N * is, PLx = Nx * is;
  // v = chi PH + (1-chi) PL, d = chi PHx + (1-chi) PLx
  const double chit = chib + (g.PH - PL) * vb + (g.PHx - PLx) * db;
  gb.PH += chi * vb;
  gb.PHx += chi * db;
  const double PLb = (1.0 - chi) * vb, PLxb = (1.0 - chi) * db;
  gb.q1 += w1 * is * PLb; gb.q2 += w2 * is * PLb; gb.q3 += w3 * is * PLb;
  gb.dq1 += w1 * is * PLxb; gb.dq2 += w2 * is * PLxb; gb.dq3 += w3 * is * PLxb;
  const double isb = N * PLb + Nx * PLxb;
  const double Sb = -is * is * isb;
  const double w1b = (g.q1 * PLb + g.dq1 * PLxb) * is + Sb;
  const double w2b = (g.q2 * PLb + g.dq2 * PLxb) * is + Sb;
  const double w3b = (g.q3 * PLb + g.dq3 * PLxb) * is + Sb;
  const double t1b = d2 * t3 * w2b + d3 * t2 * w3b;
  const double t2b = d1 * t3 * w1b + d3 * t1 * w3b;
  const double t3b = d1 * t2 * w1b + d2 * t1 * w2b;
  gb.IS1 += 2.0 * (g.IS1 + k.eps_a) * t1b;
  gb.IS2 += 2.0 * (g.IS2 + k.eps_a) * t2b;
  gb.IS3 += 2.0 * (g.IS3 + k.eps_a) * t3b;
  // chi = tanh(C alpha) / tanh C
  const double alphab = k.inv_tanhC * k.C * (1.0 - th * th) * chit;
  const double den = aH + aL;
  const double aHb = alphab * 2.0 * aL / (den * den), aLb = -alphab * 2.0 * aH / (den * den);
  const double xHb = aHb * (k.r == 1 ? 1.0 : k.r * ipow(xH, k.r - 1));
  const double xLb = aLb * (k.r == 1 ? 1.0 : k.r * ipow(xL, k.r - 1));
  // xH = tau / eH, xL = tau / eL
  const double taub = xHb * eL * inv + xLb * eH * inv;
  const double ISHb = -xHb * xH / eH, ISLb = -xLb * xL / eL;
  if (iH == 1) gb.IS1 += ISHb; else if (iH == 2) gb.IS2 += ISHb; else gb.IS3 += ISHb;
  if (iL == 1) gb.IS1 += ISLb; else if (iL == 2) gb.IS2 += ISLb; else gb.IS3 += ISLb;
  const double Xb = 0.5 * (X > 0 ? 1.0 : (X < 0 ? -1.0 : 0.0)) * taub;
  gb.IS2 += Xb;
  gb.IS3 += Xb;
  gb.IS1 += -2.0 * Xb;
}

// Adjoint of recon_iface (one component): rb = adjoints of (vl, dl, cl, vr,
// dr, cr).  Adds into qb[4], xb[4].
FDK_HD void recon_iface_b(const Consts& k, const double q[4], const double x[4], double h, double invh,
                          const double rb[6], double qb[4], double xb[4]) {
  double PHlb = 0.0, PHrb = 0.0, PHxb = 0.0;
  const double q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3];
  if (k.variant == 2) {
    PHlb = rb[0];
    PHrb = rb[3];
    PHxb = rb[1] + rb[4];
  } else {
    const double hx0 = h * x[0], hx3 = h * x[3];
    const double s2 = q0 - 2.0 * q1 + q2, s3 = q1 - 2.0 * q2 + q3;
    const double D2 = s2 * s2, D3 = s3 * s3;
    const double dmid = (q2 - q1) * invh;
    const double qc = (-q0 + 6.0 * q1 + 3.0 * q2) * 0.125;
    const double PHl = ((7.0 * q0 + 35.0 * q1 + 21.0 * q2 + q3) + (x[0] + 22.0 * x[1] - 7.0 * x[2]) * h) * (1.0 / 64.0);
    const double PHr = ((q0 + 21.0 * q1 + 35.0 * q2 + 7.0 * q3) + (7.0 * x[1] - 22.0 * x[2] - x[3]) * h) * (1.0 / 64.0);
    const double PHx = -((q0 + 45.0 * q1 - 45.0 * q2 - q3) + 9.0 * (x[1] + x[2]) * h) * (invh * (1.0 / 30.0));
    const double Al = q1 - q0 - hx0, Bl = 2.0 * (q1 - q0) - hx0, El = 3.0 * q1 - 4.0 * q2 + q3;
    const double Ar = q2 - q3 + hx3, Br = 2.0 * (q3 - q2) - hx3, Er = 3.0 * q2 - 4.0 * q1 + q0;
    GenoIn L{(13.0 / 3.0) * Al * Al + Bl * Bl, (13.0 / 12.0) * D2 + 0.25 * sqr(q2 - q0),
             (13.0 / 12.0) * D3 + 0.25 * El * El, (-5.0 * q0 + 9.0 * q1 - 3.0 * hx0) * 0.25, qc,
             (3.0 * q1 + 6.0 * q2 - q3) * 0.125, (-3.0 * q0 + 3.0 * q1 - 2.0 * hx0) * invh, dmid, dmid, PHl, PHx};
    GenoIn R{(13.0 / 3.0) * Ar * Ar + Br * Br, (13.0 / 12.0) * D3 + 0.25 * sqr(q3 - q1),
             (13.0 / 12.0) * D2 + 0.25 * Er * Er, (-5.0 * q3 + 9.0 * q2 + 3.0 * hx3) * 0.25,
             (-q3 + 6.0 * q2 + 3.0 * q1) * 0.125, qc, (-3.0 * q2 + 3.0 * q3 - 2.0 * hx3) * invh, dmid, dmid, PHr, PHx};
    GenoIn Lb{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}, Rb{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    geno_b(k, L, k.ds, k.dc, k.ds, rb[0], rb[1], rb[2], Lb);
    geno_b(k, R, k.ds, k.dc, k.ds, rb[3], rb[4], rb[5], Rb);
    PHlb = Lb.PH;
    PHrb = Rb.PH;
    PHxb = Lb.PHx + Rb.PHx;
    double hx0b = 0.0, hx3b = 0.0, D2b = 0.0, D3b = 0.0;
    const double qcb = Lb.q2 + Rb.q3, dmidb = Lb.dq2 + Lb.dq3 + Rb.dq2 + Rb.dq3;
    // right side
    qb[2] += -3.0 * invh * Rb.dq1; qb[3] += 3.0 * invh * Rb.dq1; hx3b += -2.0 * invh * Rb.dq1;
    qb[3] += -0.125 * Rb.q2; qb[2] += 0.75 * Rb.q2; qb[1] += 0.375 * Rb.q2;
    qb[3] += -1.25 * Rb.q1; qb[2] += 2.25 * Rb.q1; hx3b += 0.75 * Rb.q1;
    {
      D2b += (13.0 / 12.0) * Rb.IS3;
      const double Eb = 0.5 * Er * Rb.IS3;
      qb[2] += 3.0 * Eb; qb[1] += -4.0 * Eb; qb[0] += Eb;
      D3b += (13.0 / 12.0) * Rb.IS2;
      const double t = 0.5 * (q3 - q1) * Rb.IS2;
      qb[3] += t; qb[1] -= t;
      const double Ab = (26.0 / 3.0) * Ar * Rb.IS1, Bb = 2.0 * Br * Rb.IS1;
      qb[2] += Ab - 2.0 * Bb; qb[3] += -Ab + 2.0 * Bb; hx3b += Ab - Bb;
    }
    // left side
    qb[0] += -3.0 * invh * Lb.dq1; qb[1] += 3.0 * invh * Lb.dq1; hx0b += -2.0 * invh * Lb.dq1;
    qb[1] += 0.375 * Lb.q3; qb[2] += 0.75 * Lb.q3; qb[3] += -0.125 * Lb.q3;
    qb[0] += -1.25 * Lb.q1; qb[1] += 2.25 * Lb.q1; hx0b += -0.75 * Lb.q1;
    {
      D3b += (13.0 / 12.0) * Lb.IS3;
      const double Eb = 0.5 * El * Lb.IS3;
      qb[1] += 3.0 * Eb; qb[2] += -4.0 * Eb; qb[3] += Eb;
      D2b += (13.0 / 12.0) * Lb.IS2;
      const double t = 0.5 * (q2 - q0) * Lb.IS2;
      qb[2] += t; qb[0] -= t;
      const double Ab = (26.0 / 3.0) * Al * Lb.IS1, Bb = 2.0 * Bl * Lb.IS1;
      qb[1] += Ab + 2.0 * Bb; qb[0] += -Ab - 2.0 * Bb; hx0b += -Ab - Bb;
    }
    // shared
    qb[0] += -0.125 * qcb; qb[1] += 0.75 * qcb; qb[2] += 0.375 * qcb;
    qb[2] += invh * dmidb; qb[1] -= invh * dmidb;
    const double s3b = 2.0 * s3 * D3b, s2b = 2.0 * s2 * D2b;
    qb[1] += s3b; qb[2] += -2.0 * s3b; qb[3] += s3b;
    qb[0] += s2b; qb[1] += -2.0 * s2b; qb[2] += s2b;
    xb[0] += h * hx0b;
    xb[3] += h * hx3b;
  }
  const double c = 1.0 / 64.0, kx = -invh * (1.0 / 30.0);
  qb[0] += 7.0 * c * PHlb + c * PHrb + kx * PHxb;
  qb[1] += 35.0 * c * PHlb + 21.0 * c * PHrb + 45.0 * kx * PHxb;
  qb[2] += 21.0 * c * PHlb + 35.0 * c * PHrb - 45.0 * kx * PHxb;
  qb[3] += c * PHlb + 7.0 * c * PHrb - kx * PHxb;
  xb[0] += h * c * PHlb;
  xb[1] += 22.0 * h * c * PHlb + 7.0 * h * c * PHrb + 9.0 * h * kx * PHxb;
  xb[2] += -7.0 * h * c * PHlb - 22.0 * h * c * PHrb + 9.0 * h * kx * PHxb;
  xb[3] += -h * c * PHrb;
}

// Adjoint of recon_node: db is the adjoint of the node derivative.  Adds into
// qb[3], xb[3].
FDK_HD void recon_node_b(const Consts& k, const double q[3], const double x[3], double h, double invh, double db,
                         double qb[3], double xb[3]) {
  double PHxb = db;
  if (k.variant != 2) {
    const double q0 = q[0], q1 = q[1], q2 = q[2];
    const double hx0 = h * x[0], hx2 = h * x[2];
    const double PHx = (9.0 * (q0 - q2) + h * (x[0] + 46.0 * x[1] + x[2])) * (invh * (1.0 / 30.0));
    const double A1 = q1 - q0 - hx0, B1 = 2.0 * (q1 - q0) - hx0;
    const double A2 = q2 - q1 - hx2, B2 = 2.0 * (q2 - q1) - hx2;
    const double s = q0 - 2.0 * q1 + q2, u = q2 - q0;
    const double IS1 = (13.0 / 3.0) * A1 * A1 + B1 * B1;
    const double IS2 = (13.0 / 3.0) * A2 * A2 + B2 * B2;
    const double IS3 = (13.0 / 12.0) * s * s + 0.25 * u * u;
    GenoIn g{IS3, IS1, IS2, q1, q1, q1, (q2 - q0) * (0.5 * invh), (-2.0 * q0 + 2.0 * q1 - hx0) * invh,
             (-2.0 * q1 + 2.0 * q2 - hx2) * invh, q1, PHx};
    GenoIn gb{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    geno_b(k, g, k.dc, k.ds, k.ds, 0.0, db, 0.0, gb);
    PHxb = gb.PHx;
    double hx0b = 0.0, hx2b = 0.0;
    qb[1] += gb.q1 + gb.q2 + gb.q3 + gb.PH;
    qb[2] += 0.5 * invh * gb.dq1;
    qb[0] -= 0.5 * invh * gb.dq1;
    qb[0] += -2.0 * invh * gb.dq2; qb[1] += 2.0 * invh * gb.dq2; hx0b += -invh * gb.dq2;
    qb[1] += -2.0 * invh * gb.dq3; qb[2] += 2.0 * invh * gb.dq3; hx2b += -invh * gb.dq3;
    {
      const double sb = (13.0 / 6.0) * s * gb.IS1, ub = 0.5 * u * gb.IS1;
      qb[0] += sb - ub; qb[1] += -2.0 * sb; qb[2] += sb + ub;
      const double Ab2 = (26.0 / 3.0) * A2 * gb.IS3, Bb2 = 2.0 * B2 * gb.IS3;
      qb[2] += Ab2 + 2.0 * Bb2; qb[1] += -Ab2 - 2.0 * Bb2; hx2b += -Ab2 - Bb2;
      const double Ab1 = (26.0 / 3.0) * A1 * gb.IS2, Bb1 = 2.0 * B1 * gb.IS2;
      qb[1] += Ab1 + 2.0 * Bb1; qb[0] += -Ab1 - 2.0 * Bb1; hx0b += -Ab1 - Bb1;
    }
    xb[0] += h * hx0b;
    xb[2] += h * hx2b;
  }
  const double kx = invh * (1.0 / 30.0);
  qb[0] += 9.0 * kx * PHxb;
  qb[2] += -9.0 * kx * PHxb;
  xb[0] += h * kx * PHxb;
  xb[1] += 46.0 * h * kx * PHxb;
  xb[2] += h * kx * PHxb;
}

// ---------------------------------------------- characteristic variables
// Reverse of the 2D characteristic reconstructions (recon_iface_char<2>,
// recon_node_char<2> in gks_device.hpp): the frame (eigenvectors at the mean
// interface state, or at the node) depends on the line's values, so its
// adjoint flows back into them as well.
struct FrameB {
  double u, v, c, ic, H, b1, b2, k2;
};
FDK_HD FrameB frameb_zero() { return FrameB{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0}; }

// q = L(f) w: adds L^T qb to wb and the frame's adjoint to fb.
FDK_HD void to_char_b(const CharFrame& f, const double* w, const double* qb, double* wb, FrameB& fb) {
  const double ab = 0.5 * (qb[0] + qb[3]) - qb[1];  // a = b2 w0 + s
  const double mb = 0.5 * (qb[3] - qb[0]);           // m = ic w1 - u ic w0
  const double sb = ab;                               // s = b1 (w3 - u w1 - v w2)
  wb[0] += qb[1] - f.v * qb[2] + f.b2 * ab - f.u * f.ic * mb;
  wb[1] += f.ic * mb - f.u * f.b1 * sb;
  wb[2] += qb[2] - f.v * f.b1 * sb;
  wb[3] += f.b1 * sb;
  fb.b2 += w[0] * ab;
  fb.b1 += (w[3] - f.u * w[1] - f.v * w[2]) * sb;
  fb.ic += (w[1] - f.u * w[0]) * mb;
  fb.u += -f.ic * w[0] * mb - f.b1 * w[1] * sb;
  fb.v += -w[0] * qb[2] - f.b1 * w[2] * sb;
}

// w = R(f) q: adds R^T wb to qb and the frame's adjoint to fb.
FDK_HD void from_char_b(const CharFrame& f, const double* q, const double* wb, double* qb, FrameB& fb) {
  const double lo = q[0], en = q[1], sh = q[2], hi = q[3], sum = lo + en + hi, d = hi - lo;
  const double sb = wb[0] + f.u * wb[1] + f.v * wb[2];
  qb[0] += sb - f.c * wb[1] + (f.H - f.u * f.c) * wb[3];
  qb[1] += sb + f.k2 * wb[3];
  qb[2] += wb[2] + f.v * wb[3];
  qb[3] += sb + f.c * wb[1] + (f.H + f.u * f.c) * wb[3];
  fb.u += sum * wb[1] + f.c * d * wb[3];
  fb.v += sum * wb[2] + sh * wb[3];
  fb.c += d * wb[1] + f.u * d * wb[3];
  fb.H += (lo + hi) * wb[3];
  fb.k2 += en * wb[3];
}

// The frame from the state W: adds the adjoint of W.
FDK_HD void char_frame_b(double gamma, const double* W, const CharFrame& f, FrameB fb, double* Wb) {
  const double ir = 1.0 / W[0], gm = gamma - 1.0;
  const double p = gm * (W[3] - W[0] * f.k2), c2 = f.c * f.c;
  fb.b1 += f.k2 * fb.b2;  // b2 = b1 k2
  fb.k2 += f.b1 * fb.b2;
  double c2b = -gm / (c2 * c2) * fb.b1;                 // b1 = (gamma - 1) / c2
  fb.c += -fb.ic / c2;                                  // ic = 1 / c
  c2b += fb.c / (2.0 * f.c);                            // c = sqrt(c2)
  double pb = ir * fb.H + gamma * ir * c2b;             // H = (W3 + p) ir, c2 = gamma p ir
  double irb = (W[3] + p) * fb.H + gamma * p * c2b;
  Wb[3] += ir * fb.H + gm * pb;                         // p = (gamma - 1)(W3 - W0 k2)
  Wb[0] += -gm * f.k2 * pb;
  fb.k2 += -gm * W[0] * pb;
  fb.u += f.u * fb.k2;                                  // k2 = (u^2 + v^2) / 2
  fb.v += f.v * fb.k2;
  Wb[1] += ir * fb.u;                                   // u = W1 ir, v = W2 ir
  Wb[2] += ir * fb.v;
  irb += W[1] * fb.u + W[2] * fb.v;
  Wb[0] += -ir * ir * irb;                              // ir = 1 / W0
}

// Reverse of recon_iface_char<2>.  rb[c]: adjoints of rec[c].vl, dl, vr, dr
// (local frame); chib: adjoint of chi.  Adds into Qb, Xb.  chi's adjoint goes
// to the first of chi^l(u-c), chi^r(u-c), chi^l(u+c), chi^r(u+c) that attains
// the minimum.
FDK_HD void recon_iface_char_b(const Consts& k, const double (&Q)[4][4], const double (&X)[4][4], double h,
                               double invh, const double (&rb)[4][4], double chib, double (&Qb)[4][4],
                               double (&Xb)[4][4]) {
  double Wm[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) Wm[c] = 0.5 * (Q[c][1] + Q[c][2]);
  const CharFrame f = char_frame<2>(k.gamma, Wm);
  double qc[4][4], xc[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    double a[4], b[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) a[c] = Q[c][m];
    to_char<2>(f, a, b);
#pragma unroll
    for (int c = 0; c < 4; ++c) { qc[c][m] = b[c]; a[c] = X[c][m]; }
    to_char<2>(f, a, b);
#pragma unroll
    for (int c = 0; c < 4; ++c) xc[c][m] = b[c];
  }
  IfaceRec cr[4];
#pragma unroll
  for (int c = 0; c < 4; ++c)
    cr[c] = recon_iface<double>(k, qc[c][0], qc[c][1], qc[c][2], qc[c][3], xc[c][0], xc[c][1], xc[c][2], xc[c][3],
                                h, invh);
  // adjoints of the characteristic results (vl, dl, cl, vr, dr, cr per field)
  double crb[4][6];
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int t = 0; t < 6; ++t) crb[c][t] = 0.0;
  FrameB fb = frameb_zero();
#pragma unroll
  for (int slot = 0; slot < 4; ++slot) {  // vl, dl, vr, dr
    const int t = slot < 2 ? slot : slot + 1;
    double a[4], wb[4], ab[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      a[c] = t == 0 ? cr[c].vl : (t == 1 ? cr[c].dl : (t == 3 ? cr[c].vr : cr[c].dr));
      wb[c] = rb[c][slot];
    }
    from_char_b(f, a, wb, ab, fb);
#pragma unroll
    for (int c = 0; c < 4; ++c) crb[c][t] += ab[c];
  }
  {
    const double cand[4] = {cr[0].cl, cr[0].cr, cr[3].cl, cr[3].cr};
    int sel = 0;
#pragma unroll
    for (int a = 1; a < 4; ++a)
      if (cand[a] < cand[sel]) sel = a;
    crb[sel < 2 ? 0 : 3][sel % 2 == 0 ? 2 : 5] += chib;
  }
  double qcb[4][4], xcb[4][4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
#pragma unroll
    for (int m = 0; m < 4; ++m) { qcb[c][m] = 0.0; xcb[c][m] = 0.0; }
    recon_iface_b(k, qc[c], xc[c], h, invh, crb[c], qcb[c], xcb[c]);
  }
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    double a[4], b[4], wb[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < 4; ++c) { a[c] = Q[c][m]; b[c] = qcb[c][m]; }
    to_char_b(f, a, b, wb, fb);
#pragma unroll
    for (int c = 0; c < 4; ++c) { Qb[c][m] += wb[c]; wb[c] = 0.0; a[c] = X[c][m]; b[c] = xcb[c][m]; }
    to_char_b(f, a, b, wb, fb);
#pragma unroll
    for (int c = 0; c < 4; ++c) Xb[c][m] += wb[c];
  }
  double Wmb[4] = {0.0, 0.0, 0.0, 0.0};
  char_frame_b(k.gamma, Wm, f, fb, Wmb);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    Qb[c][1] += 0.5 * Wmb[c];
    Qb[c][2] += 0.5 * Wmb[c];
  }
}

// Reverse of recon_node_char<2>: db = adjoint of the node derivative d (local
// frame).  Adds into Qb, Xb.
FDK_HD void recon_node_char_b(const Consts& k, const double (&Q)[4][3], const double (&X)[4][3], double h,
                              double invh, const double (&db)[4], double (&Qb)[4][3], double (&Xb)[4][3]) {
  double Wc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) Wc[c] = Q[c][1];
  const CharFrame f = char_frame<2>(k.gamma, Wc);
  double qc[4][3], xc[4][3];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    double a[4], b[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) a[c] = Q[c][m];
    to_char<2>(f, a, b);
#pragma unroll
    for (int c = 0; c < 4; ++c) { qc[c][m] = b[c]; a[c] = X[c][m]; }
    to_char<2>(f, a, b);
#pragma unroll
    for (int c = 0; c < 4; ++c) xc[c][m] = b[c];
  }
  double dc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c)
    dc[c] = recon_node<double>(k, qc[c][0], qc[c][1], qc[c][2], xc[c][0], xc[c][1], xc[c][2], h, invh);
  FrameB fb = frameb_zero();
  double dcb[4] = {0.0, 0.0, 0.0, 0.0};
  from_char_b(f, dc, db, dcb, fb);
  double qcb[4][3], xcb[4][3];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
#pragma unroll
    for (int m = 0; m < 3; ++m) { qcb[c][m] = 0.0; xcb[c][m] = 0.0; }
    recon_node_b(k, qc[c], xc[c], h, invh, dcb[c], qcb[c], xcb[c]);
  }
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    double a[4], b[4], wb[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < 4; ++c) { a[c] = Q[c][m]; b[c] = qcb[c][m]; }
    to_char_b(f, a, b, wb, fb);
#pragma unroll
    for (int c = 0; c < 4; ++c) { Qb[c][m] += wb[c]; wb[c] = 0.0; a[c] = X[c][m]; b[c] = xcb[c][m]; }
    to_char_b(f, a, b, wb, fb);
#pragma unroll
    for (int c = 0; c < 4; ++c) Xb[c][m] += wb[c];
  }
  double Wcb[4] = {0.0, 0.0, 0.0, 0.0};
  char_frame_b(k.gamma, Wc, f, fb, Wcb);
#pragma unroll
  for (int c = 0; c < 4; ++c) Qb[c][1] += Wcb[c];
}

}  // namespace fdk
