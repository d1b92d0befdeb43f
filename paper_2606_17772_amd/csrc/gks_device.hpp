// Device arithmetic of the FD-CGKS stage for gfx950: compact GENO
// reconstruction and the space-time coupled BGK gas-kinetic solver.
//
// Straight-line FP64 code (FP32 optional for the gas-kinetic part), fully
// inlined so that every moment index is a compile-time constant and all
// moment tables live in VGPRs.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

// Everything here is also host-callable, so that host-side checks can run the
// same arithmetic.
#define FDK_HD __host__ __device__ __forceinline__

namespace fdk {

// Scheme constants, passed by value to every kernel.
struct Consts {
  double gamma;
  double K;           // internal degrees of freedom: (4-2g)/(g-1) in 2D, (3-g)/(g-1) in 1D
  double inv_Kd;      // 1/(K+2) in 2D, 1/(K+1) in 1D
  double mu;          // dynamic viscosity (0: Euler)
  double prfix;       // 1/Pr - 1 (applied when mu > 0)
  double C, inv_tanhC, eps, eps_a, dc, ds;  // GENO (Sec. 3.2, App. D)
  double tau_c1, tau_c2;
  int r;              // GENO exponent
  int variant;        // 0: (6-4), 1: (6-2), 2: linear
  int grad_carried;
  int flux_order;     // 6, or 8: the linear compact flux over the wider stencil
};

// ---------------------------------------------------------------- math
FDK_HD double m_erfc(double x) { return erfc(x); }
FDK_HD float m_erfc(float x) { return erfcf(x); }
FDK_HD double m_exp(double x) { return exp(x); }
FDK_HD float m_exp(float x) { return expf(x); }
FDK_HD double m_sqrt(double x) { return sqrt(x); }
FDK_HD float m_sqrt(float x) { return sqrtf(x); }
FDK_HD double m_abs(double x) { return fabs(x); }
FDK_HD float m_abs(float x) { return fabsf(x); }

template <class T> FDK_HD T sqr(T a) { return a * a; }

template <class T> FDK_HD T ipow(T x, int r) {
  T y = x;
  for (int k = 1; k < r; ++k) y = y * x;
  return y;
}

// scalar helpers (ties keep the first argument)
FDK_HD double g_abs(double a) { return fabs(a); }
FDK_HD double g_max(double a, double b) { return fmax(a, b); }
FDK_HD double g_min(double a, double b) { return fmin(a, b); }
// tanh; beyond |a| = 19.5 it rounds to +-1 in FP64 (1 - tanh(a) < 2.3e-17,
// under half an ulp of 1), so the library call is skipped there.
FDK_HD double g_tanh(double a) { return a > 19.5 ? 1.0 : (a < -19.5 ? -1.0 : tanh(a)); }
FDK_HD double val(double a) { return a; }
FDK_HD float val(float a) { return a; }

// ----------------------------------------------------- GENO, Sec. 3 / App. C
// Path function and blend of one side.  IS1 is the IS^tau reference;
// d1, d2, d3 the ideal weights; q/dq the sub-stencil value/derivative
// candidates; PH/PHx the high-order ones.  Normalised low-order weights are
// d_k / t_k^2 (t_k = IS_k + eps_a) scaled by t1^2 t2^2 t3^2, so one division
// normalises them.
template <class R> struct GenoOutT {
  R v, d, chi;
};
template <class R>
FDK_HD GenoOutT<R> geno(const Consts& k, R IS1, R IS2, R IS3, double d1, double d2, double d3,
                                            R q1, R q2, R q3, R dq1, R dq2, R dq3, R PH, R PHx) {
  R tau = 0.5 * g_abs((IS2 + IS3) - 2.0 * IS1);
  R ISH = g_max(IS1, g_max(IS2, IS3));
  R ISL = g_min(IS1, g_min(IS2, IS3));
  R eH = ISH + k.eps, eL = ISL + k.eps;
  GenoOutT<R> o;
  // Smooth data decided before any division.  With A = eH^r + tau^r and
  // B = eL^r + tau^r, alpha below equals 2 A eL^r / (A eL^r + B eH^r).  Where
  // C alpha >= 19.5 (1 + 1e-12) in that division-free form (rounding moves it
  // by a few 1e-16), the alpha computed below gives C alpha > 19.5, tanh is 1,
  // and with 1/tanh(C) = 1 the value returned is the one of the shortcut
  // further down.  Other points (and inf / NaN / underflowed products) take
  // the full path.
  if (k.inv_tanhC == 1.0) {
    R pH = eH, pL = eL, pt = tau;
    for (int q = 1; q < k.r; ++q) {
      pH = pH * eH;
      pL = pL * eL;
      pt = pt * tau;
    }
    R a = (pH + pt) * pL, b = (pL + pt) * pH;
    R lhs = (2.0 * k.C) * a, rhs = (19.5 * (1.0 + 1e-12)) * (a + b);
    if (val(rhs) >= 1e-290 && val(lhs) <= 1e300 && val(lhs) >= val(rhs)) {
      o.v = PH;
      o.d = PHx;
      o.chi = R(1.0);
      return o;
    }
  }
  R inv = 1.0 / (eH * eL);
  R xH = tau * eL * inv, xL = tau * eH * inv;
  R aH = 1.0 + ipow(xH, k.r), aL = 1.0 + ipow(xL, k.r);
  R alpha = 2.0 * aH / (aH + aL);
  R th = g_tanh(k.C * alpha);
  R chi = th * k.inv_tanhC;
  // Smooth data: tanh saturates (its derivative is 0) and chi = 1 exactly, so
  // the low-order blend has weight 0 in the value and in every derivative.
  if (val(th) == 1.0 && val(chi) == 1.0) {
    o.v = PH;
    o.d = PHx;
    o.chi = chi;
    return o;
  }
  R t1 = sqr(IS1 + k.eps_a), t2 = sqr(IS2 + k.eps_a), t3 = sqr(IS3 + k.eps_a);
  R w1 = d1 * t2 * t3, w2 = d2 * t1 * t3, w3 = d3 * t1 * t2;
  R is = 1.0 / (w1 + w2 + w3);
  R PL = (w1 * q1 + w2 * q2 + w3 * q3) * is;
  R PLx = (w1 * dq1 + w2 * dq2 + w3 * dq3) * is;
  o.v = chi * PH + (1.0 - chi) * PL;
  o.d = chi * PHx + (1.0 - chi) * PLx;
  o.chi = chi;
  return o;
}

// Interface m+1/2 of a line q0..q3 = Q_{m-1..m+2}, x0..x3 = averaged
// derivatives (Eq. 7th-compact-recons; App. C1, C2).
template <class R> struct IfaceRecT {
  R vl, dl, cl, vr, dr, cr;
};
using IfaceRec = IfaceRecT<double>;
template <class R>
FDK_HD IfaceRecT<R> recon_iface(const Consts& k, R q0, R q1, R q2, R q3, R x0, R x1, R x2, R x3,
                                                    double h, double invh) {
  IfaceRecT<R> o;
  R PHl = ((7.0 * q0 + 35.0 * q1 + 21.0 * q2 + q3) + (x0 + 22.0 * x1 - 7.0 * x2) * h) * (1.0 / 64.0);
  R PHr = ((q0 + 21.0 * q1 + 35.0 * q2 + 7.0 * q3) + (7.0 * x1 - 22.0 * x2 - x3) * h) * (1.0 / 64.0);
  R PHx = -((q0 + 45.0 * q1 - 45.0 * q2 - q3) + 9.0 * (x1 + x2) * h) * (invh * (1.0 / 30.0));
  if (k.variant == 2) {
    o.vl = PHl; o.dl = PHx; o.cl = R(1.0);
    o.vr = PHr; o.dr = PHx; o.cr = R(1.0);
    return o;
  }
  R hx0 = h * x0, hx3 = h * x3;
  R D2 = sqr(q0 - 2.0 * q1 + q2), D3 = sqr(q1 - 2.0 * q2 + q3);
  R dmid = (q2 - q1) * invh;
  R qc = (-q0 + 6.0 * q1 + 3.0 * q2) * 0.125;  // q_2^l == q_3^r
  // left (App. C1)
  R ISl1 = (13.0 / 3.0) * sqr(q1 - q0 - hx0) + sqr(2.0 * (q1 - q0) - hx0);
  R ISl2 = (13.0 / 12.0) * D2 + 0.25 * sqr(q2 - q0);
  R ISl3 = (13.0 / 12.0) * D3 + 0.25 * sqr(3.0 * q1 - 4.0 * q2 + q3);
  R ql1 = (-5.0 * q0 + 9.0 * q1 - 3.0 * hx0) * 0.25;
  R ql3 = (3.0 * q1 + 6.0 * q2 - q3) * 0.125;
  R dl1 = (-3.0 * q0 + 3.0 * q1 - 2.0 * hx0) * invh;
  GenoOutT<R> L = geno<R>(k, ISl1, ISl2, ISl3, k.ds, k.dc, k.ds, ql1, qc, ql3, dl1, dmid, dmid, PHl, PHx);
  // right (App. C2)
  R ISr1 = (13.0 / 3.0) * sqr(q2 - q3 + hx3) + sqr(2.0 * (q3 - q2) - hx3);
  R ISr2 = (13.0 / 12.0) * D3 + 0.25 * sqr(q3 - q1);
  R ISr3 = (13.0 / 12.0) * D2 + 0.25 * sqr(3.0 * q2 - 4.0 * q1 + q0);
  R qr1 = (-5.0 * q3 + 9.0 * q2 + 3.0 * hx3) * 0.25;
  R qr2 = (-q3 + 6.0 * q2 + 3.0 * q1) * 0.125;
  R dr1 = (-3.0 * q2 + 3.0 * q3 - 2.0 * hx3) * invh;
  GenoOutT<R> Rr = geno<R>(k, ISr1, ISr2, ISr3, k.ds, k.dc, k.ds, qr1, qr2, qc, dr1, dmid, dmid, PHr, PHx);
  o.vl = L.v; o.dl = L.d; o.cl = L.chi;
  o.vr = Rr.v; o.dr = Rr.d; o.cr = Rr.chi;
  return o;
}

// Node derivative from q0..q2 = Q_{j-1..j+1}, x0..x2 (Eq. 6th-compact-recons,
// App. C3; the central sub-stencil is the IS^tau reference with weight dc).
template <class R>
FDK_HD R recon_node(const Consts& k, R q0, R q1, R q2, R x0, R x1, R x2, double h, double invh) {
  R PHx = (9.0 * (q0 - q2) + h * (x0 + 46.0 * x1 + x2)) * (invh * (1.0 / 30.0));
  if (k.variant == 2) return PHx;
  R hx0 = h * x0, hx2 = h * x2;
  R IS1 = (13.0 / 3.0) * sqr(q1 - q0 - hx0) + sqr(2.0 * (q1 - q0) - hx0);
  R IS2 = (13.0 / 3.0) * sqr(q2 - q1 - hx2) + sqr(2.0 * (q2 - q1) - hx2);
  R IS3 = (13.0 / 12.0) * sqr(q0 - 2.0 * q1 + q2) + 0.25 * sqr(q2 - q0);
  R dq1 = (-2.0 * q0 + 2.0 * q1 - hx0) * invh;
  R dq2 = (-2.0 * q1 + 2.0 * q2 - hx2) * invh;
  R dq3 = (q2 - q0) * (0.5 * invh);
  GenoOutT<R> o = geno<R>(k, IS3, IS1, IS2, k.dc, k.ds, k.ds, q1, q1, q1, dq3, dq1, dq2, q1, PHx);
  return o.d;
}

// ------------------------------------- characteristic variables (Sec. 3)
// Eigenvectors of the Euler flux Jacobian along a line, in the line's local
// frame (component 1 is the momentum along the line), at a state W.  The
// columns of R are the fields u - c, u, [shears,] u + c, normalised as
// (1, u - c, [v, w,] H - u c), (1, u, [v, w,] |u|^2/2), [(0, 0, 1, 0, v),
// (0, 0, 0, 1, w),] (1, u + c, [v, w,] H + u c) (2D: no w); L = R^-1 in
// closed form with b1 = (gamma-1)/c^2 and b2 = b1 |u|^2 / 2.  The map is linear, so values and derivatives
// transform with the same matrices.  Nothing here is contracted into fused
// multiply-adds, in particular not with the callers' arithmetic: otherwise
// which products fuse would depend on the kernel the code is inlined into,
// and the path function (very sensitive to the last bit of the
// characteristic values on smooth data) would differ between kernels.
struct CharFrame {
  double u, v, c, ic, H, b1, b2, k2;  // k2 = |u|^2 / 2
  double w;                            // 3D only
};
template <int DIM> FDK_HD CharFrame char_frame(double gamma, const double* W) {
#pragma clang fp contract(off)
  CharFrame f;
  const double ir = 1.0 / W[0];
  f.u = W[1] * ir;
  f.v = DIM >= 2 ? W[2] * ir : 0.0;
  f.w = DIM == 3 ? W[3] * ir : 0.0;
  if (DIM == 3) f.k2 = 0.5 * (f.u * f.u + f.v * f.v + f.w * f.w);
  else f.k2 = 0.5 * (f.u * f.u + f.v * f.v);
  const double p = (gamma - 1.0) * (W[DIM + 1] - W[0] * f.k2);
  const double c2 = gamma * p * ir;
  f.c = sqrt(c2);
  f.ic = 1.0 / f.c;
  f.H = (W[DIM + 1] + p) * ir;
  f.b1 = (gamma - 1.0) / c2;
  f.b2 = f.b1 * f.k2;
  return f;
}
// q = L w
template <int DIM> FDK_HD void to_char(const CharFrame& f, const double* w, double* q) {
#pragma clang fp contract(off)
  const double uc = f.u * f.ic;
  double s;  // b1 (E - u m - v n [- w o])
  if (DIM == 3) s = f.b1 * (w[4] - f.u * w[1] - f.v * w[2] - f.w * w[3]);
  else s = f.b1 * (w[DIM + 1] - f.u * w[1] - (DIM == 2 ? f.v * w[2] : 0.0));
  const double a = f.b2 * w[0] + s;  // b2 rho + s
  const double m = f.ic * w[1] - uc * w[0];  // (m - u rho) / c
  q[0] = 0.5 * (a - m);
  q[1] = w[0] - a;
  if (DIM >= 2) q[2] = w[2] - f.v * w[0];
  if (DIM == 3) q[3] = w[3] - f.w * w[0];
  q[DIM + 1] = 0.5 * (a + m);
}
// w = R q
template <int DIM> FDK_HD void from_char(const CharFrame& f, const double* q, double* w) {
#pragma clang fp contract(off)
  const double lo = q[0], en = q[1], hi = q[DIM + 1];
  const double sh = DIM >= 2 ? q[2] : 0.0;
  const double sw = DIM == 3 ? q[3] : 0.0;
  const double s = lo + en + hi;
  w[0] = s;
  w[1] = f.u * s + f.c * (hi - lo);
  if (DIM >= 2) w[2] = f.v * s + sh;
  if (DIM == 3) {
    w[3] = f.w * s + sw;
    w[4] = f.H * (lo + hi) + f.u * f.c * (hi - lo) + f.k2 * en + f.v * sh + f.w * sw;
  } else {
    w[DIM + 1] = f.H * (lo + hi) + f.u * f.c * (hi - lo) + f.k2 * en + f.v * sh;
  }
}

// Interface reconstruction of a whole line of N = DIM + 2 components on
// characteristic variables.  Q[c][m], X[c][m]: values and averaged
// derivatives in the local frame at the nodes m = 0..3 around the interface;
// the eigenvectors are taken at the mean of the two interface-adjacent
// states.  rec[c] receives the local-frame results; chi is the smallest of
// the left and right path functions of the u - c and u + c fields.
template <int DIM>
FDK_HD void recon_iface_char(const Consts& k, const double (&Q)[DIM + 2][4], const double (&X)[DIM + 2][4], double h,
                             double invh, IfaceRec (&rec)[DIM + 2], double& chi) {
  constexpr int N = DIM + 2;
  double Wm[N];
  {
#pragma clang fp contract(off)
#pragma unroll
    for (int c = 0; c < N; ++c) Wm[c] = 0.5 * (Q[c][1] + Q[c][2]);
  }
  const CharFrame f = char_frame<DIM>(k.gamma, Wm);
  double qc[N][4], xc[N][4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    double a[N], b[N];
#pragma unroll
    for (int c = 0; c < N; ++c) a[c] = Q[c][m];
    to_char<DIM>(f, a, b);
#pragma unroll
    for (int c = 0; c < N; ++c) { qc[c][m] = b[c]; a[c] = X[c][m]; }
    to_char<DIM>(f, a, b);
#pragma unroll
    for (int c = 0; c < N; ++c) xc[c][m] = b[c];
  }
  IfaceRec cr[N];
#pragma unroll
  for (int c = 0; c < N; ++c)
    cr[c] = recon_iface<double>(k, qc[c][0], qc[c][1], qc[c][2], qc[c][3], xc[c][0], xc[c][1], xc[c][2], xc[c][3],
                                h, invh);
  chi = fmin(fmin(cr[0].cl, cr[0].cr), fmin(cr[N - 1].cl, cr[N - 1].cr));
  double a[N], b[N];
#pragma unroll
  for (int c = 0; c < N; ++c) a[c] = cr[c].vl;
  from_char<DIM>(f, a, b);
#pragma unroll
  for (int c = 0; c < N; ++c) { rec[c].vl = b[c]; a[c] = cr[c].dl; }
  from_char<DIM>(f, a, b);
#pragma unroll
  for (int c = 0; c < N; ++c) { rec[c].dl = b[c]; a[c] = cr[c].vr; }
  from_char<DIM>(f, a, b);
#pragma unroll
  for (int c = 0; c < N; ++c) { rec[c].vr = b[c]; a[c] = cr[c].dr; }
  from_char<DIM>(f, a, b);
#pragma unroll
  for (int c = 0; c < N; ++c) {
    rec[c].dr = b[c];
    rec[c].cl = rec[c].cr = chi;
  }
}

// Node derivatives of a whole line on characteristic variables: Q[c][m],
// X[c][m] at the nodes j-1, j, j+1 (local frame); eigenvectors at the
// node's own state.
template <int DIM>
FDK_HD void recon_node_char(const Consts& k, const double (&Q)[DIM + 2][3], const double (&X)[DIM + 2][3], double h,
                            double invh, double (&d)[DIM + 2]) {
  constexpr int N = DIM + 2;
  double Wc[N];
#pragma unroll
  for (int c = 0; c < N; ++c) Wc[c] = Q[c][1];
  const CharFrame f = char_frame<DIM>(k.gamma, Wc);
  double qc[N][3], xc[N][3];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    double a[N], b[N];
#pragma unroll
    for (int c = 0; c < N; ++c) a[c] = Q[c][m];
    to_char<DIM>(f, a, b);
#pragma unroll
    for (int c = 0; c < N; ++c) { qc[c][m] = b[c]; a[c] = X[c][m]; }
    to_char<DIM>(f, a, b);
#pragma unroll
    for (int c = 0; c < N; ++c) xc[c][m] = b[c];
  }
  double dc[N];
#pragma unroll
  for (int c = 0; c < N; ++c)
    dc[c] = recon_node<double>(k, qc[c][0], qc[c][1], qc[c][2], xc[c][0], xc[c][1], xc[c][2], h, invh);
  from_char<DIM>(f, dc, d);
}

// ------------------------------------------- Maxwellian moments (App. A)
// Per unit density: mu[n] = <u^n> (full or half line), mv[n] = <v^n>,
// x2 = <xi^2>, x4 = <xi^4>.
template <class FT> struct Mom {
  FT mu[7];
  FT mv[7];
  FT x2, x4;
};

template <class FT> FDK_HD void mu_rec(FT* m, FT U, FT i2l) {
#pragma unroll
  for (int n = 0; n < 5; ++n) m[n + 2] = U * m[n + 1] + FT(n + 1) * i2l * m[n];
}

// <u^P v^Q xi^(2R) psi>, psi = (1, u, v, (u^2+v^2+xi^2)/2), R in {0, 1}
template <int P, int Q, int R, class FT> FDK_HD void muv(const Mom<FT>& m, FT o[4]) {
  const FT xr = R == 0 ? FT(1) : m.x2;
  const FT xr1 = R == 0 ? m.x2 : m.x4;
  FT b = m.mu[P] * m.mv[Q];
  o[0] = b * xr;
  o[1] = m.mu[P + 1] * m.mv[Q] * xr;
  o[2] = m.mu[P] * m.mv[Q + 1] * xr;
  o[3] = FT(0.5) * ((m.mu[P + 2] * m.mv[Q] + m.mu[P] * m.mv[Q + 2]) * xr + b * xr1);
}
// <(s.psi) u^P v^Q psi>.  With g = s.psi = s0 + s1 u + s2 v + h3 (u^2 + v^2 +
// xi^2), h3 = s3 / 2, a moment of g splits into a u part and a v part:
//   <g u^a v^b> = mv[b] cu(a) + mu[a] cv(b),
//   cu(a) = (s0 + h3 x2) mu[a] + s1 mu[a+1] + h3 mu[a+2],  cv(b) = s2 mv[b+1] + h3 mv[b+2],
// and <g u^a v^b xi^2> = x2 <g u^a v^b> + h3 mu[a] mv[b] (x4 - x2^2): six
// one-dimensional combinations instead of the six moment vectors of psi.
template <int P, int Q, class FT> FDK_HD void ma(const FT s[4], const Mom<FT>& m, FT o[4]) {
  const FT h3 = FT(0.5) * s[3];
  const FT c0 = s[0] + h3 * m.x2;
  const FT u0 = c0 * m.mu[P] + s[1] * m.mu[P + 1] + h3 * m.mu[P + 2];
  const FT u1 = c0 * m.mu[P + 1] + s[1] * m.mu[P + 2] + h3 * m.mu[P + 3];
  const FT u2 = c0 * m.mu[P + 2] + s[1] * m.mu[P + 3] + h3 * m.mu[P + 4];
  const FT v0 = s[2] * m.mv[Q + 1] + h3 * m.mv[Q + 2];
  const FT v1 = s[2] * m.mv[Q + 2] + h3 * m.mv[Q + 3];
  const FT v2 = s[2] * m.mv[Q + 3] + h3 * m.mv[Q + 4];
  o[0] = m.mv[Q] * u0 + m.mu[P] * v0;
  o[1] = m.mv[Q] * u1 + m.mu[P + 1] * v0;
  o[2] = m.mv[Q + 1] * u0 + m.mu[P] * v1;
  const FT gx = m.x2 * o[0] + h3 * (m.mu[P] * m.mv[Q]) * (m.x4 - m.x2 * m.x2);
  o[3] = FT(0.5) * ((m.mv[Q] * u2 + m.mu[P + 2] * v0) + (m.mv[Q + 2] * u0 + m.mu[P] * v2) + gx);
}
// 1D: psi = (1, u, (u^2+xi^2)/2)
template <int P, int R, class FT> FDK_HD void mu1(const Mom<FT>& m, FT o[3]) {
  const FT xr = R == 0 ? FT(1) : m.x2;
  const FT xr1 = R == 0 ? m.x2 : m.x4;
  o[0] = m.mu[P] * xr;
  o[1] = m.mu[P + 1] * xr;
  o[2] = FT(0.5) * (m.mu[P + 2] * xr + m.mu[P] * xr1);
}
template <int P, class FT> FDK_HD void ma1(const FT s[3], const Mom<FT>& m, FT o[3]) {
  FT t0[3], t1[3], t2[3], t3[3];
  mu1<P, 0>(m, t0);
  mu1<P + 1, 0>(m, t1);
  mu1<P + 2, 0>(m, t2);
  mu1<P, 1>(m, t3);
  FT h2 = FT(0.5) * s[2];
#pragma unroll
  for (int i = 0; i < 3; ++i) o[i] = s[0] * t0[i] + s[1] * t1[i] + h2 * (t2[i] + t3[i]);
}

// Primitive variables and the shared v / xi moments of a state.
template <class FT> struct Prim {
  FT rho, irho, U, V, p, lam, i2l, ip;  // ip = 1/p
};
template <class FT, int DIM> FDK_HD Prim<FT> prim(const FT* W, FT gamma) {
  Prim<FT> s;
  s.rho = W[0];
  s.irho = FT(1) / W[0];
  s.U = W[1] * s.irho;
  s.V = DIM == 2 ? W[2] * s.irho : FT(0);
  FT rE = W[DIM + 1];
  s.p = (gamma - FT(1)) * (rE - FT(0.5) * s.rho * (s.U * s.U + s.V * s.V));
  s.i2l = s.p * s.irho;          // 1/(2 lambda) = p/rho
  s.ip = FT(1) / s.p;            // lambda = rho/(2p); 1/p also serves the collision time
  s.lam = FT(0.5) * s.rho * s.ip;
  return s;
}
template <class FT, int DIM> FDK_HD void mom_common(const Prim<FT>& s, FT K, Mom<FT>& m) {
  m.mv[0] = FT(1);
  m.mv[1] = s.V;
  if (DIM == 2) mu_rec(m.mv, s.V, s.i2l);
  m.x2 = K * s.i2l;
  m.x4 = m.x2 * (K + FT(2)) * s.i2l;
}
template <class FT> FDK_HD void mom_full(const Prim<FT>& s, Mom<FT>& m) {
  m.mu[0] = FT(1);
  m.mu[1] = s.U;
  mu_rec(m.mu, s.U, s.i2l);
}
// half line: sgn = +1 (u > 0) or -1 (u < 0)
template <class FT> FDK_HD void mom_half(const Prim<FT>& s, FT sgn, Mom<FT>& m) {
  FT sl = m_sqrt(s.lam);
  m.mu[0] = FT(0.5) * m_erfc(-sgn * sl * s.U);
  // 1/(2 sqrt(pi lambda)) = (1/(2 lambda)) sqrt(lambda) / sqrt(pi): no second square root
  m.mu[1] = s.U * m.mu[0] + sgn * m_exp(-s.lam * s.U * s.U) * (s.i2l * sl) * FT(0.56418958354775628695);
  mu_rec(m.mu, s.U, s.i2l);
}

// Micro slope s with <psi (s.psi)> = d (d per unit density): closed-form
// solution of the moment system.
template <class FT, int DIM>
FDK_HD void slope(const Prim<FT>& q, FT K, FT iKd, const FT* d, FT* s) {
  if (DIM == 2) {
    FT e = q.U * q.U + q.V * q.V + (K + FT(2)) * q.i2l;
    FT B = FT(2) * d[3] - e * d[0];
    FT A = d[1] - q.U * d[0];
    FT Cc = d[2] - q.V * d[0];
    FT tl = FT(2) * q.lam;
    s[3] = tl * tl * iKd * (B - FT(2) * q.U * A - FT(2) * q.V * Cc);
    s[2] = tl * Cc - q.V * s[3];
    s[1] = tl * A - q.U * s[3];
    s[0] = d[0] - q.U * s[1] - q.V * s[2] - FT(0.5) * s[3] * e;
  } else {
    FT e = q.U * q.U + (K + FT(1)) * q.i2l;
    FT B = FT(2) * d[2] - e * d[0];
    FT A = d[1] - q.U * d[0];
    FT tl = FT(2) * q.lam;
    s[2] = tl * tl * iKd * (B - FT(2) * q.U * A);
    s[1] = tl * A - q.U * s[2];
    s[0] = d[0] - q.U * s[1] - FT(0.5) * s[2] * e;
  }
}

// Integrated BGK time coefficients over [0, T] (equilibrium, its space and
// time slope terms, non-equilibrium initial part, its slope term) and the
// f^n / f_t^n fit of App. A1 from T = dt/2 and T = dt.
template <class FT> struct TimeCoef {
  FT c[5], ct[5], e1;  // e1 = exp(-dt/tau)
};
template <class FT> FDK_HD TimeCoef<FT> time_coef(FT dt, FT tau) {
  TimeCoef<FT> r;
  // tau = 0 (p_l = p_r without a c1 term): the tau -> 0+ limit, exp(-T/tau) = 0
  FT Eh = val(tau) > 0 ? m_exp(-FT(0.5) * dt / tau) : FT(0);
  FT Ef = Eh * Eh;
  FT Th = FT(0.5) * dt, Tf = dt;
  FT qh[5], qf[5];
  qh[0] = Th - tau * (FT(1) - Eh);
  qf[0] = Tf - tau * (FT(1) - Ef);
  qh[1] = tau * ((FT(2) * tau - Th) - (Th + FT(2) * tau) * Eh);
  qf[1] = tau * ((FT(2) * tau - Tf) - (Tf + FT(2) * tau) * Ef);
  qh[2] = FT(0.5) * Th * Th - tau * Th + tau * tau * (FT(1) - Eh);
  qf[2] = FT(0.5) * Tf * Tf - tau * Tf + tau * tau * (FT(1) - Ef);
  qh[3] = tau * (FT(1) - Eh);
  qf[3] = tau * (FT(1) - Ef);
  qh[4] = tau * ((Th + FT(2) * tau) * Eh - FT(2) * tau);
  qf[4] = tau * ((Tf + FT(2) * tau) * Ef - FT(2) * tau);
  FT idt = FT(1) / dt;
  FT idt2 = FT(4) * idt * idt;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    r.c[k] = (FT(4) * qh[k] - qf[k]) * idt;
    r.ct[k] = (qf[k] - FT(2) * qh[k]) * idt2;
  }
  r.e1 = Ef;
  return r;
}

// ----------------------------------------- gas-kinetic interface solver
// Local frame: the normal velocity is component 1 (u).  2D: W = (rho, rho u,
// rho v, rho E), tangential slope Wt; 1D: W = (rho, rho u, rho E).
// Outputs: flux F, its time derivative Ft, and the interface values
// W-hat^{l,r} and their time derivatives (Eq. W-model).  VALUES = false skips
// F and W-hat (stage 2 uses only the time derivatives).
template <class FT, int DIM> struct GksIO {
  FT WL[DIM + 2], WR[DIM + 2], nL[DIM + 2], nR[DIM + 2], Wt[DIM + 2];
  FT F[DIM + 2], Ft[DIM + 2], Wl[DIM + 2], Wr[DIM + 2], Wlt[DIM + 2], Wrt[DIM + 2];
};

// Moments of the transport and time-slope terms of one state:
// tr = <psi ((a.psi) u + (b.psi) v)>, tru = <u psi (...)>, Ap = <psi A.psi>,
// Au = <u psi A.psi> (2D; 1D drops the v terms).
template <class FT, int DIM>
FDK_HD void transport(const FT* a, const FT* b, const Mom<FT>& m, FT* tr, FT* tru) {
  if (DIM == 2) {
    FT x[4], y[4];
    ma<1, 0>(a, m, x); ma<0, 1>(b, m, y);
#pragma unroll
    for (int i = 0; i < 4; ++i) tr[i] = x[i] + y[i];
    ma<2, 0>(a, m, x); ma<1, 1>(b, m, y);
#pragma unroll
    for (int i = 0; i < 4; ++i) tru[i] = x[i] + y[i];
  } else {
    ma1<1>(a, m, tr);
    ma1<2>(a, m, tru);
  }
}
template <class FT, int DIM> FDK_HD void tslope(const FT* A, const Mom<FT>& m, FT* Ap, FT* Au) {
  if (DIM == 2) { ma<0, 0>(A, m, Ap); ma<1, 0>(A, m, Au); }
  else { ma1<0>(A, m, Ap); ma1<1>(A, m, Au); }
}
// <psi> and <u psi> of a (half or full) state
template <class FT, int DIM> FDK_HD void psi_moms(const Mom<FT>& m, FT* p, FT* u) {
  if (DIM == 2) {
    p[0] = m.mu[0]; p[1] = m.mu[1]; p[2] = m.mu[0] * m.mv[1];
    p[3] = FT(0.5) * (m.mu[2] + m.mu[0] * (m.mv[2] + m.x2));
    muv<1, 0, 0>(m, u);
  } else {
    p[0] = m.mu[0]; p[1] = m.mu[1]; p[2] = FT(0.5) * (m.mu[2] + m.mu[0] * m.x2);
    mu1<1, 0>(m, u);
  }
}

// The contribution of one side s to the moments of f^n and f_t^n:
// rho_s <phi [c3 (1 - tau A.psi) + c4 ((a.psi) u + (b.psi) v)]> over the half
// line of s, for phi = psi (We, Wet) and u psi (F, Ft); also the one-sided
// Euler time derivative Wt = -rho_s <psi (...)> over the full line.
template <class FT, int DIM, bool VALUES>
FDK_HD void side_terms(const Prim<FT>& s, const Mom<FT>& h, const FT* n, const FT* t, FT K,
                                           FT iKd, FT tau, const TimeCoef<FT>& tc, bool both, FT* F, FT* Ft, FT* We,
                                           FT* Wet, FT* Wt) {
  constexpr int N = DIM + 2;
  Mom<FT> f = h;
  mom_full(s, f);
  FT a[N], b[N], A[N], d[N], tf[N], tuf[N];
#pragma unroll
  for (int i = 0; i < N; ++i) d[i] = n[i] * s.irho;
  slope<FT, DIM>(s, K, iKd, d, a);
  if (DIM == 2) {
#pragma unroll
    for (int i = 0; i < N; ++i) d[i] = t[i] * s.irho;
    slope<FT, DIM>(s, K, iKd, d, b);
  }
  if (DIM == 2) { FT x[N], y[N]; ma<1, 0>(a, f, x); ma<0, 1>(b, f, y); for (int i = 0; i < N; ++i) tf[i] = x[i] + y[i]; }
  else ma1<1>(a, f, tf);
#pragma unroll
  for (int i = 0; i < N; ++i) { d[i] = -tf[i]; Wt[i] = -s.rho * tf[i]; }
  slope<FT, DIM>(s, K, iKd, d, A);
  FT ph[N], uh[N], tp[N], tu[N], Ap[N], Au[N];
  psi_moms<FT, DIM>(h, ph, uh);
  transport<FT, DIM>(a, b, h, tp, tu);
  tslope<FT, DIM>(A, h, Ap, Au);
  (void)tuf;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    FT nu = uh[i] - tau * Au[i], np = ph[i] - tau * Ap[i];
    Ft[i] += s.rho * (tc.ct[3] * nu + tc.ct[4] * tu[i]);
    Wet[i] += s.rho * (tc.ct[3] * np + tc.ct[4] * tp[i]);
    if (both) {
      F[i] += s.rho * (tc.c[3] * nu + tc.c[4] * tu[i]);
      We[i] += s.rho * (tc.c[3] * np + tc.c[4] * tp[i]);
    }
  }
}

template <class FT, int DIM, bool VALUES>
FDK_HD void gks_iface(const Consts& k, FT dt, GksIO<FT, DIM>& io) {
  constexpr int N = DIM + 2;
  const FT K = FT(k.K), gam = FT(k.gamma), iKd = FT(k.inv_Kd);
  const bool both = VALUES || k.mu > 0;  // F and We are needed for the values or the Prandtl fix
  Prim<FT> sL = prim<FT, DIM>(io.WL, gam), sR = prim<FT, DIM>(io.WR, gam);
  // half-line moments and the compatibility state W0
  Mom<FT> hL, hR;
  mom_common<FT, DIM>(sL, K, hL);
  mom_half(sL, FT(1), hL);
  mom_common<FT, DIM>(sR, K, hR);
  mom_half(sR, FT(-1), hR);
  FT W0[N];
  {
    FT pL[N], pR[N], u[N];
    psi_moms<FT, DIM>(hL, pL, u);
    psi_moms<FT, DIM>(hR, pR, u);
#pragma unroll
    for (int i = 0; i < N; ++i) W0[i] = sL.rho * pL[i] + sR.rho * pR[i];
  }
  Prim<FT> s0 = prim<FT, DIM>(W0, gam);
  // collision time and time coefficients
  FT tau = (k.mu > 0 ? FT(k.mu) * s0.ip : FT(k.tau_c1) * dt) +
           FT(k.tau_c2) * dt * m_abs(sL.p - sR.p) / (sL.p + sR.p);
  TimeCoef<FT> tc = time_coef(dt, tau);
  FT F[N], We[N], Wet[N], WtL[N], WtR[N];
#pragma unroll
  for (int i = 0; i < N; ++i) { F[i] = FT(0); io.Ft[i] = FT(0); We[i] = FT(0); Wet[i] = FT(0); }
  // non-equilibrium initial parts of both sides
  side_terms<FT, DIM, VALUES>(sL, hL, io.nL, io.Wt, K, iKd, tau, tc, both, F, io.Ft, We, Wet, WtL);
  side_terms<FT, DIM, VALUES>(sR, hR, io.nR, io.Wt, K, iKd, tau, tc, both, F, io.Ft, We, Wet, WtR);
  // equilibrium part: g0 with slopes from the averaged normal slope (D12) and
  // the tangential slope, time slope from compatibility
  {
    Mom<FT> m0;
    mom_common<FT, DIM>(s0, K, m0);
    mom_full(s0, m0);
    FT a0[N], b0[N], A0[N], d[N], t0[N], tu0[N], Ap0[N], Au0[N], p0[N], u0[N];
#pragma unroll
    for (int i = 0; i < N; ++i) d[i] = FT(0.5) * (io.nL[i] + io.nR[i]) * s0.irho;
    slope<FT, DIM>(s0, K, iKd, d, a0);
    if (DIM == 2) {
#pragma unroll
      for (int i = 0; i < N; ++i) d[i] = io.Wt[i] * s0.irho;
      slope<FT, DIM>(s0, K, iKd, d, b0);
    }
    transport<FT, DIM>(a0, b0, m0, t0, tu0);
#pragma unroll
    for (int i = 0; i < N; ++i) d[i] = -t0[i];
    slope<FT, DIM>(s0, K, iKd, d, A0);
    tslope<FT, DIM>(A0, m0, Ap0, Au0);
    psi_moms<FT, DIM>(m0, p0, u0);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      io.Ft[i] += s0.rho * (tc.ct[0] * u0[i] + tc.ct[1] * tu0[i] + tc.ct[2] * Au0[i]);
      Wet[i] += s0.rho * (tc.ct[0] * p0[i] + tc.ct[1] * t0[i] + tc.ct[2] * Ap0[i]);
      if (both) {
        F[i] += s0.rho * (tc.c[0] * u0[i] + tc.c[1] * tu0[i] + tc.c[2] * Au0[i]);
        We[i] += s0.rho * (tc.c[0] * p0[i] + tc.c[1] * t0[i] + tc.c[2] * Ap0[i]);
      }
    }
  }
  // Prandtl-number correction of the energy flux: (1/Pr - 1) times the heat
  // flux 1/2 <(u-U0)((u-U0)^2 + (v-V0)^2 + xi^2)> of the same distribution,
  // written with the moments of psi and u psi.
  if (k.mu > 0) {
    FT U = s0.U, V = s0.V, f = FT(k.prfix);
    if (DIM == 2) {
      FT a = FT(1.5) * U * U + FT(0.5) * V * V, b = FT(0.5) * U * (U * U + V * V);
      FT q = F[3] - U * F[1] - V * F[2] + a * F[0] - U * We[3] + U * V * We[2] - b * We[0];
      FT qt = io.Ft[3] - U * io.Ft[1] - V * io.Ft[2] + a * io.Ft[0] - U * Wet[3] + U * V * Wet[2] - b * Wet[0];
      F[3] += f * q;
      io.Ft[3] += f * qt;
    } else {
      FT a = FT(1.5) * U * U, b = FT(0.5) * U * U * U;
      FT q = F[2] - U * F[1] + a * F[0] - U * We[2] - b * We[0];
      FT qt = io.Ft[2] - U * io.Ft[1] + a * io.Ft[0] - U * Wet[2] - b * Wet[0];
      F[2] += f * q;
      io.Ft[2] += f * qt;
    }
  }
  // interface values (Eq. W-model) with the one-sided Euler time derivatives
  FT e = tc.e1, oe = FT(1) - tc.e1;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    io.Wlt[i] = oe * Wet[i] + e * WtL[i];
    io.Wrt[i] = oe * Wet[i] + e * WtR[i];
    if (VALUES) {
      io.F[i] = F[i];
      io.Wl[i] = oe * We[i] + e * io.WL[i];
      io.Wr[i] = oe * We[i] + e * io.WR[i];
    }
  }
}

// ------------------------------------------------ smooth nodal solver
// f^n = g [1 - tauN ((a.psi) u + (b.psi) v + A.psi)], f_t = (A.psi) g.
// Outputs x-flux F, Ft and (2D) y-flux G, Gt.  VALUES = false: F, G skipped.
template <class FT, int DIM, bool VALUES>
FDK_HD void gks_node(const Consts& k, const FT* W, const FT* Wx, const FT* Wy, FT* F, FT* Ft,
                                         FT* G, FT* Gt) {
  constexpr int N = DIM + 2;
  const FT K = FT(k.K), iKd = FT(k.inv_Kd);
  Prim<FT> s = prim<FT, DIM>(W, FT(k.gamma));
  Mom<FT> m;
  mom_common<FT, DIM>(s, K, m);
  mom_full(s, m);
  FT a[N], b[N], A[N], d[N], tr[N];
#pragma unroll
  for (int i = 0; i < N; ++i) d[i] = Wx[i] * s.irho;
  slope<FT, DIM>(s, K, iKd, d, a);
  if (DIM == 2) {
#pragma unroll
    for (int i = 0; i < N; ++i) d[i] = Wy[i] * s.irho;
    slope<FT, DIM>(s, K, iKd, d, b);
    FT x[N], y[N];
    ma<1, 0>(a, m, x); ma<0, 1>(b, m, y);
    for (int i = 0; i < N; ++i) tr[i] = x[i] + y[i];
  } else {
    ma1<1>(a, m, tr);
  }
#pragma unroll
  for (int i = 0; i < N; ++i) d[i] = -tr[i];
  slope<FT, DIM>(s, K, iKd, d, A);
  FT tauN = k.mu > 0 ? FT(k.mu) * s.ip : FT(0);
  const bool visc = k.mu > 0;
  FT Fu[N], Gv[N];
  if (DIM == 2) {
    FT x[N], y[N], z[N];
    ma<1, 0>(A, m, Fu);
    ma<0, 1>(A, m, Gv);
#pragma unroll
    for (int i = 0; i < N; ++i) { Ft[i] = s.rho * Fu[i]; Gt[i] = s.rho * Gv[i]; }
    if (VALUES || visc) {
      FT u0[N], v0[N];
      muv<1, 0, 0>(m, u0);
      muv<0, 1, 0>(m, v0);
      if (visc) {
        ma<2, 0>(a, m, x); ma<1, 1>(b, m, y);
        for (int i = 0; i < N; ++i) u0[i] -= tauN * (x[i] + y[i] + Fu[i]);
        ma<1, 1>(a, m, x); ma<0, 2>(b, m, z);
        for (int i = 0; i < N; ++i) v0[i] -= tauN * (x[i] + z[i] + Gv[i]);
      }
#pragma unroll
      for (int i = 0; i < N; ++i) { F[i] = s.rho * u0[i]; G[i] = s.rho * v0[i]; }
    }
    if (visc) {  // Prandtl correction with the node's velocity; W^e = W, W^e_t = -rho tr
      FT U = s.U, V = s.V, f = FT(k.prfix);
      FT ax = FT(1.5) * U * U + FT(0.5) * V * V, ay = FT(1.5) * V * V + FT(0.5) * U * U;
      FT bx = FT(0.5) * U * (U * U + V * V), by = FT(0.5) * V * (U * U + V * V);
      FT Wt0 = -s.rho * tr[0], Wt1 = -s.rho * tr[1], Wt2 = -s.rho * tr[2], Wt3 = -s.rho * tr[3];
      FT qx = F[3] - U * F[1] - V * F[2] + ax * F[0] - U * W[3] + U * V * W[2] - bx * W[0];
      FT qy = G[3] - V * G[2] - U * G[1] + ay * G[0] - V * W[3] + U * V * W[1] - by * W[0];
      FT qxt = Ft[3] - U * Ft[1] - V * Ft[2] + ax * Ft[0] - U * Wt3 + U * V * Wt2 - bx * Wt0;
      FT qyt = Gt[3] - V * Gt[2] - U * Gt[1] + ay * Gt[0] - V * Wt3 + U * V * Wt1 - by * Wt0;
      F[3] += f * qx; G[3] += f * qy; Ft[3] += f * qxt; Gt[3] += f * qyt;
    }
  } else {
    ma1<1>(A, m, Fu);
#pragma unroll
    for (int i = 0; i < N; ++i) Ft[i] = s.rho * Fu[i];
    if (VALUES || visc) {
      FT u0[N];
      mu1<1, 0>(m, u0);
      if (visc) {
        FT x[N];
        ma1<2>(a, m, x);
        for (int i = 0; i < N; ++i) u0[i] -= tauN * (x[i] + Fu[i]);
      }
#pragma unroll
      for (int i = 0; i < N; ++i) F[i] = s.rho * u0[i];
    }
    if (visc) {
      FT U = s.U, f = FT(k.prfix);
      FT a1 = FT(1.5) * U * U, b1 = FT(0.5) * U * U * U;
      FT Wt0 = -s.rho * tr[0], Wt2 = -s.rho * tr[2];
      FT q = F[2] - U * F[1] + a1 * F[0] - U * W[2] - b1 * W[0];
      FT qt = Ft[2] - U * Ft[1] + a1 * Ft[0] - U * Wt2 - b1 * Wt0;
      F[2] += f * q; Ft[2] += f * qt;
    }
  }
}

// ---------------------------------------------------------- compact flux
// Eq. fd-conservative-flux and its (6-4) / (6-2) nonlinear forms.
FDK_HD double compact_flux(int variant, double Fm, double Fc, double Fp, double N0, double N1,
                                               double chi) {
  double Fb = ((Fm + 46.0 * Fc + Fp) - 9.0 * (N0 + N1)) * (1.0 / 30.0);
  if (variant == 2) return Fb;
  double lo = variant == 1 ? Fc : (8.0 * Fc - N0 - N1) * (1.0 / 6.0);
  return lo + chi * (Fb - lo);
}
// The same with the linear flux of order 8: the averaging conditions of Eq.
// fd-conservative-flux-recons imposed also on the nodal cells j-1 and j+2
// (the wider stencil of Sec. 2.1; Nm, Np2 are the nodal fluxes there).  The
// degree-6 solution at the interface is exact to degree 7 (symmetry), error
// -h^8 F^(8) / 161280; the low-order fluxes and the blend are unchanged.
FDK_HD double compact_flux8(int variant, double Fm, double Fc, double Fp, double Nm, double N0, double N1, double Np2,
                            double chi) {
  double Fb = ((32.0 * (Fm + Fp) + 704.0 * Fc) - 171.0 * (N0 + N1) - 3.0 * (Nm + Np2)) * (1.0 / 420.0);
  if (variant == 2) return Fb;
  double lo = variant == 1 ? Fc : (8.0 * Fc - N0 - N1) * (1.0 / 6.0);
  return lo + chi * (Fb - lo);
}

}  // namespace fdk
