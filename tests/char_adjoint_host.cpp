// Host build of the reverse characteristic reconstructions (gks_adjoint.hpp,
// --cuda-host-only): for each case read from stdin
//   L gamma variant Q[4][4] X[4][4] rb[4][4] chib dQ[4][4] dX[4][4] eps
//   N gamma variant Q[4][3] X[4][3] db[4] dQ[4][3] dX[4][3] eps
// prints two numbers: <Qb, dQ> + <Xb, dX> from the reverse routine, and the
// same directional derivative by central differences of the forward
// reconstruction, <rb, (rec(+) - rec(-)) / 2 eps> (+ chib times that of chi).
#include <cmath>
#include <cstdio>
#include <cstring>

#include "../paper_2606_17772_amd/csrc/gks_device.hpp"
#include "../paper_2606_17772_amd/csrc/gks_adjoint.hpp"

static fdk::Consts consts(double gamma, int variant) {
  fdk::Consts k;
  std::memset(&k, 0, sizeof k);
  k.gamma = gamma;
  k.K = (4.0 - 2.0 * gamma) / (gamma - 1.0);
  k.inv_Kd = 1.0 / (k.K + 2.0);
  k.C = 20.0;
  k.inv_tanhC = 1.0 / std::tanh(20.0);
  k.eps = 1e-15;
  k.eps_a = 1e-6;
  k.dc = 8.0;
  k.ds = 1.0;
  k.r = 3;
  k.variant = variant;
  k.flux_order = 6;
  return k;
}

static bool read(int n, double* v) {
  for (int i = 0; i < n; ++i)
    if (std::scanf("%lf", &v[i]) != 1) return false;
  return true;
}

int main() {
  char tag[4];
  const double h = 0.05, invh = 1.0 / h;
  while (std::scanf("%3s", tag) == 1) {
    double gamma, variant;
    if (!read(1, &gamma) || !read(1, &variant)) return 1;
    const fdk::Consts k = consts(gamma, (int)variant);
    if (tag[0] == 'L') {
      double Q[4][4], X[4][4], rb[4][4], chib, dQ[4][4], dX[4][4], eps;
      if (!read(16, &Q[0][0]) || !read(16, &X[0][0]) || !read(16, &rb[0][0]) || !read(1, &chib) ||
          !read(16, &dQ[0][0]) || !read(16, &dX[0][0]) || !read(1, &eps))
        return 1;
      double Qb[4][4] = {}, Xb[4][4] = {};
      fdk::recon_iface_char_b(k, Q, X, h, invh, rb, chib, Qb, Xb);
      double an = 0.0;
      for (int c = 0; c < 4; ++c)
        for (int m = 0; m < 4; ++m) an += Qb[c][m] * dQ[c][m] + Xb[c][m] * dX[c][m];
      double val[2] = {0.0, 0.0};
      for (int sgn = 0; sgn < 2; ++sgn) {
        const double e = sgn == 0 ? eps : -eps;
        double Qe[4][4], Xe[4][4];
        for (int c = 0; c < 4; ++c)
          for (int m = 0; m < 4; ++m) { Qe[c][m] = Q[c][m] + e * dQ[c][m]; Xe[c][m] = X[c][m] + e * dX[c][m]; }
        fdk::IfaceRec rec[4];
        double chi;
        fdk::recon_iface_char<2>(k, Qe, Xe, h, invh, rec, chi);
        double s = chib * chi;
        for (int c = 0; c < 4; ++c)
          s += rb[c][0] * rec[c].vl + rb[c][1] * rec[c].dl + rb[c][2] * rec[c].vr + rb[c][3] * rec[c].dr;
        val[sgn] = s;
      }
      std::printf("%.17g %.17g\n", an, (val[0] - val[1]) / (2.0 * eps));
    } else {
      double Q[4][3], X[4][3], db[4], dQ[4][3], dX[4][3], eps;
      if (!read(12, &Q[0][0]) || !read(12, &X[0][0]) || !read(4, db) || !read(12, &dQ[0][0]) ||
          !read(12, &dX[0][0]) || !read(1, &eps))
        return 1;
      double Qb[4][3] = {}, Xb[4][3] = {};
      fdk::recon_node_char_b(k, Q, X, h, invh, db, Qb, Xb);
      double an = 0.0;
      for (int c = 0; c < 4; ++c)
        for (int m = 0; m < 3; ++m) an += Qb[c][m] * dQ[c][m] + Xb[c][m] * dX[c][m];
      double val[2] = {0.0, 0.0};
      for (int sgn = 0; sgn < 2; ++sgn) {
        const double e = sgn == 0 ? eps : -eps;
        double Qe[4][3], Xe[4][3], d[4];
        for (int c = 0; c < 4; ++c)
          for (int m = 0; m < 3; ++m) { Qe[c][m] = Q[c][m] + e * dQ[c][m]; Xe[c][m] = X[c][m] + e * dX[c][m]; }
        fdk::recon_node_char<2>(k, Qe, Xe, h, invh, d);
        val[sgn] = db[0] * d[0] + db[1] * d[1] + db[2] * d[2] + db[3] * d[3];
      }
      std::printf("%.17g %.17g\n", an, (val[0] - val[1]) / (2.0 * eps));
    }
  }
  return 0;
}
