// Host sanitizer run of the oracle: small 2D stages and steps (periodic,
// walled, characteristic, the order-8 flux on walls) and 1D runs, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_oracle_sanitized.py.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "../oracle/fdcgks_oracle.cpp"

static Par par2d(int nx, int ny, int side, int chr, int order = 6) {
  Par p{};
  p.dim = 2; p.nx = nx; p.ny = ny; p.bc = side; p.r = 3; p.recon_char = chr; p.flux_order = order;
  for (int k = 0; k < 4; ++k) p.side[k] = side;
  p.lx = 1.0; p.ly = 1.0 * ny / nx; p.gamma = 1.4; p.mu = 1e-3; p.prandtl = 0.72;
  p.C = 20.0; p.eps = 1e-15; p.eps_a = 1e-6; p.d_central = 8.0; p.d_side = 1.0; p.tau_c2 = 1.0;
  return p;
}

static void fill(std::vector<double>& A, int nx, int ny, std::mt19937& g) {
  std::uniform_real_distribution<double> u(0.5, 1.5), v(-0.3, 0.3);
  const long n = (long)nx * ny;
  for (long k = 0; k < n; ++k) {
    double rho = u(g), U = v(g), V = v(g), p = u(g);
    A[k] = rho; A[n + k] = rho * U; A[2 * n + k] = rho * V; A[3 * n + k] = p / 0.4 + 0.5 * rho * (U * U + V * V);
    for (int f = 4; f < 12; ++f) A[f * n + k] = 0.1 * v(g);
  }
}

int main() {
  std::mt19937 g(1);
  const int cases[5][3] = {{BC_PERIODIC, 0, 6}, {BC_NO_SLIP, 0, 6}, {BC_REFLECTING, 1, 6}, {BC_NO_SLIP, 0, 8},
                           {BC_ZERO_GRADIENT, 0, 8}};
  for (auto& c : cases) {
    Par p = par2d(9, 6, c[0], c[1], c[2]);
    const int bx = c[0] != BC_PERIODIC, nxd = 9 + bx, nyd = 6 + bx;
    std::vector<double> P(12 * 9 * 6), D(12 * nxd * nyd);
    fill(P, 9, 6, g);
    fill(D, nxd, nyd, g);
    std::vector<double> oP(P.size()), oD(D.size()), aP(P.size()), aD(D.size());
    orc_stage2d(&p, 1, 1e-3, P.data(), D.data(), nullptr, nullptr, oP.data(), oD.data(), aP.data(), aD.data());
    double t = 0.0;
    int k = orc_step2d(&p, P.data(), D.data(), 2, 1e-3, 0.0, 0.0, &t);
    if (k != 2 || !std::isfinite(P[0])) { std::printf("2D case failed\n"); return 1; }
  }
  Par q = par2d(40, 1, BC_REFLECTING, 0);
  q.dim = 1; q.mu = 0.0; q.dual_1d = 1;
  std::vector<double> S(2 * 6 * 40);
  for (int l = 0; l < 2; ++l)
    for (int j = 0; j < 40; ++j) {
      double x = (j + 0.5 + 0.5 * l) / 40.0, rho = 1.0 + 0.2 * std::sin(6.28 * x);
      S[l * 240 + j] = rho; S[l * 240 + 40 + j] = 0.1 * rho; S[l * 240 + 80 + j] = 2.5 + 0.005 * rho;
    }
  for (int order : {6, 8}) {
    q.flux_order = order;
    double t = 0.0;
    int k = orc_step1d(&q, S.data(), 3, 0.0, 0.5, 0.0, &t);
    if (k != 3) { std::printf("1D case failed\n"); return 1; }
  }
  std::printf("sanitized oracle runs: ok\n");
  return 0;
}
