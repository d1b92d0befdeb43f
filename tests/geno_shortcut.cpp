// The division-free smooth-data test at the top of the library's GENO
// routine (fdk::geno, gks_device.hpp) must never change its result: where it
// fires, the full path (path function, tanh and blend, Sec. 3 / App. C) gives
// the same bits.  The full path is restated here without that test and both
// run on seeded smoothness-indicator triples over the whole double range
// (log-uniform, near ties, exact zeros) for r = 1..4, C = 10, 20, 40 and
// several eps.  Prints one JSON line; host only (--cuda-host-only).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>

#include "../paper_2606_17772_amd/csrc/gks_device.hpp"

using fdk::Consts;
using fdk::GenoOutT;

static GenoOutT<double> full_path(const Consts& k, double IS1, double IS2, double IS3, double d1, double d2,
                                  double d3, double q1, double q2, double q3, double dq1, double dq2, double dq3,
                                  double PH, double PHx) {
  const double tau = 0.5 * std::fabs((IS2 + IS3) - 2.0 * IS1);
  const double eH = std::fmax(IS1, std::fmax(IS2, IS3)) + k.eps;
  const double eL = std::fmin(IS1, std::fmin(IS2, IS3)) + k.eps;
  const double inv = 1.0 / (eH * eL);
  const double aH = 1.0 + fdk::ipow(tau * eL * inv, k.r), aL = 1.0 + fdk::ipow(tau * eH * inv, k.r);
  const double th = fdk::g_tanh(k.C * (2.0 * aH / (aH + aL)));
  const double chi = th * k.inv_tanhC;
  GenoOutT<double> o;
  if (th == 1.0 && chi == 1.0) {
    o.v = PH;
    o.d = PHx;
    o.chi = chi;
    return o;
  }
  const double t1 = fdk::sqr(IS1 + k.eps_a), t2 = fdk::sqr(IS2 + k.eps_a), t3 = fdk::sqr(IS3 + k.eps_a);
  const double w1 = d1 * t2 * t3, w2 = d2 * t1 * t3, w3 = d3 * t1 * t2;
  const double is = 1.0 / (w1 + w2 + w3);
  o.v = chi * PH + (1.0 - chi) * ((w1 * q1 + w2 * q2 + w3 * q3) * is);
  o.d = chi * PHx + (1.0 - chi) * ((w1 * dq1 + w2 * dq2 + w3 * dq3) * is);
  o.chi = chi;
  return o;
}

int main() {
  std::mt19937_64 rng(20240611);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  long total = 0, saturated = 0, differ = 0;
  const double Cs[] = {20.0, 40.0, 10.0}, epss[] = {1e-15, 1e-40, 0.0, 1e-6};
  for (int r = 1; r <= 4; ++r)
    for (double C : Cs)
      for (double eps : epss) {
        Consts k{};
        k.C = C;
        k.inv_tanhC = 1.0 / std::tanh(C);
        k.eps = eps;
        k.eps_a = 1e-6;
        k.r = r;
        for (long n = 0; n < 250000; ++n) {
          double IS[3];
          const int mode = (int)(n % 4);
          for (int t = 0; t < 3; ++t) {
            const double e = mode == 1 ? -20.0 + 25.0 * U(rng) : -300.0 + 600.0 * U(rng);
            IS[t] = std::pow(10.0, e);
            if (mode == 2 && t > 0) IS[t] = IS[0] * (1.0 + 1e-3 * (U(rng) - 0.5));  // smooth: near ties
            if (mode == 3 && U(rng) < 0.2) IS[t] = 0.0;
          }
          const GenoOutT<double> a =
              fdk::geno<double>(k, IS[0], IS[1], IS[2], 0.1, 0.8, 0.1, 1.1, 2.3, 3.7, 4.1, 5.3, 6.7, 7.0, 8.0);
          const GenoOutT<double> b =
              full_path(k, IS[0], IS[1], IS[2], 0.1, 0.8, 0.1, 1.1, 2.3, 3.7, 4.1, 5.3, 6.7, 7.0, 8.0);
          ++total;
          saturated += b.v == 7.0 && b.chi == 1.0;
          differ += std::memcmp(&a, &b, sizeof a) != 0;
        }
      }
  std::printf("{\"total\": %ld, \"saturated\": %ld, \"differ\": %ld}\n", total, saturated, differ);
  return 0;
}
