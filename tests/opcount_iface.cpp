// Source-level operation count of one interface point of the stage-1
// interface sweep: the library's own reconstruction and gas-kinetic solver
// templates (gks_device.hpp) run on the host with a counting scalar.  One
// interface point is two solves (one per normal), each with the four-
// component GENO reconstruction of its line, as on the GPU; the partner blend
// and the tangential averages are added by hand below.
//
// Counts: add/sub, mul, div, sqrt and the transcendental calls (exp, erfc,
// tanh) separately, for smooth data (the GENO path functions saturate and
// the low-order blends are skipped) and for a jump in the line (every blend
// runs).  Printed as one JSON line per case.  Host only: built with
// --cuda-host-only by tests/test_opcount.py.
#include <cmath>
#include <cstdio>

#include "../paper_2606_17772_amd/csrc/gks_device.hpp"

namespace fdk {

struct Counts {
  long add = 0, mul = 0, div = 0, sqrt = 0, exp = 0, erfc = 0, tanh = 0;
};
static Counts C;

struct Cnt {
  double v;
  Cnt() : v(0.0) {}
  Cnt(double a) : v(a) {}  // NOLINT: implicit, like a double
  explicit operator double() const { return v; }
};
inline Cnt operator+(Cnt a, Cnt b) { ++C.add; return Cnt(a.v + b.v); }
inline Cnt operator-(Cnt a, Cnt b) { ++C.add; return Cnt(a.v - b.v); }
inline Cnt operator*(Cnt a, Cnt b) { ++C.mul; return Cnt(a.v * b.v); }
inline Cnt operator/(Cnt a, Cnt b) { ++C.div; return Cnt(a.v / b.v); }
inline Cnt operator+(Cnt a, double b) { return a + Cnt(b); }
inline Cnt operator+(double a, Cnt b) { return Cnt(a) + b; }
inline Cnt operator-(Cnt a, double b) { return a - Cnt(b); }
inline Cnt operator-(double a, Cnt b) { return Cnt(a) - b; }
inline Cnt operator*(Cnt a, double b) { return a * Cnt(b); }
inline Cnt operator*(double a, Cnt b) { return Cnt(a) * b; }
inline Cnt operator/(Cnt a, double b) { return a / Cnt(b); }
inline Cnt operator/(double a, Cnt b) { return Cnt(a) / b; }
inline Cnt operator-(Cnt a) { return Cnt(-a.v); }  // a sign flip, not counted
inline Cnt& operator+=(Cnt& a, Cnt b) { a = a + b; return a; }
inline Cnt& operator-=(Cnt& a, Cnt b) { a = a - b; return a; }
inline Cnt& operator*=(Cnt& a, Cnt b) { a = a * b; return a; }
inline bool operator>(Cnt a, Cnt b) { return a.v > b.v; }
inline bool operator<(Cnt a, Cnt b) { return a.v < b.v; }
inline bool operator>(Cnt a, double b) { return a.v > b; }
inline bool operator<(Cnt a, double b) { return a.v < b; }
inline bool operator==(Cnt a, double b) { return a.v == b; }
inline double val(Cnt a) { return a.v; }
inline Cnt m_erfc(Cnt a) { ++C.erfc; return Cnt(std::erfc(a.v)); }
inline Cnt m_exp(Cnt a) { ++C.exp; return Cnt(std::exp(a.v)); }
inline Cnt m_sqrt(Cnt a) { ++C.sqrt; return Cnt(std::sqrt(a.v)); }
inline Cnt m_abs(Cnt a) { return Cnt(std::fabs(a.v)); }
inline Cnt g_abs(Cnt a) { return Cnt(std::fabs(a.v)); }
inline Cnt g_max(Cnt a, Cnt b) { return b.v > a.v ? b : a; }
inline Cnt g_min(Cnt a, Cnt b) { return b.v < a.v ? b : a; }
inline Cnt g_tanh(Cnt a) {
  if (a.v > 19.5 || a.v < -19.5) return Cnt(a.v > 0 ? 1.0 : -1.0);  // as the library: no call
  ++C.tanh;
  return Cnt(std::tanh(a.v));
}

}  // namespace fdk

using fdk::Cnt;

static fdk::Consts consts() {
  fdk::Consts k{};
  k.gamma = 1.4;
  k.K = (4.0 - 2.0 * k.gamma) / (k.gamma - 1.0);
  k.inv_Kd = 1.0 / (k.K + 2.0);
  k.mu = 1e-4;
  k.prfix = 1.0 / 0.72 - 1.0;
  k.C = 20.0;
  k.inv_tanhC = 1.0 / std::tanh(20.0);
  k.eps = 1e-15;
  k.eps_a = 1e-6;
  k.dc = 8.0;
  k.ds = 1.0;
  k.tau_c1 = 0.0;
  k.tau_c2 = 1.0;
  k.r = 3;
  k.variant = 0;
  k.flux_order = 6;
  return k;
}

// One solve: the line's GENO reconstruction of the 4 components (nodes
// m-1..m+2, values q and averaged derivatives x), then the stage-1 solver.
static void one_solve(const fdk::Consts& k, double h, bool jump) {
  fdk::GksIO<Cnt, 2> io;
  const double base[4] = {1.0, 0.3, -0.05, 1.0 / (1.4 * 0.15 * 0.15) / 0.4 + 0.5 * 0.09};
  for (int c = 0; c < 4; ++c) {
    Cnt q[4], x[4];
    for (int m = 0; m < 4; ++m) {
      const double s = jump && m >= 2 ? 0.3 : 0.0;  // a jump between nodes m = 1 and 2
      q[m] = Cnt(base[c] * (1.0 + 1e-3 * (m - 1.5) + s));
      x[m] = Cnt(base[c] * 1e-3 / h);
    }
    fdk::IfaceRecT<Cnt> r = fdk::recon_iface<Cnt>(k, q[0], q[1], q[2], q[3], x[0], x[1], x[2], x[3], h, 1.0 / h);
    io.WL[c] = r.vl;
    io.WR[c] = r.vr;
    io.nL[c] = r.dl;
    io.nR[c] = r.dr;
    io.Wt[c] = 0.5 * (r.dl + r.dr);  // stands for the partner line's tangential average
  }
  fdk::gks_iface<Cnt, 2, true>(k, Cnt(1e-5), io);
}

int main() {
  const fdk::Consts k = consts();
  const double h = 1.0 / 2048.0;
  for (int jump = 0; jump < 2; ++jump) {
    fdk::C = fdk::Counts();
    for (int G = 0; G < 2; ++G) one_solve(k, h, jump != 0);
    // partner exchange and blend per solve and component: the tangential
    // average (1 add, 1 mul; counted inside one_solve), the two sums sent to
    // the partner (2 adds) and the four blended values (2 mul + 1 add each)
    fdk::C.add += 2 * 4 * (2 + 4);
    fdk::C.mul += 2 * 4 * 8;
    const fdk::Counts& c = fdk::C;
    const long arith = c.add + c.mul + c.div + c.sqrt;
    std::printf("{\"case\": \"%s\", \"add\": %ld, \"mul\": %ld, \"div\": %ld, \"sqrt\": %ld, \"exp\": %ld, "
                "\"erfc\": %ld, \"tanh\": %ld, \"arith\": %ld}\n",
                jump ? "jump" : "smooth", c.add, c.mul, c.div, c.sqrt, c.exp, c.erfc, c.tanh, arith);
  }
  return 0;
}
