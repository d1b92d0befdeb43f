// libfdcgks: gfx950 kernels and host runtime of the FD-CGKS stage sweep.
//
// Device layout (2D).  Every field is a padded plane of FP64, x fastest:
// row pitch `pitch` doubles, interior node (i, j) at (j + OY) * pitch +
// (i + OX) with OX = 8 (64-byte aligned interior rows) and OY = 3; three
// halo rows/columns on each side hold the periodic images.
//   state buffer : 24 planes, plane = grid*12 + field*4 + comp
//                  (grid 0 primary, 1 dual; field 0 W, 1 Wx, 2 Wy)
//   edge buffer  : 2 families (X, Y) x 2 normals (primary-line, dual-line)
//                  x 25 planes: F[4], Ft[4], chi, Wl[4], Wr[4], Wlt[4], Wrt[4]
//   node buffer  : 2 grids x 16 planes: F[4], Ft[4], G[4], Gt[4]
// Interface families: X(i,j) at (x0+(i+1)h, y0+(j+1/2)h) lies between the
// primary nodes (i,j), (i+1,j) along x and between the dual nodes (i,j-1),
// (i,j) along y; Y(i,j) at (x0+(i+1/2)h, y0+(j+1)h) lies between primary
// (i,j), (i,j+1) along y and dual (i-1,j), (i,j) along x (Sec. 4).
//
// One S2O4 stage = halo fill -> interface sweep (two line GENO
// reconstructions and two gas-kinetic solves per interface point) -> nodal
// sweep (nodal derivative GENO + smooth gas-kinetic flux) -> assemble+update.
// The time step lives in device memory so steps never wait on the host.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fdcgks.h"
#include "gks_device.hpp"

using fdk::Consts;

namespace {

constexpr int OX = 8, OY = 3, HALO = 3;

struct Geo {
  int nx, ny, pitch, rows;
  long plane;
  double h, invh;
};
__device__ __forceinline__ long at(const Geo& g, int j, int i) { return (long)(j + OY) * g.pitch + (i + OX); }

// Scalars of the running step, kept on the device.
struct Scal {
  double dt, t, t_end, dt_fixed;
  int stop;       // bit 0: non-physical state, bit 1: t_end reached
  int steps;      // completed steps since the counter was reset
  int fail_grid, fail_i, fail_j, fail_stage;
  int pad[2];
};

__device__ __forceinline__ int imod(int a, int m) { return ((a % m) + m) % m; }

// ------------------------------------------------------------ halo fill
// Periodic images: rows first (interior columns), then whole columns.
__global__ void k_halo_rows(double* __restrict__ S, int nplanes, Geo g, const Scal* __restrict__ sc) {
  if (sc->stop) return;
  long n = (long)nplanes * 2 * HALO * g.nx;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    int i = (int)(t % g.nx);
    long r = t / g.nx;
    int hr = (int)(r % (2 * HALO));
    int p = (int)(r / (2 * HALO));
    int j = hr < HALO ? hr - HALO : g.ny + (hr - HALO);
    double* P = S + p * g.plane;
    P[at(g, j, i)] = P[at(g, imod(j, g.ny), i)];
  }
}
__global__ void k_halo_cols(double* __restrict__ S, int nplanes, Geo g, const Scal* __restrict__ sc) {
  if (sc->stop) return;
  int rows = g.ny + 2 * HALO;
  long n = (long)nplanes * rows * 2 * HALO;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    int hc = (int)(t % (2 * HALO));
    long r = t / (2 * HALO);
    int j = (int)(r % rows) - HALO;
    int p = (int)(r / rows);
    int i = hc < HALO ? hc - HALO : g.nx + (hc - HALO);
    double* P = S + p * g.plane;
    P[at(g, j, i)] = P[at(g, j, imod(i, g.nx))];
  }
}

// ------------------------------------------------------- interface sweep
// One gas-kinetic solve at an interface point: rn is the line normal to the
// interface, rt the other line (its derivative gives the tangential slope).
// SWAP: the normal is y, so rho U and rho V trade places in the local frame.
template <bool SWAP, int STAGE, class FT>
__device__ __forceinline__ void solve_dir(const Consts& k, FT dt, const fdk::IfaceRec (&rn)[4], const double (&tang)[4],
                                          double (&F)[4], double (&Ft)[4], double (&Wl)[4], double (&Wr)[4],
                                          double (&Wlt)[4], double (&Wrt)[4]) {
  fdk::GksIO<FT, 2> io;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int q = SWAP ? (c == 1 ? 2 : (c == 2 ? 1 : c)) : c;
    io.WL[c] = (FT)rn[q].vl;
    io.WR[c] = (FT)rn[q].vr;
    io.nL[c] = (FT)rn[q].dl;
    io.nR[c] = (FT)rn[q].dr;
    io.Wt[c] = (FT)tang[q];
  }
  fdk::gks_iface<FT, 2, STAGE == 1>(k, dt, io);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int q = SWAP ? (c == 1 ? 2 : (c == 2 ? 1 : c)) : c;
    Ft[q] = (double)io.Ft[c];
    Wlt[q] = (double)io.Wlt[c];
    Wrt[q] = (double)io.Wrt[c];
    if (STAGE == 1) {
      F[q] = (double)io.F[c];
      Wl[q] = (double)io.Wl[c];
      Wr[q] = (double)io.Wr[c];
    }
  }
}

// Everything at interface point (i, j) of family FAM (0: X, 1: Y).
template <int STAGE, class FT, int FAM>
__device__ __forceinline__ void edge_point(const double* __restrict__ S, double* __restrict__ E, const Geo& g,
                                           const Consts& k, double dt, int i, int j) {
  const long pl = g.plane;
  // primary line: X along x from P(i-1,j); Y along y from P(i,j-1)
  // dual line:    X along y from D(i,j-2); Y along x from D(i-2,j)
  const long sP = FAM == 0 ? 1 : g.pitch, sD = FAM == 0 ? g.pitch : 1;
  const long oP = FAM == 0 ? at(g, j, i - 1) : at(g, j - 1, i);
  const long oD = FAM == 0 ? at(g, j - 2, i) : at(g, j, i - 2);
  constexpr int fP = FAM == 0 ? 1 : 2, fD = FAM == 0 ? 2 : 1;  // derivative field along each line
  fdk::IfaceRec rP[4], rD[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double* w = S + (0 * 12 + c) * pl + oP;
    const double* x = S + (0 * 12 + fP * 4 + c) * pl + oP;
    rP[c] = fdk::recon_iface(k, w[0], w[sP], w[2 * sP], w[3 * sP], x[0], x[sP], x[2 * sP], x[3 * sP], g.h, g.invh);
    const double* wd = S + (12 + c) * pl + oD;
    const double* xd = S + (12 + fD * 4 + c) * pl + oD;
    rD[c] = fdk::recon_iface(k, wd[0], wd[sD], wd[2 * sD], wd[3 * sD], xd[0], xd[sD], xd[2 * sD], xd[3 * sD], g.h,
                             g.invh);
  }
  double tP[4], tD[4];  // tangential slopes: mean of the left/right line derivatives
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    tP[c] = 0.5 * (rP[c].dl + rP[c].dr);
    tD[c] = 0.5 * (rD[c].dl + rD[c].dr);
  }
  double FPn[4], FPt[4], WPl[4], WPr[4], WPlt[4], WPrt[4];
  double FDn[4], FDt[4], WDl[4], WDr[4], WDlt[4], WDrt[4];
  solve_dir<FAM == 1, STAGE, FT>(k, (FT)dt, rP, tD, FPn, FPt, WPl, WPr, WPlt, WPrt);
  solve_dir<FAM == 0, STAGE, FT>(k, (FT)dt, rD, tP, FDn, FDt, WDl, WDr, WDlt, WDrt);
  // blend of the two directions (Eq. W-model-2d) and store
  double* e = E + (long)FAM * 50 * pl + at(g, j, i);
  e[8 * pl] = fmin(rP[0].cl, rP[0].cr);
  e[(25 + 8) * pl] = fmin(rD[0].cl, rD[0].cr);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double sPt = WPlt[c] + WPrt[c], sDt = WDlt[c] + WDrt[c];
    e[(4 + c) * pl] = FPt[c];
    e[(17 + c) * pl] = 0.5 * WPlt[c] + 0.25 * sDt;
    e[(21 + c) * pl] = 0.5 * WPrt[c] + 0.25 * sDt;
    e[(25 + 4 + c) * pl] = FDt[c];
    e[(25 + 17 + c) * pl] = 0.5 * WDlt[c] + 0.25 * sPt;
    e[(25 + 21 + c) * pl] = 0.5 * WDrt[c] + 0.25 * sPt;
    if (STAGE == 1) {
      double sP = WPl[c] + WPr[c], sD = WDl[c] + WDr[c];
      e[(0 + c) * pl] = FPn[c];
      e[(9 + c) * pl] = 0.5 * WPl[c] + 0.25 * sD;
      e[(13 + c) * pl] = 0.5 * WPr[c] + 0.25 * sD;
      e[(25 + 0 + c) * pl] = FDn[c];
      e[(25 + 9 + c) * pl] = 0.5 * WDl[c] + 0.25 * sP;
      e[(25 + 13 + c) * pl] = 0.5 * WDr[c] + 0.25 * sP;
    }
  }
}

// One thread per interface point.  blockIdx.z = family: X over i in [-2, nx],
// j in [-1, ny+1]; Y over i in [-1, nx+1], j in [-2, ny] (everything the
// update of the interior reads).
template <int STAGE, class FT>
__global__ __launch_bounds__(256) void k_edges2d(const double* __restrict__ S, double* __restrict__ E, Geo g,
                                                 Consts k, const Scal* __restrict__ sc) {
  const int fam = blockIdx.z;
  const int i = blockIdx.x * blockDim.x + threadIdx.x + (fam == 0 ? -2 : -1);
  const int j = blockIdx.y * blockDim.y + threadIdx.y + (fam == 0 ? -1 : -2);
  if (i > (fam == 0 ? g.nx : g.nx + 1) || j > (fam == 0 ? g.ny + 1 : g.ny)) return;
  if (sc->stop) return;
  const double dt = sc->dt;
  if (fam == 0) edge_point<STAGE, FT, 0>(S, E, g, k, dt, i, j);
  else edge_point<STAGE, FT, 1>(S, E, g, k, dt, i, j);
}

// ------------------------------------------------------------ node sweep
// Both grids (blockIdx.z), nodes i in [-1, nx], j in [-1, ny].
template <int STAGE, class FT>
__global__ __launch_bounds__(256) void k_nodes2d(const double* __restrict__ S, double* __restrict__ Nb, Geo g,
                                                 Consts k, const Scal* __restrict__ sc) {
  const int grid = blockIdx.z;
  const int i = blockIdx.x * blockDim.x + threadIdx.x - 1;
  const int j = blockIdx.y * blockDim.y + threadIdx.y - 1;
  if (i > g.nx || j > g.ny) return;
  if (sc->stop) return;
  const long pl = g.plane, o = at(g, j, i);
  const double* B = S + (long)grid * 12 * pl;
  FT W[4], Wx[4], Wy[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double* w = B + c * pl + o;
    const double* x = B + (4 + c) * pl + o;
    const double* y = B + (8 + c) * pl + o;
    W[c] = (FT)w[0];
    Wx[c] = (FT)fdk::recon_node(k, w[-1], w[0], w[1], x[-1], x[0], x[1], g.h, g.invh);
    Wy[c] = (FT)fdk::recon_node(k, w[-g.pitch], w[0], w[g.pitch], y[-g.pitch], y[0], y[g.pitch], g.h, g.invh);
  }
  FT F[4], Ft[4], G[4], Gt[4];
  fdk::gks_node<FT, 2, STAGE == 1>(k, W, Wx, Wy, F, Ft, G, Gt);
  double* n = Nb + (long)grid * 16 * pl + o;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    n[(4 + c) * pl] = (double)Ft[c];
    n[(12 + c) * pl] = (double)Gt[c];
    if (STAGE == 1) {
      n[c * pl] = (double)F[c];
      n[(8 + c) * pl] = (double)G[c];
    }
  }
}

// ------------------------------------------------------ assemble + update
// Node (i, j) of grid `grid`, axis a: the interface family and normal slot
// holding its a-fluxes, and the offset r of its right (upper) interface:
// primary x -> X, slot 0, r = 0; primary y -> Y, slot 0, r = 0;
// dual x -> Y, slot 1, r = 1;    dual y -> X, slot 1, r = 1.
template <int STAGE>
__global__ __launch_bounds__(256) void k_update2d(const double* __restrict__ S, const double* __restrict__ E,
                                                  const double* __restrict__ Nb, const double* __restrict__ Ain,
                                                  double* __restrict__ Out, double* __restrict__ Aout, Geo g,
                                                  Consts k, Scal* __restrict__ sc) {
  const int grid = blockIdx.z;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  if (i >= g.nx || j >= g.ny) return;
  if (sc->stop) return;
  const double dt = sc->dt;
  const long pl = g.plane, o = at(g, j, i);
  const int r = grid;
  double L[4] = {0, 0, 0, 0}, Lt[4] = {0, 0, 0, 0}, Gr[2][4], Grt[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const int fam = (grid == 0) ? a : 1 - a;
    const long st = a == 0 ? 1 : g.pitch;
    const double* e = E + (long)fam * 50 * pl + (long)grid * 25 * pl + o;
    const double* n = Nb + (long)grid * 16 * pl + (a == 0 ? 0 : 8) * pl + o;
    const double chiR = e[8 * pl + r * st], chiL = e[8 * pl + (r - 1) * st];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double* f = e + (0 + c) * pl;
      const double* ft = e + (4 + c) * pl;
      const double* nf = n + c * pl;
      const double* nft = n + (4 + c) * pl;
      if (STAGE == 1) {
        double FR = fdk::compact_flux(k.variant, f[(r - 1) * st], f[r * st], f[(r + 1) * st], nf[0], nf[st], chiR);
        double FL = fdk::compact_flux(k.variant, f[(r - 2) * st], f[(r - 1) * st], f[r * st], nf[-st], nf[0], chiL);
        L[c] = L[c] - (FR - FL) * g.invh;
        Gr[a][c] = (e[(9 + c) * pl + r * st] - e[(13 + c) * pl + (r - 1) * st]) * g.invh;
      }
      double FRt = fdk::compact_flux(k.variant, ft[(r - 1) * st], ft[r * st], ft[(r + 1) * st], nft[0], nft[st], chiR);
      double FLt = fdk::compact_flux(k.variant, ft[(r - 2) * st], ft[(r - 1) * st], ft[r * st], nft[-st], nft[0], chiL);
      Lt[c] = Lt[c] - (FRt - FLt) * g.invh;
      Grt[a][c] = (e[(17 + c) * pl + r * st] - e[(21 + c) * pl + (r - 1) * st]) * g.invh;
    }
  }
  const double* s = S + (long)grid * 12 * pl + o;
  double* out = Out + (long)grid * 12 * pl + o;
  double W[4];
  if (STAGE == 1) {
    double* ao = Aout + (long)grid * 12 * pl + o;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      double w = s[c * pl];
      W[c] = w + 0.5 * dt * L[c] + 0.125 * dt * dt * Lt[c];
      double gx = k.grad_carried ? s[(4 + c) * pl] : Gr[0][c];
      double gy = k.grad_carried ? s[(8 + c) * pl] : Gr[1][c];
      out[c * pl] = W[c];
      out[(4 + c) * pl] = gx + 0.5 * dt * Grt[0][c];
      out[(8 + c) * pl] = gy + 0.5 * dt * Grt[1][c];
      ao[c * pl] = w + dt * L[c] + dt * dt / 6.0 * Lt[c];
      ao[(4 + c) * pl] = gx;
      ao[(8 + c) * pl] = gy;
    }
  } else {
    const double* ai = Ain + (long)grid * 12 * pl + o;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      W[c] = ai[c * pl] + dt * dt / 3.0 * Lt[c];
      out[c * pl] = W[c];
      out[(4 + c) * pl] = ai[(4 + c) * pl] + dt * Grt[0][c];
      out[(8 + c) * pl] = ai[(8 + c) * pl] + dt * Grt[1][c];
    }
  }
  // non-physical state: rho <= 0, p <= 0 or NaN stops the run
  double p = (k.gamma - 1.0) * (W[3] - 0.5 * (W[1] * W[1] + W[2] * W[2]) / W[0]);
  if (!(W[0] > 0.0) || !(p > 0.0)) {
    if (atomicCAS(&sc->stop, 0, 1) == 0) {
      sc->fail_grid = grid;
      sc->fail_i = i;
      sc->fail_j = j;
      sc->fail_stage = STAGE;
    }
  }
}

// ------------------------------------------------------------ CFL / step
// Per-block partial max(max(|U|,|V|) + c) and min rho over both grids
// (2D: dim 2, 4 components; 1D lines: dim 1, 3 components).
template <int DIM>
__global__ __launch_bounds__(256) void k_cfl_partial(const double* __restrict__ S, Geo g, int ngrid, long gridstride,
                                                     double gamma, double* __restrict__ part,
                                                     const Scal* __restrict__ sc) {
  __shared__ double smax[256], smin[256];
  double vmax = 0.0, rmin = 1e300;
  long n = (long)ngrid * g.nx * g.ny;
  constexpr int NC = DIM + 2;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    int i = (int)(t % g.nx);
    long r = t / g.nx;
    int j = (int)(r % g.ny);
    int gr = (int)(r / g.ny);
    const double* B = S + gr * gridstride + at(g, j, i);
    double rho = B[0], U = B[g.plane] / rho;
    double V = DIM == 2 ? B[2 * g.plane] / rho : 0.0;
    double rE = B[(NC - 1) * g.plane];
    double p = (gamma - 1.0) * (rE - 0.5 * rho * (U * U + V * V));
    double c = sqrt(gamma * p / rho);
    double s = fmax(fabs(U), fabs(V)) + c;
    vmax = fmax(vmax, s);  // NaN speeds are dropped here and caught by the update's check
    rmin = fmin(rmin, rho);
  }
  smax[threadIdx.x] = vmax;
  smin[threadIdx.x] = rmin;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = smax[0];
    part[2 * blockIdx.x + 1] = smin[0];
  }
  (void)sc;
}

// Start of a step: dt from the partials (or the fixed dt), clipped to t_end;
// sets the "done" bit when t has reached t_end.
__global__ void k_step_begin(const double* __restrict__ part, int nparts, Scal* __restrict__ sc, double cfl,
                             double h, double mu, int use_cfl) {
  __shared__ double smax[256], smin[256];
  double vmax = 0.0, rmin = 1e300;
  if (use_cfl)
    for (int t = threadIdx.x; t < nparts; t += blockDim.x) {
      vmax = fmax(vmax, part[2 * t]);
      rmin = fmin(rmin, part[2 * t + 1]);
    }
  smax[threadIdx.x] = vmax;
  smin[threadIdx.x] = rmin;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (sc->stop) return;
    double dt;
    if (use_cfl) {
      dt = cfl * h / smax[0];
      if (mu > 0) dt = fmin(dt, cfl * h * h / (8.0 * mu / smin[0]));
    } else {
      dt = sc->dt_fixed;
    }
    if (sc->t_end > 0) {
      if (sc->t >= sc->t_end) { sc->stop |= 2; return; }
      if (sc->t + dt > sc->t_end) dt = sc->t_end - sc->t;
    }
    if (!(dt > 0.0)) { sc->stop |= 1; sc->fail_stage = 0; return; }
    sc->dt = dt;
  }
}
__global__ void k_step_end(Scal* __restrict__ sc) {
  if (sc->stop) return;
  sc->t += sc->dt;
  sc->steps += 1;
}

// ================================================================== host
thread_local std::string g_create_error;

struct Launch {
  dim3 grid, block;
};

}  // namespace

struct fdcgks_problem {
  fdcgks_params prm;
  Consts k;
  Geo g;
  hipStream_t stream = nullptr;
  int ngrid = 0;        // grids present (2D: 2; 1D: 1 or 2)
  int nplanes = 0;      // state planes per buffer
  double* S[2] = {nullptr, nullptr};  // ping-pong state
  double* Sstar = nullptr;
  double* Acc = nullptr;
  double* E = nullptr;
  double* Nb = nullptr;
  double* part = nullptr;
  int nparts = 0;
  Scal* sc = nullptr;
  Scal* sc_host = nullptr;  // pinned
  int cur = 0;
  bool have_state[2] = {false, false};
  std::string err;
  // optional per-kernel timing (fdcgks_step_timed): an event after every launch
  bool timing = false;
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_kind;
  int ev_used = 0;
};

namespace {

fdcgks_status fail(fdcgks_problem* pb, fdcgks_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (pb) pb->err = buf; else g_create_error = buf;
  return st;
}
#define HIPCHK(pb, call)                                                                     \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess) return fail(pb, FDCGKS_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

long state_planes(const fdcgks_params& p) { return p.dim == 2 ? 24 : 12; }

void free_all(fdcgks_problem* pb) {
  double* bufs[] = {pb->S[0], pb->S[1], pb->Sstar, pb->Acc, pb->E, pb->Nb, pb->part};
  for (double* b : bufs) if (b) (void)hipFree(b);
  if (pb->sc) (void)hipFree(pb->sc);
  if (pb->sc_host) (void)hipHostFree(pb->sc_host);
  pb->S[0] = pb->S[1] = pb->Sstar = pb->Acc = pb->E = pb->Nb = pb->part = nullptr;
  pb->sc = nullptr;
  pb->sc_host = nullptr;
}

int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

// Kernel classes reported by fdcgks_step_timed.
enum { TK_HALO = 0, TK_EDGE1, TK_NODE1, TK_UPD1, TK_EDGE2, TK_NODE2, TK_UPD2, TK_STEP, TK_COUNT };

void mark(fdcgks_problem* pb, int kind) {
  if (!pb->timing) return;
  if (pb->ev_used >= (int)pb->ev.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) { pb->timing = false; return; }
    pb->ev.push_back(e);
    pb->ev_kind.push_back(kind);
  }
  pb->ev_kind[pb->ev_used] = kind;
  (void)hipEventRecord(pb->ev[pb->ev_used++], pb->stream);
}

fdcgks_status launch_check(fdcgks_problem* pb, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(pb, FDCGKS_EHIP, "launch of %s failed: %s", what, hipGetErrorString(e));
  return FDCGKS_OK;
}

// ---- 2D stage sequence
fdcgks_status halo2d(fdcgks_problem* pb, double* S) {
  const Geo& g = pb->g;
  long nr = (long)pb->nplanes * 2 * HALO * g.nx, nc = (long)pb->nplanes * (g.ny + 2 * HALO) * 2 * HALO;
  hipLaunchKernelGGL(k_halo_rows, dim3(std::min(ceil_div(nr, 256), 4096)), dim3(256), 0, pb->stream, S,
                     pb->nplanes, g, pb->sc);
  hipLaunchKernelGGL(k_halo_cols, dim3(std::min(ceil_div(nc, 256), 4096)), dim3(256), 0, pb->stream, S,
                     pb->nplanes, g, pb->sc);
  mark(pb, TK_HALO);
  return launch_check(pb, "halo");
}

template <int STAGE>
fdcgks_status stage2d(fdcgks_problem* pb, const double* Sin, const double* Ain, double* Out, double* Aout) {
  const Geo& g = pb->g;
  fdcgks_status st = halo2d(pb, const_cast<double*>(Sin));
  if (st) return st;
  dim3 blk(64, 4);
  dim3 ge(ceil_div(g.nx + 3, 64), ceil_div(g.ny + 3, 4), 2);
  if (pb->prm.flux_precision == FDCGKS_FP32_FLUX)
    hipLaunchKernelGGL((k_edges2d<STAGE, float>), ge, blk, 0, pb->stream, Sin, pb->E, g, pb->k, pb->sc);
  else
    hipLaunchKernelGGL((k_edges2d<STAGE, double>), ge, blk, 0, pb->stream, Sin, pb->E, g, pb->k, pb->sc);
  mark(pb, STAGE == 1 ? TK_EDGE1 : TK_EDGE2);
  dim3 gn(ceil_div(g.nx + 2, 64), ceil_div(g.ny + 2, 4), 2);
  if (pb->prm.flux_precision == FDCGKS_FP32_FLUX)
    hipLaunchKernelGGL((k_nodes2d<STAGE, float>), gn, blk, 0, pb->stream, Sin, pb->Nb, g, pb->k, pb->sc);
  else
    hipLaunchKernelGGL((k_nodes2d<STAGE, double>), gn, blk, 0, pb->stream, Sin, pb->Nb, g, pb->k, pb->sc);
  mark(pb, STAGE == 1 ? TK_NODE1 : TK_NODE2);
  dim3 gu(ceil_div(g.nx, 64), ceil_div(g.ny, 4), 2);
  hipLaunchKernelGGL((k_update2d<STAGE>), gu, blk, 0, pb->stream, Sin, pb->E, pb->Nb, Ain, Out, Aout, g, pb->k,
                     pb->sc);
  mark(pb, STAGE == 1 ? TK_UPD1 : TK_UPD2);
  return launch_check(pb, "stage");
}

fdcgks_status begin_step(fdcgks_problem* pb, double dt, double cfl) {
  const Geo& g = pb->g;
  int use_cfl = dt > 0 ? 0 : 1;
  if (use_cfl) {
    long gstride = (pb->prm.dim == 2 ? 12 : 6) * g.plane;
    if (pb->prm.dim == 2)
      hipLaunchKernelGGL(k_cfl_partial<2>, dim3(pb->nparts), dim3(256), 0, pb->stream, pb->S[pb->cur], g, pb->ngrid,
                         gstride, pb->k.gamma, pb->part, pb->sc);
    else
      hipLaunchKernelGGL(k_cfl_partial<1>, dim3(pb->nparts), dim3(256), 0, pb->stream, pb->S[pb->cur], g, pb->ngrid,
                         gstride, pb->k.gamma, pb->part, pb->sc);
  }
  hipLaunchKernelGGL(k_step_begin, dim3(1), dim3(256), 0, pb->stream, pb->part, pb->nparts, pb->sc, cfl, g.h,
                     pb->k.mu, use_cfl);
  return launch_check(pb, "step_begin");
}

fdcgks_status check_params(const fdcgks_params* p) {
  if (!p) return fail(nullptr, FDCGKS_EINVAL, "params is NULL");
  if (p->dim != 1 && p->dim != 2) return fail(nullptr, FDCGKS_EINVAL, "dim must be 1 or 2 (got %d)", p->dim);
  if (p->dim == 2 && (p->nx < 4 || p->ny < 4))
    return fail(nullptr, FDCGKS_EINVAL, "2D needs nx, ny >= 4 (got %d x %d)", p->nx, p->ny);
  if (p->dim == 1 && (p->nx < 4 || p->ny != 1))
    return fail(nullptr, FDCGKS_EINVAL, "1D needs nx >= 4 and ny == 1 (got %d, %d)", p->nx, p->ny);
  if ((long)p->nx * p->ny > (1L << 28)) return fail(nullptr, FDCGKS_EINVAL, "grid too large");
  if (p->dim == 2 && p->bc != FDCGKS_BC_PERIODIC)
    return fail(nullptr, FDCGKS_EINVAL, "2D supports periodic boundaries only");
  if (p->bc != FDCGKS_BC_PERIODIC && p->bc != FDCGKS_BC_ZERO_GRADIENT)
    return fail(nullptr, FDCGKS_EINVAL, "unknown boundary condition %d", p->bc);
  if (!(p->lx > 0) || (p->dim == 2 && !(p->ly > 0))) return fail(nullptr, FDCGKS_EINVAL, "domain lengths must be > 0");
  if (p->dim == 2) {
    double hx = p->lx / p->nx, hy = p->ly / p->ny;
    if (std::fabs(hx - hy) > 1e-12 * hx) return fail(nullptr, FDCGKS_EINVAL, "2D needs lx/nx == ly/ny");
  }
  double gmax = p->dim == 2 ? 5.0 / 3.0 : 3.0;
  if (!(p->gamma > 1.0) || !(p->gamma < gmax)) return fail(nullptr, FDCGKS_EINVAL, "gamma out of range");
  if (!(p->mu >= 0)) return fail(nullptr, FDCGKS_EINVAL, "mu must be >= 0");
  if (p->mu > 0 && !(p->prandtl > 0)) return fail(nullptr, FDCGKS_EINVAL, "prandtl must be > 0");
  if (p->flux_variant < 0 || p->flux_variant > 2) return fail(nullptr, FDCGKS_EINVAL, "bad flux_variant");
  if (p->flux_precision != FDCGKS_FP64 && p->flux_precision != FDCGKS_FP32_FLUX)
    return fail(nullptr, FDCGKS_EINVAL, "bad flux_precision");
  if (p->grad_update != FDCGKS_GRAD_REEVAL && p->grad_update != FDCGKS_GRAD_CARRIED)
    return fail(nullptr, FDCGKS_EINVAL, "bad grad_update");
  if (p->geno_r < 1 || p->geno_r > 8) return fail(nullptr, FDCGKS_EINVAL, "geno_r must be in 1..8");
  if (!(p->geno_C > 0) || !(p->geno_eps > 0) || !(p->geno_eps_a > 0) || !(p->geno_d_central > 0) ||
      !(p->geno_d_side > 0))
    return fail(nullptr, FDCGKS_EINVAL, "GENO constants must be > 0");
  if (!(p->tau_c1 >= 0) || !(p->tau_c2 >= 0)) return fail(nullptr, FDCGKS_EINVAL, "tau constants must be >= 0");
  if (p->reserved != 0) return fail(nullptr, FDCGKS_EINVAL, "reserved must be 0");
  return FDCGKS_OK;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

void fdcgks_default_params(fdcgks_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->dim = 2;
  p->nx = p->ny = 64;
  p->bc = FDCGKS_BC_PERIODIC;
  p->flux_variant = FDCGKS_FLUX_6_4;
  p->flux_precision = FDCGKS_FP64;
  p->grad_update = FDCGKS_GRAD_REEVAL;
  p->geno_r = 3;
  p->lx = p->ly = 1.0;
  p->gamma = 1.4;
  p->prandtl = 1.0;
  p->geno_C = 20.0;
  p->geno_eps = 1e-15;
  p->geno_eps_a = 1e-6;
  p->geno_d_central = 8.0;
  p->geno_d_side = 1.0;
  p->tau_c1 = 0.0;
  p->tau_c2 = 1.0;
}

fdcgks_status fdcgks_create(const fdcgks_params* p, void* hip_stream, fdcgks_problem** out) {
  if (!out) return fail(nullptr, FDCGKS_EINVAL, "out is NULL");
  *out = nullptr;
  fdcgks_status st = check_params(p);
  if (st) return st;
  fdcgks_problem* pb = new fdcgks_problem();
  pb->prm = *p;
  pb->stream = (hipStream_t)hip_stream;
  Geo& g = pb->g;
  g.nx = p->nx;
  g.ny = p->ny;
  g.pitch = ((p->nx + 2 * OX) + 15) / 16 * 16;
  g.rows = p->ny + 2 * OY;
  g.plane = (long)g.pitch * g.rows;
  g.h = p->lx / p->nx;
  g.invh = 1.0 / g.h;
  Consts& k = pb->k;
  k.gamma = p->gamma;
  k.K = p->dim == 2 ? (4.0 - 2.0 * p->gamma) / (p->gamma - 1.0) : (3.0 - p->gamma) / (p->gamma - 1.0);
  k.mu = p->mu;
  k.prfix = p->mu > 0 ? 1.0 / p->prandtl - 1.0 : 0.0;
  k.C = p->geno_C;
  k.inv_tanhC = 1.0 / std::tanh(p->geno_C);
  k.eps = p->geno_eps;
  k.eps_a = p->geno_eps_a;
  k.dc = p->geno_d_central;
  k.ds = p->geno_d_side;
  k.tau_c1 = p->tau_c1;
  k.tau_c2 = p->tau_c2;
  k.r = p->geno_r;
  k.variant = p->flux_variant;
  k.grad_carried = p->grad_update == FDCGKS_GRAD_CARRIED;
  pb->ngrid = p->dim == 2 ? 2 : (p->dual_1d ? 2 : 1);
  pb->nplanes = (int)state_planes(*p);
  if (p->dim == 1) {
    delete pb;
    return fail(nullptr, FDCGKS_EINVAL, "1D problems are not available in this build");
  }
  size_t sbytes = (size_t)pb->nplanes * g.plane * sizeof(double);
  size_t ebytes = (size_t)100 * g.plane * sizeof(double);
  size_t nbytes = (size_t)32 * g.plane * sizeof(double);
  pb->nparts = 512;
  hipError_t e = hipSuccess;
  double** tgt[] = {&pb->S[0], &pb->S[1], &pb->Sstar, &pb->Acc};
  for (double** t : tgt)
    if (e == hipSuccess) e = hipMalloc((void**)t, sbytes);
  if (e == hipSuccess) e = hipMalloc((void**)&pb->E, ebytes);
  if (e == hipSuccess) e = hipMalloc((void**)&pb->Nb, nbytes);
  if (e == hipSuccess) e = hipMalloc((void**)&pb->part, (size_t)2 * pb->nparts * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&pb->sc, sizeof(Scal));
  if (e == hipSuccess) e = hipHostMalloc((void**)&pb->sc_host, sizeof(Scal), hipHostMallocDefault);
  if (e == hipSuccess) {
    // zero everything once so that halo / unused padding never holds garbage
    for (double** t : tgt) if (e == hipSuccess) e = hipMemsetAsync(*t, 0, sbytes, pb->stream);
    if (e == hipSuccess) e = hipMemsetAsync(pb->E, 0, ebytes, pb->stream);
    if (e == hipSuccess) e = hipMemsetAsync(pb->Nb, 0, nbytes, pb->stream);
    if (e == hipSuccess) e = hipMemsetAsync(pb->sc, 0, sizeof(Scal), pb->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(pb->stream);
  }
  if (e != hipSuccess) {
    fdcgks_status code = (e == hipErrorOutOfMemory) ? FDCGKS_ENOMEM : FDCGKS_EHIP;
    fail(nullptr, code, "device allocation failed: %s", hipGetErrorString(e));
    free_all(pb);
    delete pb;
    return code;
  }
  *out = pb;
  return FDCGKS_OK;
}

static fdcgks_status copy_grid(fdcgks_problem* pb, int grid, double* const* ptrs, int to_device_state,
                               int on_device) {
  const Geo& g = pb->g;
  int ncomp = pb->prm.dim == 2 ? 4 : 3;
  int nfield = pb->prm.dim == 2 ? 3 : 2;
  double* base = pb->S[pb->cur] + (long)grid * (pb->prm.dim == 2 ? 12 : 6) * g.plane;
  size_t row = (size_t)g.nx * sizeof(double);
  hipMemcpyKind kind = to_device_state ? (on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice)
                                       : (on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost);
  for (int f = 0; f < nfield; ++f)
    for (int c = 0; c < ncomp; ++c) {
      double* dev = base + (long)(f * (pb->prm.dim == 2 ? 4 : 3) + c) * g.plane + (long)OY * g.pitch + OX;
      double* usr = ptrs[f] + (long)c * g.nx * g.ny;
      if (to_device_state)
        HIPCHK(pb, hipMemcpy2DAsync(dev, (size_t)g.pitch * sizeof(double), usr, row, row, g.ny, kind, pb->stream));
      else
        HIPCHK(pb, hipMemcpy2DAsync(usr, row, dev, (size_t)g.pitch * sizeof(double), row, g.ny, kind, pb->stream));
    }
  if (!on_device) HIPCHK(pb, hipStreamSynchronize(pb->stream));
  return FDCGKS_OK;
}

fdcgks_status fdcgks_set_state(fdcgks_problem* pb, int32_t grid, const double* W, const double* Wx, const double* Wy,
                               int32_t on_device) {
  if (!pb) return fail(nullptr, FDCGKS_EINVAL, "problem is NULL");
  if (grid < 0 || grid >= pb->ngrid) return fail(pb, FDCGKS_EINVAL, "grid %d not present", grid);
  if (!W || !Wx || (pb->prm.dim == 2 && !Wy)) return fail(pb, FDCGKS_EINVAL, "state pointer is NULL");
  double* ptrs[3] = {const_cast<double*>(W), const_cast<double*>(Wx), const_cast<double*>(Wy)};
  fdcgks_status st = copy_grid(pb, grid, ptrs, 1, on_device);
  if (st) return st;
  pb->have_state[grid] = true;
  return FDCGKS_OK;
}

fdcgks_status fdcgks_get_state(const fdcgks_problem* cpb, int32_t grid, double* W, double* Wx, double* Wy,
                               int32_t on_device) {
  fdcgks_problem* pb = const_cast<fdcgks_problem*>(cpb);
  if (!pb) return fail(nullptr, FDCGKS_EINVAL, "problem is NULL");
  if (grid < 0 || grid >= pb->ngrid) return fail(pb, FDCGKS_EINVAL, "grid %d not present", grid);
  if (!W || !Wx || (pb->prm.dim == 2 && !Wy)) return fail(pb, FDCGKS_EINVAL, "state pointer is NULL");
  double* ptrs[3] = {W, Wx, Wy};
  return copy_grid(pb, grid, ptrs, 0, on_device);
}

static bool state_ready(const fdcgks_problem* pb) {
  for (int g = 0; g < pb->ngrid; ++g)
    if (!pb->have_state[g]) return false;
  return true;
}

static fdcgks_status read_scal(fdcgks_problem* pb) {
  HIPCHK(pb, hipMemcpyAsync(pb->sc_host, pb->sc, sizeof(Scal), hipMemcpyDeviceToHost, pb->stream));
  HIPCHK(pb, hipStreamSynchronize(pb->stream));
  return FDCGKS_OK;
}
static fdcgks_status write_scal(fdcgks_problem* pb) {
  HIPCHK(pb, hipMemcpyAsync(pb->sc, pb->sc_host, sizeof(Scal), hipMemcpyHostToDevice, pb->stream));
  return FDCGKS_OK;
}

fdcgks_status fdcgks_compute_dt(fdcgks_problem* pb, double cfl, double* dt_out) {
  if (!pb || !dt_out) return fail(pb, FDCGKS_EINVAL, "NULL argument");
  if (!(cfl > 0)) return fail(pb, FDCGKS_EINVAL, "cfl must be > 0");
  if (!state_ready(pb)) return fail(pb, FDCGKS_ESTATE, "set_state has not been called for every grid");
  std::memset(pb->sc_host, 0, sizeof(Scal));
  fdcgks_status st = write_scal(pb);
  if (!st) st = begin_step(pb, 0.0, cfl);
  if (!st) st = read_scal(pb);
  if (st) return st;
  if (pb->sc_host->stop) return fail(pb, FDCGKS_ENONPHYS, "state gives no positive time step");
  *dt_out = pb->sc_host->dt;
  return FDCGKS_OK;
}

fdcgks_status fdcgks_step(fdcgks_problem* pb, double dt, double cfl, int32_t nsteps, double t_end, double* t_inout,
                          int32_t* steps_done) {
  if (!pb) return fail(nullptr, FDCGKS_EINVAL, "problem is NULL");
  if (!t_inout) return fail(pb, FDCGKS_EINVAL, "t_inout is NULL");
  if (nsteps < 0) return fail(pb, FDCGKS_EINVAL, "nsteps < 0");
  if (!(dt > 0) && !(cfl > 0)) return fail(pb, FDCGKS_EINVAL, "need dt > 0 or cfl > 0");
  if (!std::isfinite(dt) || !std::isfinite(*t_inout) || !std::isfinite(t_end))
    return fail(pb, FDCGKS_EINVAL, "dt, t and t_end must be finite");
  if (!state_ready(pb)) return fail(pb, FDCGKS_ESTATE, "set_state has not been called for every grid");
  if (steps_done) *steps_done = 0;
  Scal* h = pb->sc_host;
  std::memset(h, 0, sizeof(Scal));
  h->t = *t_inout;
  h->t_end = t_end;
  h->dt_fixed = dt;
  fdcgks_status st = write_scal(pb);
  if (st) return st;
  const int cur0 = pb->cur;
  int cur = cur0;
  pb->ev_used = 0;
  mark(pb, TK_STEP);
  for (int s = 0; s < nsteps; ++s) {
    pb->cur = cur;
    st = begin_step(pb, dt, cfl);
    mark(pb, TK_STEP);
    if (!st) st = stage2d<1>(pb, pb->S[cur], nullptr, pb->Sstar, pb->Acc);
    if (!st) st = stage2d<2>(pb, pb->Sstar, pb->Acc, pb->S[1 - cur], nullptr);
    if (st) break;
    hipLaunchKernelGGL(k_step_end, dim3(1), dim3(1), 0, pb->stream, pb->sc);
    mark(pb, TK_STEP);
    cur = 1 - cur;
  }
  fdcgks_status st2 = read_scal(pb);
  if (st) return st;
  if (st2) return st2;
  int done = h->steps;
  pb->cur = cur0 ^ (done & 1);
  *t_inout = h->t;
  if (steps_done) *steps_done = done;
  if (h->stop & 1)
    return fail(pb, FDCGKS_ENONPHYS, "non-physical state in step %d stage %d at grid %d node (%d, %d)", done + 1,
                h->fail_stage, h->fail_grid, h->fail_i, h->fail_j);
  return FDCGKS_OK;
}

fdcgks_status fdcgks_destroy(fdcgks_problem* pb) {
  if (!pb) return FDCGKS_OK;
  if (pb->stream || true) (void)hipStreamSynchronize(pb->stream);
  free_all(pb);
  for (hipEvent_t e : pb->ev) (void)hipEventDestroy(e);
  delete pb;
  return FDCGKS_OK;
}

fdcgks_status fdcgks_step_timed(fdcgks_problem* pb, double dt, double cfl, int32_t nsteps, double t_end,
                                double* t_inout, int32_t* steps_done, double* kernel_ms) {
  if (!pb || !kernel_ms) return fail(pb, FDCGKS_EINVAL, "NULL argument");
  for (int k = 0; k < TK_COUNT; ++k) kernel_ms[k] = 0.0;
  pb->timing = true;
  fdcgks_status st = fdcgks_step(pb, dt, cfl, nsteps, t_end, t_inout, steps_done);
  pb->timing = false;
  if (st != FDCGKS_OK && st != FDCGKS_ENONPHYS) return st;
  for (int e = 1; e < pb->ev_used; ++e) {
    float ms = 0.f;
    HIPCHK(pb, hipEventElapsedTime(&ms, pb->ev[e - 1], pb->ev[e]));
    kernel_ms[pb->ev_kind[e]] += ms;
  }
  return st;
}

const char* fdcgks_last_error(const fdcgks_problem* pb) {
  return pb ? pb->err.c_str() : g_create_error.c_str();
}

fdcgks_status fdcgks_debug_stage(fdcgks_problem* pb, int32_t stage, double dt, double* out_state, double* out_acc) {
  if (!pb || !out_state) return fail(pb, FDCGKS_EINVAL, "NULL argument");
  if (stage != 1 && stage != 2) return fail(pb, FDCGKS_EINVAL, "stage must be 1 or 2");
  if (!(dt > 0)) return fail(pb, FDCGKS_EINVAL, "dt must be > 0");
  if (!state_ready(pb)) return fail(pb, FDCGKS_ESTATE, "set_state has not been called for every grid");
  std::memset(pb->sc_host, 0, sizeof(Scal));
  pb->sc_host->dt = dt;
  fdcgks_status st = write_scal(pb);
  double* scratch = pb->S[1 - pb->cur];  // the next-state buffer is free between steps
  if (!st) {
    if (stage == 1) st = stage2d<1>(pb, pb->S[pb->cur], nullptr, pb->Sstar, pb->Acc);
    else st = stage2d<2>(pb, pb->Sstar, pb->Acc, scratch, nullptr);
  }
  if (st) return st;
  const Geo& g = pb->g;
  const double* src = stage == 1 ? pb->Sstar : scratch;
  size_t row = (size_t)g.nx * sizeof(double), pitchb = (size_t)g.pitch * sizeof(double);
  long n = (long)g.nx * g.ny;
  for (int p = 0; p < pb->nplanes; ++p) {
    HIPCHK(pb, hipMemcpy2DAsync(out_state + p * n, row, src + p * g.plane + (long)OY * g.pitch + OX, pitchb, row,
                                g.ny, hipMemcpyDeviceToHost, pb->stream));
    if (stage == 1 && out_acc)
      HIPCHK(pb, hipMemcpy2DAsync(out_acc + p * n, row, pb->Acc + p * g.plane + (long)OY * g.pitch + OX, pitchb, row,
                                  g.ny, hipMemcpyDeviceToHost, pb->stream));
  }
  return read_scal(pb);
}

fdcgks_status fdcgks_debug_intermediates(fdcgks_problem* pb, double dt, double* edge_x, double* edge_y,
                                         double* node_p, double* node_d) {
  if (!pb || !edge_x || !edge_y || !node_p || !node_d) return fail(pb, FDCGKS_EINVAL, "NULL argument");
  if (pb->prm.dim != 2) return fail(pb, FDCGKS_EINVAL, "2D only");
  if (!(dt > 0)) return fail(pb, FDCGKS_EINVAL, "dt must be > 0");
  if (!state_ready(pb)) return fail(pb, FDCGKS_ESTATE, "set_state has not been called for every grid");
  std::memset(pb->sc_host, 0, sizeof(Scal));
  pb->sc_host->dt = dt;
  fdcgks_status st = write_scal(pb);
  if (!st) st = stage2d<1>(pb, pb->S[pb->cur], nullptr, pb->Sstar, pb->Acc);
  if (st) return st;
  const Geo& g = pb->g;
  size_t row = (size_t)g.nx * sizeof(double), pitchb = (size_t)g.pitch * sizeof(double);
  long n = (long)g.nx * g.ny;
  // device edge planes are [family][slot primary/dual][25]; the output is
  // [family][normal x/y][25]: X: primary line = x, dual = y; Y: the reverse
  for (int fam = 0; fam < 2; ++fam)
    for (int ax = 0; ax < 2; ++ax) {
      int slot = fam == 0 ? ax : 1 - ax;
      double* dst = (fam == 0 ? edge_x : edge_y) + (long)ax * 25 * n;
      for (int q = 0; q < 25; ++q)
        HIPCHK(pb, hipMemcpy2DAsync(dst + q * n, row,
                                    pb->E + ((long)fam * 50 + slot * 25 + q) * g.plane + (long)OY * g.pitch + OX,
                                    pitchb, row, g.ny, hipMemcpyDeviceToHost, pb->stream));
    }
  for (int gr = 0; gr < 2; ++gr)
    for (int q = 0; q < 16; ++q)
      HIPCHK(pb, hipMemcpy2DAsync((gr == 0 ? node_p : node_d) + q * n, row,
                                  pb->Nb + ((long)gr * 16 + q) * g.plane + (long)OY * g.pitch + OX, pitchb, row, g.ny,
                                  hipMemcpyDeviceToHost, pb->stream));
  return read_scal(pb);
}

}  // extern "C"
