// libfdcgks, 3D: gfx950 kernels and host runtime of the 3D FD-CGKS stage on
// the four-grid lattice (primary grid plus the three face-offset duals).
//
// Device layout.  All buffers are SoA planes of n = nx*ny*nz doubles, x
// fastest, cell (i, j, k) at (k*ny + j)*nx + i; all axes periodic.
//   state buffer : 4 grids x 20 planes (W[5], Wx[5], Wy[5], Wz[5])
//   edge buffer  : 4 interface classes x 3 normal axes x 31 planes:
//                  F[5], Ft[5], chi, Wl[5], Wr[5], Wlt[5], Wrt[5] (blended)
//   node buffer  : 4 grids x 30 planes: per axis F[5], Ft[5]
// Parities along (x, y, z) as bit masks (bit a set: even coordinate along a):
// grids P 000, Dxy 011, Dxz 101, Dyz 110; interface classes 001, 010, 100,
// 111.  The line along axis a through a point flips bit a: it joins an
// interface point to the nodes of one grid, and a node to the interface
// points of one class.
//
// One S2O4 stage = interface sweep (three line reconstructions and three
// gas-kinetic solves per interface point, one thread per solve, the three
// threads of a point exchanging tangential slopes and interface values in
// LDS) -> node sweep (three derivative reconstructions + smooth nodal
// solver) -> update (compact fluxes along the three axes, averaged gradients,
// S2O4 combination).

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fdcgks3d.h"
#include "gks3d_device.hpp"
#include "gks_device.hpp"

using fdk::Consts;

namespace {

constexpr int NSP = 20;   // state planes per grid
constexpr int NEP = 31;   // edge planes per (class, axis)
constexpr int NNP = 30;   // node-flux planes per grid
constexpr int EDGE_THREADS = 256;   // interface sweep block: four waves
constexpr int EDGE_WAVE_POINTS = 21;  // interface points per wave (63 busy lanes, 3 solves per point)
constexpr int EDGE_POINTS = 4 * EDGE_WAVE_POINTS;  // interface points per block
// Minimum waves per SIMD of the interface and node sweeps.  Measured on a
// 128^3 Navier-Stokes step: the interface sweep is fastest at 1 (about 440
// registers, no spills; 2 waves spill 192 registers and take 40% longer),
// the node sweep at 2 (17% faster than at 1).
#ifndef FDCGKS3D_EDGE_WAVES
#define FDCGKS3D_EDGE_WAVES 1
#endif
#ifndef FDCGKS3D_NODE_WAVES
#define FDCGKS3D_NODE_WAVES 2
#endif
constexpr int NODE_BLOCK = 128;
constexpr int UPD_BLOCK = 128;

struct Geo3 {
  int nx, ny, nz;
  long n;  // nodes per grid
  double h, invh;
};

__host__ __device__ constexpr int grid_mask(int g) { return g == 0 ? 0 : (g == 1 ? 3 : (g == 2 ? 5 : 6)); }
__host__ __device__ constexpr int class_mask(int q) { return q == 0 ? 1 : (q == 1 ? 2 : (q == 2 ? 4 : 7)); }
__host__ __device__ constexpr int grid_of(int m) { return m == 0 ? 0 : (m == 3 ? 1 : (m == 5 ? 2 : 3)); }
__host__ __device__ constexpr int class_of(int m) { return m == 1 ? 0 : (m == 2 ? 1 : (m == 4 ? 2 : 3)); }

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Stored index of the point at odd lattice offset o along an axis from a
// point with stored index i, whose coordinate there is even (2i+2) or odd
// (2i+1).
__device__ __forceinline__ int odd_step(int i, int o, bool even) { return even ? i + (o + 1) / 2 : i + (o - 1) / 2; }

struct Cell {
  int c[3];  // i, j, k
};

__device__ __forceinline__ long cell_index(const Geo3& g, int i, int j, int k) { return ((long)k * g.ny + j) * g.nx + i; }

// One axis seen from a cell: its coordinate, extent and cell-index stride
// (selected without indexing an array, so a runtime axis needs no scratch).
struct Axis {
  int coord, n;
  long stride;
};
__device__ __forceinline__ Axis axis_of(const Geo3& g, const Cell& c, int ax) {
  Axis a;
  a.coord = ax == 0 ? c.c[0] : (ax == 1 ? c.c[1] : c.c[2]);
  a.n = ax == 0 ? g.nx : (ax == 1 ? g.ny : g.nz);
  a.stride = ax == 0 ? 1L : (ax == 1 ? (long)g.nx : (long)g.nx * g.ny);
  return a;
}
// Cell index of the point at stored index m along the axis from `cell`.
__device__ __forceinline__ long cell_along(long cell, const Axis& a, int m) {
  return cell + (long)(wrap(m, a.n) - a.coord) * a.stride;
}

// Local frame of a line along axis ax: components 1 and 1 + ax swapped (the
// momentum along the line becomes component 1).  Local component cc is global
// component lperm(ax, cc) and vice versa (the swap is its own inverse).
__device__ __forceinline__ int lperm(int ax, int cc) { return cc == 1 ? 1 + ax : (cc == 1 + ax ? 1 : cc); }

// Orders the LDS accesses of one wave: writes before the call are seen by
// every lane of the wave after it.  A wave's LDS operations execute in order;
// the fences keep the compiler from moving accesses across the call.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// --------------------------------------------------------- interface sweep
// One thread per (interface point, normal axis): lane l < 63 of wave w takes
// point 21 w + l / 3 of EDGE_POINTS consecutive points of one class (cells in
// x-fastest order) and normal axis l % 3; lane 63 idles.  The three solves of
// a point thus sit in neighbouring lanes of one wave, which exchange data
// through LDS with wave-level ordering only (no block barrier, so a wave never
// waits for the other waves of its block).  A block is four waves: the solver
// needs about 440 registers, one wave per SIMD, and a four-wave block keeps all
// four SIMDs of a compute unit busy (a three-wave block left one idle).
// The axis varies across a wave, so every component permutation goes through
// LDS (addresses are free to compute; registers cannot be indexed at run
// time):
//   phase 1: line reconstruction -> LDS (global component order);
//   phase 2: the solve's inputs read from LDS in the line's local frame, the
//            tangential slopes from the other two lines' entries;
//   phase 3: the solve; fluxes to HBM, interface values -> LDS;
//   phase 4: blend of the interface values over the three directions.
template <bool VALUES, bool CHAR>
__global__ __launch_bounds__(EDGE_THREADS, FDCGKS3D_EDGE_WAVES) void k_edges3d(Consts k, Geo3 g, double dt,
                                                                              const double* __restrict__ S,
                                                                              double* __restrict__ E) {
  __shared__ double xs[20][EDGE_THREADS];
  const int t = threadIdx.x;
  const int lane = t % 64, wv = t / 64;
  const bool busy = lane < 3 * EDGE_WAVE_POINTS;
  const int ax = busy ? lane % 3 : 0;
  const int base = t - ax;  // slot of this point's x solve (the idle lane reads its own slots)
  const int q = blockIdx.y;
  const long P = (long)blockIdx.x * EDGE_POINTS + wv * EDGE_WAVE_POINTS + lane / 3;
  const bool live = busy && P < g.n;
  const long cell = live ? P : 0;
  Cell c;
  c.c[0] = (int)(cell % g.nx);
  c.c[1] = (int)((cell / g.nx) % g.ny);
  c.c[2] = (int)(cell / ((long)g.nx * g.ny));
  const int qm = class_mask(q);
  const bool even = (qm >> ax) & 1;
  const int gl = grid_of(qm ^ (1 << ax));  // grid of this line's nodes
  const double* Sg = S + (long)gl * NSP * g.n;
  const Axis A = axis_of(g, c, ax);
  // phase 1: line reconstruction (conservative: chi from the density line;
  // characteristic: in the line's local frame, chi from the u -+ c fields)
  double chi;
  if (CHAR) {
    long at[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) at[m] = cell_along(cell, A, odd_step(A.coord, 2 * m - 3, even));
    double Q[5][4], X[5][4];
#pragma unroll
    for (int cc = 0; cc < 5; ++cc) {
      const int p = lperm(ax, cc);
      const double* W = Sg + (long)p * g.n;
      const double* Xp = Sg + (long)(5 * (1 + ax) + p) * g.n;
#pragma unroll
      for (int m = 0; m < 4; ++m) { Q[cc][m] = W[at[m]]; X[cc][m] = Xp[at[m]]; }
    }
    fdk::IfaceRec rec[5];
    fdk::recon_iface_char<3>(k, Q, X, g.h, g.invh, rec, chi);
#pragma unroll
    for (int cc = 0; cc < 5; ++cc) {
      const int p = lperm(ax, cc);
      xs[p][t] = rec[cc].vl;
      xs[5 + p][t] = rec[cc].vr;
      xs[10 + p][t] = rec[cc].dl;
      xs[15 + p][t] = rec[cc].dr;
    }
  } else {
    long at[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) at[m] = cell_along(cell, A, odd_step(A.coord, 2 * m - 3, even));
    // all 40 stencil values are loaded before the first reconstruction, so a
    // wave waits for memory once rather than once per component
    double Q[5][4], X[5][4];
#pragma unroll
    for (int cc = 0; cc < 5; ++cc) {
      const double* W = Sg + (long)cc * g.n;
      const double* Xp = Sg + (long)(5 * (1 + ax) + cc) * g.n;
#pragma unroll
      for (int m = 0; m < 4; ++m) { Q[cc][m] = W[at[m]]; X[cc][m] = Xp[at[m]]; }
    }
#pragma unroll
    for (int cc = 0; cc < 5; ++cc) {
      fdk::IfaceRec r = fdk::recon_iface<double>(k, Q[cc][0], Q[cc][1], Q[cc][2], Q[cc][3], X[cc][0], X[cc][1],
                                                 X[cc][2], X[cc][3], g.h, g.invh);
      xs[cc][t] = r.vl;
      xs[5 + cc][t] = r.vr;
      xs[10 + cc][t] = r.dl;
      xs[15 + cc][t] = r.dr;
      if (cc == 0) chi = fdk::g_min(r.cl, r.cr);
    }
  }
  wave_sync();
  // phase 2: inputs in the local frame; the local v and w are the velocities
  // of axes av and aw, whose lines give the tangential slopes (mean of their
  // l and r derivatives)
  const int tv = base + (ax == 1 ? 0 : 1), tw = base + (ax == 2 ? 0 : 2);
  fdk3::GksIO3 io;
#pragma unroll
  for (int cc = 0; cc < 5; ++cc) {
    const int p = lperm(ax, cc);
    io.WL[cc] = xs[p][t];
    io.WR[cc] = xs[5 + p][t];
    io.nL[cc] = xs[10 + p][t];
    io.nR[cc] = xs[15 + p][t];
    io.Wt[cc] = 0.5 * (xs[10 + p][tv] + xs[15 + p][tv]);
    io.Wt2[cc] = 0.5 * (xs[10 + p][tw] + xs[15 + p][tw]);
  }
  wave_sync();
  // phase 3: the solve; fluxes go out, interface values to LDS (global order)
  fdk3::gks_iface<VALUES>(k, dt, io);
  double* Eo = E + (long)(q * 3 + ax) * NEP * g.n + cell;
#pragma unroll
  for (int cc = 0; cc < 5; ++cc) {
    const int p = lperm(ax, cc);
    xs[10 + p][t] = io.Wlt[cc];
    xs[15 + p][t] = io.Wrt[cc];
    if (VALUES) {
      xs[p][t] = io.Wl[cc];
      xs[5 + p][t] = io.Wr[cc];
    }
    if (live) {
      Eo[(long)(5 + p) * g.n] = io.Ft[cc];
      if (VALUES) Eo[(long)p * g.n] = io.F[cc];
    }
  }
  wave_sync();
  // phase 4: blend, weight 1/3 per direction (the normal one with its own
  // side, the tangential ones with the mean of l and r)
  const int b1 = base + (ax == 0 ? 1 : 0), b2 = base + (ax == 2 ? 1 : 2);  // the other axes, increasing
  if (!live) return;
#pragma unroll
  for (int cc = 0; cc < 5; ++cc) {
    const double st = (xs[10 + cc][b1] + xs[15 + cc][b1]) + (xs[10 + cc][b2] + xs[15 + cc][b2]);
    Eo[(21 + cc) * g.n] = xs[10 + cc][t] / 3.0 + st / 6.0;
    Eo[(26 + cc) * g.n] = xs[15 + cc][t] / 3.0 + st / 6.0;
    if (VALUES) {
      const double sv = (xs[cc][b1] + xs[5 + cc][b1]) + (xs[cc][b2] + xs[5 + cc][b2]);
      Eo[(11 + cc) * g.n] = xs[cc][t] / 3.0 + sv / 6.0;
      Eo[(16 + cc) * g.n] = xs[5 + cc][t] / 3.0 + sv / 6.0;
    }
  }
  Eo[10 * g.n] = chi;
}

// -------------------------------------------------------------- node sweep
template <bool VALUES, bool CHAR>
__global__ __launch_bounds__(NODE_BLOCK, FDCGKS3D_NODE_WAVES) void k_nodes3d(Consts k, Geo3 g, const double* __restrict__ S,
                                                        double* __restrict__ Nb) {
  const int nbx = (g.nx + NODE_BLOCK - 1) / NODE_BLOCK;
  const int row = blockIdx.x / nbx;
  const int i = (blockIdx.x % nbx) * NODE_BLOCK + threadIdx.x;
  if (i >= g.nx) return;
  const int gr = blockIdx.y;
  Cell c;
  c.c[0] = i;
  c.c[1] = row % g.ny;
  c.c[2] = row / g.ny;
  const long cell = cell_index(g, c.c[0], c.c[1], c.c[2]);
  const double* Sg = S + (long)gr * NSP * g.n;
  double W[5], D[3][5];
#pragma unroll
  for (int cc = 0; cc < 5; ++cc) W[cc] = Sg[(long)cc * g.n + cell];
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const Axis A = axis_of(g, c, ax);
    const long am = cell_along(cell, A, A.coord - 1), ap = cell_along(cell, A, A.coord + 1);
    if (CHAR) {  // in the line's local frame (ax is a compile-time index here)
      double Q[5][3], X[5][3], d[5];
#pragma unroll
      for (int cc = 0; cc < 5; ++cc) {
        const int p = lperm(ax, cc);
        const double* Wp = Sg + (long)p * g.n;
        const double* Xp = Sg + (long)(5 * (1 + ax) + p) * g.n;
        Q[cc][0] = Wp[am]; Q[cc][1] = Wp[cell]; Q[cc][2] = Wp[ap];
        X[cc][0] = Xp[am]; X[cc][1] = Xp[cell]; X[cc][2] = Xp[ap];
      }
      fdk::recon_node_char<3>(k, Q, X, g.h, g.invh, d);
#pragma unroll
      for (int cc = 0; cc < 5; ++cc) D[ax][lperm(ax, cc)] = d[cc];
      continue;
    }
    // the axis's 25 stencil values are loaded before the first reconstruction,
    // so a wave waits for memory once per axis rather than once per component
    double Wm[5], Wq[5], Xm[5], X0[5], Xq[5];
#pragma unroll
    for (int cc = 0; cc < 5; ++cc) {
      const double* Wp = Sg + (long)cc * g.n;
      const double* X = Sg + (long)(5 * (1 + ax) + cc) * g.n;
      Wm[cc] = Wp[am]; Wq[cc] = Wp[ap];
      Xm[cc] = X[am]; X0[cc] = X[cell]; Xq[cc] = X[ap];
    }
#pragma unroll
    for (int cc = 0; cc < 5; ++cc)
      D[ax][cc] = fdk::recon_node<double>(k, Wm[cc], W[cc], Wq[cc], Xm[cc], X0[cc], Xq[cc], g.h, g.invh);
  }
  double F[3][5], Ft[3][5];
  fdk3::gks_node<VALUES>(k, W, D[0], D[1], D[2], F, Ft);
  double* No = Nb + (long)gr * NNP * g.n + cell;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax)
#pragma unroll
    for (int cc = 0; cc < 5; ++cc) {
      No[(10 * ax + 5 + cc) * g.n] = Ft[ax][cc];
      if (VALUES) No[(10 * ax + cc) * g.n] = F[ax][cc];
    }
}

// ------------------------------------------------------------------ update
__device__ __forceinline__ double cflux(const Consts& k, double Fm, double Fc, double Fp, double Nm, double N0,
                                        double N1, double Np2, double chi) {
  return k.flux_order == 8 ? fdk::compact_flux8(k.variant, Fm, Fc, Fp, Nm, N0, N1, Np2, chi)
                           : fdk::compact_flux(k.variant, Fm, Fc, Fp, N0, N1, chi);
}

// Stage 1: Out = W*, grad W*; AccOut = W + dt L + dt^2/6 L_t and the base
// gradient.  Stage 2: Out = W^{n+1}, grad W^{n+1} from the stage-1
// accumulators Acc.  bad is set when an output node has rho <= 0, p <= 0 or
// a NaN.  The axes are taken one at a time (not unrolled) and each axis's
// gradient outputs are written as soon as they are known, so that only L and
// L_t stay live across axes: the kernel then runs at 4 waves per SIMD
// without spilling.
template <int STAGE>
__global__ __launch_bounds__(UPD_BLOCK, 4) void k_update3d(Consts k, Geo3 g, double dt, const double* __restrict__ S,
                                                           const double* __restrict__ Acc, const double* __restrict__ E,
                                                           const double* __restrict__ Nb, double* __restrict__ Out,
                                                           double* __restrict__ AccOut, int* bad) {
  const int nbx = (g.nx + UPD_BLOCK - 1) / UPD_BLOCK;
  const int row = blockIdx.x / nbx;
  const int i = (blockIdx.x % nbx) * UPD_BLOCK + threadIdx.x;
  if (i >= g.nx) return;
  const int gr = blockIdx.y;
  const int gm = grid_mask(gr);
  Cell c;
  c.c[0] = i;
  c.c[1] = row % g.ny;
  c.c[2] = row / g.ny;
  const long cell = cell_index(g, c.c[0], c.c[1], c.c[2]);
  const bool wide = k.flux_order == 8;
  const double* Sg = S + (long)gr * NSP * g.n + cell;
  const double* Ag = (STAGE == 1 ? AccOut : Acc) + (long)gr * NSP * g.n + cell;
  double* Og = Out + (long)gr * NSP * g.n + cell;
  double* Aw = STAGE == 1 ? AccOut + (long)gr * NSP * g.n + cell : nullptr;
  double L[5], Lt[5];
#pragma unroll
  for (int cc = 0; cc < 5; ++cc) { L[cc] = 0.0; Lt[cc] = 0.0; }
#pragma unroll 1
  for (int ax = 0; ax < 3; ++ax) {
    const bool even = (gm >> ax) & 1;
    const int q = class_of(gm ^ (1 << ax));
    const double* Eq = E + (long)(q * 3 + ax) * NEP * g.n;
    const Axis A = axis_of(g, c, ax);
    const long em3 = cell_along(cell, A, odd_step(A.coord, -3, even));
    const long em1 = cell_along(cell, A, odd_step(A.coord, -1, even));
    const long ep1 = cell_along(cell, A, odd_step(A.coord, 1, even));
    const long ep3 = cell_along(cell, A, odd_step(A.coord, 3, even));
    const long nm = cell_along(cell, A, A.coord - 1), np = cell_along(cell, A, A.coord + 1);
    const long nm2 = wide ? cell_along(cell, A, A.coord - 2) : cell;
    const long np2 = wide ? cell_along(cell, A, A.coord + 2) : cell;
    const double* Ng = Nb + (long)gr * NNP * g.n + (long)(10 * ax) * g.n;
    const double chiR = Eq[10 * g.n + ep1], chiL = Eq[10 * g.n + em1];
#pragma unroll
    for (int cc = 0; cc < 5; ++cc) {
      const double* Ft = Eq + (long)(5 + cc) * g.n;
      const double* Nt = Ng + (long)(5 + cc) * g.n;
      const double FRt = cflux(k, Ft[em1], Ft[ep1], Ft[ep3], Nt[nm], Nt[cell], Nt[np], Nt[np2], chiR);
      const double FLt = cflux(k, Ft[em3], Ft[em1], Ft[ep1], Nt[nm2], Nt[nm], Nt[cell], Nt[np], chiL);
      Lt[cc] -= (FRt - FLt) * g.invh;
      const double Gt = (Eq[(21 + cc) * g.n + ep1] - Eq[(26 + cc) * g.n + em1]) * g.invh;
      const int f = 5 * (1 + ax) + cc;
      if (STAGE == 1) {
        const double* F = Eq + (long)cc * g.n;
        const double* Nf = Ng + (long)cc * g.n;
        const double FR = cflux(k, F[em1], F[ep1], F[ep3], Nf[nm], Nf[cell], Nf[np], Nf[np2], chiR);
        const double FL = cflux(k, F[em3], F[em1], F[ep1], Nf[nm2], Nf[nm], Nf[cell], Nf[np], chiL);
        L[cc] -= (FR - FL) * g.invh;
        const double G = (Eq[(11 + cc) * g.n + ep1] - Eq[(16 + cc) * g.n + em1]) * g.invh;
        const double gb = k.grad_carried ? Sg[f * g.n] : G;
        Og[f * g.n] = gb + 0.5 * dt * Gt;
        Aw[f * g.n] = gb;
      } else {
        Og[f * g.n] = Ag[f * g.n] + dt * Gt;
      }
    }
  }
  double o[5];
#pragma unroll
  for (int cc = 0; cc < 5; ++cc) {
    if (STAGE == 1) {
      const double w = Sg[cc * g.n];
      o[cc] = w + 0.5 * dt * L[cc] + 0.125 * dt * dt * Lt[cc];
      Aw[cc * g.n] = w + dt * L[cc] + dt * dt / 6.0 * Lt[cc];
    } else {
      o[cc] = Ag[cc * g.n] + dt * dt / 3.0 * Lt[cc];
    }
    Og[cc * g.n] = o[cc];
  }
  const double ke = 0.5 * (o[1] * o[1] + o[2] * o[2] + o[3] * o[3]) / o[0];
  const double p = (k.gamma - 1.0) * (o[4] - ke);
  if (!(o[0] > 0.0) || !(p > 0.0)) atomicOr(bad, 1);
}

// ------------------------------------------------------- CFL, diagnostics
// red[0]: max over nodes of max(|U|,|V|,|W|) + c, red[1]: min rho, both as
// the bit patterns of non-negative doubles (which order like the doubles).
__global__ void k_red_init(unsigned long long* red) {
  if (threadIdx.x == 0) {
    red[0] = 0ull;
    red[1] = (unsigned long long)__double_as_longlong(1e300);
  }
}

__global__ __launch_bounds__(256) void k_cfl3d(Geo3 g, double gamma, const double* __restrict__ S,
                                               unsigned long long* red) {
  __shared__ double smax[256], rmin[256];
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  double s = 0.0, r = 1e300;
  if (t < 4 * g.n) {
    const long gr = t / g.n, cell = t % g.n;
    const double* W = S + gr * NSP * g.n + cell;
    const double rho = W[0], U = W[g.n] / rho, V = W[2 * g.n] / rho, Wv = W[3 * g.n] / rho;
    const double p = (gamma - 1.0) * (W[4 * g.n] - 0.5 * rho * (U * U + V * V + Wv * Wv));
    const double cs = sqrt(gamma * p / rho);
    s = fmax(fabs(U), fmax(fabs(V), fabs(Wv))) + cs;
    r = rho;
    if (!(s >= 0.0)) s = 1e300;  // NaN: the step is refused downstream
  }
  smax[threadIdx.x] = s;
  rmin[threadIdx.x] = r;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
      rmin[threadIdx.x] = fmin(rmin[threadIdx.x], rmin[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicMax(red, (unsigned long long)__double_as_longlong(smax[0]));
    if (rmin[0] > 0.0) atomicMin(red + 1, (unsigned long long)__double_as_longlong(rmin[0]));
  }
}

__global__ void k_zero_int(int* p) {
  if (threadIdx.x == 0) *p = 0;
}

}  // namespace

struct fdcgks3d_problem {
  fdcgks3d_params prm;
  Consts k;
  Geo3 g;
  hipStream_t stream = nullptr;
  double* S[2] = {nullptr, nullptr};
  double* Sstar = nullptr;
  double* Acc = nullptr;
  double* E = nullptr;
  double* Nb = nullptr;
  unsigned long long* red = nullptr;  // CFL reduction slots (2)
  int* bad = nullptr;                 // non-physical flag
  unsigned long long* host = nullptr; // pinned readback (2 reduction slots + flag)
  int cur = 0;
  bool chr = false;  // characteristic reconstruction
  bool have[4] = {false, false, false, false};
  std::string err;
  std::vector<hipEvent_t> ev;
};

namespace {

thread_local char g_create_error3[512];

fdcgks_status fail(fdcgks3d_problem* pb, fdcgks_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (pb) pb->err = buf; else std::snprintf(g_create_error3, sizeof g_create_error3, "%s", buf);
  return st;
}
#define HIPCHK3(pb, call)                                                                    \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess) return fail(pb, FDCGKS_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

fdcgks_status launched(fdcgks3d_problem* pb, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(pb, FDCGKS_EHIP, "launch of %s failed: %s", what, hipGetErrorString(e));
  return FDCGKS_OK;
}

void free_all(fdcgks3d_problem* pb) {
  double* bufs[] = {pb->S[0], pb->S[1], pb->Sstar, pb->Acc, pb->E, pb->Nb};
  for (double* b : bufs) if (b) (void)hipFree(b);
  if (pb->red) (void)hipFree(pb->red);
  if (pb->bad) (void)hipFree(pb->bad);
  if (pb->host) (void)hipHostFree(pb->host);
  for (hipEvent_t e : pb->ev) (void)hipEventDestroy(e);
  pb->ev.clear();
  pb->S[0] = pb->S[1] = pb->Sstar = pb->Acc = pb->E = pb->Nb = nullptr;
  pb->red = nullptr;
  pb->bad = nullptr;
  pb->host = nullptr;
}

fdcgks_status check(const fdcgks3d_params* p) {
  if (!p) return fail(nullptr, FDCGKS_EINVAL, "params is NULL");
  if (p->nx < 4 || p->ny < 4 || p->nz < 4)
    return fail(nullptr, FDCGKS_EINVAL, "3D needs nx, ny, nz >= 4 (got %d x %d x %d)", p->nx, p->ny, p->nz);
  if ((long)p->nx * p->ny * p->nz > (1L << 26)) return fail(nullptr, FDCGKS_EINVAL, "grid too large");
  if (p->recon_vars != FDCGKS_RECON_CONSERVATIVE && p->recon_vars != FDCGKS_RECON_CHARACTERISTIC)
    return fail(nullptr, FDCGKS_EINVAL, "bad recon_vars");
  if (!(p->lx > 0)) return fail(nullptr, FDCGKS_EINVAL, "lx must be > 0");
  if (!(p->gamma > 1.0) || !(p->gamma < 5.0 / 3.0)) return fail(nullptr, FDCGKS_EINVAL, "gamma out of range");
  if (!(p->mu >= 0)) return fail(nullptr, FDCGKS_EINVAL, "mu must be >= 0");
  if (p->mu > 0 && !(p->prandtl > 0)) return fail(nullptr, FDCGKS_EINVAL, "prandtl must be > 0");
  if (p->flux_variant < 0 || p->flux_variant > 2) return fail(nullptr, FDCGKS_EINVAL, "bad flux_variant");
  if (p->flux_order != 6 && p->flux_order != 8) return fail(nullptr, FDCGKS_EINVAL, "flux_order must be 6 or 8");
  if (p->grad_update != FDCGKS_GRAD_REEVAL && p->grad_update != FDCGKS_GRAD_CARRIED)
    return fail(nullptr, FDCGKS_EINVAL, "bad grad_update");
  if (p->geno_r < 1 || p->geno_r > 8) return fail(nullptr, FDCGKS_EINVAL, "geno_r must be in 1..8");
  if (!(p->geno_C > 0) || !(p->geno_eps > 0) || !(p->geno_eps_a > 0) || !(p->geno_d_central > 0) ||
      !(p->geno_d_side > 0))
    return fail(nullptr, FDCGKS_EINVAL, "GENO constants must be > 0");
  if (!(p->tau_c1 >= 0) || !(p->tau_c2 >= 0)) return fail(nullptr, FDCGKS_EINVAL, "tau constants must be >= 0");
  return FDCGKS_OK;
}

void setup(const fdcgks3d_params& p, Geo3& g, Consts& k) {
  g.nx = p.nx;
  g.ny = p.ny;
  g.nz = p.nz;
  g.n = (long)p.nx * p.ny * p.nz;
  g.h = p.lx / p.nx;
  g.invh = 1.0 / g.h;
  std::memset(&k, 0, sizeof k);
  k.gamma = p.gamma;
  k.K = (5.0 - 3.0 * p.gamma) / (p.gamma - 1.0);
  k.inv_Kd = 1.0 / (k.K + 3.0);
  k.mu = p.mu;
  k.prfix = p.mu > 0 ? 1.0 / p.prandtl - 1.0 : 0.0;
  k.C = p.geno_C;
  k.inv_tanhC = 1.0 / std::tanh(p.geno_C);
  k.eps = p.geno_eps;
  k.eps_a = p.geno_eps_a;
  k.dc = p.geno_d_central;
  k.ds = p.geno_d_side;
  k.tau_c1 = p.tau_c1;
  k.tau_c2 = p.tau_c2;
  k.r = p.geno_r;
  k.variant = p.flux_variant;
  k.grad_carried = p.grad_update == FDCGKS_GRAD_CARRIED;
  k.flux_order = p.flux_order;
}

// Blocks along the flattened (x tiles, y, z) axis of a sweep: each block
// takes `width` consecutive points of one row of x.
unsigned blocks_x(const Geo3& g, int width) {
  return (unsigned)(((g.nx + width - 1) / width) * (long)g.ny * g.nz);
}

enum { T3_EDGE1 = 0, T3_NODE1, T3_UPD1, T3_EDGE2, T3_NODE2, T3_UPD2, T3_STEP, T3_COUNT };

struct Timer {
  fdcgks3d_problem* pb;
  bool on;
  int used = 0;
  std::vector<int> kind;
  void mark(int kd) {
    if (!on) return;
    if (used >= (int)pb->ev.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) { on = false; return; }
      pb->ev.push_back(e);
    }
    kind.push_back(kd);
    (void)hipEventRecord(pb->ev[used++], pb->stream);
  }
};

// One stage: Sin (and Ain for stage 2) -> Out (and Aout for stage 1).
fdcgks_status stage3d(fdcgks3d_problem* pb, int stage, double dt, const double* Sin, const double* Ain, double* Out,
                      double* Aout, Timer* tm) {
  const Geo3& g = pb->g;
  const dim3 eg((unsigned)((g.n + EDGE_POINTS - 1) / EDGE_POINTS), 4), eb(EDGE_THREADS);
  const dim3 ng(blocks_x(g, NODE_BLOCK), 4), nb(NODE_BLOCK);
  const dim3 ug(blocks_x(g, UPD_BLOCK), 4), ub(UPD_BLOCK);
  if (stage == 1) {
    if (pb->chr) hipLaunchKernelGGL((k_edges3d<true, true>), eg, eb, 0, pb->stream, pb->k, g, dt, Sin, pb->E);
    else hipLaunchKernelGGL((k_edges3d<true, false>), eg, eb, 0, pb->stream, pb->k, g, dt, Sin, pb->E);
    if (tm) tm->mark(T3_EDGE1);
    if (pb->chr) hipLaunchKernelGGL((k_nodes3d<true, true>), ng, nb, 0, pb->stream, pb->k, g, Sin, pb->Nb);
    else hipLaunchKernelGGL((k_nodes3d<true, false>), ng, nb, 0, pb->stream, pb->k, g, Sin, pb->Nb);
    if (tm) tm->mark(T3_NODE1);
    hipLaunchKernelGGL(k_update3d<1>, ug, ub, 0, pb->stream, pb->k, g, dt, Sin, (const double*)nullptr, pb->E,
                       pb->Nb, Out, Aout, pb->bad);
    if (tm) tm->mark(T3_UPD1);
  } else {
    if (pb->chr) hipLaunchKernelGGL((k_edges3d<false, true>), eg, eb, 0, pb->stream, pb->k, g, dt, Sin, pb->E);
    else hipLaunchKernelGGL((k_edges3d<false, false>), eg, eb, 0, pb->stream, pb->k, g, dt, Sin, pb->E);
    if (tm) tm->mark(T3_EDGE2);
    if (pb->chr) hipLaunchKernelGGL((k_nodes3d<false, true>), ng, nb, 0, pb->stream, pb->k, g, Sin, pb->Nb);
    else hipLaunchKernelGGL((k_nodes3d<false, false>), ng, nb, 0, pb->stream, pb->k, g, Sin, pb->Nb);
    if (tm) tm->mark(T3_NODE2);
    hipLaunchKernelGGL(k_update3d<2>, ug, ub, 0, pb->stream, pb->k, g, dt, Sin, Ain, pb->E, pb->Nb, Out,
                       (double*)nullptr, pb->bad);
    if (tm) tm->mark(T3_UPD2);
  }
  return launched(pb, "3D stage kernels");
}

fdcgks_status cfl_dt(fdcgks3d_problem* pb, const double* S, double cfl, double* dt) {
  const Geo3& g = pb->g;
  hipLaunchKernelGGL(k_red_init, dim3(1), dim3(64), 0, pb->stream, pb->red);
  const long nthr = 4 * g.n;
  hipLaunchKernelGGL(k_cfl3d, dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, pb->stream, g, pb->k.gamma, S,
                     pb->red);
  fdcgks_status st = launched(pb, "CFL reduction");
  if (st != FDCGKS_OK) return st;
  HIPCHK3(pb, hipMemcpyAsync(pb->host, pb->red, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, pb->stream));
  HIPCHK3(pb, hipStreamSynchronize(pb->stream));
  double smax, rmin;
  std::memcpy(&smax, &pb->host[0], sizeof smax);
  std::memcpy(&rmin, &pb->host[1], sizeof rmin);
  if (!(smax > 0.0) || !(smax < 1e299) || !(rmin > 0.0) || !(rmin < 1e299))
    return fail(pb, FDCGKS_ENONPHYS, "non-physical state: no finite CFL time step");
  double d = cfl * g.h / smax;
  if (pb->k.mu > 0) d = std::min(d, cfl * g.h * g.h / (8.0 * pb->k.mu / rmin));
  *dt = d;
  return FDCGKS_OK;
}

bool all_set(const fdcgks3d_problem* pb) { return pb->have[0] && pb->have[1] && pb->have[2] && pb->have[3]; }

// A pointer handed over with on_device = 1 must be device memory: a host
// pointer in a device-to-device copy would be read by the GPU.
bool device_memory(const void* p) {
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice;
}

fdcgks_status run(fdcgks3d_problem* pb, double dt, double cfl, int32_t nsteps, double t_end, double* t_inout,
                  int32_t* steps_done, double* kernel_ms) {
  if (steps_done) *steps_done = 0;
  if (!t_inout) return fail(pb, FDCGKS_EINVAL, "t_inout is NULL");
  if (nsteps < 0) return fail(pb, FDCGKS_EINVAL, "nsteps must be >= 0");
  if (!all_set(pb)) return fail(pb, FDCGKS_ESTATE, "set the state of all four grids first");
  if (dt <= 0 && !(cfl > 0)) return fail(pb, FDCGKS_EINVAL, "cfl must be > 0 when dt <= 0");
  if (!std::isfinite(dt) || !std::isfinite(*t_inout) || !std::isfinite(t_end))
    return fail(pb, FDCGKS_EINVAL, "dt, t and t_end must be finite");
  Timer tm{pb, kernel_ms != nullptr};
  std::vector<double> acc(T3_COUNT, 0.0);
  if (kernel_ms)
    for (int q = 0; q < T3_COUNT; ++q) kernel_ms[q] = 0.0;
  double t = *t_inout;
  int done = 0;
  fdcgks_status st = FDCGKS_OK;
  for (; done < nsteps; ++done) {
    if (t_end > 0 && t >= t_end) break;
    tm.used = 0;
    tm.kind.clear();
    tm.mark(-1);
    double* Sc = pb->S[pb->cur];
    double* Sn = pb->S[1 - pb->cur];
    double d = dt;
    if (d <= 0) {
      st = cfl_dt(pb, Sc, cfl, &d);
      if (st != FDCGKS_OK) break;
    }
    if (t_end > 0 && t + d > t_end) d = t_end - t;
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, pb->stream, pb->bad);
    tm.mark(T3_STEP);
    if ((st = stage3d(pb, 1, d, Sc, nullptr, pb->Sstar, pb->Acc, &tm)) != FDCGKS_OK) break;
    if ((st = stage3d(pb, 2, d, pb->Sstar, pb->Acc, Sn, nullptr, &tm)) != FDCGKS_OK) break;
    hipError_t e = hipMemcpyAsync(pb->host + 2, pb->bad, sizeof(int), hipMemcpyDeviceToHost, pb->stream);
    tm.mark(T3_STEP);
    if (e == hipSuccess) e = hipStreamSynchronize(pb->stream);
    if (e != hipSuccess) { st = fail(pb, FDCGKS_EHIP, "step: %s", hipGetErrorString(e)); break; }
    if (tm.on) {
      for (int q = 1; q < tm.used; ++q) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, pb->ev[q - 1], pb->ev[q]) == hipSuccess) acc[tm.kind[q]] += ms;
      }
    }
    int badv;
    std::memcpy(&badv, pb->host + 2, sizeof badv);
    if (badv) {
      st = fail(pb, FDCGKS_ENONPHYS, "step %d at t = %.17g produced rho <= 0, p <= 0 or NaN", done, t);
      break;
    }
    pb->cur = 1 - pb->cur;
    t += d;
  }
  if (kernel_ms)
    for (int q = 0; q < T3_COUNT; ++q) kernel_ms[q] = acc[q];
  *t_inout = t;
  if (steps_done) *steps_done = done;
  return st;
}

}  // namespace

extern "C" {

void fdcgks3d_default_params(fdcgks3d_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->nx = p->ny = p->nz = 32;
  p->flux_variant = FDCGKS_FLUX_6_4;
  p->flux_order = 6;
  p->grad_update = FDCGKS_GRAD_REEVAL;
  p->geno_r = 3;
  p->lx = 1.0;
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

fdcgks_status fdcgks3d_create(const fdcgks3d_params* p, void* hip_stream, fdcgks3d_problem** out) {
  if (!out) return fail(nullptr, FDCGKS_EINVAL, "out is NULL");
  *out = nullptr;
  fdcgks_status st = check(p);
  if (st != FDCGKS_OK) return st;
  fdcgks3d_problem* pb = new fdcgks3d_problem();
  pb->prm = *p;
  setup(*p, pb->g, pb->k);
  pb->chr = p->recon_vars == FDCGKS_RECON_CHARACTERISTIC;
  pb->stream = (hipStream_t)hip_stream;
  const long n = pb->g.n;
  const size_t state = (size_t)4 * NSP * n * sizeof(double);
  struct { double** ptr; size_t bytes; } allocs[] = {
      {&pb->S[0], state}, {&pb->S[1], state}, {&pb->Sstar, state}, {&pb->Acc, state},
      {&pb->E, (size_t)12 * NEP * n * sizeof(double)}, {&pb->Nb, (size_t)4 * NNP * n * sizeof(double)}};
  for (auto& a : allocs) {
    if (hipMalloc(a.ptr, a.bytes) != hipSuccess) {
      *a.ptr = nullptr;
      (void)hipGetLastError();
      free_all(pb);
      delete pb;
      return fail(nullptr, FDCGKS_ENOMEM, "device allocation of %zu bytes failed", a.bytes);
    }
  }
  if (hipMalloc(&pb->red, 2 * sizeof(unsigned long long)) != hipSuccess || hipMalloc(&pb->bad, sizeof(int)) != hipSuccess ||
      hipHostMalloc(&pb->host, 4 * sizeof(unsigned long long)) != hipSuccess) {
    (void)hipGetLastError();
    free_all(pb);
    delete pb;
    return fail(nullptr, FDCGKS_ENOMEM, "allocation of the step scalars failed");
  }
  *out = pb;
  return FDCGKS_OK;
}

fdcgks_status fdcgks3d_set_state(fdcgks3d_problem* pb, int32_t grid, const double* S, int32_t on_device) {
  if (!pb) return fail(nullptr, FDCGKS_EINVAL, "problem is NULL");
  if (grid < 0 || grid > 3) return fail(pb, FDCGKS_EINVAL, "grid must be 0..3");
  if (!S) return fail(pb, FDCGKS_EINVAL, "state pointer is NULL");
  if (on_device && !device_memory(S)) return fail(pb, FDCGKS_EINVAL, "on_device = 1 needs device memory");
  const size_t bytes = (size_t)NSP * pb->g.n * sizeof(double);
  double* dst = pb->S[pb->cur] + (long)grid * NSP * pb->g.n;
  if (on_device) HIPCHK3(pb, hipMemcpyAsync(dst, S, bytes, hipMemcpyDeviceToDevice, pb->stream));
  else {
    HIPCHK3(pb, hipMemcpyAsync(dst, S, bytes, hipMemcpyHostToDevice, pb->stream));
    HIPCHK3(pb, hipStreamSynchronize(pb->stream));
  }
  pb->have[grid] = true;
  return FDCGKS_OK;
}

fdcgks_status fdcgks3d_get_state(const fdcgks3d_problem* cpb, int32_t grid, double* S, int32_t on_device) {
  fdcgks3d_problem* pb = const_cast<fdcgks3d_problem*>(cpb);
  if (!pb) return fail(nullptr, FDCGKS_EINVAL, "problem is NULL");
  if (grid < 0 || grid > 3) return fail(pb, FDCGKS_EINVAL, "grid must be 0..3");
  if (!S) return fail(pb, FDCGKS_EINVAL, "state pointer is NULL");
  if (!pb->have[grid]) return fail(pb, FDCGKS_ESTATE, "grid %d has no state", grid);
  if (on_device && !device_memory(S)) return fail(pb, FDCGKS_EINVAL, "on_device = 1 needs device memory");
  const size_t bytes = (size_t)NSP * pb->g.n * sizeof(double);
  const double* src = pb->S[pb->cur] + (long)grid * NSP * pb->g.n;
  if (on_device) HIPCHK3(pb, hipMemcpyAsync(S, src, bytes, hipMemcpyDeviceToDevice, pb->stream));
  else {
    HIPCHK3(pb, hipMemcpyAsync(S, src, bytes, hipMemcpyDeviceToHost, pb->stream));
    HIPCHK3(pb, hipStreamSynchronize(pb->stream));
  }
  return FDCGKS_OK;
}

fdcgks_status fdcgks3d_compute_dt(fdcgks3d_problem* pb, double cfl, double* dt_out) {
  if (!pb) return fail(nullptr, FDCGKS_EINVAL, "problem is NULL");
  if (!dt_out || !(cfl > 0)) return fail(pb, FDCGKS_EINVAL, "need dt_out and cfl > 0");
  if (!all_set(pb)) return fail(pb, FDCGKS_ESTATE, "set the state of all four grids first");
  return cfl_dt(pb, pb->S[pb->cur], cfl, dt_out);
}

fdcgks_status fdcgks3d_diagnostics(fdcgks3d_problem* pb, double* out) {
  if (!pb) return fail(nullptr, FDCGKS_EINVAL, "problem is NULL");
  if (!out) return fail(pb, FDCGKS_EINVAL, "out is NULL");
  if (!all_set(pb)) return fail(pb, FDCGKS_ESTATE, "set the state of all four grids first");
  const long n = pb->g.n;
  std::vector<double> h((size_t)5 * n);
  double rmin = 1e300, pmin = 1e300;
  for (int gr = 0; gr < 4; ++gr) {
    HIPCHK3(pb, hipMemcpyAsync(h.data(), pb->S[pb->cur] + (long)gr * NSP * n, h.size() * sizeof(double),
                               hipMemcpyDeviceToHost, pb->stream));
    HIPCHK3(pb, hipStreamSynchronize(pb->stream));
    for (int c = 0; c < 5; ++c) {
      double s = 0.0;
      for (long q = 0; q < n; ++q) s += h[c * n + q];
      out[5 * gr + c] = s;
    }
    for (long q = 0; q < n; ++q) {
      const double rho = h[q];
      const double ke = 0.5 * (h[n + q] * h[n + q] + h[2 * n + q] * h[2 * n + q] + h[3 * n + q] * h[3 * n + q]) / rho;
      rmin = std::min(rmin, rho);
      pmin = std::min(pmin, (pb->k.gamma - 1.0) * (h[4 * n + q] - ke));
    }
  }
  out[20] = rmin;
  out[21] = pmin;
  return FDCGKS_OK;
}

fdcgks_status fdcgks3d_step(fdcgks3d_problem* pb, double dt, double cfl, int32_t nsteps, double t_end,
                            double* t_inout, int32_t* steps_done) {
  if (!pb) return fail(nullptr, FDCGKS_EINVAL, "problem is NULL");
  return run(pb, dt, cfl, nsteps, t_end, t_inout, steps_done, nullptr);
}

fdcgks_status fdcgks3d_step_timed(fdcgks3d_problem* pb, double dt, double cfl, int32_t nsteps, double t_end,
                                  double* t_inout, int32_t* steps_done, double* kernel_ms) {
  if (!pb) return fail(nullptr, FDCGKS_EINVAL, "problem is NULL");
  if (!kernel_ms) return fail(pb, FDCGKS_EINVAL, "kernel_ms is NULL");
  return run(pb, dt, cfl, nsteps, t_end, t_inout, steps_done, kernel_ms);
}

fdcgks_status fdcgks3d_debug_stage(fdcgks3d_problem* pb, int32_t stage, double dt, double* out_state,
                                   double* out_acc) {
  if (!pb) return fail(nullptr, FDCGKS_EINVAL, "problem is NULL");
  if (stage != 1 && stage != 2) return fail(pb, FDCGKS_EINVAL, "stage must be 1 or 2");
  if (!out_state || !(dt > 0)) return fail(pb, FDCGKS_EINVAL, "need out_state and dt > 0");
  if (!all_set(pb)) return fail(pb, FDCGKS_ESTATE, "set the state of all four grids first");
  const size_t bytes = (size_t)4 * NSP * pb->g.n * sizeof(double);
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, pb->stream, pb->bad);
  fdcgks_status st;
  if (stage == 1) {
    st = stage3d(pb, 1, dt, pb->S[pb->cur], nullptr, pb->Sstar, pb->Acc, nullptr);
    if (st != FDCGKS_OK) return st;
    HIPCHK3(pb, hipMemcpyAsync(out_state, pb->Sstar, bytes, hipMemcpyDeviceToHost, pb->stream));
    if (out_acc) HIPCHK3(pb, hipMemcpyAsync(out_acc, pb->Acc, bytes, hipMemcpyDeviceToHost, pb->stream));
  } else {
    double* scratch = pb->S[1 - pb->cur];
    st = stage3d(pb, 2, dt, pb->Sstar, pb->Acc, scratch, nullptr, nullptr);
    if (st != FDCGKS_OK) return st;
    HIPCHK3(pb, hipMemcpyAsync(out_state, scratch, bytes, hipMemcpyDeviceToHost, pb->stream));
  }
  HIPCHK3(pb, hipStreamSynchronize(pb->stream));
  return FDCGKS_OK;
}

fdcgks_status fdcgks3d_debug_intermediates(fdcgks3d_problem* pb, double dt, double* edges, double* nodes) {
  if (!pb) return fail(nullptr, FDCGKS_EINVAL, "problem is NULL");
  if (!edges || !nodes || !(dt > 0)) return fail(pb, FDCGKS_EINVAL, "need edges, nodes and dt > 0");
  if (!all_set(pb)) return fail(pb, FDCGKS_ESTATE, "set the state of all four grids first");
  const Geo3& g = pb->g;
  const dim3 eg((unsigned)((g.n + EDGE_POINTS - 1) / EDGE_POINTS), 4), eb(EDGE_THREADS);
  const dim3 ng(blocks_x(g, NODE_BLOCK), 4), nb(NODE_BLOCK);
  if (pb->chr) {
    hipLaunchKernelGGL((k_edges3d<true, true>), eg, eb, 0, pb->stream, pb->k, g, dt, pb->S[pb->cur], pb->E);
    hipLaunchKernelGGL((k_nodes3d<true, true>), ng, nb, 0, pb->stream, pb->k, g, pb->S[pb->cur], pb->Nb);
  } else {
    hipLaunchKernelGGL((k_edges3d<true, false>), eg, eb, 0, pb->stream, pb->k, g, dt, pb->S[pb->cur], pb->E);
    hipLaunchKernelGGL((k_nodes3d<true, false>), ng, nb, 0, pb->stream, pb->k, g, pb->S[pb->cur], pb->Nb);
  }
  fdcgks_status st = launched(pb, "3D interface / node sweeps");
  if (st != FDCGKS_OK) return st;
  HIPCHK3(pb, hipMemcpyAsync(edges, pb->E, (size_t)12 * NEP * g.n * sizeof(double), hipMemcpyDeviceToHost,
                             pb->stream));
  HIPCHK3(pb, hipMemcpyAsync(nodes, pb->Nb, (size_t)4 * NNP * g.n * sizeof(double), hipMemcpyDeviceToHost,
                             pb->stream));
  HIPCHK3(pb, hipStreamSynchronize(pb->stream));
  return FDCGKS_OK;
}

fdcgks_status fdcgks3d_destroy(fdcgks3d_problem* pb) {
  if (!pb) return FDCGKS_OK;
  free_all(pb);
  delete pb;
  return FDCGKS_OK;
}

const char* fdcgks3d_last_error(const fdcgks3d_problem* pb) { return pb ? pb->err.c_str() : g_create_error3; }

}  // extern "C"
