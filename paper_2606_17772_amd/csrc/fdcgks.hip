// libfdcgks: gfx950 kernels and host runtime of the FD-CGKS stage sweep.
//
// Device layout (2D).  Every field is a padded plane of FP64, x fastest:
// row pitch `pitch` doubles, interior node (i, j) at (j + OY) * pitch +
// (i + OX) with OX = 16 (interior rows start on a 128-byte cache line, so
// the 128-wide update tiles touch whole lines) and OY = 3; three halo
// rows/columns on each side hold the periodic images or the ghosts of
// bounded sides.
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

#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
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

constexpr int OX = 16, OY = 3, HALO = 3;

// Bounded axes: along an axis whose sides are not periodic the dual grid has
// nx + 1 (ny + 1) nodes, the first and last on the boundary lines.  Kernels
// index dual nodes as on a periodic grid, i in [-1, nx - 1] there, and reach
// the dual planes through `dshift` = sx + sy * pitch (stored dual node 0 is
// kernel node -1).  side: x-low, x-high, y-low, y-high (FDCGKS_BC_*).
struct Geo {
  int nx, ny, pitch, rows;
  long plane;
  double h, invh;
  int sx = 0, sy = 0;
  long dshift = 0;
  int side[4] = {0, 0, 0, 0};
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

// XCD-aware tile order.  The GPU deals consecutive workgroup ids round robin
// to its 8 XCDs, each with its own L2, so row-major tiles put vertically
// neighbouring tiles (which read the same stencil rows) on different L2s.
// Instead every XCD takes a contiguous band of tiles: launch id (over ntiles
// rounded up to a multiple of 8) -> tile; false for the padding ids.
constexpr int NXCD = 8;
__device__ __forceinline__ bool xcd_tile(int id, int padded, int ntiles, int& tile) {
  tile = (id % NXCD) * (padded / NXCD) + id / NXCD;
  return tile < ntiles;
}

// ------------------------------------------------------------ halo fill
// Ghost index a along an axis of n real nodes of one grid: the node it copies
// and the factor.  Periodic: the periodic image.  Zero-gradient: the end node,
// the derivative normal to the side zeroed.  Reflecting / no-slip: the mirror
// image about the boundary line, which lies half a mesh beyond the end node
// (primary) or through it (dual, on_line); the normal momentum is odd
// (no-slip: both momenta) and a derivative normal to the side has the
// opposite parity of its component.
__device__ __forceinline__ int ghost_src(int a, int n, int lo, int hi, bool on_line, bool normal_deriv, bool odd_refl,
                                         bool odd_noslip, double& fac) {
  fac = 1.0;
  if (lo == FDCGKS_BC_PERIODIC) return imod(a, n);
  const int type = a < 0 ? lo : hi;
  if (type == FDCGKS_BC_ZERO_GRADIENT) {
    if (normal_deriv) fac = 0.0;
    return a < 0 ? 0 : n - 1;
  }
  const bool odd = type == FDCGKS_BC_NO_SLIP ? odd_noslip : odd_refl;
  fac = odd != normal_deriv ? -1.0 : 1.0;
  if (on_line) return a < 0 ? -a : 2 * (n - 1) - a;
  return a < 0 ? -1 - a : 2 * n - 1 - a;
}

// Plane p of the 2D state (grid * 12 + field * 4 + comp), in stored node
// coordinates: rows first (real columns), then whole columns.
struct PlaneInfo {
  int mx, my, field, comp;
  bool dual;
};
__device__ __forceinline__ PlaneInfo plane_info(const Geo& g, int p) {
  PlaneInfo q;
  q.dual = p >= 12;
  q.field = (p % 12) / 4;
  q.comp = p % 4;
  q.mx = g.nx + (q.dual ? g.sx : 0);
  q.my = g.ny + (q.dual ? g.sy : 0);
  return q;
}
__global__ void k_halo_rows(double* __restrict__ S, int nplanes, Geo g, const Scal* __restrict__ sc) {
  if (sc->stop) return;
  const int W = g.nx + g.sx;
  long n = (long)nplanes * 2 * HALO * W;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    int i = (int)(t % W);
    long r = t / W;
    int hr = (int)(r % (2 * HALO));
    int p = (int)(r / (2 * HALO));
    const PlaneInfo q = plane_info(g, p);
    if (i >= q.mx) continue;
    int j = hr < HALO ? hr - HALO : q.my + (hr - HALO);
    double fac;
    int js = ghost_src(j, q.my, g.side[2], g.side[3], q.dual && g.sy, q.field == 2, q.comp == 2,
                       q.comp == 1 || q.comp == 2, fac);
    double* P = S + p * g.plane;
    P[at(g, j, i)] = fac * P[at(g, js, i)];
  }
}
__global__ void k_halo_cols(double* __restrict__ S, int nplanes, Geo g, const Scal* __restrict__ sc) {
  if (sc->stop) return;
  int rows = g.ny + g.sy + 2 * HALO;
  long n = (long)nplanes * rows * 2 * HALO;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    int hc = (int)(t % (2 * HALO));
    long r = t / (2 * HALO);
    int j = (int)(r % rows) - HALO;
    int p = (int)(r / rows);
    const PlaneInfo q = plane_info(g, p);
    if (j >= q.my + HALO) continue;
    int i = hc < HALO ? hc - HALO : q.mx + (hc - HALO);
    double fac;
    int is = ghost_src(i, q.mx, g.side[0], g.side[1], q.dual && g.sx, q.field == 1, q.comp == 1,
                       q.comp == 1 || q.comp == 2, fac);
    double* P = S + p * g.plane;
    P[at(g, j, i)] = fac * P[at(g, j, is)];
  }
}

// ------------------------------------------------------- interface sweep
// One gas-kinetic solve at an interface point: rn is the line normal to the
// interface, rt the other line (its derivative gives the tangential slope).
// swap: the normal is y, so rho U and rho V trade places in the local frame.
// The swap is applied to the data (selects), not by a second copy of the
// solver: the interface sweep's code then fits the instruction cache.
template <int STAGE, class FT>
__device__ __forceinline__ void solve_dir(const Consts& k, FT dt, bool swap, const fdk::IfaceRec (&rn)[4],
                                          const double (&tang)[4], double (&F)[4], double (&Ft)[4], double (&Wl)[4],
                                          double (&Wr)[4], double (&Wlt)[4], double (&Wrt)[4]) {
  fdk::GksIO<FT, 2> io;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int q = c == 1 ? 2 : (c == 2 ? 1 : c);
    const bool sw = swap && q != c;
    io.WL[c] = (FT)(sw ? rn[q].vl : rn[c].vl);
    io.WR[c] = (FT)(sw ? rn[q].vr : rn[c].vr);
    io.nL[c] = (FT)(sw ? rn[q].dl : rn[c].dl);
    io.nR[c] = (FT)(sw ? rn[q].dr : rn[c].dr);
    io.Wt[c] = (FT)(sw ? tang[q] : tang[c]);
  }
  fdk::gks_iface<FT, 2, STAGE == 1>(k, dt, io);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int q = c == 1 ? 2 : (c == 2 ? 1 : c);
    const bool sw = swap && q != c;
    Ft[c] = (double)(sw ? io.Ft[q] : io.Ft[c]);
    Wlt[c] = (double)(sw ? io.Wlt[q] : io.Wlt[c]);
    Wrt[c] = (double)(sw ? io.Wrt[q] : io.Wrt[c]);
    if (STAGE == 1) {
      F[c] = (double)(sw ? io.F[q] : io.F[c]);
      Wl[c] = (double)(sw ? io.Wl[q] : io.Wl[c]);
      Wr[c] = (double)(sw ? io.Wr[q] : io.Wr[c]);
    }
  }
}

// Reconstruction of one interface line.  Family fam (0: X, 1: Y), grid G
// (0: primary, 1: dual).  The line runs along y when fam != G: X-primary
// along x from P(i-1,j); X-dual along y from D(i,j-2); Y-primary along y
// from P(i,j-1); Y-dual along x from D(i-2,j).  fam and G are runtime values
// (uniform over a wave) so that one copy of the code serves all four lines.
// CHAR: reconstruct characteristic variables (every rec[c].cl/cr then holds
// the path function of the line).
template <bool CHAR = false>
__device__ __forceinline__ void edge_recon(const double* __restrict__ S, const Geo& g, const Consts& k, int i, int j,
                                           int fam, int G, fdk::IfaceRec (&rec)[4]) {
  const bool ALONG_Y = (fam ^ G) != 0;
  const int back = G == 0 ? 1 : 2;
  const long st = ALONG_Y ? g.pitch : 1;
  const long o = (ALONG_Y ? at(g, j - back, i) : at(g, j, i - back)) + (G ? g.dshift : 0);
  const int f = ALONG_Y ? 2 : 1;  // derivative field along the line
  const long pl = g.plane;
  if constexpr (CHAR) {
    // local frame of the line: the momentum along it is component 1
    double Q[4][4], X[4][4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int q = ALONG_Y ? (c == 1 ? 2 : (c == 2 ? 1 : c)) : c;
      const double* w = S + (G * 12 + q) * pl + o;
      const double* x = S + (G * 12 + f * 4 + q) * pl + o;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        Q[c][m] = w[m * st];
        X[c][m] = x[m * st];
      }
    }
    fdk::IfaceRec loc[4];
    double chi;
    fdk::recon_iface_char<2>(k, Q, X, g.h, g.invh, loc, chi);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int q = c == 1 ? 2 : (c == 2 ? 1 : c);
      rec[c] = ALONG_Y && q != c ? loc[q] : loc[c];
    }
  } else {
    // all 32 stencil values are loaded before the first reconstruction, so a
    // wave waits for memory once rather than once per component
    double Q[4][4], X[4][4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double* w = S + (G * 12 + c) * pl + o;
      const double* x = S + (G * 12 + f * 4 + c) * pl + o;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        Q[c][m] = w[m * st];
        X[c][m] = x[m * st];
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
      rec[c] = fdk::recon_iface(k, Q[c][0], Q[c][1], Q[c][2], Q[c][3], X[c][0], X[c][1], X[c][2], X[c][3], g.h,
                                g.invh);
  }
}

// One thread per (interface point, normal): blockDim (TX, TY) with TX a
// multiple of 64 or 32 and TY even, threadIdx.y = 2 * row + G, so the two
// solves of one point sit in neighbouring rows of threads (with TX >= 64,
// neighbouring waves).  fam: X covers i in [-2, nx], j in [-1 - sy, ny+1]; Y
// covers i in [-1 - sx, nx+1], j in [-2, ny] (everything the update of the
// nodes reads, the dual boundary nodes of bounded axes included); block
// (bx, by) covers TX points in i from ix0 + bx TX (threads outside the
// family's range stay idle but join the barriers) and TY/2 in j.  The
// partners exchange tangential slopes and blend sums through LDS.  Every
// thread of the block must call this.
// IN_LOOP (work loops of the persistent batch kernel): the thread indices and
// block shape as values formed at each call, so that nothing derived from
// them is hoisted in front of the loop and held through the solve.
template <int STAGE, class FT, bool CHAR = false, bool IN_LOOP = false>
__device__ __forceinline__ void edge_block(const double* __restrict__ S, double* __restrict__ E, const Geo& g,
                                           const Consts& k, double dt, int bx, int by, int fam, int ix0) {
  // LDS slots per thread: 0-3 tangential slope, 4-7 Wlt + Wrt, 8-11 Wl + Wr
  __shared__ double xch[12 * 256];
  int tx = threadIdx.x, ty = threadIdx.y, TX = blockDim.x, TY = blockDim.y;
  if (IN_LOOP) asm volatile("" : "+v"(tx), "+v"(ty), "+s"(TX), "+s"(TY));
  const int G = ty & 1;
#define XCH(c, r) xch[((c) * TY + (r)) * TX + tx]
  const int i = bx * TX + tx + ix0;
  const int j = by * (TY >> 1) + (ty >> 1) + (fam == 0 ? -1 - g.sy : -2);
  const bool valid = i >= (fam == 0 ? -2 : -1 - g.sx) && i <= (fam == 0 ? g.nx : g.nx + 1) &&
                     j <= (fam == 0 ? g.ny + 1 : g.ny);
  fdk::IfaceRec rec[4];
  if (valid) {
    edge_recon<CHAR>(S, g, k, i, j, fam, G, rec);
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) rec[c] = fdk::IfaceRec{1.0, 0.0, 1.0, 1.0, 0.0, 1.0};
  }
  double* e = E + ((long)fam * 50 + G * 25) * g.plane + at(g, j, i);
  const long pl = g.plane;
  // what needs no partner goes out at once (non-temporal stores: the
  // interface, node and state buffers are read back only by the next kernel,
  // from HBM, so they are kept out of the caches); the path function of the
  // density (or acoustic) line before the solve, so that it is not held
  // through it
  if (valid) __builtin_nontemporal_store(fmin(rec[0].cl, rec[0].cr), &e[8 * pl]);
#pragma unroll
  for (int c = 0; c < 4; ++c) XCH(c, ty) = 0.5 * (rec[c].dl + rec[c].dr);
  __syncthreads();
  double tang[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) tang[c] = XCH(c, ty ^ 1);
  double F[4] = {0, 0, 0, 0}, Ft[4] = {0, 0, 0, 0}, Wl[4] = {0, 0, 0, 0}, Wr[4] = {0, 0, 0, 0};
  double Wlt[4] = {0, 0, 0, 0}, Wrt[4] = {0, 0, 0, 0};
  if (valid) {
    // the normal is y when FAM != G (rho U and rho V swap in the local frame)
    solve_dir<STAGE, FT>(k, (FT)dt, fam != G, rec, tang, F, Ft, Wl, Wr, Wlt, Wrt);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      __builtin_nontemporal_store((double)(Ft[c]), &e[(4 + c) * pl]);
      if (STAGE == 1) __builtin_nontemporal_store((double)(F[c]), &e[c * pl]);
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    XCH(4 + c, ty) = Wlt[c] + Wrt[c];
    if (STAGE == 1) XCH(8 + c, ty) = Wl[c] + Wr[c];
  }
  __syncthreads();
  if (valid) {
    // blend with the partner direction (Eq. W-model-2d)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double st = XCH(4 + c, ty ^ 1);
      __builtin_nontemporal_store((double)(0.5 * Wlt[c] + 0.25 * st), &e[(17 + c) * pl]);
      __builtin_nontemporal_store((double)(0.5 * Wrt[c] + 0.25 * st), &e[(21 + c) * pl]);
      if (STAGE == 1) {
        const double sv = XCH(8 + c, ty ^ 1);
        __builtin_nontemporal_store((double)(0.5 * Wl[c] + 0.25 * sv), &e[(9 + c) * pl]);
        __builtin_nontemporal_store((double)(0.5 * Wr[c] + 0.25 * sv), &e[(13 + c) * pl]);
      }
    }
  }
  __syncthreads();  // the block may reuse xch for its next work item
#undef XCH
}

// Waves per SIMD the interface sweep is compiled for (register budget).
#ifndef FDCGKS_EDGE_WAVES
#define FDCGKS_EDGE_WAVES 2
#endif
template <int STAGE, class FT, bool CHAR>
__global__ __launch_bounds__(256, FDCGKS_EDGE_WAVES) void k_edges2d(const double* __restrict__ S, double* __restrict__ E, Geo g,
                                                    Consts k, const Scal* __restrict__ sc, int tiles_x,
                                                    int ntiles) {
  if (sc->stop) return;  // grid-uniform
  int t;
  if (!xcd_tile(blockIdx.x, gridDim.x, ntiles, t)) return;  // block-uniform
  edge_block<STAGE, FT, CHAR>(S, E, g, k, sc->dt, t % tiles_x, t / tiles_x, blockIdx.z, -OX);
}

// ------------------------------------------------------------ node sweep
// Derivatives along x and y at node offset o of grid base B (3-point
// reconstructions), component-wise or on characteristic variables (then in
// each line's local frame, eigenvectors at the node's state).
template <bool CHAR, class FT>
__device__ __forceinline__ void node_derivs(const double* __restrict__ B, const Geo& g, const Consts& k, long o,
                                            FT (&Wx)[4], FT (&Wy)[4]) {
  const long pl = g.plane;
  if constexpr (CHAR) {
#pragma unroll
    for (int ax = 0; ax < 2; ++ax) {
      const long st = ax == 0 ? 1 : g.pitch;
      double Q[4][3], X[4][3], d[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int q = ax == 1 ? (c == 1 ? 2 : (c == 2 ? 1 : c)) : c;
        const double* w = B + q * pl + o;
        const double* x = B + ((ax + 1) * 4 + q) * pl + o;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          Q[c][m] = w[(m - 1) * st];
          X[c][m] = x[(m - 1) * st];
        }
      }
      fdk::recon_node_char<2>(k, Q, X, g.h, g.invh, d);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int q = ax == 1 ? (c == 1 ? 2 : (c == 2 ? 1 : c)) : c;
        (ax == 0 ? Wx : Wy)[q] = (FT)d[c];
      }
    }
  } else {
    // the stencil is loaded before the first reconstruction (one wait for
    // memory rather than one per component and axis)
    double w[4][5], x[4][3], y[4][3];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double* pw = B + c * pl + o;
      const double* px = B + (4 + c) * pl + o;
      const double* py = B + (8 + c) * pl + o;
      w[c][0] = pw[-1], w[c][1] = pw[0], w[c][2] = pw[1], w[c][3] = pw[-g.pitch], w[c][4] = pw[g.pitch];
      x[c][0] = px[-1], x[c][1] = px[0], x[c][2] = px[1];
      y[c][0] = py[-g.pitch], y[c][1] = py[0], y[c][2] = py[g.pitch];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      Wx[c] = (FT)fdk::recon_node(k, w[c][0], w[c][1], w[c][2], x[c][0], x[c][1], x[c][2], g.h, g.invh);
      Wy[c] = (FT)fdk::recon_node(k, w[c][3], w[c][1], w[c][4], y[c][0], y[c][1], y[c][2], g.h, g.invh);
    }
  }
}

// Nodes whose fluxes the update reads beyond a grid's own nodes: one along
// each axis, two for the order-8 flux.
__host__ __device__ __forceinline__ int node_reach(const Consts& k) { return k.flux_order == 8 ? 2 : 1; }

// Nodes i in [-w - sx, nx - 1 + w], j in [-w - sy, ny - 1 + w] of the dual
// grid and i, j in [-w, n - 1 + w] of the primary grid (w = node_reach;
// batches pass 1): w beyond the grid's own nodes, whose dual nodes start at
// -1 on a bounded axis.  (A primary row at -w - 1 would read state row -w - 2,
// beyond the 3-row halo when w = 2.)  Block (bx, by) of blockDim.x x
// blockDim.y nodes, x from ix0 + bx blockDim.x (threads outside the range
// return).
template <int STAGE, class FT, bool CHAR = false>
__device__ __forceinline__ void node_block(const double* __restrict__ S, double* __restrict__ Nb, const Geo& g,
                                           const Consts& k, int bx, int by, int grid, int w, int ix0) {
  const int i = bx * blockDim.x + threadIdx.x + ix0;
  const int j = by * blockDim.y + threadIdx.y - w - (grid ? g.sy : 0);
  if (i < -w - (grid ? g.sx : 0) || i > g.nx - 1 + w || j > g.ny - 1 + w) return;
  const long pl = g.plane, o = at(g, j, i);
  const double* B = S + (long)grid * 12 * pl + (grid ? g.dshift : 0);
  FT W[4], Wx[4], Wy[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) W[c] = (FT)B[c * pl + o];
  node_derivs<CHAR, FT>(B, g, k, o, Wx, Wy);
  FT F[4], Ft[4], G[4], Gt[4];
  fdk::gks_node<FT, 2, STAGE == 1>(k, W, Wx, Wy, F, Ft, G, Gt);
  double* n = Nb + (long)grid * 16 * pl + o;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    __builtin_nontemporal_store((double)((double)Ft[c]), &n[(4 + c) * pl]);
    __builtin_nontemporal_store((double)((double)Gt[c]), &n[(12 + c) * pl]);
    if (STAGE == 1) {
      __builtin_nontemporal_store((double)((double)F[c]), &n[c * pl]);
      __builtin_nontemporal_store((double)((double)G[c]), &n[(8 + c) * pl]);
    }
  }
}

template <int STAGE, class FT, bool CHAR>
__global__ __launch_bounds__(256) void k_nodes2d(const double* __restrict__ S, double* __restrict__ Nb, Geo g,
                                                 Consts k, const Scal* __restrict__ sc, int tiles_x, int ntiles) {
  if (sc->stop) return;
  int t;
  if (!xcd_tile(blockIdx.x, gridDim.x, ntiles, t)) return;
  node_block<STAGE, FT, CHAR>(S, Nb, g, k, t % tiles_x, t / tiles_x, blockIdx.z, node_reach(k), -OX);
}

// ------------------------------------------------------ assemble + update
// Node (i, j) of grid `grid`, axis a: the interface family and normal slot
// holding its a-fluxes, and the offset r of its right (upper) interface:
// primary x -> X, slot 0, r = 0; primary y -> Y, slot 0, r = 0;
// dual x -> Y, slot 1, r = 1;    dual y -> X, slot 1, r = 1.
// The nodal fluxes come through an accessor nf(a, q, off): component q of
// (F, F_t) along x (a = 0) or (G, G_t) along y (a = 1), q = 0..3 values and
// 4..7 time derivatives, at the node `off` = -1, 0, +1 along the axis (-2 and
// +2 as well for the order-8 flux, WIDE: a template argument, so that the
// order-6 kernels keep their register budget).  A
// non-physical result (rho <= 0, p <= 0, NaN) sets the stop flag and records
// where (`member` names the batch member, 0 for a single problem).
// Components are processed one at a time (the loop is not unrolled): each
// reads its own ~20 planes and writes its outputs before the next starts, so
// few values are live and the HBM-bound kernel runs at high occupancy.
#ifndef FDCGKS_UPDATE_UNROLL
#define FDCGKS_UPDATE_UNROLL 1
#endif
// The wall condition of dual node (i, j) on a reflecting / no-slip side: the
// normal momentum (no-slip: both momenta) and its derivative along the wall
// are zero after every stage.  Bit c clears component c, bit 4 + c its
// x-derivative, bit 8 + c its y-derivative; 0 off the walls.
__device__ __forceinline__ int wall_mask(const Geo& g, int grid, int i, int j) {
  int zero = 0;
  if (grid == 1 && (g.sx | g.sy)) {
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const bool bnd = a == 0 ? g.sx != 0 : g.sy != 0;
      const int pos = a == 0 ? i : j, n = a == 0 ? g.nx : g.ny;
      const int type = !bnd ? FDCGKS_BC_PERIODIC
                            : (pos == -1 ? g.side[2 * a] : (pos == n - 1 ? g.side[2 * a + 1] : FDCGKS_BC_PERIODIC));
      if (type != FDCGKS_BC_REFLECTING && type != FDCGKS_BC_NO_SLIP) continue;
      const int along = 2 - a;  // field of the derivative along the wall
#pragma unroll
      for (int c = 1; c <= 2; ++c)
        if (type == FDCGKS_BC_NO_SLIP || c == 1 + a) zero |= (1 << c) | (1 << (4 * along + c));
    }
  }
  return zero;
}

template <int STAGE, class NF, bool WIDE = false>
__device__ __forceinline__ void update_node(const double* __restrict__ S, const double* __restrict__ E,
                                            const NF& nf, const double* __restrict__ Ain, double* __restrict__ Out,
                                            double* __restrict__ Aout, const Geo& g, const Consts& k, double dt,
                                            int i, int j, int grid, Scal* sc, int member, bool want_cfl,
                                            double& cfl_s, double& cfl_r) {
  const long pl = g.plane, o = at(g, j, i);
  const int r = grid;
  const long so = o + (grid ? g.dshift : 0);  // the dual planes are shifted along bounded axes
  const double* s = S + (long)grid * 12 * pl + so;
  double* out = Out + (long)grid * 12 * pl + so;
  const int zero = wall_mask(g, grid, i, j);
  double rho = 0.0, mom2 = 0.0, ener = 0.0, mU = 0.0, mV = 0.0;  // the new values
#pragma unroll FDCGKS_UPDATE_UNROLL
  for (int c = 0; c < 4; ++c) {
    double L = 0.0, Lt = 0.0, Gr[2], Grt[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int fam = (grid == 0) ? a : 1 - a;
      const long st = a == 0 ? 1 : g.pitch;
      const double* e = E + (long)fam * 50 * pl + (long)grid * 25 * pl + o;
      const double chiR = e[8 * pl + r * st], chiL = e[8 * pl + (r - 1) * st];
      const double* f = e + (0 + c) * pl;
      const double* ft = e + (4 + c) * pl;
      if constexpr (WIDE) {
        if (STAGE == 1) {
          const double n0 = nf(a, c, 0), nm = nf(a, c, -1), np = nf(a, c, 1);
          double FR = fdk::compact_flux8(k.variant, f[(r - 1) * st], f[r * st], f[(r + 1) * st], nm, n0, np,
                                         nf(a, c, 2), chiR);
          double FL = fdk::compact_flux8(k.variant, f[(r - 2) * st], f[(r - 1) * st], f[r * st], nf(a, c, -2), nm,
                                         n0, np, chiL);
          L = L - (FR - FL) * g.invh;
          Gr[a] = (e[(9 + c) * pl + r * st] - e[(13 + c) * pl + (r - 1) * st]) * g.invh;
        }
        const double nt0 = nf(a, 4 + c, 0), ntm = nf(a, 4 + c, -1), ntp = nf(a, 4 + c, 1);
        double FRt = fdk::compact_flux8(k.variant, ft[(r - 1) * st], ft[r * st], ft[(r + 1) * st], ntm, nt0, ntp,
                                        nf(a, 4 + c, 2), chiR);
        double FLt = fdk::compact_flux8(k.variant, ft[(r - 2) * st], ft[(r - 1) * st], ft[r * st], nf(a, 4 + c, -2),
                                        ntm, nt0, ntp, chiL);
        Lt = Lt - (FRt - FLt) * g.invh;
      } else {
        if (STAGE == 1) {
          const double n0 = nf(a, c, 0);
          double FR = fdk::compact_flux(k.variant, f[(r - 1) * st], f[r * st], f[(r + 1) * st], n0, nf(a, c, 1), chiR);
          double FL = fdk::compact_flux(k.variant, f[(r - 2) * st], f[(r - 1) * st], f[r * st], nf(a, c, -1), n0, chiL);
          L = L - (FR - FL) * g.invh;
          Gr[a] = (e[(9 + c) * pl + r * st] - e[(13 + c) * pl + (r - 1) * st]) * g.invh;
        }
        const double nt0 = nf(a, 4 + c, 0);
        double FRt = fdk::compact_flux(k.variant, ft[(r - 1) * st], ft[r * st], ft[(r + 1) * st], nt0,
                                       nf(a, 4 + c, 1), chiR);
        double FLt = fdk::compact_flux(k.variant, ft[(r - 2) * st], ft[(r - 1) * st], ft[r * st], nf(a, 4 + c, -1),
                                       nt0, chiL);
        Lt = Lt - (FRt - FLt) * g.invh;
      }
      Grt[a] = (e[(17 + c) * pl + r * st] - e[(21 + c) * pl + (r - 1) * st]) * g.invh;
    }
    double W, GX, GY;
    if (STAGE == 1) {
      double* ao = Aout + (long)grid * 12 * pl + so;
      const double w = s[c * pl];
      W = w + 0.5 * dt * L + 0.125 * dt * dt * Lt;
      const double gx = k.grad_carried ? s[(4 + c) * pl] : Gr[0];
      const double gy = k.grad_carried ? s[(8 + c) * pl] : Gr[1];
      GX = gx + 0.5 * dt * Grt[0];
      GY = gy + 0.5 * dt * Grt[1];
      __builtin_nontemporal_store((double)(w + dt * L + dt * dt / 6.0 * Lt), &ao[c * pl]);
      __builtin_nontemporal_store((double)(gx), &ao[(4 + c) * pl]);
      __builtin_nontemporal_store((double)(gy), &ao[(8 + c) * pl]);
    } else {
      const double* ai = Ain + (long)grid * 12 * pl + so;
      W = ai[c * pl] + dt * dt / 3.0 * Lt;
      GX = ai[(4 + c) * pl] + dt * Grt[0];
      GY = ai[(8 + c) * pl] + dt * Grt[1];
    }
    if (zero & (1 << c)) W = 0.0;
    if (zero & (1 << (4 + c))) GX = 0.0;
    if (zero & (1 << (8 + c))) GY = 0.0;
    __builtin_nontemporal_store((double)(W), &out[c * pl]);
    __builtin_nontemporal_store((double)(GX), &out[(4 + c) * pl]);
    __builtin_nontemporal_store((double)(GY), &out[(8 + c) * pl]);
    if (c == 0) rho = W;
    else if (c == 3) ener = W;
    else {
      mom2 = mom2 + W * W;
      if (c == 1) mU = W;
      else mV = W;
    }
  }
  if (want_cfl) {
    // wave speed and density of the new state, written as the CFL reduction
    // (k_cfl_partial) writes them, so the next step's dt is bit for bit the same
    const double U = mU / rho, V = mV / rho;
    const double pc = (k.gamma - 1.0) * (ener - 0.5 * rho * (U * U + V * V));
    const double c = sqrt(k.gamma * pc / rho);
    cfl_s = fmax(fabs(U), fabs(V)) + c;
    cfl_r = rho;
  }
  // non-physical state: rho <= 0, p <= 0 or NaN stops the run
  double p = (k.gamma - 1.0) * (ener - 0.5 * mom2 / rho);
  if (!(rho > 0.0) || !(p > 0.0)) {
    if (atomicCAS(&sc->stop, 0, 1) == 0) {
      sc->fail_grid = grid + 2 * member;
      sc->fail_i = i;
      sc->fail_j = j;
      sc->fail_stage = STAGE;
    }
  }
}

// Nodal fluxes from the node buffer (planes grid*16 + a*8 + q).
struct NodeFluxGlobal {
  const double* n;  // Nb + grid*16*plane + o
  long pl, pitch;
  __device__ __forceinline__ double operator()(int a, int q, int off) const {
    return n[(long)(a * 8 + q) * pl + off * (a == 0 ? 1 : pitch)];
  }
};

// Block (bx, by) of blockDim.x x blockDim.y nodes; the dual grid starts at
// i = -sx, j = -sy (its boundary nodes on bounded axes).
template <int STAGE, bool WIDE>
__device__ __forceinline__ void update_block(const double* __restrict__ S, const double* __restrict__ E,
                                             const double* __restrict__ Nb, const double* __restrict__ Ain,
                                             double* __restrict__ Out, double* __restrict__ Aout, const Geo& g,
                                             const Consts& k, double dt, int bx, int by, int grid, Scal* sc,
                                             int member, bool want_cfl, double& cfl_s, double& cfl_r) {
  const int i = bx * blockDim.x + threadIdx.x - (grid ? g.sx : 0);
  const int j = by * blockDim.y + threadIdx.y - (grid ? g.sy : 0);
  if (i >= g.nx || j >= g.ny) return;
  const NodeFluxGlobal nf{Nb + (long)grid * 16 * g.plane + at(g, j, i), g.plane, g.pitch};
  update_node<STAGE, NodeFluxGlobal, WIDE>(S, E, nf, Ain, Out, Aout, g, k, dt, i, j, grid, sc, member, want_cfl,
                                           cfl_s, cfl_r);
}

// Folds a wave's CFL contributions (largest wave speed, smallest density)
// into the partials slot of its block, so that the next step's time step
// needs no separate pass over the state.  Both are reduced as k_cfl_partial
// reduces them (speeds from 0, NaN speeds dropped).  Speeds are >= 0 and the
// densities kept are > 0, so their bit patterns order like their values.
__device__ __forceinline__ void cfl_fold(double* __restrict__ part, int nparts, double s, double r) {
  s = fmax(0.0, s);
  if (!(r > 0.0)) r = 1e300;  // a non-physical density has already stopped the run
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    s = fmax(s, __shfl_xor(s, off));
    r = fmin(r, __shfl_xor(r, off));
  }
  if (((threadIdx.y * blockDim.x + threadIdx.x) & 63) == 0) {
    const int slot = (int)((blockIdx.x + (long)gridDim.x * (blockIdx.y + (long)gridDim.y * blockIdx.z)) % nparts);
    atomicMax(reinterpret_cast<unsigned long long*>(part + 2 * slot), (unsigned long long)__double_as_longlong(s));
    atomicMin(reinterpret_cast<unsigned long long*>(part + 2 * slot + 1),
              (unsigned long long)__double_as_longlong(r));
  }
}

// ------------------------------------------- node sweep fused into update
// One block (64 x 4 threads) owns a 64 x 4 tile of grid blockIdx.z: it
// evaluates the nodal fluxes of the tile and of a one-node halo along each
// axis (F, F_t on rows j0..j0+3, columns i0-1..i0+64; G, G_t on columns
// i0..i0+63, rows j0-1..j0+4) into LDS, then assembles and updates its nodes
// from there.  The node buffer is neither written nor read.  Periodic
// problems with the order-6 flux only (the host takes the separate kernels
// for bounded axes and for the order-8 flux, which reads two nodes away).
constexpr int FT_X = 66, FT_Y = 6;
struct NodeFluxShared {
  const double* xs;  // [8][4][66]
  const double* ys;  // [8][6][64]
  int tx, ty;
  __device__ __forceinline__ double operator()(int a, int q, int off) const {
    return a == 0 ? xs[(q * 4 + ty) * FT_X + tx + 1 + off] : ys[(q * FT_Y + ty + 1 + off) * 64 + tx];
  }
};

template <int STAGE, class FT, bool CHAR>
__global__ __launch_bounds__(256) void k_nodeupd2d(const double* __restrict__ S, const double* __restrict__ E,
                                                   const double* __restrict__ Ain, double* __restrict__ Out,
                                                   double* __restrict__ Aout, Geo g, Consts k, Scal* __restrict__ sc) {
  if (sc->stop) return;  // grid-uniform
  __shared__ double xs[8 * 4 * FT_X];
  __shared__ double ys[8 * FT_Y * 64];
  const int grid = blockIdx.z, i0 = blockIdx.x * 64, j0 = blockIdx.y * 4;
  const int tid = threadIdx.y * 64 + threadIdx.x;
  const long pl = g.plane;
  const double* B = S + (long)grid * 12 * pl;
  // 4 x 66 positions on the tile rows (F and, inside, G), then 2 x 64 on the rows above and below (G)
  for (int q = tid; q < 4 * FT_X + 2 * 64; q += 256) {
    int r, c;
    if (q < 4 * FT_X) {
      r = q / FT_X;
      c = q % FT_X - 1;
    } else {
      r = (q - 4 * FT_X) < 64 ? -1 : 4;
      c = (q - 4 * FT_X) % 64;
    }
    const int i = i0 + c, j = j0 + r;
    if (i > g.nx || j > g.ny) continue;  // beyond the fluxes any interior node of the tile reads
    const long o = at(g, j, i);
    FT W[4], Wx[4], Wy[4];
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) W[cc] = (FT)B[cc * pl + o];
    node_derivs<CHAR, FT>(B, g, k, o, Wx, Wy);
    FT F[4], Ft[4], Gv[4], Gt[4];
    fdk::gks_node<FT, 2, STAGE == 1>(k, W, Wx, Wy, F, Ft, Gv, Gt);
    const bool xrow = r >= 0 && r < 4, ycol = c >= 0 && c < 64;
#pragma unroll
    for (int cc = 0; cc < 4; ++cc) {
      if (xrow) {
        xs[((4 + cc) * 4 + r) * FT_X + c + 1] = (double)Ft[cc];
        if (STAGE == 1) xs[(cc * 4 + r) * FT_X + c + 1] = (double)F[cc];
      }
      if (ycol) {
        ys[((4 + cc) * FT_Y + r + 1) * 64 + c] = (double)Gt[cc];
        if (STAGE == 1) ys[(cc * FT_Y + r + 1) * 64 + c] = (double)Gv[cc];
      }
    }
  }
  __syncthreads();
  const int i = i0 + threadIdx.x, j = j0 + threadIdx.y;
  if (i >= g.nx || j >= g.ny) return;
  const NodeFluxShared nf{xs, ys, (int)threadIdx.x, (int)threadIdx.y};
  double cs = 0.0, cr = 0.0;  // no CFL fold in the fused kernel
  update_node<STAGE>(S, E, nf, Ain, Out, Aout, g, k, sc->dt, i, j, grid, sc, 0, false, cs, cr);
}

template <int STAGE, bool WIDE>
// stage 2 reads and writes half the planes of stage 1 and folds the CFL
// partials: up to 96 VGPRs, 5 waves/SIMD; the order-8 assembly holds two more
// nodal fluxes per axis: one wave fewer
__global__ __launch_bounds__(256, (STAGE == 2 ? 5 : 4) - (WIDE ? 1 : 0)) void k_update2d(const double* __restrict__ S, const double* __restrict__ E,
                                                  const double* __restrict__ Nb, const double* __restrict__ Ain,
                                                  double* __restrict__ Out, double* __restrict__ Aout, Geo g,
                                                  Consts k, Scal* __restrict__ sc, double* __restrict__ part,
                                                  int nparts) {
  if (sc->stop) return;  // grid-uniform
  // part (stage 2 of a CFL step after the first): fold the new state's wave
  // speeds into the time-step partials; every lane reaches the fold
  double s = 0.0, r = 1e300;
  const bool fold = STAGE == 2 && part != nullptr;
  update_block<STAGE, WIDE>(S, E, Nb, Ain, Out, Aout, g, k, sc->dt, blockIdx.x, blockIdx.y, blockIdx.z, sc, 0, fold,
                            s, r);
  if (fold) cfl_fold(part, nparts, s, r);
}


// ------------------------------------ interface sweep fused with the update
// Periodic problems with the order-6 flux.  A block of 64 x 4 threads owns a
// strip of FS_W node columns [i0, i0 + FS_W) of both grids and a chunk of
// node rows [jlo, jhi), and marches up the rows.  Row step J evaluates the
// interface points of row J with the interface sweep's own code
// (reconstruction, solver, blend; thread row ty = 2 * family + normal):
//   ty 0: X(i0 - 2 + lane, J), primary-line normal: x-fluxes of primary nodes
//   ty 1: X(i0 - 2 + lane, J), dual-line normal:    y-fluxes of dual nodes
//   ty 2: Y(i0 - 1 + lane, J), primary-line normal: y-fluxes of primary nodes
//   ty 3: Y(i0 - 1 + lane, J), dual-line normal:    x-fluxes of dual nodes
// and then, without an interface buffer:
//   ty 0: x-flux difference and x-gradients of primary row J (neighbouring
//         interfaces by lane shuffles); the flux difference waits a step in LDS;
//   ty 3: the same for dual row J (it waits two steps);
//   ty 2: y-flux of primary row J-1 from the column's last three Y rows (an
//         LDS ring private to the lane), y-gradients of primary row J, and the
//         S2O4 update of primary row J-1;
//   ty 1: y-flux of dual row J-2 from the last three X rows, y-gradients of
//         dual row J-1, and the S2O4 update of dual row J-2.
// Nodal fluxes come from the node buffer (the node sweep runs first).  Every
// value is formed by the same expressions as in the separate interface sweep
// and update, so the results are bitwise those of the separate kernels.
constexpr int FS_W = 61;

template <int STAGE>
struct FusedLds {
  static constexpr int NV = STAGE == 1 ? 8 : 4;  // F[4], Ft[4] (stage 2: Ft[4]); also L[4], Lt[4] (Lt[4])
  static constexpr int NX = STAGE == 1 ? 12 : 8;  // exchange slots per thread
  // per lane: two rows of fluxes, the last path function, the last W-tilde-r
  // (and _t), the last compact flux (and _t)
  static constexpr int RS = 2 * NV + 1 + NV + NV;
  static constexpr int CHI = 2 * NV, WR = 2 * NV + 1, FB = 3 * NV + 1;
  double xch[NX * 256];
  double ring[2][RS * 64];     // [0]: ty 2 (Y rows), [1]: ty 1 (X rows); field-major, lane fastest
  double partP[2][NV * 64];    // x-flux differences of primary rows J, J-1
  double partD[3][NV * 64];    // of dual rows J, J-1, J-2
};

// One interface point (both normals of the point are the partner rows ty,
// ty ^ 1 of the block), values kept in registers: fluxes, the path function
// of the density (or acoustic) line and the blended interface values.
struct IfaceVals {
  double F[4], Ft[4], chi, Wl[4], Wr[4], Wlt[4], Wrt[4];
};
template <int STAGE, class FT, bool CHAR>
__device__ __forceinline__ void fused_iface(const double* __restrict__ S, const Geo& g, const Consts& k, double dt,
                                            int i, int j, int fam, bool valid, double* xch, IfaceVals& o, int tx,
                                            int ty) {
  const int G = ty & 1;
  constexpr int TX = 64, TY = 4;
#define XCH(c, r) xch[((c) * TY + (r)) * TX + tx]
  fdk::IfaceRec rec[4];
  if (valid) {
    edge_recon<CHAR>(S, g, k, i, j, fam, G, rec);
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) rec[c] = fdk::IfaceRec{1.0, 0.0, 1.0, 1.0, 0.0, 1.0};
  }
  o.chi = fmin(rec[0].cl, rec[0].cr);
#pragma unroll
  for (int c = 0; c < 4; ++c) XCH(c, ty) = 0.5 * (rec[c].dl + rec[c].dr);
  __syncthreads();
  double tang[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) tang[c] = XCH(c, ty ^ 1);
  double Wl[4] = {0, 0, 0, 0}, Wr[4] = {0, 0, 0, 0}, Wlt[4] = {0, 0, 0, 0}, Wrt[4] = {0, 0, 0, 0};
#pragma unroll
  for (int c = 0; c < 4; ++c) { o.F[c] = 0.0; o.Ft[c] = 0.0; }
  if (valid) solve_dir<STAGE, FT>(k, (FT)dt, fam != G, rec, tang, o.F, o.Ft, Wl, Wr, Wlt, Wrt);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    XCH(4 + c, ty) = Wlt[c] + Wrt[c];
    if (STAGE == 1) XCH(8 + c, ty) = Wl[c] + Wr[c];
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double st = XCH(4 + c, ty ^ 1);
    o.Wlt[c] = 0.5 * Wlt[c] + 0.25 * st;
    o.Wrt[c] = 0.5 * Wrt[c] + 0.25 * st;
    if (STAGE == 1) {
      const double sv = XCH(8 + c, ty ^ 1);
      o.Wl[c] = 0.5 * Wl[c] + 0.25 * sv;
      o.Wr[c] = 0.5 * Wr[c] + 0.25 * sv;
    } else {
      o.Wl[c] = o.Wr[c] = 0.0;
    }
  }
#undef XCH
}

// S2O4 update of node (i, j) of `grid` from its complete L (and Lt) per
// component (the gradients are written by the caller), with the
// non-physical check and the CFL contribution of update_node.  pre[c] is the
// node's state component c (stage 1) or its stage-1 accumulator (stage 2),
// loaded by the caller together with the row's other operands.
template <int STAGE>
__device__ __forceinline__ void fused_node_update(double* __restrict__ Out, double* __restrict__ Aout, const Geo& g,
                                                  const Consts& k, double dt, int i, int j, int grid,
                                                  const double (&pre)[4], const double (&L)[4],
                                                  const double (&Lt)[4], Scal* sc, bool want_cfl, double& cfl_s,
                                                  double& cfl_r) {
  const long pl = g.plane, o = at(g, j, i);
  double* out = Out + (long)grid * 12 * pl + o;
  double rho = 0.0, mom2 = 0.0, ener = 0.0, mU = 0.0, mV = 0.0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double W;
    if (STAGE == 1) {
      double* ao = Aout + (long)grid * 12 * pl + o;
      const double w = pre[c];
      W = w + 0.5 * dt * L[c] + 0.125 * dt * dt * Lt[c];
      __builtin_nontemporal_store((double)(w + dt * L[c] + dt * dt / 6.0 * Lt[c]), &ao[c * pl]);
    } else {
      W = pre[c] + dt * dt / 3.0 * Lt[c];
    }
    __builtin_nontemporal_store((double)(W), &out[c * pl]);
    if (c == 0) rho = W;
    else if (c == 3) ener = W;
    else {
      mom2 = mom2 + W * W;
      if (c == 1) mU = W;
      else mV = W;
    }
  }
  if (want_cfl) {
    const double U = mU / rho, V = mV / rho;
    const double pc = (k.gamma - 1.0) * (ener - 0.5 * rho * (U * U + V * V));
    const double c = sqrt(k.gamma * pc / rho);
    cfl_s = fmax(cfl_s, fmax(0.0, fmax(fabs(U), fabs(V)) + c));
    cfl_r = fmin(cfl_r, rho > 0.0 ? rho : 1e300);
  }
  double p = (k.gamma - 1.0) * (ener - 0.5 * mom2 / rho);
  if (!(rho > 0.0) || !(p > 0.0)) {
    if (atomicCAS(&sc->stop, 0, 1) == 0) {
      sc->fail_grid = grid;
      sc->fail_i = i;
      sc->fail_j = j;
      sc->fail_stage = STAGE;
    }
  }
}

// Gradients of node (i, j) of `grid` along axis a from the Gauss differences
// Gr (stage 1) and Grt, written to Out (and the stage-1 accumulators).
// pre[c] is the node's carried gradient (stage 1, carried gradients only) or
// its stage-1 accumulator (stage 2) of component c along a, loaded by the
// caller (fused_grad_load).
template <int STAGE>
__device__ __forceinline__ void fused_grad(double* __restrict__ Out, double* __restrict__ Aout, const Geo& g,
                                           const Consts& k, double dt, int i, int j, int grid, int a,
                                           const double (&pre)[4], const double (&Gr)[4], const double (&Grt)[4]) {
  const long pl = g.plane, o = at(g, j, i);
  const int f = 4 + 4 * a;  // field of the derivative along axis a
  double* out = Out + (long)grid * 12 * pl + o;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    double GA;
    if (STAGE == 1) {
      double* ao = Aout + (long)grid * 12 * pl + o;
      const double gx = k.grad_carried ? pre[c] : Gr[c];
      GA = gx + 0.5 * dt * Grt[c];
      __builtin_nontemporal_store((double)(gx), &ao[(f + c) * pl]);
    } else {
      GA = pre[c] + dt * Grt[c];
    }
    __builtin_nontemporal_store((double)(GA), &out[(f + c) * pl]);
  }
}

// The stored operands of fused_node_update (fields 0..3) or fused_grad (the
// derivative fields along axis a) of node (i, j) of `grid`, read when `on`
// (else zeros): the state at stage 1, the stage-1 accumulators at stage 2.
// A row's loads are issued together, before any of them is used, so a wave
// waits for memory once per row rather than once per helper.
template <int STAGE>
__device__ __forceinline__ void fused_pre_load(const double* __restrict__ S, const double* __restrict__ Ain,
                                               const Geo& g, int i, int j, int grid, int field0, bool on,
                                               double (&pre)[4]) {
  const long pl = g.plane;
  const double* p = (STAGE == 1 ? S : Ain) + (long)grid * 12 * pl + at(g, j, i) + field0 * pl;
#pragma unroll
  for (int c = 0; c < 4; ++c) pre[c] = on ? p[c * pl] : 0.0;
}

// Copies of loop-invariant values the compiler cannot see through: formed
// inside a loop, everything computed from them stays inside it.
__device__ __forceinline__ Geo opaque_strides(const Geo& g) {
  Geo q = g;
  asm volatile("" : "+s"(q.plane), "+s"(q.pitch), "+s"(q.h), "+s"(q.invh));
  return q;
}
__device__ __forceinline__ Consts opaque_consts(const Consts& k) {
  Consts q = k;
  asm volatile("" : "+s"(q.gamma), "+s"(q.K), "+s"(q.inv_Kd), "+s"(q.mu), "+s"(q.prfix));
  asm volatile("" : "+s"(q.C), "+s"(q.inv_tanhC), "+s"(q.eps), "+s"(q.eps_a), "+s"(q.dc), "+s"(q.ds));
  asm volatile("" : "+s"(q.tau_c1), "+s"(q.tau_c2));
  return q;
}
__device__ __forceinline__ double opaque_uniform(double x) {
  asm volatile("" : "+s"(x));
  return x;
}
__device__ __forceinline__ int opaque_lane(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

template <int STAGE, class FT, bool CHAR>
__global__ __launch_bounds__(256, 2) void k_fused2d(const double* __restrict__ S, const double* __restrict__ Nb,
                                                    const double* __restrict__ Ain, double* __restrict__ Out,
                                                    double* __restrict__ Aout, Geo g_in, Consts k_in,
                                                    Scal* __restrict__ sc, double* __restrict__ part, int nparts,
                                                    int nstrips, int nchunks, int rows) {
  const Geo& g0 = g_in;
  if (sc->stop) return;  // grid-uniform
  int t;
  if (!xcd_tile(blockIdx.x, gridDim.x, nstrips * nchunks, t)) return;  // block-uniform
  using LD = FusedLds<STAGE>;
  constexpr int NV = LD::NV;
  __shared__ LD lds;
  const int strip = t / nchunks, chunk = t % nchunks;
  const int i0 = strip * FS_W;
  const int jlo = chunk * rows, jhi = min(g0.ny, jlo + rows);
  const int fam = threadIdx.y >> 1;
  const int i_lane = (fam == 0 ? i0 - 2 : i0 - 1) + threadIdx.x;  // the lane's interface column
  const double dt_in = sc->dt;
  const bool fold = STAGE == 2 && part != nullptr;
  double cfl_s = 0.0, cfl_r = 1e300;
  for (int J = jlo - 2; J <= jhi + 1; ++J) {
    // the strides, scheme constants, time step and lane indices as values the compiler cannot see through, so
    // that what is computed from them is formed inside the loop: hoisted in front of it (plane offsets, dt and
    // constant expressions), about 45 values would hold registers through the interface solve and spill
    const Geo g = opaque_strides(g_in);
    const Consts k = opaque_consts(k_in);
    const double dt = opaque_uniform(dt_in);
    const int lane = opaque_lane(threadIdx.x), i = opaque_lane(i_lane), ty = opaque_lane(threadIdx.y);
    const long pl = g.plane;
    // X rows jlo-1 .. jhi+1, Y rows jlo-2 .. jhi (block-uniform per wave pair)
    const bool row_ok = fam == 0 ? J >= jlo - 1 : J <= jhi;
    const bool valid = row_ok && i <= (fam == 0 ? g.nx : g.nx + 1);
    IfaceVals v;
    fused_iface<STAGE, FT, CHAR>(S, g, k, dt, i, J, fam, valid, lds.xch, v, lane, ty);
    if (ty == 0 || ty == 3) {
      // x-flux differences and x-gradients of row J: primary (ty 0, nodes
      // i = i0 - 2 + lane, lanes 2..62) or dual (ty 3, nodes i = i0 - 1 + lane,
      // lanes 1..61)
      const bool dual = ty == 3;
      const int off = dual ? 1 : 2;
      const int node = i0 + lane - off;  // the node this lane updates
      const bool doit = J >= jlo && J < jhi;  // wave-uniform
      if (doit) {
        // compact flux at this lane's interface m: primary F~(X m) uses nodal
        // fluxes at P(m), P(m + 1); dual F~(Y m) at D(m - 1), D(m)
        const int m = i;
        const bool need = lane >= 1 && lane <= 62 && (dual ? m <= g.nx : m <= g.nx - 1);
        const bool upd = lane >= off && lane < off + FS_W && node < g.nx;
        // every load of the row first: nodal fluxes, then the gradient operands
        const double* nb = Nb + (dual ? 16 * pl : 0) + at(g, J, dual ? m - 1 : m);
        double nbl[NV], nbr[NV], gpre[4];
#pragma unroll
        for (int q = 0; q < NV; ++q) {
          const int qq = STAGE == 1 ? q : 4 + q;  // plane of F (q < 4) or Ft
          nbl[q] = need ? nb[qq * pl] : 0.0;
          nbr[q] = need ? nb[qq * pl + 1] : 0.0;
        }
        fused_pre_load<STAGE>(S, Ain, g, node, J, dual ? 1 : 0, 4, upd && (STAGE == 2 || k.grad_carried), gpre);
        double Fb[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) {
          const int qq = STAGE == 1 ? q : 4 + q;  // plane of F (q < 4) or Ft
          const int c = qq & 3;
          const double f0 = qq < 4 ? v.F[c] : v.Ft[c];
          const double fm = __shfl_up(f0, 1), fp = __shfl_down(f0, 1);
          Fb[q] = need ? fdk::compact_flux(k.variant, fm, f0, fp, nbl[q], nbr[q], v.chi) : 0.0;
        }
        double Lx[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) {
          // primary node: FR = F~(lane), FL = F~(lane - 1); dual: FR = F~(lane + 1), FL = F~(lane)
          const double FR = dual ? __shfl_down(Fb[q], 1) : Fb[q];
          const double FL = dual ? Fb[q] : __shfl_up(Fb[q], 1);
          double Lq = 0.0;
          Lq = Lq - (FR - FL) * g.invh;
          Lx[q] = Lq;
        }
        double Gr[4], Grt[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          // primary: W~l(X node) - W~r(X node - 1); dual: W~l(Y node + 1) - W~r(Y node)
          const double wlt = dual ? __shfl_down(v.Wlt[c], 1) : v.Wlt[c];
          const double wrt = dual ? v.Wrt[c] : __shfl_up(v.Wrt[c], 1);
          Grt[c] = (wlt - wrt) * g.invh;
          if (STAGE == 1) {
            const double wl = dual ? __shfl_down(v.Wl[c], 1) : v.Wl[c];
            const double wr = dual ? v.Wr[c] : __shfl_up(v.Wr[c], 1);
            Gr[c] = (wl - wr) * g.invh;
          } else {
            Gr[c] = 0.0;
          }
        }
        if (upd) {
          double* pp = dual ? lds.partD[J % 3] : lds.partP[J & 1];
#pragma unroll
          for (int q = 0; q < NV; ++q) pp[q * 64 + (node - i0)] = Lx[q];
          fused_grad<STAGE>(Out, Aout, g, k, dt, node, J, dual ? 1 : 0, 0, gpre, Gr, Grt);
        }
      }
    } else {
      // y-direction: primary column (ty 2, i = i0 - 1 + lane, lanes 1..61) or
      // dual column (ty 1, i = i0 - 2 + lane, lanes 2..62); the ring holds the
      // last two rows of this column's interfaces
      const bool dual = ty == 1;
      const int off = dual ? 2 : 1;
      const bool col = lane >= off && lane < off + FS_W && i < g.nx;
      double* rg = lds.ring[dual ? 1 : 0];
#define RING(f) rg[(f) * 64 + lane]
      // compact flux at row J - 1 of this column: primary F~(Y J-1) between
      // P(J-1), P(J); dual F~(X J-1) between D(J-2), D(J-1)
      const bool flux = dual ? (J >= jlo + 1 && J <= jhi + 1) : (J >= jlo && J <= jhi);
      const int r0 = dual ? J - 2 : J - 1;  // lower node row of the flux, and the row updated now
      const int rg_row = dual ? J - 1 : J;  // the row whose y-gradients are formed now
      const bool do_flux = flux && col, do_upd = do_flux && r0 >= jlo;
      const bool do_grad = rg_row >= jlo && rg_row < jhi && col;
      // every load of the row first: nodal fluxes, the update's state or
      // accumulators, the gradient operands
      double nbl[NV], nbu[NV], upre[4], gpre[4];
      {
        const double* nb = Nb + (dual ? 16 * pl : 0) + at(g, r0, i);
#pragma unroll
        for (int q = 0; q < NV; ++q) {
          const int qq = STAGE == 1 ? q : 4 + q;
          nbl[q] = do_flux ? nb[(8 + qq) * pl] : 0.0;
          nbu[q] = do_flux ? nb[(8 + qq) * pl + g.pitch] : 0.0;
        }
      }
      fused_pre_load<STAGE>(S, Ain, g, i, r0, dual ? 1 : 0, 0, do_upd, upre);
      fused_pre_load<STAGE>(S, Ain, g, i, rg_row, dual ? 1 : 0, 8, do_grad && (STAGE == 2 || k.grad_carried), gpre);
      if (do_flux) {
        double Fb[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) {
          const int qq = STAGE == 1 ? q : 4 + q;
          const int c = qq & 3;
          const double f2 = qq < 4 ? v.F[c] : v.Ft[c];
          const double f0 = RING((J & 1) * NV + q), f1 = RING(((J - 1) & 1) * NV + q);
          Fb[q] = fdk::compact_flux(k.variant, f0, f1, f2, nbl[q], nbu[q], RING(LD::CHI));
        }
        const int ru = r0;
        if (ru >= jlo) {
          const double* pp = dual ? lds.partD[ru % 3] : lds.partP[ru & 1];
          double L[4] = {0, 0, 0, 0}, Lt[4];
#pragma unroll
          for (int q = 0; q < NV; ++q) {
            double Lq = pp[q * 64 + (i - i0)];
            Lq = Lq - (Fb[q] - RING(LD::FB + q)) * g.invh;
            if (STAGE == 1) {
              if (q < 4) L[q] = Lq;
              else Lt[q - 4] = Lq;
            } else {
              Lt[q] = Lq;
            }
          }
          fused_node_update<STAGE>(Out, Aout, g, k, dt, i, ru, dual ? 1 : 0, upre, L, Lt, sc, fold, cfl_s, cfl_r);
        }
#pragma unroll
        for (int q = 0; q < NV; ++q) RING(LD::FB + q) = Fb[q];
      }
      // y-gradients of primary row J (W~l(Y J) - W~r(Y J-1)) or dual row J-1
      // (W~l(X J) - W~r(X J-1))
      if (do_grad) {
        double Gr[4], Grt[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          Grt[c] = (v.Wlt[c] - RING(LD::WR + (STAGE == 1 ? 4 : 0) + c)) * g.invh;
          Gr[c] = STAGE == 1 ? (v.Wl[c] - RING(LD::WR + c)) * g.invh : 0.0;
        }
        fused_grad<STAGE>(Out, Aout, g, k, dt, i, rg_row, dual ? 1 : 0, 1, gpre, Gr, Grt);
      }
      if (valid && col) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
          const int qq = STAGE == 1 ? q : 4 + q;
          RING((J & 1) * NV + q) = qq < 4 ? v.F[qq & 3] : v.Ft[qq & 3];
        }
        RING(LD::CHI) = v.chi;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if (STAGE == 1) {
            RING(LD::WR + c) = v.Wr[c];
            RING(LD::WR + 4 + c) = v.Wrt[c];
          } else {
            RING(LD::WR + c) = v.Wrt[c];
          }
        }
      }
#undef RING
    }
  }
  if (fold) cfl_fold(part, nparts, cfl_s, cfl_r);
}

// ================================================================== 1D
// A 1D problem is one line (grid 0) or two independent lines (grid 1 = the
// copy on nodes shifted by h/2).  Planes have one interior row (j = 0):
// state plane = line*6 + field*3 + comp (field 0 W, 1 Wx); interface buffer
// plane = line*19 + q for the interface j+1/2 stored at column j, j in
// [-2, N]: F[3], Ft[3], chi, Wl[3], Wr[3], Wlt[3], Wrt[3]; node buffer plane
// = line*6 + q at column j in [-w, N - 1 + w] (w = node_reach): F[3], Ft[3].
// One workgroup advances every line of the problem through whole steps:
// block barriers separate halo fill, interface and node sweeps, and update;
// interface and node results stay in global memory (cache resident at these
// sizes).

// ghost cells: periodic, zero-gradient (copy W, zero derivative) or
// reflecting (mirror about the face half a mesh beyond the end node: the
// momentum and the other components' derivatives odd)
__device__ __forceinline__ void halo1d(double* __restrict__ S, const Geo& g, int lines, int bc) {
  const long pl = g.plane;
  for (int q = threadIdx.x; q < lines * 6 * 2 * HALO; q += blockDim.x) {
    int gh = q % (2 * HALO), p = q / (2 * HALO);
    int f = (p % 6) / 3, c = (p % 6) % 3;
    int i = gh < HALO ? gh - HALO : g.nx + (gh - HALO);
    double* P = S + p * pl;
    double fac;
    const int src = ghost_src(i, g.nx, bc, bc, false, f == 1, c == 1, c == 1, fac);
    P[at(g, 0, i)] = fac * P[at(g, 0, src)];
  }
}

template <int STAGE, class FT, bool CHAR>
__device__ void stage1d_block(double* __restrict__ S, const double* __restrict__ Ain, double* __restrict__ Out,
                              double* __restrict__ Aout, double* __restrict__ E, double* __restrict__ Nb,
                              const Geo& g, const Consts& k, int lines, int bc, double dt, int* sfail,
                              Scal* __restrict__ sc) {
  const long pl = g.plane;
  const int N = g.nx;
  halo1d(S, g, lines, bc);
  __syncthreads();
  // interfaces j+1/2 for j in [-2, N]
  for (int q = threadIdx.x; q < lines * (N + 3); q += blockDim.x) {
    const int l = q / (N + 3), j = q % (N + 3) - 2;
    const double* B = S + (long)l * 6 * pl;
    fdk::GksIO<FT, 1> io;
    double chi = 1.0;
    if constexpr (CHAR) {
      double Q[3][4], X[3][4];
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          Q[c][m] = B[c * pl + at(g, 0, j - 1 + m)];
          X[c][m] = B[(3 + c) * pl + at(g, 0, j - 1 + m)];
        }
      fdk::IfaceRec r[3];
      fdk::recon_iface_char<1>(k, Q, X, g.h, g.invh, r, chi);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        io.WL[c] = (FT)r[c].vl; io.WR[c] = (FT)r[c].vr; io.nL[c] = (FT)r[c].dl; io.nR[c] = (FT)r[c].dr;
        io.Wt[c] = FT(0);
      }
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double* w = B + c * pl + at(g, 0, j - 1);
        const double* x = B + (3 + c) * pl + at(g, 0, j - 1);
        fdk::IfaceRec r = fdk::recon_iface(k, w[0], w[1], w[2], w[3], x[0], x[1], x[2], x[3], g.h, g.invh);
        io.WL[c] = (FT)r.vl; io.WR[c] = (FT)r.vr; io.nL[c] = (FT)r.dl; io.nR[c] = (FT)r.dr; io.Wt[c] = FT(0);
        if (c == 0) chi = fmin(r.cl, r.cr);
      }
    }
    fdk::gks_iface<FT, 1, STAGE == 1>(k, (FT)dt, io);
    double* e = E + (long)l * 19 * pl + at(g, 0, j);
    e[6 * pl] = chi;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      e[(3 + c) * pl] = (double)io.Ft[c];
      e[(13 + c) * pl] = (double)io.Wlt[c];
      e[(16 + c) * pl] = (double)io.Wrt[c];
      if (STAGE == 1) {
        e[c * pl] = (double)io.F[c];
        e[(7 + c) * pl] = (double)io.Wl[c];
        e[(10 + c) * pl] = (double)io.Wr[c];
      }
    }
  }
  // nodes j in [-w, N - 1 + w]
  const int w = node_reach(k);
  for (int q = threadIdx.x; q < lines * (N + 2 * w); q += blockDim.x) {
    const int l = q / (N + 2 * w), j = q % (N + 2 * w) - w;
    const double* B = S + (long)l * 6 * pl;
    FT W[3], Wx[3], F[3], Ft[3];
    if constexpr (CHAR) {
      double Q[3][3], X[3][3], d[3];
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          Q[c][m] = B[c * pl + at(g, 0, j - 1 + m)];
          X[c][m] = B[(3 + c) * pl + at(g, 0, j - 1 + m)];
        }
      fdk::recon_node_char<1>(k, Q, X, g.h, g.invh, d);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        W[c] = (FT)Q[c][1];
        Wx[c] = (FT)d[c];
      }
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double* w = B + c * pl + at(g, 0, j);
        const double* x = B + (3 + c) * pl + at(g, 0, j);
        W[c] = (FT)w[0];
        Wx[c] = (FT)fdk::recon_node(k, w[-1], w[0], w[1], x[-1], x[0], x[1], g.h, g.invh);
      }
    }
    fdk::gks_node<FT, 1, STAGE == 1>(k, W, Wx, (const FT*)nullptr, F, Ft, (FT*)nullptr, (FT*)nullptr);
    double* n = Nb + (long)l * 6 * pl + at(g, 0, j);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      n[(3 + c) * pl] = (double)Ft[c];
      if (STAGE == 1) n[c * pl] = (double)F[c];
    }
  }
  __syncthreads();
  // assemble + S2O4 update of the interior nodes
  for (int q = threadIdx.x; q < lines * N; q += blockDim.x) {
    const int l = q / N, j = q % N;
    const double* e = E + (long)l * 19 * pl + at(g, 0, j);
    const double* n = Nb + (long)l * 6 * pl + at(g, 0, j);
    const double* s = S + (long)l * 6 * pl + at(g, 0, j);
    double* out = Out + (long)l * 6 * pl + at(g, 0, j);
    const double chiR = e[6 * pl], chiL = e[6 * pl - 1];
    double W[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double* f = e + c * pl;
      const double* ft = e + (3 + c) * pl;
      const double* nf = n + c * pl;
      const double* nft = n + (3 + c) * pl;
      const bool wide = k.flux_order == 8;
      double FRt = wide ? fdk::compact_flux8(k.variant, ft[-1], ft[0], ft[1], nft[-1], nft[0], nft[1], nft[2], chiR)
                        : fdk::compact_flux(k.variant, ft[-1], ft[0], ft[1], nft[0], nft[1], chiR);
      double FLt = wide ? fdk::compact_flux8(k.variant, ft[-2], ft[-1], ft[0], nft[-2], nft[-1], nft[0], nft[1], chiL)
                        : fdk::compact_flux(k.variant, ft[-2], ft[-1], ft[0], nft[-1], nft[0], chiL);
      double Lt = -(FRt - FLt) * g.invh;
      double Gt = (e[(13 + c) * pl] - e[(16 + c) * pl - 1]) * g.invh;
      if (STAGE == 1) {
        double FR = wide ? fdk::compact_flux8(k.variant, f[-1], f[0], f[1], nf[-1], nf[0], nf[1], nf[2], chiR)
                         : fdk::compact_flux(k.variant, f[-1], f[0], f[1], nf[0], nf[1], chiR);
        double FL = wide ? fdk::compact_flux8(k.variant, f[-2], f[-1], f[0], nf[-2], nf[-1], nf[0], nf[1], chiL)
                         : fdk::compact_flux(k.variant, f[-2], f[-1], f[0], nf[-1], nf[0], chiL);
        double L = -(FR - FL) * g.invh;
        double G = (e[(7 + c) * pl] - e[(10 + c) * pl - 1]) * g.invh;
        if (k.grad_carried) G = s[(3 + c) * pl];
        double w = s[c * pl];
        double* ao = Aout + (long)l * 6 * pl + at(g, 0, j);
        W[c] = w + 0.5 * dt * L + 0.125 * dt * dt * Lt;
        out[c * pl] = W[c];
        out[(3 + c) * pl] = G + 0.5 * dt * Gt;
        __builtin_nontemporal_store((double)(w + dt * L + dt * dt / 6.0 * Lt), &ao[c * pl]);
        ao[(3 + c) * pl] = G;
      } else {
        const double* ai = Ain + (long)l * 6 * pl + at(g, 0, j);
        W[c] = ai[c * pl] + dt * dt / 3.0 * Lt;
        out[c * pl] = W[c];
        out[(3 + c) * pl] = ai[(3 + c) * pl] + dt * Gt;
      }
    }
    double p = (k.gamma - 1.0) * (W[2] - 0.5 * W[1] * W[1] / W[0]);
    if (!(W[0] > 0.0) || !(p > 0.0)) {
      if (atomicCAS(sfail, 0, 1) == 0) {
        sc->fail_grid = l;
        sc->fail_i = j;
        sc->fail_j = 0;
        sc->fail_stage = STAGE;
      }
    }
  }
  __syncthreads();
}

// Whole 1D run in one workgroup.  mode 0: up to nsteps steps, ping-pong
// between S0 and S1 starting from S0; mode 1 / 2: one stage at sc->dt into
// Sstar/Acc (1) or S1 (2), not committed.
template <class FT, bool CHAR>
__global__ __launch_bounds__(256) void k_run1d(double* S0, double* S1, double* Sstar, double* Acc, double* E,
                                               double* Nb, Geo g, Consts k, Scal* sc, int lines, int bc,
                                               int nsteps, double cfl, int use_cfl, int mode) {
  __shared__ double rmax[256], rmin[256];
  __shared__ double sdt;
  __shared__ int sfail, sstop;
  if (threadIdx.x == 0) { sfail = 0; sstop = sc->stop; }
  __syncthreads();
  if (sstop) return;
  if (mode == 1 || mode == 2) {
    const double dt = sc->dt;
    if (mode == 1) stage1d_block<1, FT, CHAR>(S0, nullptr, Sstar, Acc, E, Nb, g, k, lines, bc, dt, &sfail, sc);
    else stage1d_block<2, FT, CHAR>(Sstar, Acc, S1, nullptr, E, Nb, g, k, lines, bc, dt, &sfail, sc);
    if (threadIdx.x == 0 && sfail) sc->stop |= 1;
    return;
  }
  double* cur = S0;
  double* nxt = S1;
  const long pl = g.plane;
  for (int st = 0; st < nsteps; ++st) {
    // time step: CFL over every node of every line (or the fixed dt), clipped to t_end
    double vmax = 0.0, rm = 1e300;
    if (use_cfl)
      for (int q = threadIdx.x; q < lines * g.nx; q += blockDim.x) {
        const int l = q / g.nx, j = q % g.nx;
        const double* B = cur + (long)l * 6 * pl + at(g, 0, j);
        double rho = B[0], U = B[pl] / rho, rE = B[2 * pl];
        double p = (k.gamma - 1.0) * (rE - 0.5 * rho * U * U);
        vmax = fmax(vmax, fabs(U) + sqrt(k.gamma * p / rho));
        rm = fmin(rm, rho);
      }
    rmax[threadIdx.x] = vmax;
    rmin[threadIdx.x] = rm;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) {
        rmax[threadIdx.x] = fmax(rmax[threadIdx.x], rmax[threadIdx.x + w]);
        rmin[threadIdx.x] = fmin(rmin[threadIdx.x], rmin[threadIdx.x + w]);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      double dt = sc->dt_fixed;
      if (use_cfl) {
        dt = cfl * g.h / rmax[0];
        if (k.mu > 0) dt = fmin(dt, cfl * g.h * g.h / (8.0 * k.mu / rmin[0]));
      }
      int stop = 0;
      if (sc->t_end > 0) {
        if (sc->t >= sc->t_end) stop = 2;
        else if (sc->t + dt > sc->t_end) dt = sc->t_end - sc->t;
      }
      if (!stop && !(dt > 0.0)) { stop = 1; sc->fail_stage = 0; }
      sc->stop |= stop;
      sstop = stop;
      sdt = dt;
      sc->dt = dt;
    }
    __syncthreads();
    if (sstop) break;
    const double dt = sdt;
    stage1d_block<1, FT, CHAR>(cur, nullptr, Sstar, Acc, E, Nb, g, k, lines, bc, dt, &sfail, sc);
    if (sfail) break;
    stage1d_block<2, FT, CHAR>(Sstar, Acc, nxt, nullptr, E, Nb, g, k, lines, bc, dt, &sfail, sc);
    if (sfail) break;
    if (threadIdx.x == 0) {
      sc->t += dt;
      sc->steps += 1;
    }
    double* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  if (threadIdx.x == 0 && sfail) sc->stop |= 1;
}

// ------------------------------------------------ state from point samples
// Nodal values are the samples; averaged derivatives are the Gauss
// differences of the samples at the two bounding interfaces divided by h
// (Eq. define-averaged-gradient), with periodic wrap.  2D samples
// S[c][2ny][2nx]: sample (kx, ky) at (x0 + (kx+1) h/2, y0 + (ky+1) h/2);
// primary node (i, j) is sample (2i, 2j), dual node (i, j) sample (2i+1, 2j+1).
__global__ void k_from_samples2d(const double* __restrict__ S, double* __restrict__ St, Geo g) {
  const int NX = 2 * g.nx, NY = 2 * g.ny;
  const long n = 2L * 4 * g.nx * g.ny;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    const int i = (int)(t % g.nx);
    long r = t / g.nx;
    const int j = (int)(r % g.ny);
    r /= g.ny;
    const int c = (int)(r % 4), gr = (int)(r / 4);
    const int kx = 2 * i + gr, ky = 2 * j + gr;
    const double* P = S + (long)c * NY * NX;
    const double w = P[(long)ky * NX + kx];
    const double wx = (P[(long)ky * NX + imod(kx + 1, NX)] - P[(long)ky * NX + imod(kx - 1, NX)]) / g.h;
    const double wy = (P[(long)imod(ky + 1, NY) * NX + kx] - P[(long)imod(ky - 1, NY) * NX + kx]) / g.h;
    const long o = at(g, j, i);
    St[(long)(gr * 12 + c) * g.plane + o] = w;
    St[(long)(gr * 12 + 4 + c) * g.plane + o] = wx;
    St[(long)(gr * 12 + 8 + c) * g.plane + o] = wy;
  }
}
// 1D samples S[c][2nx]: node j of line l (0 primary, 1 the shifted copy) is
// sample 2j + l.
__global__ void k_from_samples1d(const double* __restrict__ S, double* __restrict__ St, Geo g, int lines) {
  const int NX = 2 * g.nx;
  const long n = (long)lines * 3 * g.nx;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    const int j = (int)(t % g.nx);
    const int c = (int)((t / g.nx) % 3), l = (int)(t / (3L * g.nx));
    const int k = 2 * j + l;
    const double* P = S + (long)c * NX;
    const long o = at(g, 0, j);
    St[(long)(l * 6 + c) * g.plane + o] = P[k];
    St[(long)(l * 6 + 3 + c) * g.plane + o] = (P[imod(k + 1, NX)] - P[imod(k - 1, NX)]) / g.h;
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
  // stored nodes; the dual grid has one more column (row) along a bounded
  // axis.  A block takes whole rows (no per-node index division), its
  // threads the columns.
  const int W = g.nx + g.sx, H = g.ny + g.sy;
  constexpr int NC = DIM + 2;
  for (int row = blockIdx.x; row < ngrid * H; row += gridDim.x) {
    const int gr = row / H, j = row - gr * H;
    if (gr == 0 && j >= g.ny) continue;  // block-uniform
    const int w = gr == 0 ? g.nx : W;
    const double* B = S + gr * gridstride + at(g, j, 0);
    for (int i = threadIdx.x; i < w; i += blockDim.x) {
      double rho = B[i], U = B[g.plane + i] / rho;
      double V = DIM == 2 ? B[2 * g.plane + i] / rho : 0.0;
      double rE = B[(NC - 1) * g.plane + i];
      double p = (gamma - 1.0) * (rE - 0.5 * rho * (U * U + V * V));
      double c = sqrt(gamma * p / rho);
      double s = fmax(fabs(U), fabs(V)) + c;
      vmax = fmax(vmax, s);  // NaN speeds are dropped here and caught by the update's check
      rmin = fmin(rmin, rho);
    }
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

// Per-block partial diagnostics over the stored nodes of every grid: sums of
// each conserved component per grid, min rho and min p.  part[block * NQ + q]
// with q = grid * (DIM + 2) + comp, then NQ - 2 (min rho) and NQ - 1 (min p).
template <int DIM>
__global__ __launch_bounds__(256) void k_diag_partial(const double* __restrict__ S, Geo g, int ngrid, long gridstride,
                                                      double gamma, double* __restrict__ part) {
  __shared__ double red[256];
  constexpr int NC = DIM + 2;
  const int W = g.nx + g.sx, H = g.ny + g.sy;
  const long n = (long)ngrid * W * H;
  double s0[NC], s1[NC], rmin = 1e300, pmin = 1e300;
#pragma unroll
  for (int c = 0; c < NC; ++c) s0[c] = s1[c] = 0.0;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    const int i = (int)(t % W);
    long r = t / W;
    const int j = (int)(r % H);
    const int gr = (int)(r / H);
    if (gr == 0 && (i >= g.nx || j >= g.ny)) continue;
    const double* B = S + gr * gridstride + at(g, j, i);
    double w[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) w[c] = B[c * g.plane];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if (gr == 0) s0[c] += w[c];
      else s1[c] += w[c];
    }
    const double rho = w[0], U = w[1] / rho, V = DIM == 2 ? w[2] / rho : 0.0;
    const double p = (gamma - 1.0) * (w[NC - 1] - 0.5 * rho * (U * U + V * V));
    rmin = fmin(rmin, rho);
    pmin = fmin(pmin, p);
  }
  const int NQ = ngrid * NC + 2;
  for (int q = 0; q < NQ; ++q) {
    double v = q < NC ? s0[q] : (q < 2 * NC && ngrid == 2 ? s1[q - NC] : (q == NQ - 2 ? rmin : pmin));
    const bool is_min = q >= NQ - 2;
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w)
        red[threadIdx.x] = is_min ? fmin(red[threadIdx.x], red[threadIdx.x + w]) : red[threadIdx.x] + red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(long)blockIdx.x * NQ + q] = red[0];
    __syncthreads();
  }
}

// Start of a step: dt from the partials (or the fixed dt), clipped to t_end;
// sets the "done" bit when t has reached t_end.
__global__ void k_step_begin(double* __restrict__ part, int nparts, Scal* __restrict__ sc, double cfl,
                             double h, double mu, int use_cfl) {
  __shared__ double smax[256], smin[256];
  double vmax = 0.0, rmin = 1e300;
  if (use_cfl)
    for (int t = threadIdx.x; t < nparts; t += blockDim.x) {
      vmax = fmax(vmax, part[2 * t]);
      rmin = fmin(rmin, part[2 * t + 1]);
      // emptied for the fold of the next state by this step's stage-2 update
      part[2 * t] = 0.0;
      part[2 * t + 1] = 1e300;
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

// ============================================================ batched 2D
// Many independent periodic 2D problems of different sizes advanced together:
// one cooperative persistent launch per stage.  Work items of every phase
// are listed on the host (member, family/grid, block x, block y) and taken
// round-robin by the resident workgroups; grid-wide barriers separate the
// phases.  Each member keeps its own padded planes, mesh size and CFL time
// step; all members share the scheme constants.
struct BMember {
  Geo g;
  double* S[2];
  double* Sstar;
  double* Acc;
  double* E;
  double* Nb;
};
struct BItem {
  int m, z, bx, by;
};
struct BArgs {
  const BMember* mem;
  int count;
  const BItem* items;  // concatenated: cfl, halo, edges, nodes, updates
  int n_cfl, n_halo, n_edge, n_node, n_upd;
  double cfl;
  int parity;          // step parity: selects the CFL slots of this step
  int cur;             // which of S[0], S[1] holds the state at the start of the step
  unsigned long long* slots;  // [2 parities][2: max speed, min rho][count] as ordered bit patterns
  double* t;           // per-member time
  double* dt_last;     // per-member last dt
  Scal* sc;            // shared stop flag / failure record
};

__device__ __forceinline__ double member_dt(const BArgs& a, int m, const Consts& k) {
  const unsigned long long* sl = a.slots + (long)a.parity * 2 * a.count;
  double smax = __longlong_as_double((long long)sl[m]);
  double rmin = __longlong_as_double((long long)sl[a.count + m]);
  const Geo& g = a.mem[m].g;
  double dt = a.cfl * g.h / smax;
  if (k.mu > 0) dt = fmin(dt, a.cfl * g.h * g.h / (8.0 * k.mu / rmin));
  return dt;
}

// CFL partial of one member over stored rows [16 by, 16 by + 16) of both
// grids (the dual grid has one more row and column along a bounded axis).
__device__ __forceinline__ void cfl_block(const BArgs& a, const Consts& k, const BItem& it, double* red) {
  const BMember& M = a.mem[it.m];
  const Geo& g = M.g;
  const double* S = M.S[a.cur];
  const int nthr = blockDim.x * blockDim.y, tid = threadIdx.y * blockDim.x + threadIdx.x;
  double vmax = 0.0, rmin = 1e300;
  const int H = g.ny + g.sy, W = g.nx + g.sx;
  const int j0 = it.by * 16, j1 = min(H, j0 + 16);
  for (int q = tid; q < 2 * (j1 - j0) * W; q += nthr) {
    int i = q % W, r = q / W, j = j0 + r % (j1 - j0), gr = r / (j1 - j0);
    if (gr == 0 && (i >= g.nx || j >= g.ny)) continue;
    const double* B = S + (long)gr * 12 * g.plane + at(g, j, i);
    double rho = B[0], U = B[g.plane] / rho, V = B[2 * g.plane] / rho;
    double p = (k.gamma - 1.0) * (B[3 * g.plane] - 0.5 * rho * (U * U + V * V));
    vmax = fmax(vmax, fmax(fabs(U), fabs(V)) + sqrt(k.gamma * p / rho));
    rmin = fmin(rmin, rho);
  }
  red[tid] = vmax;
  red[nthr + tid] = rmin;
  __syncthreads();
  for (int w = nthr / 2; w > 0; w >>= 1) {
    if (tid < w) {
      red[tid] = fmax(red[tid], red[tid + w]);
      red[nthr + tid] = fmin(red[nthr + tid], red[nthr + tid + w]);
    }
    __syncthreads();
  }
  if (tid == 0) {
    unsigned long long* sl = a.slots + (long)a.parity * 2 * a.count;
    // positive doubles order like their bit patterns
    atomicMax(&sl[it.m], (unsigned long long)__double_as_longlong(red[0]));
    atomicMin(&sl[a.count + it.m], (unsigned long long)__double_as_longlong(red[nthr]));
  }
  __syncthreads();
}

// Halo of state plane p of a member (rows over the real columns, then whole
// columns): periodic images or the ghosts of bounded sides, as k_halo_rows /
// k_halo_cols fill them for a single problem.
__device__ __forceinline__ void halo_plane_block(double* __restrict__ S, const Geo& g, int p) {
  const int nthr = blockDim.x * blockDim.y, tid = threadIdx.y * blockDim.x + threadIdx.x;
  const PlaneInfo q = plane_info(g, p);
  double* P = S + (long)p * g.plane;
  for (int t = tid; t < 2 * HALO * q.mx; t += nthr) {
    const int i = t % q.mx, hr = t / q.mx;
    const int j = hr < HALO ? hr - HALO : q.my + (hr - HALO);
    double fac;
    const int js = ghost_src(j, q.my, g.side[2], g.side[3], q.dual && g.sy, q.field == 2, q.comp == 2,
                             q.comp == 1 || q.comp == 2, fac);
    P[at(g, j, i)] = fac * P[at(g, js, i)];
  }
  __syncthreads();
  for (int t = tid; t < (q.my + 2 * HALO) * 2 * HALO; t += nthr) {
    const int hc = t % (2 * HALO), j = t / (2 * HALO) - HALO;
    const int i = hc < HALO ? hc - HALO : q.mx + (hc - HALO);
    double fac;
    const int is = ghost_src(i, q.mx, g.side[0], g.side[1], q.dual && g.sx, q.field == 1, q.comp == 1,
                             q.comp == 1 || q.comp == 2, fac);
    P[at(g, j, i)] = fac * P[at(g, j, is)];
  }
  __syncthreads();
}

// End of a batched step (one block): every member's time advances by its dt
// and the step counts, unless a stage stopped it.
// The stop flag as other workgroups of the same launch left it (coherent load).
__device__ __forceinline__ int load_stop(const Scal* sc) {
  return __hip_atomic_load(&sc->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void batch_step_end(const BArgs& a, const Consts& k) {
  if (load_stop(a.sc)) return;
  for (int q = threadIdx.y * blockDim.x + threadIdx.x; q < a.count; q += blockDim.x * blockDim.y) {
    const double dt = member_dt(a, q, k);
    a.t[q] += dt;
    a.dt_last[q] = dt;
  }
  if (threadIdx.x == 0 && threadIdx.y == 0) a.sc->steps += 1;
}

template <int STAGE, class FT, bool CHAR, bool WIDE>
__global__ __launch_bounds__(256, 2) void k_batch_stage(BArgs a, Consts k) {
  namespace cg = cooperative_groups;
  cg::grid_group grid = cg::this_grid();
  __shared__ double red[512];
  const BItem* it = a.items;
  const int nb = gridDim.x;
  // phase A: (stage 1) CFL partials of every member, reset of the next
  // step's slots; halo of the stage input
  if (STAGE == 1) {
    if (blockIdx.x == 0)
      for (int q = threadIdx.y * blockDim.x + threadIdx.x; q < a.count; q += blockDim.x * blockDim.y) {
        unsigned long long* nx = a.slots + (long)(a.parity ^ 1) * 2 * a.count;
        nx[q] = 0ull;
        nx[a.count + q] = (unsigned long long)__double_as_longlong(1e300);
      }
    for (int q = blockIdx.x; q < a.n_cfl; q += nb) cfl_block(a, k, it[q], red);
  }
  it += a.n_cfl;
  for (int q = blockIdx.x; q < a.n_halo; q += nb) {
    const BMember& M = a.mem[it[q].m];
    halo_plane_block(STAGE == 1 ? M.S[a.cur] : M.Sstar, M.g, it[q].z);
  }
  it += a.n_halo;
  grid.sync();
  // phase B: interfaces and nodes
  const bool stopped = load_stop(a.sc) != 0;
  if (!stopped) {
    for (int q = blockIdx.x; q < a.n_edge; q += nb) {
      const BItem& w = it[q];
      const BMember& M = a.mem[w.m];
      // the scheme constants as values formed inside the loop (hoisted in front of it, constant expressions of
      // them would hold registers through the interface solve)
      const Consts kq = opaque_consts(k);
      edge_block<STAGE, FT, CHAR, true>(STAGE == 1 ? M.S[a.cur] : M.Sstar, M.E, M.g, kq, member_dt(a, w.m, kq),
                                        w.bx, w.by, w.z, w.z == 0 ? -2 : -1 - M.g.sx);
    }
  }
  it += a.n_edge;
  if (!stopped) {
    for (int q = blockIdx.x; q < a.n_node; q += nb) {
      const BItem& w = it[q];
      const BMember& M = a.mem[w.m];
      node_block<STAGE, FT, CHAR>(STAGE == 1 ? M.S[a.cur] : M.Sstar, M.Nb, M.g, k, w.bx, w.by, w.z, node_reach(k),
                                  -OX);
    }
  }
  it += a.n_node;
  grid.sync();
  // phase C: assemble + update
  if (!stopped) {
    for (int q = blockIdx.x; q < a.n_upd; q += nb) {
      const BItem& w = it[q];
      const BMember& M = a.mem[w.m];
      const double dt = member_dt(a, w.m, k);
      double cs = 0.0, cr = 0.0;  // batches reduce their time steps themselves
      if (STAGE == 1)
        update_block<1, WIDE>(M.S[a.cur], M.E, M.Nb, nullptr, M.Sstar, M.Acc, M.g, k, dt, w.bx, w.by, w.z, a.sc,
                              w.m, false, cs, cr);
      else
        update_block<2, WIDE>(M.Sstar, M.E, M.Nb, M.Acc, M.S[a.cur ^ 1], nullptr, M.g, k, dt, w.bx, w.by, w.z,
                              a.sc, w.m, false, cs, cr);
    }
  }
  if (STAGE == 2) {
    // the step counts only if no update of this stage stopped it
    grid.sync();
    if (blockIdx.x == 0) batch_step_end(a, k);
  }
}

// ---- the same stage as separate launches, one per phase (grid = work items)
template <int STAGE>
__global__ __launch_bounds__(256) void k_bphase_halo(BArgs a, Consts k) {
  if (a.sc->stop) return;
  __shared__ double red[512];
  const int q = blockIdx.x;
  if (STAGE == 1 && q == 0)
    for (int m = threadIdx.y * blockDim.x + threadIdx.x; m < a.count; m += blockDim.x * blockDim.y) {
      unsigned long long* nx = a.slots + (long)(a.parity ^ 1) * 2 * a.count;
      nx[m] = 0ull;
      nx[a.count + m] = (unsigned long long)__double_as_longlong(1e300);
    }
  if (STAGE == 1 && q < a.n_cfl) {
    cfl_block(a, k, a.items[q], red);
    return;
  }
  const BItem& it = a.items[a.n_cfl + q - (STAGE == 1 ? a.n_cfl : 0)];
  const BMember& M = a.mem[it.m];
  halo_plane_block(STAGE == 1 ? M.S[a.cur] : M.Sstar, M.g, it.z);
}
// CHAR: characteristic reconstruction; WIDE: the order-8 flux (node reach 2).
template <int STAGE, class FT, bool CHAR>
__global__ __launch_bounds__(256, FDCGKS_EDGE_WAVES) void k_bphase_edges(BArgs a, Consts k) {
  if (a.sc->stop) return;
  const BItem& w = a.items[a.n_cfl + a.n_halo + blockIdx.x];
  const BMember& M = a.mem[w.m];
  edge_block<STAGE, FT, CHAR>(STAGE == 1 ? M.S[a.cur] : M.Sstar, M.E, M.g, k, member_dt(a, w.m, k), w.bx, w.by,
                              w.z, w.z == 0 ? -2 : -1 - M.g.sx);
}
template <int STAGE, class FT, bool CHAR>
__global__ __launch_bounds__(256) void k_bphase_nodes(BArgs a, Consts k) {
  if (a.sc->stop) return;
  const BItem& w = a.items[a.n_cfl + a.n_halo + a.n_edge + blockIdx.x];
  const BMember& M = a.mem[w.m];
  node_block<STAGE, FT, CHAR>(STAGE == 1 ? M.S[a.cur] : M.Sstar, M.Nb, M.g, k, w.bx, w.by, w.z, node_reach(k), -OX);
}
template <int STAGE, bool WIDE>
__global__ __launch_bounds__(256) void k_bphase_update(BArgs a, Consts k) {
  if (a.sc->stop) return;
  const BItem& w = a.items[a.n_cfl + a.n_halo + a.n_edge + a.n_node + blockIdx.x];
  const BMember& M = a.mem[w.m];
  const double dt = member_dt(a, w.m, k);
  double cs = 0.0, cr = 0.0;  // batches reduce their time steps themselves
  if (STAGE == 1)
    update_block<1, WIDE>(M.S[a.cur], M.E, M.Nb, nullptr, M.Sstar, M.Acc, M.g, k, dt, w.bx, w.by, w.z, a.sc, w.m,
                          false, cs, cr);
  else
    update_block<2, WIDE>(M.Sstar, M.E, M.Nb, M.Acc, M.S[a.cur ^ 1], nullptr, M.g, k, dt, w.bx, w.by, w.z, a.sc,
                          w.m, false, cs, cr);
}
__global__ void k_bphase_end(BArgs a, Consts k) { batch_step_end(a, k); }


// ------------------------------------------- allocation-free 1D run
// fdcgks_step1d_static keeps every buffer of a 1D run in one file-scope
// device array: the four state buffers (12 planes each), the interface
// buffer (19 planes per line) and the node buffer (6 planes per line) of a
// problem of at most STATIC1D_MAX_NX nodes per line, then the step scalars.
// The array is per device and lives until the process ends.
constexpr int STATIC1D_MAX_NX = 2048;
constexpr long STATIC1D_PLANE = (long)(((STATIC1D_MAX_NX + 2 * OX) + 15) / 16 * 16) * (1 + 2 * OY);
constexpr long STATIC1D_PLANES = 4 * 12 + 2 * 19 + 2 * 6;
constexpr long STATIC1D_DOUBLES = STATIC1D_PLANES * STATIC1D_PLANE + 64;
static_assert(sizeof(Scal) <= 64 * sizeof(double), "step scalars exceed their slot");
static __device__ __align__(256) double scratch[STATIC1D_DOUBLES];

// Step scalars of a run: t, t_end and the fixed dt set, everything else zero.
__global__ void k_static1d_begin(Scal* __restrict__ sc, double t, double t_end, double dt_fixed) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Scal z = {};
  z.t = t;
  z.t_end = t_end;
  z.dt_fixed = dt_fixed;
  *sc = z;
}

// Dense caller state [lines][6][nx] (W[3], Wx[3]) to the padded planes of S0
// (dir 0), or back from the buffer holding the last completed step (dir 1:
// S0 after an even number of steps, S1 after an odd one).
__global__ void k_static1d_io(double* __restrict__ dense, double* __restrict__ S0, const double* __restrict__ S1,
                              Geo g, int lines, const Scal* __restrict__ sc, int dir) {
  const long n = (long)lines * 6 * g.nx;
  const double* src = dir == 1 && (sc->steps & 1) ? S1 : S0;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    const long p = t / g.nx;
    const int i = (int)(t % g.nx);
    const long o = p * g.plane + at(g, 0, i);
    if (dir == 0) S0[o] = dense[t];
    else dense[t] = src[o];
  }
}
}  // namespace

#include "gks_adjoint.hpp"
#include "adjoint.inc.hip"

namespace {

// ================================================================== host
// errors of calls without a problem handle (create, the allocation-free run):
// a fixed buffer, so that reporting one allocates nothing
thread_local char g_create_error[512];

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
  // launch shapes of the interface, node and update kernels (x, y threads):
  // fdcgks_autotune's pick on the 2048^2 shear layer
  dim3 tile[3] = {dim3(64, 2), dim3(64, 1), dim3(128, 1)};
  // captured whole steps (one graph per ping-pong parity), replayed by fdcgks_step
  int graph_steps = 16;  // steps per captured graph; 0: separate launches
  bool fuse_nodes = false;  // node sweep inside the update kernel
  int fuse_stage = 2;       // interface sweep and update in one marching kernel (k_fused2d): 0 off, 1 on, 2 auto
  int fused_rows = 0;       // node rows per block of k_fused2d (0: from the CU count)
  int ncu = 256;            // compute units of the device
  bool cfl_fold = false;    // the stage-2 update being launched folds the CFL partials
  hipStream_t cap = nullptr;
  hipGraphExec_t gx[2] = {nullptr, nullptr};
  bool g_valid = false;
  int g_use_cfl = -1;
  int g_steps = 0;
  double g_cfl = 0.0;
  // adjoint workspace (fdcgks_step_vjp), allocated on first use
  double* adj = nullptr;
  double *E1 = nullptr, *Nb1 = nullptr, *Lo = nullptr, *Op = nullptr, *LE = nullptr, *LN = nullptr;
  double *LSs = nullptr, *LAcc = nullptr, *LS0 = nullptr;
};

namespace {

fdcgks_status fail(fdcgks_problem* pb, fdcgks_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (pb) pb->err = buf; else std::snprintf(g_create_error, sizeof g_create_error, "%s", buf);
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
  if (pb->adj) (void)hipFree(pb->adj);
  pb->adj = nullptr;
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
  long nr = (long)pb->nplanes * 2 * HALO * (g.nx + g.sx);
  long nc = (long)pb->nplanes * (g.ny + g.sy + 2 * HALO) * 2 * HALO;
  hipLaunchKernelGGL(k_halo_rows, dim3(std::min(ceil_div(nr, 256), 4096)), dim3(256), 0, pb->stream, S,
                     pb->nplanes, g, pb->sc);
  hipLaunchKernelGGL(k_halo_cols, dim3(std::min(ceil_div(nc, 256), 4096)), dim3(256), 0, pb->stream, S,
                     pb->nplanes, g, pb->sc);
  mark(pb, TK_HALO);
  return launch_check(pb, "halo");
}

// Launches of the three stage kernels with a given block shape (x, y).
template <int STAGE>
void launch_edges(fdcgks_problem* pb, const double* Sin, dim3 blk) {
  const Geo& g = pb->g;
  // x tiles start at i = -OX (column 0 of the padded row), so every wave's
  // row segment starts on a cache line; the last point is i = nx + 1
  const int tx = ceil_div(g.nx + 2 + OX, blk.x), nt = tx * ceil_div(g.ny + 3 + g.sy, blk.y / 2);
  dim3 ge(ceil_div(nt, NXCD) * NXCD, 1, 2);  // tiles in XCD bands (xcd_tile)
  const bool f32 = pb->prm.flux_precision == FDCGKS_FP32_FLUX;
  const bool ch = pb->prm.recon_vars == FDCGKS_RECON_CHARACTERISTIC;
  auto fn = f32 ? (ch ? k_edges2d<STAGE, float, true> : k_edges2d<STAGE, float, false>)
                : (ch ? k_edges2d<STAGE, double, true> : k_edges2d<STAGE, double, false>);
  hipLaunchKernelGGL(fn, ge, blk, 0, pb->stream, Sin, pb->E, g, pb->k, pb->sc, tx, nt);
}
template <int STAGE>
void launch_nodes(fdcgks_problem* pb, const double* Sin, dim3 blk) {
  const Geo& g = pb->g;
  const int w = node_reach(pb->k);
  // x tiles start at i = -OX (a cache-line boundary); the last node is nx - 1 + w
  const int tx = ceil_div(g.nx + w + OX, blk.x), nt = tx * ceil_div(g.ny + 2 * w + g.sy, blk.y);
  dim3 gn(ceil_div(nt, NXCD) * NXCD, 1, 2);  // tiles in XCD bands (xcd_tile)
  const bool f32 = pb->prm.flux_precision == FDCGKS_FP32_FLUX;
  const bool ch = pb->prm.recon_vars == FDCGKS_RECON_CHARACTERISTIC;
  auto fn = f32 ? (ch ? k_nodes2d<STAGE, float, true> : k_nodes2d<STAGE, float, false>)
                : (ch ? k_nodes2d<STAGE, double, true> : k_nodes2d<STAGE, double, false>);
  hipLaunchKernelGGL(fn, gn, blk, 0, pb->stream, Sin, pb->Nb, g, pb->k, pb->sc, tx, nt);
}
template <int STAGE>
void launch_update(fdcgks_problem* pb, const double* Sin, const double* Ain, double* Out, double* Aout, dim3 blk) {
  const Geo& g = pb->g;
  dim3 gu(ceil_div(g.nx + g.sx, blk.x), ceil_div(g.ny + g.sy, blk.y), 2);
  auto fn = pb->k.flux_order == 8 ? k_update2d<STAGE, true> : k_update2d<STAGE, false>;
  double* fold = STAGE == 2 && pb->cfl_fold ? pb->part : nullptr;
  hipLaunchKernelGGL(fn, gu, blk, 0, pb->stream, Sin, pb->E, pb->Nb, Ain, Out, Aout, g, pb->k, pb->sc, fold,
                     pb->nparts);
}

// Launch of the fused interface sweep + update (k_fused2d): strips of FS_W
// node columns, each cut into chunks of rows so that about two blocks per CU
// run at once.
template <int STAGE>
void launch_fused(fdcgks_problem* pb, const double* Sin, const double* Ain, double* Out, double* Aout) {
  const Geo& g = pb->g;
  const int nstrips = ceil_div(g.nx, FS_W);
  int rows = pb->fused_rows;
  if (rows <= 0) {
    const int nch = std::max(1, 2 * pb->ncu / nstrips);
    rows = std::max(16, ceil_div(g.ny, nch));
  }
  rows = std::min(rows, g.ny);
  const int nchunks = ceil_div(g.ny, rows);
  const int nblk = nstrips * nchunks;
  const bool f32 = pb->prm.flux_precision == FDCGKS_FP32_FLUX;
  const bool ch = pb->prm.recon_vars == FDCGKS_RECON_CHARACTERISTIC;
  auto fn = f32 ? (ch ? k_fused2d<STAGE, float, true> : k_fused2d<STAGE, float, false>)
                : (ch ? k_fused2d<STAGE, double, true> : k_fused2d<STAGE, double, false>);
  double* fold = STAGE == 2 && pb->cfl_fold ? pb->part : nullptr;
  hipLaunchKernelGGL(fn, dim3(ceil_div(nblk, NXCD) * NXCD), dim3(64, 4), 0, pb->stream, Sin, pb->Nb, Ain, Out, Aout,
                     g, pb->k, pb->sc, fold, pb->nparts, nstrips, nchunks, rows);
}

// How a stage is launched: 0 separate interface sweep, node sweep and
// update; 1 the node sweep inside the update kernel; 2 the interface sweep
// fused with the update after the node sweep.  Both fusions need periodic
// axes and the order-6 flux; otherwise the separate kernels run.
enum { STAGE_SEPARATE = 0, STAGE_FUSE_NODES = 1, STAGE_FUSE_IFACE = 2 };
// Whether the fused stage kernel beats the separate sweeps (the automatic
// choice): its blocks march the rows of one strip of columns in lock step,
// so it needs tall row chunks at about two blocks per compute unit, here at
// least 64 rows each.  Measured: 2048^2 5.42 against 5.92 ms per step; 512^2
// 0.72 against 0.52 ms (16-row chunks).
bool fused_pays(const fdcgks_problem* pb) {
  const long strips = ceil_div(pb->g.nx, FS_W);
  return (long)pb->g.ny * strips >= 64L * 2 * pb->ncu;
}
int stage_mode(const fdcgks_problem* pb) {
  if ((pb->g.sx | pb->g.sy) || pb->k.flux_order == 8 || pb->prm.dim != 2) return STAGE_SEPARATE;
  if (pb->fuse_stage == 1 || (pb->fuse_stage == 2 && fused_pays(pb))) return STAGE_FUSE_IFACE;
  return pb->fuse_nodes ? STAGE_FUSE_NODES : STAGE_SEPARATE;
}

// One stage in launch mode `mode` (stage_mode; callers that read the
// interface or node buffers afterwards pass STAGE_SEPARATE).
template <int STAGE>
fdcgks_status stage2d(fdcgks_problem* pb, const double* Sin, const double* Ain, double* Out, double* Aout,
                      int mode) {
  const Geo& g = pb->g;
  fdcgks_status st = halo2d(pb, const_cast<double*>(Sin));
  if (st) return st;
  if (mode == STAGE_FUSE_IFACE) {
    launch_nodes<STAGE>(pb, Sin, pb->tile[1]);
    mark(pb, STAGE == 1 ? TK_NODE1 : TK_NODE2);
    launch_fused<STAGE>(pb, Sin, Ain, Out, Aout);
    mark(pb, STAGE == 1 ? TK_UPD1 : TK_UPD2);
    return launch_check(pb, "stage");
  }
  launch_edges<STAGE>(pb, Sin, pb->tile[0]);
  mark(pb, STAGE == 1 ? TK_EDGE1 : TK_EDGE2);
  if (mode == STAGE_FUSE_NODES) {
    dim3 gu(ceil_div(g.nx, 64), ceil_div(g.ny, 4), 2);
    const bool f32 = pb->prm.flux_precision == FDCGKS_FP32_FLUX;
    const bool ch = pb->prm.recon_vars == FDCGKS_RECON_CHARACTERISTIC;
    auto fn = f32 ? (ch ? k_nodeupd2d<STAGE, float, true> : k_nodeupd2d<STAGE, float, false>)
                  : (ch ? k_nodeupd2d<STAGE, double, true> : k_nodeupd2d<STAGE, double, false>);
    hipLaunchKernelGGL(fn, gu, dim3(64, 4), 0, pb->stream, Sin, pb->E, Ain, Out, Aout, g, pb->k, pb->sc);
    mark(pb, STAGE == 1 ? TK_UPD1 : TK_UPD2);
    return launch_check(pb, "stage");
  }
  launch_nodes<STAGE>(pb, Sin, pb->tile[1]);
  mark(pb, STAGE == 1 ? TK_NODE1 : TK_NODE2);
  launch_update<STAGE>(pb, Sin, Ain, Out, Aout, pb->tile[2]);
  mark(pb, STAGE == 1 ? TK_UPD1 : TK_UPD2);
  return launch_check(pb, "stage");
}

// Whether a CFL step's stage-2 update folds the partials for the next step:
// 2D steps with the separate node sweep (the fused node kernel does not fold).
bool fold_ok(const fdcgks_problem* pb, double dt) {
  return !(dt > 0) && pb->prm.dim == 2 && stage_mode(pb) != STAGE_FUSE_NODES;
}

// fresh: reduce the CFL partials from the state (the first step of a call or
// graph); otherwise the previous step's stage-2 update folded them.
fdcgks_status begin_step(fdcgks_problem* pb, double dt, double cfl, bool fresh = true) {
  const Geo& g = pb->g;
  int use_cfl = dt > 0 ? 0 : 1;
  if (use_cfl && fresh) {
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

fdcgks_status launch_run1d(fdcgks_problem* pb, int mode, int nsteps, double dt, double cfl) {
  const int use_cfl = dt > 0 ? 0 : 1;
  double* S0 = pb->S[pb->cur];
  double* S1 = pb->S[1 - pb->cur];
  const bool f32 = pb->prm.flux_precision == FDCGKS_FP32_FLUX;
  const bool ch = pb->prm.recon_vars == FDCGKS_RECON_CHARACTERISTIC;
  auto fn = f32 ? (ch ? k_run1d<float, true> : k_run1d<float, false>)
                : (ch ? k_run1d<double, true> : k_run1d<double, false>);
  hipLaunchKernelGGL(fn, dim3(1), dim3(256), 0, pb->stream, S0, S1, pb->Sstar, pb->Acc, pb->E, pb->Nb, pb->g, pb->k,
                     pb->sc, pb->ngrid, pb->prm.bc, nsteps, cfl, use_cfl, mode);
  return launch_check(pb, "run1d");
}

// ---- captured steps
void graph_invalidate(fdcgks_problem* pb) {
  for (hipGraphExec_t& x : pb->gx)
    if (x) {
      (void)hipGraphExecDestroy(x);
      x = nullptr;
    }
  pb->g_valid = false;
}

// One whole 2D step (dt reduction, two stages, step end) captured per
// ping-pong parity on a private stream and replayed on the problem's stream.
// The graphs depend only on the buffers, the launch shapes and (cfl,
// use_cfl): the fixed dt, t and t_end are read from device memory.
fdcgks_status capture_steps(fdcgks_problem* pb, double dt, double cfl) {
  const int use_cfl = dt > 0 ? 0 : 1;
  if (pb->g_valid && pb->g_use_cfl == use_cfl && (!use_cfl || pb->g_cfl == cfl) && pb->g_steps == pb->graph_steps)
    return FDCGKS_OK;
  graph_invalidate(pb);
  if (!pb->cap) HIPCHK(pb, hipStreamCreateWithFlags(&pb->cap, hipStreamNonBlocking));
  hipStream_t user = pb->stream;
  const int cur0 = pb->cur;
  for (int c = 0; c < 2; ++c) {
    HIPCHK(pb, hipStreamBeginCapture(pb->cap, hipStreamCaptureModeThreadLocal));
    pb->stream = pb->cap;
    fdcgks_status st = FDCGKS_OK;
    for (int q = 0, cc = c; q < pb->graph_steps && !st; ++q, cc = 1 - cc) {
      pb->cur = cc;
      st = begin_step(pb, dt, cfl, q == 0 || !fold_ok(pb, dt));
      if (!st) st = stage2d<1>(pb, pb->S[cc], nullptr, pb->Sstar, pb->Acc, stage_mode(pb));
      pb->cfl_fold = fold_ok(pb, dt);
      if (!st) st = stage2d<2>(pb, pb->Sstar, pb->Acc, pb->S[1 - cc], nullptr, stage_mode(pb));
      pb->cfl_fold = false;
      if (!st) {
        hipLaunchKernelGGL(k_step_end, dim3(1), dim3(1), 0, pb->stream, pb->sc);
        st = launch_check(pb, "step_end");
      }
    }
    hipGraph_t gr = nullptr;
    hipError_t e = hipStreamEndCapture(pb->cap, &gr);
    pb->stream = user;
    pb->cur = cur0;
    if (!st && e != hipSuccess) st = fail(pb, FDCGKS_EHIP, "step capture: %s", hipGetErrorString(e));
    if (!st) {
      e = hipGraphInstantiate(&pb->gx[c], gr, nullptr, nullptr, 0);
      if (e != hipSuccess) st = fail(pb, FDCGKS_EHIP, "step graph instantiation: %s", hipGetErrorString(e));
    }
    if (gr) (void)hipGraphDestroy(gr);
    if (st) {
      graph_invalidate(pb);
      return st;
    }
  }
  pb->g_valid = true;
  pb->g_steps = pb->graph_steps;
  pb->g_use_cfl = use_cfl;
  pb->g_cfl = cfl;
  return FDCGKS_OK;
}

// ---- launch shapes
// A shape is valid for kernel class c (0 interface, 1 node, 2 update) when it
// has whole waves, at most 256 threads, x in {32, 64, 128, 256} and, for the
// interface sweep, an even y (the two normals of a point are paired rows).
bool tile_ok(int c, unsigned x, unsigned y) {
  if (!(x == 32 || x == 64 || x == 128 || x == 256) || y < 1 || x * y > 256 || (x * y) % 64 != 0) return false;
  return c != 0 || y % 2 == 0;
}

// Device milliseconds of `reps` launches of one stage-1 kernel with shape blk.
float time_tile(fdcgks_problem* pb, int c, dim3 blk, int reps, hipEvent_t e0, hipEvent_t e1) {
  auto one = [&]() {
    if (c == 0) launch_edges<1>(pb, pb->S[pb->cur], blk);
    else if (c == 1) launch_nodes<1>(pb, pb->S[pb->cur], blk);
    else launch_update<1>(pb, pb->S[pb->cur], nullptr, pb->Sstar, pb->Acc, blk);
  };
  one();  // warm-up
  (void)hipEventRecord(e0, pb->stream);
  for (int r = 0; r < reps; ++r) one();
  (void)hipEventRecord(e1, pb->stream);
  if (hipEventSynchronize(e1) != hipSuccess) return -1.f;
  float ms = -1.f;
  if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.f;
  return ms;
}

// Boundary of 2D side k (x-low, x-high, y-low, y-high): its own entry, or bc.
int side_bc(const fdcgks_params& p, int k) { return p.side[k] >= 0 ? p.side[k] : p.bc; }

// Padded-plane geometry and scheme constants of a problem (validated params).
void setup_geometry(const fdcgks_params& prm, Geo& g, Consts& k) {
  const fdcgks_params* p = &prm;
  g.nx = p->nx;
  g.ny = p->ny;
  g.pitch = ((p->nx + 2 * OX) + 15) / 16 * 16;
  if (p->dim == 2) {
    for (int q = 0; q < 4; ++q) g.side[q] = side_bc(*p, q);
    g.sx = g.side[0] != FDCGKS_BC_PERIODIC;
    g.sy = g.side[2] != FDCGKS_BC_PERIODIC;
  }
  g.rows = p->ny + 2 * OY + g.sy;  // a bounded y axis adds the dual boundary row
  g.dshift = g.sx + (long)g.sy * g.pitch;
  g.plane = (long)g.pitch * g.rows;
  g.h = p->lx / p->nx;
  g.invh = 1.0 / g.h;
  k.gamma = p->gamma;
  k.K = p->dim == 2 ? (4.0 - 2.0 * p->gamma) / (p->gamma - 1.0) : (3.0 - p->gamma) / (p->gamma - 1.0);
  k.inv_Kd = 1.0 / (k.K + (p->dim == 2 ? 2.0 : 1.0));
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
  k.flux_order = p->flux_order;
}


fdcgks_status check_params(const fdcgks_params* p) {
  if (!p) return fail(nullptr, FDCGKS_EINVAL, "params is NULL");
  if (p->dim != 1 && p->dim != 2) return fail(nullptr, FDCGKS_EINVAL, "dim must be 1 or 2 (got %d)", p->dim);
  if (p->dim == 2 && (p->nx < 4 || p->ny < 4))
    return fail(nullptr, FDCGKS_EINVAL, "2D needs nx, ny >= 4 (got %d x %d)", p->nx, p->ny);
  if (p->dim == 1 && (p->nx < 4 || p->ny != 1))
    return fail(nullptr, FDCGKS_EINVAL, "1D needs nx >= 4 and ny == 1 (got %d, %d)", p->nx, p->ny);
  if ((long)p->nx * p->ny > (1L << 28)) return fail(nullptr, FDCGKS_EINVAL, "grid too large");
  if (p->bc < FDCGKS_BC_PERIODIC || p->bc > FDCGKS_BC_NO_SLIP)
    return fail(nullptr, FDCGKS_EINVAL, "unknown boundary condition %d", p->bc);
  if (p->dim == 1 && p->bc == FDCGKS_BC_NO_SLIP)
    return fail(nullptr, FDCGKS_EINVAL, "1D walls are reflecting (no tangential velocity)");
  if (p->dim == 2) {
    for (int k = 0; k < 4; ++k)
      if (p->side[k] < -1 || p->side[k] > FDCGKS_BC_NO_SLIP)
        return fail(nullptr, FDCGKS_EINVAL, "unknown boundary condition %d on side %d", p->side[k], k);
    for (int a = 0; a < 2; ++a)
      if ((side_bc(*p, 2 * a) == FDCGKS_BC_PERIODIC) != (side_bc(*p, 2 * a + 1) == FDCGKS_BC_PERIODIC))
        return fail(nullptr, FDCGKS_EINVAL, "a periodic side needs a periodic opposite side (axis %d)", a);
  }
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
  if (p->recon_vars != FDCGKS_RECON_CONSERVATIVE && p->recon_vars != FDCGKS_RECON_CHARACTERISTIC)
    return fail(nullptr, FDCGKS_EINVAL, "bad recon_vars");
  if (p->flux_order != 6 && p->flux_order != 8) return fail(nullptr, FDCGKS_EINVAL, "flux_order must be 6 or 8");
  return FDCGKS_OK;
}


// ---- adjoint of one step (2D, FP64 fluxes)
constexpr int ADJ_PLANES = 100 + 32 + 24 + 48 + 100 + 32 + 24 + 24 + 24;

fdcgks_status adj_alloc(fdcgks_problem* pb) {
  if (pb->adj) return FDCGKS_OK;
  const long pl = pb->g.plane;
  size_t bytes = (size_t)ADJ_PLANES * pl * sizeof(double);
  hipError_t e = hipMalloc((void**)&pb->adj, bytes);
  if (e != hipSuccess) {
    pb->adj = nullptr;
    return fail(pb, e == hipErrorOutOfMemory ? FDCGKS_ENOMEM : FDCGKS_EHIP, "adjoint workspace: %s",
                hipGetErrorString(e));
  }
  HIPCHK(pb, hipMemsetAsync(pb->adj, 0, bytes, pb->stream));
  double* q = pb->adj;
  auto take = [&](double*& dst, int planes) { dst = q; q += (long)planes * pl; };
  take(pb->E1, 100);
  take(pb->Nb1, 32);
  take(pb->Lo, 24);
  take(pb->Op, 48);
  take(pb->LE, 100);
  take(pb->LN, 32);
  take(pb->LSs, 24);
  take(pb->LAcc, 24);
  take(pb->LS0, 24);
  return FDCGKS_OK;
}

void adj_fold(fdcgks_problem* pb, double* L) {
  const Geo& g = pb->g;
  long nc = 24L * (g.ny + g.sy + 2 * HALO) * 2 * HALO, nr = 24L * 2 * HALO * (g.nx + g.sx);
  hipLaunchKernelGGL(k_adj_fold_cols, dim3(std::min(ceil_div(nc, 256), 4096)), dim3(256), 0, pb->stream, L, 24, g);
  hipLaunchKernelGGL(k_adj_fold_rows, dim3(std::min(ceil_div(nr, 256), 4096)), dim3(256), 0, pb->stream, L, 24, g);
}

// Reverse of one stage.  Sin, E, Nb: the stage's input state and its
// interface / node results; lam_out (and lam_acc for stage 1): adjoint of the
// stage outputs; direct: receives the adjoint of the accumulators (stage 2)
// or of Sin (stage 1); scatter: receives the adjoint of Sin through the
// reconstructions and solvers (stage 2: LSs; stage 1: the same buffer as
// direct).
template <int STAGE>
fdcgks_status adj_stage(fdcgks_problem* pb, double dt, const double* Sin, const double* E, const double* Nb,
                        const double* lam_out, const double* lam_acc, double* direct, double* scatter) {
  const Geo& g = pb->g;
  const dim3 blk(64, 4);
  if (STAGE == 2) HIPCHK(pb, hipMemsetAsync(scatter, 0, 24 * g.plane * sizeof(double), pb->stream));
  else HIPCHK(pb, hipMemsetAsync(direct, 0, 24 * g.plane * sizeof(double), pb->stream));
  // the ranges of the forward launches (bounded axes add the dual grid's boundary nodes), as tiles in XCD
  // bands (xcd_tile3)
  auto bands = [](const Tiles3& t) { return dim3(ceil_div(t.gx * t.gy * t.gz, NXCD) * NXCD); };
  const Tiles3 tu{ceil_div(g.nx + g.sx, 64), ceil_div(g.ny + g.sy, 4), 2};
  hipLaunchKernelGGL((k_adj_update<STAGE>), bands(tu), blk, 0, pb->stream, lam_out, lam_acc, pb->Op, direct, g, pb->k,
                     dt, tu);
  const Tiles3 ta{ceil_div(g.nx + 3 + g.sx, 64), ceil_div(g.ny + 3 + g.sy, 4), 4};
  hipLaunchKernelGGL((k_adj_assemble<STAGE>), bands(ta), blk, 0, pb->stream, pb->Op, E, Nb, pb->LE, g, pb->k, ta);
  const int w = node_reach(pb->k);  // nodes whose fluxes the forward sweep computes beyond the grid's own
  const Tiles3 tn{ceil_div(g.nx + 2 * w + g.sx, 64), ceil_div(g.ny + 2 * w + g.sy, 4), 2};
  hipLaunchKernelGGL((k_adj_nodeflux<STAGE>), bands(tn), blk, 0, pb->stream, pb->Op, E, pb->LN, g, pb->k, tn);
  const bool chr = pb->prm.recon_vars == FDCGKS_RECON_CHARACTERISTIC;
  const Tiles3 te{ceil_div(g.nx + 3 + g.sx, 64), ceil_div(g.ny + 3 + g.sy, 2), 2};
  hipLaunchKernelGGL((chr ? k_adj_edges<STAGE, true> : k_adj_edges<STAGE, false>), bands(te), blk, 0, pb->stream,
                     Sin, pb->LE, scatter, g, pb->k, dt, te);
  hipLaunchKernelGGL((chr ? k_adj_nodes<STAGE, true> : k_adj_nodes<STAGE, false>), bands(tn), blk, 0, pb->stream,
                     Sin, pb->LN, scatter, g, pb->k, tn);
  adj_fold(pb, scatter);
  return launch_check(pb, "adjoint stage");
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
  for (int k = 0; k < 4; ++k) p->side[k] = -1;
  p->flux_variant = FDCGKS_FLUX_6_4;
  p->flux_order = 6;
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
  setup_geometry(*p, pb->g, pb->k);
  const Geo& g = pb->g;
  pb->ngrid = p->dim == 2 ? 2 : (p->dual_1d ? 2 : 1);
  pb->nplanes = (int)state_planes(*p);
  {
    int dev = 0, cu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cu > 0)
      pb->ncu = cu;
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
  // CFL partials (2 per block) and diagnostics partials (up to 10 per block)
  if (e == hipSuccess) e = hipMalloc((void**)&pb->part, (size_t)10 * pb->nparts * sizeof(double));
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

// Stored nodes of a grid: the dual grid has one more column (row) along a
// bounded axis.
static int grid_nx(const fdcgks_problem* pb, int grid) { return pb->g.nx + (grid == 1 ? pb->g.sx : 0); }
static int grid_ny(const fdcgks_problem* pb, int grid) { return pb->g.ny + (grid == 1 ? pb->g.sy : 0); }

static fdcgks_status copy_grid(fdcgks_problem* pb, int grid, double* const* ptrs, int to_device_state,
                               int64_t row_stride, int on_device) {
  const Geo& g = pb->g;
  int ncomp = pb->prm.dim == 2 ? 4 : 3;
  int nfield = pb->prm.dim == 2 ? 3 : 2;
  const int mx = grid_nx(pb, grid), my = grid_ny(pb, grid);
  if (row_stride == 0) row_stride = mx;
  if (row_stride < mx) return fail(pb, FDCGKS_EINVAL, "row_stride %ld below the row length %d", (long)row_stride, mx);
  double* base = pb->S[pb->cur] + (long)grid * (pb->prm.dim == 2 ? 12 : 6) * g.plane;
  size_t row = (size_t)mx * sizeof(double), upitch = (size_t)row_stride * sizeof(double);
  if (!on_device && row_stride == mx) {
    // Dense host arrays: one contiguous host transfer per field through the
    // interface buffer (idle between steps, 100 planes, room for the ncomp
    // dense planes of a field), and the padded layout by device-to-device 2D
    // copies.  Pageable 2D host copies row by row are several times slower.
    double* stage = pb->E;
    const size_t plane_dense = (size_t)mx * my, field_bytes = plane_dense * ncomp * sizeof(double);
    for (int f = 0; f < nfield; ++f) {
      double* dev0 = base + (long)f * ncomp * g.plane + (long)OY * g.pitch + OX;
      if (to_device_state)
        HIPCHK(pb, hipMemcpyAsync(stage, ptrs[f], field_bytes, hipMemcpyHostToDevice, pb->stream));
      for (int c = 0; c < ncomp; ++c) {
        double* dev = dev0 + (long)c * g.plane;
        double* st = stage + (long)c * plane_dense;
        if (to_device_state)
          HIPCHK(pb, hipMemcpy2DAsync(dev, (size_t)g.pitch * sizeof(double), st, row, row, my,
                                      hipMemcpyDeviceToDevice, pb->stream));
        else
          HIPCHK(pb, hipMemcpy2DAsync(st, row, dev, (size_t)g.pitch * sizeof(double), row, my,
                                      hipMemcpyDeviceToDevice, pb->stream));
      }
      if (!to_device_state)
        HIPCHK(pb, hipMemcpyAsync(ptrs[f], stage, field_bytes, hipMemcpyDeviceToHost, pb->stream));
    }
    HIPCHK(pb, hipStreamSynchronize(pb->stream));
    return FDCGKS_OK;
  }
  hipMemcpyKind kind = to_device_state ? (on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice)
                                       : (on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost);
  for (int f = 0; f < nfield; ++f)
    for (int c = 0; c < ncomp; ++c) {
      double* dev = base + (long)(f * (pb->prm.dim == 2 ? 4 : 3) + c) * g.plane + (long)OY * g.pitch + OX;
      double* usr = ptrs[f] + (long)c * row_stride * my;
      if (to_device_state)
        HIPCHK(pb, hipMemcpy2DAsync(dev, (size_t)g.pitch * sizeof(double), usr, upitch, row, my, kind, pb->stream));
      else
        HIPCHK(pb, hipMemcpy2DAsync(usr, upitch, dev, (size_t)g.pitch * sizeof(double), row, my, kind, pb->stream));
    }
  if (!on_device) HIPCHK(pb, hipStreamSynchronize(pb->stream));
  return FDCGKS_OK;
}

fdcgks_status fdcgks_set_state(fdcgks_problem* pb, int32_t grid, const double* W, const double* Wx, const double* Wy,
                               int64_t row_stride, int32_t on_device) {
  if (!pb) return fail(nullptr, FDCGKS_EINVAL, "problem is NULL");
  if (grid < 0 || grid >= pb->ngrid) return fail(pb, FDCGKS_EINVAL, "grid %d not present", grid);
  if (!W || !Wx || (pb->prm.dim == 2 && !Wy)) return fail(pb, FDCGKS_EINVAL, "state pointer is NULL");
  double* ptrs[3] = {const_cast<double*>(W), const_cast<double*>(Wx), const_cast<double*>(Wy)};
  fdcgks_status st = copy_grid(pb, grid, ptrs, 1, row_stride, on_device);
  if (st) return st;
  pb->have_state[grid] = true;
  return FDCGKS_OK;
}

fdcgks_status fdcgks_get_state(const fdcgks_problem* cpb, int32_t grid, double* W, double* Wx, double* Wy,
                               int64_t row_stride, int32_t on_device) {
  fdcgks_problem* pb = const_cast<fdcgks_problem*>(cpb);
  if (!pb) return fail(nullptr, FDCGKS_EINVAL, "problem is NULL");
  if (grid < 0 || grid >= pb->ngrid) return fail(pb, FDCGKS_EINVAL, "grid %d not present", grid);
  if (!W || !Wx || (pb->prm.dim == 2 && !Wy)) return fail(pb, FDCGKS_EINVAL, "state pointer is NULL");
  double* ptrs[3] = {W, Wx, Wy};
  return copy_grid(pb, grid, ptrs, 0, row_stride, on_device);
}

fdcgks_status fdcgks_set_state_from_samples(fdcgks_problem* pb, const double* S, int32_t on_device) {
  if (!pb) return fail(nullptr, FDCGKS_EINVAL, "problem is NULL");
  if (!S) return fail(pb, FDCGKS_EINVAL, "samples pointer is NULL");
  const Geo& g = pb->g;
  if (g.sx | g.sy || (pb->prm.dim == 1 && pb->prm.bc != FDCGKS_BC_PERIODIC))
    return fail(pb, FDCGKS_EINVAL, "state from samples needs periodic sides");
  const int ncomp = pb->prm.dim == 2 ? 4 : 3;
  const long nS = (long)ncomp * 2 * g.nx * (pb->prm.dim == 2 ? 2 * g.ny : 1);
  const double* src = S;
  if (!on_device) {
    // stage the host samples in the stage buffer (free between steps; it
    // holds nplanes padded planes, more than the nS samples)
    HIPCHK(pb, hipMemcpyAsync(pb->Sstar, S, (size_t)nS * sizeof(double), hipMemcpyHostToDevice, pb->stream));
    src = pb->Sstar;
  }
  if (pb->prm.dim == 2) {
    const long n = 2L * 4 * g.nx * g.ny;
    hipLaunchKernelGGL(k_from_samples2d, dim3(std::min(ceil_div(n, 256), 65535)), dim3(256), 0, pb->stream, src,
                       pb->S[pb->cur], g);
  } else {
    const long n = (long)pb->ngrid * 3 * g.nx;
    hipLaunchKernelGGL(k_from_samples1d, dim3(std::min(ceil_div(n, 256), 65535)), dim3(256), 0, pb->stream, src,
                       pb->S[pb->cur], g, pb->ngrid);
  }
  fdcgks_status st = launch_check(pb, "from_samples");
  if (st) return st;
  if (!on_device) HIPCHK(pb, hipStreamSynchronize(pb->stream));
  for (int gr = 0; gr < pb->ngrid; ++gr) pb->have_state[gr] = true;
  return FDCGKS_OK;
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

fdcgks_status fdcgks_diagnostics(fdcgks_problem* pb, double* out) {
  if (!pb || !out) return fail(pb, FDCGKS_EINVAL, "NULL argument");
  if (!state_ready(pb)) return fail(pb, FDCGKS_ESTATE, "set_state has not been called for every grid");
  const Geo& g = pb->g;
  const int nc = pb->prm.dim == 2 ? 4 : 3, NQ = pb->ngrid * nc + 2;
  const long gstride = (pb->prm.dim == 2 ? 12 : 6) * g.plane;
  if (pb->prm.dim == 2)
    hipLaunchKernelGGL(k_diag_partial<2>, dim3(pb->nparts), dim3(256), 0, pb->stream, pb->S[pb->cur], g, pb->ngrid,
                       gstride, pb->k.gamma, pb->part);
  else
    hipLaunchKernelGGL(k_diag_partial<1>, dim3(pb->nparts), dim3(256), 0, pb->stream, pb->S[pb->cur], g, pb->ngrid,
                       gstride, pb->k.gamma, pb->part);
  fdcgks_status st = launch_check(pb, "diagnostics");
  if (st) return st;
  std::vector<double> h((size_t)pb->nparts * NQ);
  HIPCHK(pb, hipMemcpyAsync(h.data(), pb->part, h.size() * sizeof(double), hipMemcpyDeviceToHost, pb->stream));
  HIPCHK(pb, hipStreamSynchronize(pb->stream));
  for (int q = 0; q < NQ; ++q) out[q] = q >= NQ - 2 ? 1e300 : 0.0;
  for (int b = 0; b < pb->nparts; ++b)  // fixed order: the result does not depend on timing
    for (int q = 0; q < NQ; ++q) {
      const double v = h[(size_t)b * NQ + q];
      out[q] = q >= NQ - 2 ? std::fmin(out[q], v) : out[q] + v;
    }
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
  if (pb->prm.dim == 1 && nsteps > 0) {
    st = launch_run1d(pb, 0, nsteps, dt, cfl);
    mark(pb, TK_STEP);
    nsteps = 0;
  }
  const int K = pb->graph_steps;
  if (pb->prm.dim == 2 && K > 0 && nsteps >= K && !pb->timing) {
    st = capture_steps(pb, dt, cfl);
    for (; !st && nsteps >= K; nsteps -= K) {
      hipError_t e = hipGraphLaunch(pb->gx[cur], pb->stream);
      if (e != hipSuccess) st = fail(pb, FDCGKS_EHIP, "step graph launch: %s", hipGetErrorString(e));
      cur ^= K & 1;
    }
    if (st) nsteps = 0;
  }
  for (int s = 0; s < nsteps; ++s) {
    pb->cur = cur;
    st = begin_step(pb, dt, cfl, s == 0 || !fold_ok(pb, dt));
    mark(pb, TK_STEP);
    if (!st) st = stage2d<1>(pb, pb->S[cur], nullptr, pb->Sstar, pb->Acc, stage_mode(pb));
    pb->cfl_fold = fold_ok(pb, dt);
    if (!st) st = stage2d<2>(pb, pb->Sstar, pb->Acc, pb->S[1 - cur], nullptr, stage_mode(pb));
    pb->cfl_fold = false;
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

// Device address of `scratch` on each device, looked up once per device with
// that device current.
static std::atomic<double*> g_static_ptr[64];

fdcgks_status fdcgks_step1d_static(const fdcgks_params* p, double* state, double dt, double cfl, int32_t nsteps,
                                   double t_end, double* t_inout, int32_t* steps_done, void* hip_stream) {
  fdcgks_status st = check_params(p);
  if (st) return st;
  if (p->dim != 1) return fail(nullptr, FDCGKS_EINVAL, "the allocation-free run is 1D only");
  if (p->nx > STATIC1D_MAX_NX)
    return fail(nullptr, FDCGKS_EINVAL, "the allocation-free run takes at most %d nodes per line (got %d)",
                STATIC1D_MAX_NX, p->nx);
  if (!state || !t_inout) return fail(nullptr, FDCGKS_EINVAL, "state and t_inout must not be NULL");
  if (nsteps < 0) return fail(nullptr, FDCGKS_EINVAL, "nsteps < 0");
  if (!(dt > 0) && !(cfl > 0)) return fail(nullptr, FDCGKS_EINVAL, "need dt > 0 or cfl > 0");
  if (!std::isfinite(dt) || !std::isfinite(*t_inout) || !std::isfinite(t_end))
    return fail(nullptr, FDCGKS_EINVAL, "dt, t and t_end must be finite");
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, state) != hipSuccess || attr.type != hipMemoryTypeDevice) {
    (void)hipGetLastError();
    return fail(nullptr, FDCGKS_EINVAL, "state must be device memory");
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
    return fail(nullptr, FDCGKS_EHIP, "no usable current device");
  if (attr.device != dev) return fail(nullptr, FDCGKS_EINVAL, "state lives on device %d, not the current %d",
                                      attr.device, dev);
  const int lines = p->dual_1d ? 2 : 1;
  {
    // the caller's array must hold lines * 6 * nx doubles inside its allocation
    hipDeviceptr_t lo = nullptr;
    size_t len = 0;
    if (hipMemGetAddressRange(&lo, &len, state) != hipSuccess) {
      (void)hipGetLastError();
      return fail(nullptr, FDCGKS_EINVAL, "state is not a device allocation");
    }
    const char* end = reinterpret_cast<const char*>(state) + (size_t)lines * 6 * p->nx * sizeof(double);
    if (end > static_cast<const char*>(lo) + len)
      return fail(nullptr, FDCGKS_EINVAL, "state allocation is smaller than %d x 6 x %d doubles", lines, p->nx);
  }
  double* base = g_static_ptr[dev].load();
  if (!base) {
    void* a = nullptr;
    hipError_t e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !a)
      return fail(nullptr, FDCGKS_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    base = static_cast<double*>(a);
    g_static_ptr[dev].store(base);
  }
  Geo g;
  Consts k;
  setup_geometry(*p, g, k);
  const long pl = g.plane;  // <= STATIC1D_PLANE since nx <= STATIC1D_MAX_NX
  double* S0 = base;
  double* S1 = base + 12 * pl;
  double* Sstar = base + 24 * pl;
  double* Acc = base + 36 * pl;
  double* E = base + 48 * pl;
  double* Nb = base + 86 * pl;
  Scal* sc = reinterpret_cast<Scal*>(base + STATIC1D_PLANES * pl);
  hipStream_t stream = (hipStream_t)hip_stream;
  const int use_cfl = dt > 0 ? 0 : 1;
  const bool f32 = p->flux_precision == FDCGKS_FP32_FLUX;
  const bool ch = p->recon_vars == FDCGKS_RECON_CHARACTERISTIC;
  auto fn = f32 ? (ch ? k_run1d<float, true> : k_run1d<float, false>)
                : (ch ? k_run1d<double, true> : k_run1d<double, false>);
  const int ioblocks = ceil_div((long)lines * 6 * g.nx, 256);
  hipLaunchKernelGGL(k_static1d_begin, dim3(1), dim3(64), 0, stream, sc, *t_inout, t_end, dt);
  hipLaunchKernelGGL(k_static1d_io, dim3(ioblocks), dim3(256), 0, stream, state, S0, S1, g, lines, sc, 0);
  if (nsteps > 0)
    hipLaunchKernelGGL(fn, dim3(1), dim3(256), 0, stream, S0, S1, Sstar, Acc, E, Nb, g, k, sc, lines, p->bc, nsteps,
                       cfl, use_cfl, 0);
  hipLaunchKernelGGL(k_static1d_io, dim3(ioblocks), dim3(256), 0, stream, state, S0, S1, g, lines, sc, 1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(nullptr, FDCGKS_EHIP, "launch failed: %s", hipGetErrorString(e));
  Scal h;
  e = hipMemcpyAsync(&h, sc, sizeof(Scal), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return fail(nullptr, FDCGKS_EHIP, "reading the step scalars: %s", hipGetErrorString(e));
  *t_inout = h.t;
  if (steps_done) *steps_done = h.steps;
  if (h.stop & 1)
    return fail(nullptr, FDCGKS_ENONPHYS, "non-physical state in step %d stage %d at line %d node %d", h.steps + 1,
                h.fail_stage, h.fail_grid, h.fail_i);
  return FDCGKS_OK;
}

fdcgks_status fdcgks_destroy(fdcgks_problem* pb) {
  if (!pb) return FDCGKS_OK;
  (void)hipStreamSynchronize(pb->stream);
  graph_invalidate(pb);
  if (pb->cap) (void)hipStreamDestroy(pb->cap);
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
  return pb ? pb->err.c_str() : g_create_error;
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
    if (pb->prm.dim == 1) st = launch_run1d(pb, stage, 0, dt, 0.0);
    else if (stage == 1) st = stage2d<1>(pb, pb->S[pb->cur], nullptr, pb->Sstar, pb->Acc, stage_mode(pb));
    else st = stage2d<2>(pb, pb->Sstar, pb->Acc, scratch, nullptr, stage_mode(pb));
  }
  if (st) return st;
  const Geo& g = pb->g;
  const double* src = stage == 1 ? pb->Sstar : scratch;
  size_t pitchb = (size_t)g.pitch * sizeof(double);
  const int npg = pb->prm.dim == 2 ? 12 : 6;  // planes per grid
  long off = 0;
  for (int gr = 0; gr < pb->ngrid; ++gr) {
    const int mx = grid_nx(pb, gr), my = grid_ny(pb, gr);
    const size_t row = (size_t)mx * sizeof(double);
    for (int q = 0; q < npg; ++q, off += (long)mx * my) {
      const long p = (long)gr * npg + q;
      HIPCHK(pb, hipMemcpy2DAsync(out_state + off, row, src + p * g.plane + (long)OY * g.pitch + OX, pitchb, row, my,
                                  hipMemcpyDeviceToHost, pb->stream));
      if (stage == 1 && out_acc)
        HIPCHK(pb, hipMemcpy2DAsync(out_acc + off, row, pb->Acc + p * g.plane + (long)OY * g.pitch + OX, pitchb, row,
                                    my, hipMemcpyDeviceToHost, pb->stream));
    }
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
  if (!st) st = stage2d<1>(pb, pb->S[pb->cur], nullptr, pb->Sstar, pb->Acc, STAGE_SEPARATE);
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

fdcgks_status fdcgks_step_vjp(fdcgks_problem* pb, double dt, const double* lam_out, double* lam_in,
                              int32_t on_device) {
  if (!pb || !lam_out || !lam_in) return fail(pb, FDCGKS_EINVAL, "NULL argument");
  if (pb->prm.dim != 2) return fail(pb, FDCGKS_EINVAL, "the step adjoint is implemented for 2D problems");
  if (pb->prm.flux_precision != FDCGKS_FP64) return fail(pb, FDCGKS_EINVAL, "the step adjoint needs FP64 fluxes");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(pb, FDCGKS_EINVAL, "dt must be finite and > 0");
  if (!state_ready(pb)) return fail(pb, FDCGKS_ESTATE, "set_state has not been called for every grid");
  fdcgks_status st = adj_alloc(pb);
  if (st) return st;
  const Geo& g = pb->g;
  const size_t pitchb = (size_t)g.pitch * sizeof(double);
  const long interior = (long)OY * g.pitch + OX;
  // dense layout: grid 0's 12 planes, then grid 1's (one more node along a bounded axis)
  const int mx[2] = {g.nx, g.nx + g.sx}, my[2] = {g.ny, g.ny + g.sy};
  const long total = 12L * ((long)mx[0] * my[0] + (long)mx[1] * my[1]);
  auto dense_plane = [&](int p) {  // offset of plane p (grid p / 12) in the dense layout
    return p < 12 ? (long)p * mx[0] * my[0] : 12L * mx[0] * my[0] + (long)(p - 12) * mx[1] * my[1];
  };
  // adjoint of the step output into the padded layout (halo stays zero)
  // host input: one contiguous transfer into the interface buffer (written
  // by the forward recompute only after these copies, in stream order), then
  // device-to-device 2D copies into the padded layout
  const double* lsrc = lam_out;
  if (!on_device) {
    HIPCHK(pb, hipMemcpyAsync(pb->E, lam_out, (size_t)total * sizeof(double), hipMemcpyHostToDevice, pb->stream));
    lsrc = pb->E;
  }
  for (int p = 0; p < 24; ++p) {
    const size_t row = (size_t)mx[p / 12] * sizeof(double);
    HIPCHK(pb, hipMemcpy2DAsync(pb->Lo + p * g.plane + interior, pitchb, lsrc + dense_plane(p), row, row,
                                my[p / 12], hipMemcpyDeviceToDevice, pb->stream));
  }
  // forward recompute at the frozen dt: stage-1 results into E1/Nb1, stage-2 into E/Nb
  std::memset(pb->sc_host, 0, sizeof(Scal));
  pb->sc_host->dt = dt;
  st = write_scal(pb);
  double* E0 = pb->E;
  double* N0 = pb->Nb;
  double* scratch = pb->S[1 - pb->cur];
  pb->E = pb->E1;
  pb->Nb = pb->Nb1;
  if (!st) st = stage2d<1>(pb, pb->S[pb->cur], nullptr, pb->Sstar, pb->Acc, STAGE_SEPARATE);
  pb->E = E0;
  pb->Nb = N0;
  if (!st) st = stage2d<2>(pb, pb->Sstar, pb->Acc, scratch, nullptr, STAGE_SEPARATE);
  if (!st) st = read_scal(pb);
  if (st) return st;
  if (pb->sc_host->stop & 1)
    return fail(pb, FDCGKS_ENONPHYS, "non-physical state in the forward step (stage %d, grid %d, node (%d, %d))",
                pb->sc_host->fail_stage, pb->sc_host->fail_grid, pb->sc_host->fail_i, pb->sc_host->fail_j);
  // reverse: stage 2 then stage 1
  st = adj_stage<2>(pb, dt, pb->Sstar, pb->E, pb->Nb, pb->Lo, nullptr, pb->LAcc, pb->LSs);
  if (!st) st = adj_stage<1>(pb, dt, pb->S[pb->cur], pb->E1, pb->Nb1, pb->LSs, pb->LAcc, pb->LS0, pb->LS0);
  if (st) return st;
  // host output: dense through the interface buffer (free once the reverse
  // sweeps are done), then one contiguous transfer
  double* ldst = on_device ? lam_in : pb->E;
  for (int p = 0; p < 24; ++p) {
    const size_t row = (size_t)mx[p / 12] * sizeof(double);
    HIPCHK(pb, hipMemcpy2DAsync(ldst + dense_plane(p), row, pb->LS0 + p * g.plane + interior, pitchb, row,
                                my[p / 12], hipMemcpyDeviceToDevice, pb->stream));
  }
  if (!on_device) {
    HIPCHK(pb, hipMemcpyAsync(lam_in, pb->E, (size_t)total * sizeof(double), hipMemcpyDeviceToHost, pb->stream));
    HIPCHK(pb, hipStreamSynchronize(pb->stream));
  }
  return FDCGKS_OK;
}

fdcgks_status fdcgks_set_option(fdcgks_problem* pb, int32_t option, int64_t value) {
  if (!pb) return fail(nullptr, FDCGKS_EINVAL, "problem is NULL");
  switch (option) {
    case FDCGKS_OPT_GRAPH:
      if (value < 0 || value > 64) return fail(pb, FDCGKS_EINVAL, "steps per graph must be in 0..64");
      pb->graph_steps = (int)value;
      graph_invalidate(pb);
      return FDCGKS_OK;
    case FDCGKS_OPT_FUSE_NODES:
      if (value != 0 && value != 1) return fail(pb, FDCGKS_EINVAL, "node-fusion option must be 0 or 1");
      pb->fuse_nodes = value != 0;
      graph_invalidate(pb);
      return FDCGKS_OK;
    case FDCGKS_OPT_FUSE_STAGE:
      if (value < 0 || value > 2) return fail(pb, FDCGKS_EINVAL, "stage-fusion option must be 0, 1 or 2");
      pb->fuse_stage = (int)value;
      graph_invalidate(pb);
      return FDCGKS_OK;
    case FDCGKS_OPT_FUSED_ROWS:
      if (value < 0 || value > (1 << 20)) return fail(pb, FDCGKS_EINVAL, "rows per fused block must be >= 0");
      pb->fused_rows = (int)value;
      graph_invalidate(pb);
      return FDCGKS_OK;
    case FDCGKS_OPT_TILE_EDGE:
    case FDCGKS_OPT_TILE_NODE:
    case FDCGKS_OPT_TILE_UPDATE: {
      const int c = option - FDCGKS_OPT_TILE_EDGE;
      const unsigned x = (unsigned)(value & 0xffff), y = (unsigned)((value >> 16) & 0xffff);
      if (value < 0 || (value >> 32) != 0 || !tile_ok(c, x, y))
        return fail(pb, FDCGKS_EINVAL, "invalid launch shape %u x %u for kernel class %d", x, y, c);
      pb->tile[c] = dim3(x, y);
      graph_invalidate(pb);
      return FDCGKS_OK;
    }
    default:
      return fail(pb, FDCGKS_EINVAL, "unknown option %d", option);
  }
}

fdcgks_status fdcgks_get_option(const fdcgks_problem* cpb, int32_t option, int64_t* value) {
  fdcgks_problem* pb = const_cast<fdcgks_problem*>(cpb);
  if (!pb || !value) return fail(pb, FDCGKS_EINVAL, "NULL argument");
  if (option == FDCGKS_OPT_GRAPH) {
    *value = pb->graph_steps;
    return FDCGKS_OK;
  }
  if (option == FDCGKS_OPT_FUSE_NODES) {
    *value = pb->fuse_nodes ? 1 : 0;
    return FDCGKS_OK;
  }
  if (option == FDCGKS_OPT_FUSE_STAGE) {
    *value = pb->fuse_stage;
    return FDCGKS_OK;
  }
  if (option == FDCGKS_OPT_FUSED_ROWS) {
    *value = pb->fused_rows;
    return FDCGKS_OK;
  }
  if (option >= FDCGKS_OPT_TILE_EDGE && option <= FDCGKS_OPT_TILE_UPDATE) {
    const dim3 t = pb->tile[option - FDCGKS_OPT_TILE_EDGE];
    *value = (int64_t)t.x | ((int64_t)t.y << 16);
    return FDCGKS_OK;
  }
  return fail(pb, FDCGKS_EINVAL, "unknown option %d", option);
}

fdcgks_status fdcgks_autotune(fdcgks_problem* pb, int32_t reps) {
  if (!pb) return fail(nullptr, FDCGKS_EINVAL, "problem is NULL");
  if (reps < 1 || reps > 1000) return fail(pb, FDCGKS_EINVAL, "reps must be in 1..1000");
  if (pb->prm.dim != 2) return FDCGKS_OK;  // the 1D path runs in one workgroup: nothing to tune
  if (!state_ready(pb)) return fail(pb, FDCGKS_ESTATE, "set_state has not been called for every grid");
  double dt = 0.0;
  fdcgks_status st = fdcgks_compute_dt(pb, 0.4, &dt);
  if (st) return st;
  // one real stage 1 so that the update reads valid interface and node results
  std::memset(pb->sc_host, 0, sizeof(Scal));
  pb->sc_host->dt = dt;
  st = write_scal(pb);
  if (!st) st = stage2d<1>(pb, pb->S[pb->cur], nullptr, pb->Sstar, pb->Acc, STAGE_SEPARATE);
  if (st) return st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(pb, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(pb, FDCGKS_EHIP, "event creation failed");
  }
  static const unsigned cand[][2] = {{64, 4}, {64, 2}, {128, 2}, {32, 8}, {256, 1}, {128, 1}, {64, 1}, {32, 4}};
  for (int c = 0; c < 3 && !st; ++c) {
    float best = -1.f;
    dim3 pick = pb->tile[c];
    for (const auto& xy : cand) {
      if (!tile_ok(c, xy[0], xy[1])) continue;
      const float ms = time_tile(pb, c, dim3(xy[0], xy[1]), reps, e0, e1);
      if (ms < 0.f) {
        st = launch_check(pb, "autotune");
        if (!st) st = fail(pb, FDCGKS_EHIP, "autotune timing failed");
        break;
      }
      if (best < 0.f || ms < best) {
        best = ms;
        pick = dim3(xy[0], xy[1]);
      }
    }
    pb->tile[c] = pick;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  graph_invalidate(pb);
  if (st) return st;
  st = read_scal(pb);
  if (st) return st;
  if (pb->sc_host->stop & 1) return fail(pb, FDCGKS_ENONPHYS, "non-physical state during autotuning");
  return FDCGKS_OK;
}

}  // extern "C"

// ============================================================ batch host
struct fdcgks_batch {
  int count = 0;
  fdcgks_params prm0;
  Consts k;
  hipStream_t stream = nullptr;
  std::vector<BMember> mem;
  BMember* mem_d = nullptr;
  std::vector<void*> allocs;
  BItem* items_d = nullptr;
  int n_cfl = 0, n_halo = 0, n_edge = 0, n_node = 0, n_upd = 0;
  unsigned long long* slots = nullptr;
  double* t = nullptr;
  double* dt_last = nullptr;
  Scal* sc = nullptr;
  Scal* sc_host = nullptr;
  int cur = 0, parity = 0;
  int blocks = 0;
  int mode = FDCGKS_BATCH_GRAPH;
  // FDCGKS_BATCH_GRAPH: BATCH_GRAPH_STEPS phased steps captured as one HIP
  // graph per start parity (cur, parity), on a private stream, for one cfl
  hipStream_t cap = nullptr;
  hipGraphExec_t gx[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  double g_cfl[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  std::vector<char> have_state;
  std::string err;
};

namespace {
fdcgks_status bfail(fdcgks_batch* b, fdcgks_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (b) b->err = buf; else std::snprintf(g_create_error, sizeof g_create_error, "%s", buf);
  return st;
}
#define BHIPCHK(b, call)                                                                      \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) return bfail(b, FDCGKS_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

void batch_graphs_free(fdcgks_batch* b) {
  for (auto& row : b->gx)
    for (hipGraphExec_t& x : row)
      if (x) {
        (void)hipGraphExecDestroy(x);
        x = nullptr;
      }
}

void batch_free(fdcgks_batch* b) {
  batch_graphs_free(b);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  b->cap = nullptr;
  for (void* p : b->allocs) (void)hipFree(p);
  b->allocs.clear();
  if (b->sc_host) (void)hipHostFree(b->sc_host);
  b->sc_host = nullptr;
}

bool same_scheme(const fdcgks_params& a, const fdcgks_params& b) {
  return a.gamma == b.gamma && a.mu == b.mu && a.prandtl == b.prandtl && a.flux_variant == b.flux_variant &&
         a.flux_precision == b.flux_precision && a.grad_update == b.grad_update && a.geno_r == b.geno_r &&
         a.geno_C == b.geno_C && a.geno_eps == b.geno_eps && a.geno_eps_a == b.geno_eps_a &&
         a.geno_d_central == b.geno_d_central && a.geno_d_side == b.geno_d_side && a.tau_c1 == b.tau_c1 &&
         a.tau_c2 == b.tau_c2 && a.recon_vars == b.recon_vars && a.flux_order == b.flux_order;
}

// Steps per captured batch graph (even, so that a graph keeps the parity).
constexpr int BATCH_GRAPH_STEPS = 16;

// One batched step as one launch per phase on `stream`.
template <class FT, bool CHAR, bool WIDE>
void batch_phased_step_t(const BArgs& a, const Consts& k, hipStream_t stream) {
  const dim3 blk(64, 4);
  hipLaunchKernelGGL(k_bphase_halo<1>, dim3(a.n_cfl + a.n_halo), blk, 0, stream, a, k);
  hipLaunchKernelGGL((k_bphase_edges<1, FT, CHAR>), dim3(a.n_edge), blk, 0, stream, a, k);
  hipLaunchKernelGGL((k_bphase_nodes<1, FT, CHAR>), dim3(a.n_node), blk, 0, stream, a, k);
  hipLaunchKernelGGL((k_bphase_update<1, WIDE>), dim3(a.n_upd), blk, 0, stream, a, k);
  hipLaunchKernelGGL(k_bphase_halo<2>, dim3(a.n_halo), blk, 0, stream, a, k);
  hipLaunchKernelGGL((k_bphase_edges<2, FT, CHAR>), dim3(a.n_edge), blk, 0, stream, a, k);
  hipLaunchKernelGGL((k_bphase_nodes<2, FT, CHAR>), dim3(a.n_node), blk, 0, stream, a, k);
  hipLaunchKernelGGL((k_bphase_update<2, WIDE>), dim3(a.n_upd), blk, 0, stream, a, k);
  hipLaunchKernelGGL(k_bphase_end, dim3(1), blk, 0, stream, a, k);
}
void batch_phased_step(const BArgs& a, const Consts& k, bool fp32, bool chr, hipStream_t stream) {
  using Step = void (*)(const BArgs&, const Consts&, hipStream_t);
  static const Step steps[2][2][2] = {
      {{batch_phased_step_t<double, false, false>, batch_phased_step_t<double, false, true>},
       {batch_phased_step_t<double, true, false>, batch_phased_step_t<double, true, true>}},
      {{batch_phased_step_t<float, false, false>, batch_phased_step_t<float, false, true>},
       {batch_phased_step_t<float, true, false>, batch_phased_step_t<float, true, true>}}};
  steps[fp32][chr][k.flux_order == 8](a, k, stream);
}

// The cooperative persistent kernel of one stage for the batch's scheme.
template <int STAGE> void* batch_kernel_t(bool fp32, bool chr, bool wide) {
  static void* const fns[2][2][2] = {
      {{reinterpret_cast<void*>(k_batch_stage<STAGE, double, false, false>),
        reinterpret_cast<void*>(k_batch_stage<STAGE, double, false, true>)},
       {reinterpret_cast<void*>(k_batch_stage<STAGE, double, true, false>),
        reinterpret_cast<void*>(k_batch_stage<STAGE, double, true, true>)}},
      {{reinterpret_cast<void*>(k_batch_stage<STAGE, float, false, false>),
        reinterpret_cast<void*>(k_batch_stage<STAGE, float, false, true>)},
       {reinterpret_cast<void*>(k_batch_stage<STAGE, float, true, false>),
        reinterpret_cast<void*>(k_batch_stage<STAGE, float, true, true>)}}};
  return fns[fp32][chr][wide];
}
void* batch_kernel(int stage, bool fp32, bool chr, bool wide) {
  return stage == 1 ? batch_kernel_t<1>(fp32, chr, wide) : batch_kernel_t<2>(fp32, chr, wide);
}
}  // namespace

extern "C" {

fdcgks_status fdcgks_batch_create(int32_t count, const fdcgks_params* params, void* hip_stream, fdcgks_batch** out) {
  if (!out) return bfail(nullptr, FDCGKS_EINVAL, "out is NULL");
  *out = nullptr;
  if (count < 1 || !params) return bfail(nullptr, FDCGKS_EINVAL, "need count >= 1 and a params array");
  for (int m = 0; m < count; ++m) {
    fdcgks_status st = check_params(&params[m]);
    if (st) return bfail(nullptr, st, "member %d: %s", m, std::string(g_create_error).c_str());
    if (params[m].dim != 2) return bfail(nullptr, FDCGKS_EINVAL, "member %d: batches are 2D only", m);
    if (!same_scheme(params[0], params[m]))
      return bfail(nullptr, FDCGKS_EINVAL, "member %d: scheme constants differ from member 0", m);
  }
  int dev = 0, coop = 0, ncu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return bfail(nullptr, FDCGKS_EHIP, "device query failed: %s", hipGetErrorString(e));
  if (!coop) return bfail(nullptr, FDCGKS_EHIP, "device does not support cooperative launches");
  fdcgks_batch* b = new fdcgks_batch();
  b->count = count;
  b->prm0 = params[0];
  b->stream = (hipStream_t)hip_stream;
  // scheme constants (shared)
  const fdcgks_params& p = params[0];
  Consts& k = b->k;
  std::memset(&k, 0, sizeof k);
  k.gamma = p.gamma;
  k.K = (4.0 - 2.0 * p.gamma) / (p.gamma - 1.0);
  k.inv_Kd = 1.0 / (k.K + 2.0);
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
  // per-member buffers and work lists
  std::vector<BItem> cfl, halo, edge, node, upd;
  b->mem.resize(count);
  b->have_state.assign(2 * count, 0);
  auto alloc = [&](size_t bytes) -> double* {
    void* ptr = nullptr;
    if (e == hipSuccess) e = hipMalloc(&ptr, bytes);
    if (e == hipSuccess) {
      b->allocs.push_back(ptr);
      e = hipMemsetAsync(ptr, 0, bytes, b->stream);
    }
    return (double*)ptr;
  };
  for (int m = 0; m < count && e == hipSuccess; ++m) {
    Geo& g = b->mem[m].g;
    Consts km;  // the shared constants are b->k
    setup_geometry(params[m], g, km);
    size_t sb = (size_t)24 * g.plane * sizeof(double);
    b->mem[m].S[0] = alloc(sb);
    b->mem[m].S[1] = alloc(sb);
    b->mem[m].Sstar = alloc(sb);
    b->mem[m].Acc = alloc(sb);
    b->mem[m].E = alloc((size_t)100 * g.plane * sizeof(double));
    b->mem[m].Nb = alloc((size_t)32 * g.plane * sizeof(double));
    // ranges of the single-problem launches; a bounded axis adds the dual
    // grid's boundary row / column
    for (int by = 0; by < ceil_div(g.ny + g.sy, 16); ++by) cfl.push_back({m, 0, 0, by});
    for (int pl = 0; pl < 24; ++pl) halo.push_back({m, pl, 0, 0});
    for (int z = 0; z < 2; ++z)
      for (int by = 0; by < ceil_div(g.ny + 3 + g.sy, 2); ++by)
        for (int bx = 0; bx < ceil_div(g.nx + 3 + g.sx, 64); ++bx) edge.push_back({m, z, bx, by});
    const int w = node_reach(k);  // nodes beyond the grid's own that the update reads
    for (int z = 0; z < 2; ++z)
      for (int by = 0; by < ceil_div(g.ny + 2 * w + g.sy, 4); ++by)
        for (int bx = 0; bx < ceil_div(g.nx + w + OX, 64); ++bx) node.push_back({m, z, bx, by});  // from i = -OX
    for (int z = 0; z < 2; ++z)
      for (int by = 0; by < ceil_div(g.ny + g.sy, 4); ++by)
        for (int bx = 0; bx < ceil_div(g.nx + g.sx, 64); ++bx) upd.push_back({m, z, bx, by});
  }
  b->n_cfl = (int)cfl.size();
  b->n_halo = (int)halo.size();
  b->n_edge = (int)edge.size();
  b->n_node = (int)node.size();
  b->n_upd = (int)upd.size();
  std::vector<BItem> all;
  for (auto* v : {&cfl, &halo, &edge, &node, &upd}) all.insert(all.end(), v->begin(), v->end());
  b->mem_d = (BMember*)alloc(sizeof(BMember) * count);
  b->items_d = (BItem*)alloc(sizeof(BItem) * all.size());
  b->slots = (unsigned long long*)alloc(sizeof(unsigned long long) * 4 * count);
  b->t = alloc(sizeof(double) * count);
  b->dt_last = alloc(sizeof(double) * count);
  b->sc = (Scal*)alloc(sizeof(Scal));
  if (e == hipSuccess) e = hipHostMalloc((void**)&b->sc_host, sizeof(Scal), hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->mem_d, b->mem.data(), sizeof(BMember) * count, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->items_d, all.data(), sizeof(BItem) * all.size(), hipMemcpyHostToDevice, b->stream);
  // CFL slots of both parities: max speed 0, min rho +big
  std::vector<unsigned long long> sl(4 * count, 0ull);
  double big = 1e300;
  unsigned long long bigbits;
  std::memcpy(&bigbits, &big, sizeof big);
  for (int q = 0; q < 2; ++q)
    for (int m = 0; m < count; ++m) sl[(2 * q + 1) * count + m] = bigbits;
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->slots, sl.data(), sizeof(unsigned long long) * sl.size(), hipMemcpyHostToDevice,
                       b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  // resident workgroups of the cooperative grid
  if (e == hipSuccess) {
    int nb1 = 0, nb2 = 0;
    const bool fp32 = p.flux_precision == FDCGKS_FP32_FLUX, chr = p.recon_vars == FDCGKS_RECON_CHARACTERISTIC;
    const bool wide = p.flux_order == 8;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb1, batch_kernel(1, fp32, chr, wide), 256, 0);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb2, batch_kernel(2, fp32, chr, wide), 256, 0);
    b->blocks = std::max(1, std::min(nb1, nb2)) * ncu;
  }
  if (e != hipSuccess) {
    fdcgks_status code = (e == hipErrorOutOfMemory) ? FDCGKS_ENOMEM : FDCGKS_EHIP;
    bfail(nullptr, code, "batch setup failed: %s", hipGetErrorString(e));
    batch_free(b);
    delete b;
    return code;
  }
  *out = b;
  return FDCGKS_OK;
}

static fdcgks_status batch_copy(fdcgks_batch* b, int m, int grid, double* const* ptrs, int to_dev, int on_device) {
  const Geo& g = b->mem[m].g;
  double* base = b->mem[m].S[b->cur] + (long)grid * 12 * g.plane;
  const int mx = g.nx + (grid ? g.sx : 0), my = g.ny + (grid ? g.sy : 0);  // stored nodes of the grid
  size_t row = (size_t)mx * sizeof(double);
  const size_t dense = (size_t)mx * my;
  // host arrays go through the member's interface buffer (idle between
  // steps) as one contiguous transfer per field, like single problems
  for (int f = 0; f < 3; ++f) {
    double* stage = on_device ? ptrs[f] : b->mem[m].E;
    if (to_dev && !on_device)
      BHIPCHK(b, hipMemcpyAsync(stage, ptrs[f], 4 * dense * sizeof(double), hipMemcpyHostToDevice, b->stream));
    for (int c = 0; c < 4; ++c) {
      double* dev = base + (long)(f * 4 + c) * g.plane + (long)OY * g.pitch + OX;
      double* usr = stage + (long)c * dense;
      if (to_dev)
        BHIPCHK(b, hipMemcpy2DAsync(dev, (size_t)g.pitch * sizeof(double), usr, row, row, my,
                                    hipMemcpyDeviceToDevice, b->stream));
      else
        BHIPCHK(b, hipMemcpy2DAsync(usr, row, dev, (size_t)g.pitch * sizeof(double), row, my,
                                    hipMemcpyDeviceToDevice, b->stream));
    }
    if (!to_dev && !on_device)
      BHIPCHK(b, hipMemcpyAsync(ptrs[f], stage, 4 * dense * sizeof(double), hipMemcpyDeviceToHost, b->stream));
  }
  if (!on_device) BHIPCHK(b, hipStreamSynchronize(b->stream));
  return FDCGKS_OK;
}

fdcgks_status fdcgks_batch_set_state(fdcgks_batch* b, int32_t member, int32_t grid, const double* W, const double* Wx,
                                     const double* Wy, int32_t on_device) {
  if (!b) return bfail(nullptr, FDCGKS_EINVAL, "batch is NULL");
  if (member < 0 || member >= b->count || grid < 0 || grid > 1)
    return bfail(b, FDCGKS_EINVAL, "member %d / grid %d out of range", member, grid);
  if (!W || !Wx || !Wy) return bfail(b, FDCGKS_EINVAL, "state pointer is NULL");
  double* ptrs[3] = {const_cast<double*>(W), const_cast<double*>(Wx), const_cast<double*>(Wy)};
  fdcgks_status st = batch_copy(b, member, grid, ptrs, 1, on_device);
  if (!st) b->have_state[2 * member + grid] = 1;
  return st;
}

fdcgks_status fdcgks_batch_get_state(const fdcgks_batch* cb, int32_t member, int32_t grid, double* W, double* Wx,
                                     double* Wy, int32_t on_device) {
  fdcgks_batch* b = const_cast<fdcgks_batch*>(cb);
  if (!b) return bfail(nullptr, FDCGKS_EINVAL, "batch is NULL");
  if (member < 0 || member >= b->count || grid < 0 || grid > 1)
    return bfail(b, FDCGKS_EINVAL, "member %d / grid %d out of range", member, grid);
  if (!W || !Wx || !Wy) return bfail(b, FDCGKS_EINVAL, "state pointer is NULL");
  double* ptrs[3] = {W, Wx, Wy};
  return batch_copy(b, member, grid, ptrs, 0, on_device);
}

fdcgks_status fdcgks_batch_step(fdcgks_batch* b, double cfl, int32_t nsteps, double* t_out, double* dt_out,
                                int32_t* steps_done) {
  if (!b) return bfail(nullptr, FDCGKS_EINVAL, "batch is NULL");
  if (!(cfl > 0) || nsteps < 0) return bfail(b, FDCGKS_EINVAL, "need cfl > 0 and nsteps >= 0");
  for (char c : b->have_state)
    if (!c) return bfail(b, FDCGKS_ESTATE, "set_state has not been called for every member and grid");
  std::memset(b->sc_host, 0, sizeof(Scal));
  BHIPCHK(b, hipMemcpyAsync(b->sc, b->sc_host, sizeof(Scal), hipMemcpyHostToDevice, b->stream));
  const int cur0 = b->cur, par0 = b->parity;
  BArgs a;
  a.mem = b->mem_d;
  a.count = b->count;
  a.items = b->items_d;
  a.n_cfl = b->n_cfl;
  a.n_halo = b->n_halo;
  a.n_edge = b->n_edge;
  a.n_node = b->n_node;
  a.n_upd = b->n_upd;
  a.cfl = cfl;
  a.slots = b->slots;
  a.t = b->t;
  a.dt_last = b->dt_last;
  a.sc = b->sc;
  const bool fp32 = b->prm0.flux_precision == FDCGKS_FP32_FLUX;
  const bool chr = b->prm0.recon_vars == FDCGKS_RECON_CHARACTERISTIC;
  int s = 0;
  if (b->mode == FDCGKS_BATCH_GRAPH && nsteps >= BATCH_GRAPH_STEPS) {
    // whole graphs of BATCH_GRAPH_STEPS (even) steps leave cur and parity unchanged
    hipGraphExec_t& gx = b->gx[cur0][par0];
    if (gx && b->g_cfl[cur0][par0] != cfl) {
      (void)hipGraphExecDestroy(gx);
      gx = nullptr;
    }
    if (!gx) {
      if (!b->cap) BHIPCHK(b, hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
      BHIPCHK(b, hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
      for (int q = 0; q < BATCH_GRAPH_STEPS; ++q) {
        a.cur = cur0 ^ (q & 1);
        a.parity = par0 ^ (q & 1);
        batch_phased_step(a, b->k, fp32, chr, b->cap);
      }
      hipGraph_t gr = nullptr;
      hipError_t e = hipStreamEndCapture(b->cap, &gr);
      if (e == hipSuccess) e = hipGetLastError();
      if (e == hipSuccess) e = hipGraphInstantiate(&gx, gr, nullptr, nullptr, 0);
      if (gr) (void)hipGraphDestroy(gr);
      if (e != hipSuccess) {
        gx = nullptr;
        return bfail(b, FDCGKS_EHIP, "batched step capture: %s", hipGetErrorString(e));
      }
      b->g_cfl[cur0][par0] = cfl;
    }
    for (; s + BATCH_GRAPH_STEPS <= nsteps; s += BATCH_GRAPH_STEPS)
      BHIPCHK(b, hipGraphLaunch(gx, b->stream));
  }
  for (; s < nsteps; ++s) {
    a.cur = cur0 ^ (s & 1);
    a.parity = par0 ^ (s & 1);
    if (b->mode == FDCGKS_BATCH_PERSISTENT) {
      void* args[2] = {&a, &b->k};
      for (int stage = 1; stage <= 2; ++stage) {
        void* fn = batch_kernel(stage, fp32, chr, b->k.flux_order == 8);
        BHIPCHK(b, hipLaunchCooperativeKernel(fn, dim3(b->blocks), dim3(64, 4), args, 0, b->stream));
      }
      continue;
    }
    batch_phased_step(a, b->k, fp32, chr, b->stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return bfail(b, FDCGKS_EHIP, "batched launch failed: %s", hipGetErrorString(e));
  }
  BHIPCHK(b, hipMemcpyAsync(b->sc_host, b->sc, sizeof(Scal), hipMemcpyDeviceToHost, b->stream));
  if (t_out) BHIPCHK(b, hipMemcpyAsync(t_out, b->t, sizeof(double) * b->count, hipMemcpyDeviceToHost, b->stream));
  if (dt_out)
    BHIPCHK(b, hipMemcpyAsync(dt_out, b->dt_last, sizeof(double) * b->count, hipMemcpyDeviceToHost, b->stream));
  BHIPCHK(b, hipStreamSynchronize(b->stream));
  const int done = b->sc_host->steps;
  b->cur = cur0 ^ (done & 1);
  b->parity = par0 ^ (done & 1);
  if (steps_done) *steps_done = done;
  if (b->sc_host->stop & 1) {
    // the failing step's input is intact; the next step must start from clean CFL slots
    std::vector<unsigned long long> sl(4 * b->count, 0ull);
    double big = 1e300;
    unsigned long long bigbits;
    std::memcpy(&bigbits, &big, sizeof big);
    for (int q = 0; q < 2; ++q)
      for (int m = 0; m < b->count; ++m) sl[(2 * q + 1) * b->count + m] = bigbits;
    BHIPCHK(b, hipMemcpy(b->slots, sl.data(), sizeof(unsigned long long) * sl.size(), hipMemcpyHostToDevice));
    return bfail(b, FDCGKS_ENONPHYS, "non-physical state in step %d stage %d: member %d grid %d node (%d, %d)",
                 done + 1, b->sc_host->fail_stage, b->sc_host->fail_grid / 2, b->sc_host->fail_grid % 2,
                 b->sc_host->fail_i, b->sc_host->fail_j);
  }
  return FDCGKS_OK;
}

fdcgks_status fdcgks_batch_destroy(fdcgks_batch* b) {
  if (!b) return FDCGKS_OK;
  (void)hipStreamSynchronize(b->stream);
  batch_free(b);
  delete b;
  return FDCGKS_OK;
}

const char* fdcgks_batch_last_error(const fdcgks_batch* b) { return b ? b->err.c_str() : g_create_error; }

fdcgks_status fdcgks_batch_set_mode(fdcgks_batch* b, int32_t mode) {
  if (!b) return bfail(nullptr, FDCGKS_EINVAL, "batch is NULL");
  if (mode != FDCGKS_BATCH_PERSISTENT && mode != FDCGKS_BATCH_PHASED && mode != FDCGKS_BATCH_GRAPH)
    return bfail(b, FDCGKS_EINVAL, "unknown batch mode %d", mode);
  b->mode = mode;
  return FDCGKS_OK;
}

}  // extern "C"
