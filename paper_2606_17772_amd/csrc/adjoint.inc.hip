// Adjoint of one S2O4 step (vector-Jacobian product at a frozen time step).
// Included by fdcgks.hip after the forward kernels, whose layouts it uses.
//
// Reverse of a stage, for every node and interface point:
//   update^T     lambda of the stage outputs -> lambda of L, L_t, the averaged
//                gradients and their time derivatives (and direct terms);
//   assembly^T   -> lambda of the interface fluxes, path functions, blended
//                interface values and nodal fluxes (compact flux of
//                Eq. fd-conservative-flux with the (6-4)/(6-2) blend; Gauss
//                gradients of Eq. define-averaged-gradient);
//   blend^T      -> lambda of the interface values of each direction
//                (Eq. W-model-2d);
//   solver^T     local Jacobian-transpose products of the gas-kinetic
//                interface and nodal solvers;
//   GENO^T       of the line and nodal reconstructions, scattered to the
//                nodes they read (atomic adds), then the periodic halo is
//                folded back onto its images.
// The local transposes of the two nonlinear pointwise maps (gas-kinetic
// solvers, GENO reconstructions) are the reverse-mode routines of
// gks_adjoint.hpp.  min/max ties take the first argument and d|x|/dx = 0 at 0.

namespace {

// Planes of the per-node operator adjoint: L[4], Lt[4], Gx[4], Gy[4],
// Gxt[4], Gyt[4] per grid.
constexpr int OPN = 24;

// The reverse sweeps' tiles in XCD bands, as the forward sweeps': a 1D
// launch over gx * gy * gz tiles (rounded up to a multiple of 8); tile
// (bx, by, bz), bz slowest; false for the padding ids.
struct Tiles3 {
  int gx, gy, gz;
};
__device__ __forceinline__ bool xcd_tile3(const Tiles3& t, int& bx, int& by, int& bz) {
  int tile;
  if (!xcd_tile(blockIdx.x, gridDim.x, t.gx * t.gy * t.gz, tile)) return false;
  bx = tile % t.gx;
  by = (tile / t.gx) % t.gy;
  bz = tile / (t.gx * t.gy);
  return true;
}

// ---------------------------------------------------------- update^T
// lam_out: adjoint of the stage output state (24 planes); lam_acc: adjoint
// of the stage-1 accumulators (stage 1 only).  Writes lam_op (interior) and
// the direct terms: stage 1 -> lam_in (W planes, and the gradient planes
// when the stored gradient is carried); stage 2 -> lam_acc_out (copy).
template <int STAGE>
__global__ __launch_bounds__(256) void k_adj_update(const double* __restrict__ lam_out,
                                                    const double* __restrict__ lam_acc, double* __restrict__ lam_op,
                                                    double* __restrict__ lam_direct, Geo g, Consts k, double dt, Tiles3 tl) {
  int bx, by, bz;
  if (!xcd_tile3(tl, bx, by, bz)) return;  // block-uniform
  const int grid = bz;
  // the nodes the forward update writes: the dual grid starts at -sx, -sy
  const int i = bx * 64 + threadIdx.x - (grid ? g.sx : 0);
  const int j = by * 4 + threadIdx.y - (grid ? g.sy : 0);
  if (i >= g.nx || j >= g.ny) return;
  const long pl = g.plane, o = at(g, j, i), so = o + (grid ? g.dshift : 0);  // state planes: shifted dual
  const double* lo = lam_out + (long)grid * 12 * pl + so;
  double* op = lam_op + (long)grid * OPN * pl + o;
  double* dir = lam_direct + (long)grid * 12 * pl + so;
  // outputs the wall condition sets to zero depend on nothing
  const int zero = wall_mask(g, grid, i, j);
  for (int c = 0; c < 4; ++c) {
    const double lW = zero & (1 << c) ? 0.0 : lo[c * pl];
    const double lX = zero & (1 << (4 + c)) ? 0.0 : lo[(4 + c) * pl];
    const double lY = zero & (1 << (8 + c)) ? 0.0 : lo[(8 + c) * pl];
    if (STAGE == 2) {
      dir[c * pl] = lW;  // acc_W
      dir[(4 + c) * pl] = lX;
      dir[(8 + c) * pl] = lY;
      op[c * pl] = 0.0;
      op[(4 + c) * pl] = dt * dt / 3.0 * lW;
      op[(8 + c) * pl] = 0.0;
      op[(12 + c) * pl] = 0.0;
      op[(16 + c) * pl] = dt * lX;
      op[(20 + c) * pl] = dt * lY;
    } else {
      const double* la = lam_acc + (long)grid * 12 * pl + so;
      const double aW = la[c * pl], aX = la[(4 + c) * pl], aY = la[(8 + c) * pl];
      dir[c * pl] = lW + aW;
      op[c * pl] = 0.5 * dt * lW + dt * aW;
      op[(4 + c) * pl] = 0.125 * dt * dt * lW + dt * dt / 6.0 * aW;
      op[(16 + c) * pl] = 0.5 * dt * lX;
      op[(20 + c) * pl] = 0.5 * dt * lY;
      if (k.grad_carried) {
        dir[(4 + c) * pl] = lX + aX;
        dir[(8 + c) * pl] = lY + aY;
        op[(8 + c) * pl] = 0.0;
        op[(12 + c) * pl] = 0.0;
      } else {
        dir[(4 + c) * pl] = 0.0;
        dir[(8 + c) * pl] = 0.0;
        op[(8 + c) * pl] = lX + aX;
        op[(12 + c) * pl] = lY + aY;
      }
    }
  }
}

// Partial derivatives of the compact flux CF(Fm, Fc, Fp, [Nm,] N0, N1, [Np2,]
// chi) of order 6 (Eq. fd-conservative-flux) or 8 (wide = true: the nodal
// fluxes Nm, Np2 one node further out), with the (6-4)/(6-2) blend.
struct CFd {
  double dm, dc, dp, dn, dw;  // dn: N0 and N1; dw: Nm and Np2 (order 8)
};
__device__ __forceinline__ CFd cf_partials(int variant, double chi, bool wide) {
  // the linear flux Fbar = (a (Fm + Fp) + b Fc + c (N0 + N1) + e (Nm + Np2)) / den
  const double den = wide ? 420.0 : 30.0, a = wide ? 32.0 : 1.0, b = wide ? 704.0 : 46.0;
  const double c = wide ? -171.0 : -9.0, e = wide ? -3.0 : 0.0;
  const double x = variant == 2 ? 1.0 : chi;  // the linear variant is Fbar itself
  const double clo = variant == 1 ? 1.0 : 8.0 / 6.0, nlo = variant == 1 ? 0.0 : -1.0 / 6.0;
  CFd d;
  d.dm = d.dp = x * a / den;
  d.dc = (1.0 - x) * clo + x * b / den;
  d.dn = (1.0 - x) * nlo + x * c / den;
  d.dw = x * e / den;
  return d;
}
// d CF / d chi = Fbar - lo (0 for the linear variant).
__device__ __forceinline__ double cf_dchi(int variant, double Fm, double Fc, double Fp, double Nm, double N0,
                                          double N1, double Np2, bool wide) {
  if (variant == 2) return 0.0;
  const double Fb = wide ? ((32.0 * (Fm + Fp) + 704.0 * Fc) - 171.0 * (N0 + N1) - 3.0 * (Nm + Np2)) * (1.0 / 420.0)
                         : ((Fm + 46.0 * Fc + Fp) - 9.0 * (N0 + N1)) * (1.0 / 30.0);
  const double lo = variant == 1 ? Fc : (8.0 * Fc - N0 - N1) * (1.0 / 6.0);
  return Fb - lo;
}

// ---------------------------------------------------------- assembly^T
// One thread per (interface point, slot) over the forward interface ranges:
// lambda of F, Ft, chi, Wl, Wr, Wlt, Wrt of the slot (25 planes, like E).
// The slot's grid is G = slot; its axis is y when fam != G; the interface's
// left / right nodes (along the axis, grid G) sit at offsets -G and 1-G.
template <int STAGE>
__global__ __launch_bounds__(256) void k_adj_assemble(const double* __restrict__ lam_op, const double* __restrict__ E,
                                                      const double* __restrict__ Nb, double* __restrict__ lamE, Geo g,
                                                      Consts k, Tiles3 tl) {
  int bx, by, bz;
  if (!xcd_tile3(tl, bx, by, bz)) return;  // block-uniform
  const int fam = bz >> 1, G = bz & 1;
  const int i = bx * 64 + threadIdx.x + (fam == 0 ? -2 : -1 - g.sx);
  const int j = by * 4 + threadIdx.y + (fam == 0 ? -1 - g.sy : -2);
  if (i > (fam == 0 ? g.nx : g.nx + 1) || j > (fam == 0 ? g.ny + 1 : g.ny)) return;
  const bool ay = (fam ^ G) != 0;
  const long pl = g.plane, st = ay ? g.pitch : 1, o = at(g, j, i);
  const double* e = E + ((long)fam * 50 + G * 25) * pl + o;
  const double* op = lam_op + (long)G * OPN * pl + o;            // node planes, indexed at this interface
  const double* nf = Nb + (long)G * 16 * pl + (ay ? 8 : 0) * pl + o;
  double* le = lamE + ((long)fam * 50 + G * 25) * pl + o;
  const long nL = -(long)G * st, nR = (long)(1 - G) * st;         // node offsets of interface e
  const int gop = ay ? 12 : 8, gopt = ay ? 20 : 16;               // gradient planes of this axis in lam_op
  const bool wide = k.flux_order == 8;
  double lchi = 0.0;
  for (int c = 0; c < 4; ++c) {
    for (int tpart = (STAGE == 1 ? 0 : 1); tpart < 2; ++tpart) {
      const double* f = e + (tpart * 4 + c) * pl;
      const double* n = nf + (tpart * 4 + c) * pl;
      const double* lL = op + (tpart * 4 + c) * pl;
      double lF = 0.0;
      // interfaces e' = e - st, e, e + st; lambda of CF(e') = (lam L(right node) - lam L(left node)) / h
      for (int q = -1; q <= 1; ++q) {
        const long eo = q * st;
        const double lcf = (lL[eo + nR] - lL[eo + nL]) * g.invh;
        const double chi = e[8 * pl + eo];
        const CFd d = cf_partials(k.variant, chi, wide);
        lF += (q == -1 ? d.dp : (q == 0 ? d.dc : d.dm)) * lcf;
        // interfaces next to no updated node have lcf = 0, and their outer nodal fluxes are not computed
        if (q == 0 && lcf != 0.0)
          lchi += cf_dchi(k.variant, f[-st], f[0], f[st], wide ? n[nL - st] : 0.0, n[nL], n[nR],
                          wide ? n[nR + st] : 0.0, wide) * lcf;
      }
      le[(tpart * 4 + c) * pl] = lF;
    }
    // gradients: G(left node) uses Wl(e), G(right node) uses -Wr(e)
    if (STAGE == 1) {
      le[(9 + c) * pl] = op[(gop + c) * pl + nL] * g.invh;
      le[(13 + c) * pl] = -op[(gop + c) * pl + nR] * g.invh;
    } else {
      le[c * pl] = 0.0;
      le[(9 + c) * pl] = 0.0;
      le[(13 + c) * pl] = 0.0;
    }
    le[(17 + c) * pl] = op[(gopt + c) * pl + nL] * g.invh;
    le[(21 + c) * pl] = -op[(gopt + c) * pl + nR] * g.invh;
  }
  le[8 * pl] = lchi;
}

// Lambda of the nodal fluxes: node n is the left node (N0) of its right
// interface e_R = n + G st and the right node (N1) of e_L = e_R - st; with
// the order-8 flux also Nm of e_R + st and Np2 of e_L - st.  Nodes i, j in
// [-w, n - 1 + w] (w = node reach; the dual grid's range starts one node
// lower along a bounded axis): the nodes whose fluxes the forward sweep
// computes.  Only interfaces next to an updated node carry a flux adjoint.
template <int STAGE>
__global__ __launch_bounds__(256) void k_adj_nodeflux(const double* __restrict__ lam_op, const double* __restrict__ E,
                                                      double* __restrict__ lamN, Geo g, Consts k, Tiles3 tl) {
  int bx, by, bz;
  if (!xcd_tile3(tl, bx, by, bz)) return;  // block-uniform
  const int G = bz, w = node_reach(k);
  const bool wide = w == 2;
  const int sx = G ? g.sx : 0, sy = G ? g.sy : 0;  // the dual grid starts at -sx, -sy
  const int i = bx * 64 + threadIdx.x - w - sx, j = by * 4 + threadIdx.y - w - sy;
  if (i > g.nx - 1 + w || j > g.ny - 1 + w) return;
  const long pl = g.plane, o = at(g, j, i);
  const double* op = lam_op + (long)G * OPN * pl + o;
  double* ln = lamN + (long)G * 16 * pl + o;
  for (int a = 0; a < 2; ++a) {
    const int fam = (G == 0) ? a : 1 - a;
    const long st = a == 0 ? 1 : g.pitch;
    // node index along the axis; the grid's updated nodes along it are [lo, nn - 1]
    const int idx = a == 0 ? i : j, nn = a == 0 ? g.nx : g.ny, lo = a == 0 ? -sx : -sy;
    const double* e = E + ((long)fam * 50 + G * 25) * pl + o;
    const long eR = (long)G * st, eL = eR - st;
    // interface between nodes idx + m and idx + m + 1 (m = -2..1): at e offset eR + m st; it has an updated
    // node when idx + m + 1 >= lo and idx + m <= nn - 1
    auto has = [&](int m) { return idx + m + 1 >= lo && idx + m <= nn - 1; };
    const CFd dR = has(0) ? cf_partials(k.variant, e[8 * pl + eR], wide) : CFd{0, 0, 0, 0, 0};
    const CFd dL = has(-1) ? cf_partials(k.variant, e[8 * pl + eL], wide) : CFd{0, 0, 0, 0, 0};
    const CFd dR2 = wide && has(1) ? cf_partials(k.variant, e[8 * pl + eR + st], wide) : CFd{0, 0, 0, 0, 0};
    const CFd dL2 = wide && has(-2) ? cf_partials(k.variant, e[8 * pl + eL - st], wide) : CFd{0, 0, 0, 0, 0};
    for (int c = 0; c < 4; ++c)
      for (int tpart = (STAGE == 1 ? 0 : 1); tpart < 2; ++tpart) {
        const double* lL = op + (tpart * 4 + c) * pl;
        // lambda of CF at the interface between nodes idx + m and idx + m + 1
        auto lcf = [&](int m) { return has(m) ? (lL[(m + 1) * st] - lL[m * st]) * g.invh : 0.0; };
        double v = dR.dn * lcf(0) + dL.dn * lcf(-1);
        if (wide) v += dR2.dw * lcf(1) + dL2.dw * lcf(-2);
        ln[(a * 8 + tpart * 4 + c) * pl] = v;
      }
    if (STAGE == 2)
      for (int c = 0; c < 4; ++c) ln[(a * 8 + c) * pl] = 0.0;
  }
}

// ------------------------------------------------------- solver^T, GENO^T
// GENO^T of one line: lam of (vl, dl, cl, vr, dr, cr) per component ->
// scatter onto the line's nodes (W plane and derivative plane).  fam and G
// are runtime values (wave-uniform): one copy of the code serves all lines.
// CHAR: the line was reconstructed on characteristic variables in its local
// frame (edge_recon<true>); lv's cl, cr entries are unused and chib is the
// adjoint of the line's single path function.
template <bool CHAR>
__device__ __forceinline__ void line_adjoint(const double* __restrict__ S, double* __restrict__ lamS, const Geo& g,
                                             const Consts& k, int i, int j, int fam, int G,
                                             const double (&lv)[4][6], double chib) {
  const bool ALONG_Y = (fam ^ G) != 0;
  const int back = G == 0 ? 1 : 2;
  const long st = ALONG_Y ? g.pitch : 1;
  const long o = (ALONG_Y ? at(g, j - back, i) : at(g, j, i - back)) + (G ? g.dshift : 0);  // shifted dual planes
  const int f = ALONG_Y ? 2 : 1;
  const long pl = g.plane;
  if constexpr (CHAR) {
    // local component c holds global component q (rho U and rho V trade places along y), as in edge_recon
    double Q[4][4], X[4][4], rb[4][4], Qb[4][4], Xb[4][4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int q = ALONG_Y ? (c == 1 ? 2 : (c == 2 ? 1 : c)) : c;
      const double* w = S + (G * 12 + q) * pl + o;
      const double* x = S + (G * 12 + f * 4 + q) * pl + o;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        Q[c][m] = w[m * st];
        X[c][m] = x[m * st];
        Qb[c][m] = Xb[c][m] = 0.0;
      }
      rb[c][0] = lv[q][0];
      rb[c][1] = lv[q][1];
      rb[c][2] = lv[q][3];
      rb[c][3] = lv[q][4];
    }
    fdk::recon_iface_char_b(k, Q, X, g.h, g.invh, rb, chib, Qb, Xb);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int q = ALONG_Y ? (c == 1 ? 2 : (c == 2 ? 1 : c)) : c;
      double* lw = lamS + (G * 12 + q) * pl + o;
      double* lx = lamS + (G * 12 + f * 4 + q) * pl + o;
      for (int m = 0; m < 4; ++m) {
        if (Qb[c][m] != 0.0) atomicAdd(lw + m * st, Qb[c][m]);
        if (Xb[c][m] != 0.0) atomicAdd(lx + m * st, Xb[c][m]);
      }
    }
    return;
  }
  for (int c = 0; c < 4; ++c) {
    const double* w = S + (G * 12 + c) * pl + o;
    const double* x = S + (G * 12 + f * 4 + c) * pl + o;
    const double q[4] = {w[0], w[st], w[2 * st], w[3 * st]};
    const double xv[4] = {x[0], x[st], x[2 * st], x[3 * st]};
    double qb[4] = {0, 0, 0, 0}, xb[4] = {0, 0, 0, 0};
    fdk::recon_iface_b(k, q, xv, g.h, g.invh, lv[c], qb, xb);
    double* lw = lamS + (G * 12 + c) * pl + o;
    double* lx = lamS + (G * 12 + f * 4 + c) * pl + o;
    for (int m = 0; m < 4; ++m) {
      if (qb[m] != 0.0) atomicAdd(lw + m * st, qb[m]);
      if (xb[m] != 0.0) atomicAdd(lx + m * st, xb[m]);
    }
  }
}

// Reverse of the interface sweep: same thread layout as the forward sweep
// (two threads per point, partners in neighbouring waves).  The adjoint of a
// solve runs in phases (see gks_iface_b) whose largest needs about 380
// registers; the solve's inputs, their adjoint accumulators, the moment
// adjoints and the time-coefficient adjoints live in LDS (155 KB per block:
// one block of four waves per CU, one wave per SIMD), so that only a few
// values spill.
// The normal along y (fam != G) swaps rho U and rho V in the local frame:
// the swap is applied to the data, so one copy of the solver adjoint serves
// both normals.
template <int STAGE, bool CHAR>
__global__ __launch_bounds__(256, 1) void k_adj_edges(const double* __restrict__ S, const double* __restrict__ lamE,
                                                      double* __restrict__ lamS, Geo g, Consts k, double dt, Tiles3 tl) {
  __shared__ double xch[4][4][64];
  __shared__ fdk::SolveIO s_in[256], s_inb[256];
  __shared__ fdk::AccB s_ab[256];
  int bx, by, bz;
  if (!xcd_tile3(tl, bx, by, bz)) return;  // block-uniform
  const int fam = bz;
  const int tx = threadIdx.x, ty = threadIdx.y, G = ty & 1, tid = ty * 64 + tx;
  const int i = bx * 64 + tx + (fam == 0 ? -2 : -1 - g.sx);
  const int j = by * 2 + (ty >> 1) + (fam == 0 ? -1 - g.sy : -2);
  const bool valid = i <= (fam == 0 ? g.nx : g.nx + 1) && j <= (fam == 0 ? g.ny + 1 : g.ny);
  const bool swap = fam != G;
  fdk::SolveIO& in = s_in[tid];
  fdk::SolveIO& inb = s_inb[tid];
  bool chi_right = false;  // chi = min(chi_l, chi_r) of the density line took chi_r (ties: left)
  {
    fdk::IfaceRec rec[4];
    if (valid) {
      edge_recon<CHAR>(S, g, k, i, j, fam, G, rec);
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c) rec[c] = fdk::IfaceRec{1.0, 0.0, 1.0, 1.0, 0.0, 1.0};
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) xch[ty][c][tx] = 0.5 * (rec[c].dl + rec[c].dr);
    __syncthreads();
    // solve inputs in the local frame (global component of local slot c: q0 when swapped)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int q0 = c == 1 ? 2 : (c == 2 ? 1 : c);
      const int q = swap ? q0 : c;
      in.WL[c] = rec[q].vl;
      in.WR[c] = rec[q].vr;
      in.nL[c] = rec[q].dl;
      in.nR[c] = rec[q].dr;
      in.Wt[c] = xch[ty ^ 1][q][tx];
      inb.WL[c] = inb.WR[c] = inb.nL[c] = inb.nR[c] = inb.Wt[c] = 0.0;
    }
    chi_right = rec[0].cr < rec[0].cl;
  }
  __syncthreads();
  double lchi = 0.0;
  if (valid) {
    const long pl = g.plane, o = at(g, j, i);
    const double* le0 = lamE + ((long)fam * 50 + G * 25) * pl + o;
    const double* lp0 = lamE + ((long)fam * 50 + (1 - G) * 25) * pl + o;  // partner slot
    // output adjoints, read inside the solver adjoint's first phase (the
    // addresses are formed there too: hoisted out of its phase loop they
    // would hold 32 registers through every phase)
    auto obload = [&](fdk::GksIO<double, 2>& ob) {
      const double* le = fdk::opaque_ptr(le0);
      const double* lp = fdk::opaque_ptr(lp0);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        // blend^T: W~(own) = W^/2 + (partner W^l + W^r)/4 and W~(partner) = W^p/2 + (own W^l + W^r)/4
        const int q0 = c == 1 ? 2 : (c == 2 ? 1 : c);
        const int q = swap ? q0 : c;
        const double ps = lp[(9 + q) * pl] + lp[(13 + q) * pl], pst = lp[(17 + q) * pl] + lp[(21 + q) * pl];
        ob.Ft[c] = le[(4 + q) * pl];
        ob.Wlt[c] = 0.5 * le[(17 + q) * pl] + 0.25 * pst;
        ob.Wrt[c] = 0.5 * le[(21 + q) * pl] + 0.25 * pst;
        ob.F[c] = STAGE == 1 ? le[q * pl] : 0.0;
        ob.Wl[c] = STAGE == 1 ? 0.5 * le[(9 + q) * pl] + 0.25 * ps : 0.0;
        ob.Wr[c] = STAGE == 1 ? 0.5 * le[(13 + q) * pl] + 0.25 * ps : 0.0;
      }
    };
    lchi = le0[8 * pl];
    fdk::gks_iface_b(k, dt, in, obload, inb, s_ab[tid]);
  }
  // the tangential slope of this solve came from the partner line: send its lambda
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int q0 = c == 1 ? 2 : (c == 2 ? 1 : c);
    xch[ty][c][tx] = swap && q0 != c ? inb.Wt[q0] : inb.Wt[c];  // global component c
  }
  __syncthreads();
  if (valid) {
    double lv[4][6];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int q0 = c == 1 ? 2 : (c == 2 ? 1 : c);
      const int q = swap ? q0 : c;  // local slot of global component c
      const double lt = 0.5 * xch[ty ^ 1][c][tx];  // partner's tangential slope = mean of my dl, dr
      lv[c][0] = inb.WL[q];
      lv[c][1] = inb.nL[q] + lt;
      lv[c][2] = 0.0;
      lv[c][3] = inb.WR[q];
      lv[c][4] = inb.nR[q] + lt;
      lv[c][5] = 0.0;
    }
    if (!CHAR) {
      if (chi_right) lv[0][5] = lchi; else lv[0][2] = lchi;
    }
    line_adjoint<CHAR>(S, lamS, g, k, i, j, fam, G, lv, CHAR ? lchi : 0.0);
  }
}

// Reverse of the node sweep: lambda of the nodal fluxes -> lambda of the
// node's W and of the 3-point lines its derivative reconstructions read.
// Block 64 x 4 nodes, one wave per row.  A node's reverse adds to 12 planes
// of itself and to 8 planes of each neighbour along x and y (W and that
// axis's derivative plane).  Each thread parks its contributions in LDS
// slots of its own as they are produced; after a barrier every node sums
// what it received from the adjacent lanes and rows of the block and adds
// the 12 sums atomically (neighbouring blocks add to the same nodes), and
// only contributions that leave the block go out one by one.
template <int STAGE, bool CHAR>
__global__ __launch_bounds__(256) void k_adj_nodes(const double* __restrict__ S, const double* __restrict__ lamN,
                                                   double* __restrict__ lamS, Geo g, Consts k, Tiles3 tl) {
  // [slot][thread]: own[p] = plane p of this node; to_xm / to_xp / to_ym / to_yp [s] = the node at i -/+ 1 or
  // j -/+ 1, plane s for s < 4 (W), else the axis's derivative plane (4 + s along x, 8 + (s - 4) along y)
  __shared__ double own[12][256], to_xm[8][256], to_xp[8][256], to_ym[8][256], to_yp[8][256];
  int bx, by, bz;
  if (!xcd_tile3(tl, bx, by, bz)) return;  // block-uniform
  const int grid = bz, w = node_reach(k), tx = threadIdx.x, ty = threadIdx.y, t = ty * 64 + tx;
  const int i = bx * 64 + tx - w - (grid ? g.sx : 0);
  const int j = by * 4 + ty - w - (grid ? g.sy : 0);
  for (int p = 0; p < 12; ++p) own[p][t] = 0.0;
  for (int s8 = 0; s8 < 8; ++s8) { to_xm[s8][t] = 0.0; to_xp[s8][t] = 0.0; to_ym[s8][t] = 0.0; to_yp[s8][t] = 0.0; }
  const long pl = g.plane, o = at(g, j, i);
  const long ds = grid ? g.dshift : 0;  // state planes: shifted dual
  // the nodes whose fluxes the forward sweep computed; the rest of the block
  // only collects what its neighbours hand over
  if (i <= g.nx - 1 + w && j <= g.ny - 1 + w) {
    const double* B = S + (long)grid * 12 * pl + ds;
    const double* ln = lamN + (long)grid * 16 * pl + o;
    double W[4], Wx[4], Wy[4];
    for (int c = 0; c < 4; ++c) W[c] = B[c * pl + o];
    node_derivs<CHAR, double>(B, g, k, o, Wx, Wy);
    double lF[4], lFt[4], lG[4], lGt[4];
    for (int c = 0; c < 4; ++c) {
      lF[c] = ln[c * pl];
      lFt[c] = ln[(4 + c) * pl];
      lG[c] = ln[(8 + c) * pl];
      lGt[c] = ln[(12 + c) * pl];
    }
    // nodal solver^T (stage 2 has no F, G outputs)
    double Wb[4] = {0, 0, 0, 0}, Wxb[4] = {0, 0, 0, 0}, Wyb[4] = {0, 0, 0, 0};
    if (STAGE == 2)
      for (int c = 0; c < 4; ++c) { lF[c] = 0.0; lG[c] = 0.0; }
    fdk::gks_node_b(k, W, Wx, Wy, lF, lFt, lG, lGt, Wb, Wxb, Wyb);
#pragma unroll
    for (int c = 0; c < 4; ++c) own[c][t] += Wb[c];
    // the 3-point line of axis a, component q: adjoints of W (qb) and of the axis's derivative plane (xb) at
    // offsets -1, 0, +1
    auto park = [&](int a, int q, const double* qb, const double* xb) {
      own[q][t] += qb[1];
      own[(a + 1) * 4 + q][t] += xb[1];
      if (a == 0) {
        to_xm[q][t] = qb[0]; to_xm[4 + q][t] = xb[0]; to_xp[q][t] = qb[2]; to_xp[4 + q][t] = xb[2];
      } else {
        to_ym[q][t] = qb[0]; to_ym[4 + q][t] = xb[0]; to_yp[q][t] = qb[2]; to_yp[4 + q][t] = xb[2];
      }
    };
    if constexpr (CHAR) {
      // derivative reconstructions along x and y on characteristic variables (local frame of each axis: rho U
      // and rho V trade places along y, as in node_derivs)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const long st = a == 0 ? 1 : g.pitch;
        double Q[4][3], X[4][3], db[4], Qb[4][3], Xb[4][3];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int q = a == 1 ? (c == 1 ? 2 : (c == 2 ? 1 : c)) : c;
          const double* wp = B + q * pl + o;
          const double* xq = B + ((a + 1) * 4 + q) * pl + o;
#pragma unroll
          for (int m = 0; m < 3; ++m) {
            Q[c][m] = wp[(m - 1) * st];
            X[c][m] = xq[(m - 1) * st];
            Qb[c][m] = Xb[c][m] = 0.0;
          }
          db[c] = a == 0 ? Wxb[q] : Wyb[q];
        }
        fdk::recon_node_char_b(k, Q, X, g.h, g.invh, db, Qb, Xb);
#pragma unroll
        for (int c = 0; c < 4; ++c) park(a, a == 1 ? (c == 1 ? 2 : (c == 2 ? 1 : c)) : c, Qb[c], Xb[c]);
      }
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          // derivative reconstructions along x and y
          const double la = a == 0 ? Wxb[c] : Wyb[c];
          if (la == 0.0) continue;
          const long st = a == 0 ? 1 : g.pitch;
          const double* wp = B + c * pl + o;
          const double* xq = B + ((a + 1) * 4 + c) * pl + o;
          const double q[3] = {wp[-st], wp[0], wp[st]}, xv[3] = {xq[-st], xq[0], xq[st]};
          double qb[3] = {0, 0, 0}, xb[3] = {0, 0, 0};
          fdk::recon_node_b(k, q, xv, g.h, g.invh, la, qb, xb);
          park(a, c, qb, xb);
        }
    }
  }
  __syncthreads();
  double* lS = lamS + (long)grid * 12 * pl + ds + o;
  // contributions that leave the block
  for (int s8 = 0; s8 < 8; ++s8) {
    const int py = s8 < 4 ? s8 : s8 + 4;
    double v;
    if (tx == 0 && (v = to_xm[s8][t]) != 0.0) atomicAdd(lS + s8 * pl - 1, v);
    if (tx == 63 && (v = to_xp[s8][t]) != 0.0) atomicAdd(lS + s8 * pl + 1, v);
    if (ty == 0 && (v = to_ym[s8][t]) != 0.0) atomicAdd(lS + py * pl - g.pitch, v);
    if (ty == 3 && (v = to_yp[s8][t]) != 0.0) atomicAdd(lS + py * pl + g.pitch, v);
  }
  // this node's sums (nodes beyond the computed range hold what a computed neighbour handed over, or nothing)
  if (i > g.nx + w || j > g.ny + w) return;
  for (int p = 0; p < 12; ++p) {
    double v = own[p][t];
    if (p < 8) {
      if (tx > 0) v += to_xp[p][t - 1];
      if (tx < 63) v += to_xm[p][t + 1];
    }
    if (p < 4 || p >= 8) {
      const int s8 = p < 4 ? p : p - 4;
      if (ty > 0) v += to_yp[s8][t - 64];
      if (ty < 3) v += to_ym[s8][t + 64];
    }
    if (v != 0.0) atomicAdd(lS + p * pl, v);
  }
}

// Transpose of the halo fill (k_halo_rows, then k_halo_cols): a ghost value
// fac * P[src] hands its adjoint to its source, columns first (their ghost
// rows included), then rows.  Stored node coordinates, as the state planes.
__global__ void k_adj_fold_cols(double* __restrict__ L, int nplanes, Geo g) {
  const int rows = g.ny + g.sy + 2 * HALO;
  const long n = (long)nplanes * rows * 2 * HALO;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    const int hc = (int)(t % (2 * HALO));
    const long r = t / (2 * HALO);
    const int j = (int)(r % rows) - HALO;
    const int p = (int)(r / rows);
    const PlaneInfo q = plane_info(g, p);
    if (j >= q.my + HALO) continue;
    const int i = hc < HALO ? hc - HALO : q.mx + (hc - HALO);
    double fac;
    const int is = ghost_src(i, q.mx, g.side[0], g.side[1], q.dual && g.sx, q.field == 1, q.comp == 1,
                             q.comp == 1 || q.comp == 2, fac);
    double* P = L + p * g.plane;
    const double v = fac * P[at(g, j, i)];
    if (v != 0.0) atomicAdd(&P[at(g, j, is)], v);
    P[at(g, j, i)] = 0.0;
  }
}
__global__ void k_adj_fold_rows(double* __restrict__ L, int nplanes, Geo g) {
  const int W = g.nx + g.sx;
  const long n = (long)nplanes * 2 * HALO * W;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    const int i = (int)(t % W);
    const long r = t / W;
    const int hr = (int)(r % (2 * HALO));
    const int p = (int)(r / (2 * HALO));
    const PlaneInfo q = plane_info(g, p);
    if (i >= q.mx) continue;
    const int j = hr < HALO ? hr - HALO : q.my + (hr - HALO);
    double fac;
    const int js = ghost_src(j, q.my, g.side[2], g.side[3], q.dual && g.sy, q.field == 2, q.comp == 2,
                             q.comp == 1 || q.comp == 2, fac);
    double* P = L + p * g.plane;
    const double v = fac * P[at(g, j, i)];
    if (v != 0.0) atomicAdd(&P[at(g, js, i)], v);
    P[at(g, j, i)] = 0.0;
  }
}

}  // namespace
