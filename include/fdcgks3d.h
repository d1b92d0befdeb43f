/* fdcgks3d.h - C ABI of the 3D FD-CGKS solver in libfdcgks.so (gfx950).
 *
 * The paper develops the scheme in 2D and states that the extension to three
 * dimensions is straightforward (Sec. 4, opening paragraph) without giving
 * its grid.  This is the library's reading of that extension:
 *
 *   - Half-spacing lattice: point (I, J, L) at (x0 + I h/2, y0 + J h/2,
 *     z0 + L h/2).  Points with zero or two even coordinates are nodes of four
 *     grids, updated alike: grid 0 = primary P (odd, odd, odd), grid 1 = Dxy
 *     (even, even, odd), grid 2 = Dxz (even, odd, even), grid 3 = Dyz (odd,
 *     even, even), i.e. the primary grid and the three duals offset by half a
 *     mesh along two axes.  Points with one or three even coordinates are
 *     virtual interfaces.
 *   - Every interface point lies on three lines (one per axis, each of a
 *     different grid) and hosts one gas-kinetic solve per axis (App. A with
 *     psi = (1, u, v, w, (u^2+v^2+w^2+xi^2)/2) and K + 3 = 2/(gamma - 1)).
 *     Left/right states and normal derivatives come from the GENO
 *     reconstruction along the solve's own line (Sec. 3, App. C1-C2); the
 *     tangential derivatives are the means of the left and right derivatives
 *     of the two other lines through the point (Sec. 4 item 1(b)).
 *   - The interface values used by the gradient update generalise
 *     Eq. W-model-2d with weight 1/3 per direction:
 *       W~^l = W^^{l,(n)}/3 + (W^^{l,(t1)} + W^^{r,(t1)} + W^^{l,(t2)} + W^^{r,(t2)})/6,
 *     and likewise W~^r and the time derivatives.
 *   - Nodal fluxes come from three-point derivative reconstructions along
 *     x, y, z (App. C3) and the smooth nodal solver; each node is advanced by
 *     the 3D form of Eq. eq-conservation-law-2d with the compact flux of
 *     Eq. fd-conservative-flux (or its order-8 variant) along each axis, and
 *     the S2O4 update of values and averaged gradients (Eqs. eq-nodal-update,
 *     eq-interface-update).
 *
 * All sides are periodic and the gas-kinetic solver runs in FP64.  The GENO
 * reconstruction works on conservative variables or, as in 2D, on the
 * characteristic variables of the Euler flux Jacobian along each line (local
 * frame, eigenvectors at the mean of the two interface-adjacent states or at
 * the node, path function the smallest of the u -+ c fields' left and right
 * values).
 *
 * State layout at the boundary: one grid is 20 contiguous planes of
 * nz*ny*nx doubles, x fastest,
 *   element (f, k, j, i) at  f*nz*ny*nx + (k*ny + j)*nx + i,
 * with planes 0-4 = W = (rho, rho U, rho V, rho W, rho E), 5-9 = Wx, 10-14 =
 * Wy, 15-19 = Wz: the derivatives averaged over the interval between the
 * node's two interfaces along x, y, z (Eq. define-averaged-gradient).
 * Stored node i along an axis sits at lattice coordinate 2i+1 where the grid
 * is odd along that axis and 2i+2 where it is even.
 *
 * Every call returns an fdcgks_status (fdcgks.h); no call aborts.  Pointers
 * passed in are only used during the call.  Data are IEEE binary64.
 */
#ifndef FDCGKS3D_H
#define FDCGKS3D_H

#include <stdint.h>

#include "fdcgks.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdcgks3d_params {
  int32_t nx, ny, nz;     /* nodes per grid along x, y, z; each >= 4; nx*ny*nz <= 2^26 */
  int32_t flux_variant;   /* FDCGKS_FLUX_* (fdcgks.h) */
  int32_t flux_order;     /* 6 (default) or 8, as for 2D problems */
  int32_t grad_update;    /* FDCGKS_GRAD_* */
  int32_t geno_r;         /* GENO exponent r, 1..8 (default 3) */
  int32_t recon_vars;     /* FDCGKS_RECON_* (fdcgks.h): conservative (default) or characteristic, as in 2D */
  double x0, y0, z0;      /* domain origin */
  double lx;              /* x length; h = lx / nx, the y and z lengths are h ny, h nz */
  double gamma;           /* ratio of specific heats, 1 < gamma < 5/3 */
  double mu;              /* dynamic viscosity; 0 = Euler */
  double prandtl;         /* Prandtl number (used when mu > 0) */
  double geno_C, geno_eps, geno_eps_a, geno_d_central, geno_d_side;  /* as in fdcgks_params */
  double tau_c1, tau_c2;  /* Euler collision time, as in fdcgks_params */
} fdcgks3d_params;

typedef struct fdcgks3d_problem fdcgks3d_problem; /* opaque, owned by the library */

/* Defaults: 32^3 on [0,1]^3, gamma 1.4, Euler, (6-4) flux of order 6, the
 * GENO constants of fdcgks_default_params. */
void fdcgks3d_default_params(fdcgks3d_params* p);

/* Validate *p, allocate the device buffers on the current HIP device and bind
 * the problem to hip_stream (NULL = the null stream).  Device memory: 812
 * doubles (6.5 KB) per cell of the nx*ny*nz cells (two state copies, the
 * stage-1 state and accumulators, interface and nodal-flux buffers).  *out is
 * NULL on error (message in fdcgks3d_last_error(NULL)). */
fdcgks_status fdcgks3d_create(const fdcgks3d_params* p, void* hip_stream, fdcgks3d_problem** out);

/* Copy one grid (0..3) in or out: 20 planes of nz*ny*nx doubles (layout
 * above).  on_device = 1: device pointers (EINVAL for anything else),
 * enqueued on the problem's stream; 0: host pointers, synchronous.  Values
 * with rho <= 0, p <= 0 or NaN are accepted and reported by the first step or
 * compute_dt as FDCGKS_ENONPHYS.  get_state before any set_state of that grid:
 * FDCGKS_ESTATE. */
fdcgks_status fdcgks3d_set_state(fdcgks3d_problem* pb, int32_t grid, const double* S, int32_t on_device);
fdcgks_status fdcgks3d_get_state(const fdcgks3d_problem* pb, int32_t grid, double* S, int32_t on_device);

/* CFL time step of the current state: dt = cfl h / max over all nodes of
 * (max(|U|, |V|, |W|) + c); with mu > 0 also dt <= cfl h^2 / (8 mu / rho_min).
 * Synchronous. */
fdcgks_status fdcgks3d_compute_dt(fdcgks3d_problem* pb, double cfl, double* dt_out);

/* Sums of the five conserved components over each grid (out[5 g + c]), then
 * the smallest rho and the smallest pressure over all nodes: 22 doubles.
 * Synchronous; sums in a fixed order. */
fdcgks_status fdcgks3d_diagnostics(fdcgks3d_problem* pb, double* out);

/* Advance up to nsteps S2O4 steps (dt > 0 fixed, dt <= 0 the CFL step of
 * each step's start state; t_end > 0 clips the last step and stops there).
 * EINVAL for non-finite dt, t or t_end, nsteps < 0, or dt <= 0 without
 * cfl > 0; ESTATE until all four grids have a state.
 * Each step synchronises the stream once to check it: on FDCGKS_ENONPHYS
 * (rho <= 0, p <= 0 or NaN at some node) the state is the one after the last
 * good step and *t_inout, *steps_done describe it. */
fdcgks_status fdcgks3d_step(fdcgks3d_problem* pb, double dt, double cfl, int32_t nsteps, double t_end,
                            double* t_inout, int32_t* steps_done);

/* fdcgks3d_step with per-kernel device times (HIP events on the problem's
 * stream): kernel_ms[7] = interface sweep, node sweep, update of stage 1;
 * the same three of stage 2; step bookkeeping (CFL reduction and the
 * non-physical check). */
fdcgks_status fdcgks3d_step_timed(fdcgks3d_problem* pb, double dt, double cfl, int32_t nsteps, double t_end,
                                  double* t_inout, int32_t* steps_done, double* kernel_ms);

/* One stage without committing it: stage 1 from the current state, stage 2
 * from the stage-1 buffers left by the previous stage-1 call (same dt).
 * Host outputs: out_state[4][20][nz][ny][nx], out_acc (stage 1, may be NULL)
 * the accumulators W + dt L + dt^2/6 L_t and the base gradients. */
fdcgks_status fdcgks3d_debug_stage(fdcgks3d_problem* pb, int32_t stage, double dt, double* out_state,
                                   double* out_acc);

/* Stage-1 intermediates at step dt from the current state.  Host outputs:
 *   edges[4][3][31][nz][ny][nx]: interface classes q = 0..3 = (even, odd,
 *     odd), (odd, even, odd), (odd, odd, even), (even, even, even), cell
 *     (i, j, k) at the lattice point with coordinate 2i+2 where even and 2i+1
 *     where odd; per normal axis: F[5], F_t[5], chi (path function of rho,
 *     min of left/right), blended values W~l[5], W~r[5], W~l_t[5], W~r_t[5];
 *   nodes[4][30][nz][ny][nx]: per grid the x-, y-, z-fluxes F[5], F_t[5]. */
fdcgks_status fdcgks3d_debug_intermediates(fdcgks3d_problem* pb, double dt, double* edges, double* nodes);

/* Free the problem's device memory.  NULL is accepted. */
fdcgks_status fdcgks3d_destroy(fdcgks3d_problem* pb);

/* Message of the last failed call on pb (pb = NULL: of the last failed
 * create).  Valid until the next call on the same problem. */
const char* fdcgks3d_last_error(const fdcgks3d_problem* pb);

#ifdef __cplusplus
}
#endif

#endif /* FDCGKS3D_H */
