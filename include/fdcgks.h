/* fdcgks.h - C ABI of the MI355X (gfx950) FD-CGKS library (libfdcgks.so).
 *
 * The library advances the compressible Euler / Navier-Stokes equations with
 * the finite-difference compact gas-kinetic scheme of Zhao, Chen & Xu,
 * "Finite difference implementation of a high-order space-time coupled compact
 * gas-kinetic scheme":
 *   - conservative compact finite differences, Eq. (fd-conservative-form) and
 *     (eq-conservation-law-2d), with the compact numerical flux of
 *     Eq. (fd-conservative-flux) and its nonlinear (6-4) / (6-2) forms,
 *     Eqs. (fd-conservative-flux-2) / (fd-conservative-flux-1);
 *   - nodal values and interval-averaged derivatives evolved on a primary
 *     grid and a dual grid offset by half a mesh size (Sec. 4);
 *   - compact GENO reconstruction at virtual interfaces and nodes (Sec. 3,
 *     App. C, App. D);
 *   - the space-time coupled BGK gas-kinetic interface and nodal solver
 *     (App. A), giving fluxes, their time derivatives and time-accurate
 *     interface values;
 *   - the two-stage fourth-order (S2O4) update of values and averaged
 *     gradients, Eqs. (eq-nodal-update) and (eq-interface-update).
 *
 * Every call returns an fdcgks_status; no call aborts the process.  Pointers
 * passed in are only read or written during the call (the library keeps no
 * reference to caller memory).  All floating-point data are IEEE binary64.
 *
 * State layout at the boundary.  For one grid, W, Wx, Wy are each
 * ncomp contiguous planes of ny*nx doubles, x fastest:
 *   element (c, j, i) at  c*ny*nx + j*nx + i,
 * with ncomp = 4 in 2D (rho, rho U, rho V, rho E) and 3 in 1D (rho, rho U,
 * rho E).  Wx (Wy) holds the derivative averaged over the interval between
 * the node's two x (y) interfaces, i.e. the Gauss difference of the interface
 * values divided by the mesh size (Eq. define-averaged-gradient).
 * Grid 0 is the primary grid: node (i, j) at (x0+(i+1/2)h, y0+(j+1/2)h).
 * Grid 1 is the dual grid:    node (i, j) at (x0+(i+1)h,   y0+(j+1)h).
 * In 1D grid 1 is an independent copy on the shifted nodes, advanced only when
 * dual_1d is set.
 *
 * Bounded 2D axes.  A side that is not periodic lies half a mesh beyond the
 * end primary nodes, so the dual grid has nodes on it: along a bounded x axis
 * the dual grid has nx + 1 nodes, node i at x0 + i h (i = 0..nx), and its
 * planes are (ny or ny + 1) x (nx + 1); likewise along y.  Every dual-grid
 * array at the boundary (set_state, get_state, debug_stage) has that shape.
 */
#ifndef FDCGKS_H
#define FDCGKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FDCGKS_OK = 0,
  FDCGKS_EINVAL = -1,   /* bad argument: sizes, NULL pointers, parameters out of range */
  FDCGKS_ENOMEM = -2,   /* device allocation failed */
  FDCGKS_EHIP = -3,     /* a HIP runtime call failed (message in fdcgks_last_error) */
  FDCGKS_ENONPHYS = -4, /* a stage produced rho <= 0, p <= 0 or a NaN; state rolled back */
  FDCGKS_ESTATE = -5    /* call out of order (e.g. step before set_state) */
} fdcgks_status;

/* Boundary conditions (the paper uses walls and outflow sides in Sec. 5
 * without defining their ghost nodes; this is the library's reading):
 *   PERIODIC: periodic images (both sides of an axis);
 *   ZERO_GRADIENT: ghosts copy the end node of their grid, with the
 *     derivative normal to the side set to zero;
 *   REFLECTING: slip wall / symmetry plane: ghosts are the mirror image about
 *     the side, the normal momentum odd, the other components even, and a
 *     derivative normal to the side of the opposite parity to its component;
 *     dual nodes on the side keep zero normal momentum and zero derivative of
 *     it along the side;
 *   NO_SLIP: adiabatic no-slip wall (2D): as REFLECTING with both momenta
 *     odd, and both momenta (and their derivatives along the side) zero at
 *     the dual nodes on the side. */
enum { FDCGKS_BC_PERIODIC = 0, FDCGKS_BC_ZERO_GRADIENT = 1, FDCGKS_BC_REFLECTING = 2, FDCGKS_BC_NO_SLIP = 3 };
/* Numerical flux: (6-4) = Eq. fd-conservative-flux-2 with its low-order term
 * divided by 6; (6-2) = Eq. fd-conservative-flux-1; LINEAR = linear compact
 * flux and linear reconstruction (no GENO). */
enum { FDCGKS_FLUX_6_4 = 0, FDCGKS_FLUX_6_2 = 1, FDCGKS_FLUX_LINEAR = 2 };
/* Width of the linear compact flux (flux_order): 6 = Eq. fd-conservative-flux
 * (nodal fluxes at j, j+1); 8 = the wider stencil Sec. 2.1 mentions, read as
 * the averaging conditions of Eq. fd-conservative-flux-recons imposed also on
 * the nodal cells j-1 and j+2:
 *   F = (32 (F_{j-1/2} + F_{j+3/2}) + 704 F_{j+1/2} - 171 (F_j + F_{j+1})
 *        - 3 (F_{j-1} + F_{j+2})) / 420,
 * exact to degree 7.  The flux variant's low-order term and blend are the same
 * for both.  Order 8 is available to fdcgks_problem steps (1D and 2D, every
 * boundary), to batches and to the step adjoint. */
/* Precision of the gas-kinetic solver; reconstruction and update stay FP64. */
enum { FDCGKS_FP64 = 0, FDCGKS_FP32_FLUX = 1 };
/* Base of the averaged-gradient update (Eq. eq-interface-update): the gradient
 * re-evaluated from the stage-1 interface values (default) or the stored one. */
enum { FDCGKS_GRAD_REEVAL = 0, FDCGKS_GRAD_CARRIED = 1 };
/* Variables the GENO reconstruction works on (Sec. 3): each conservative
 * component on its own (the path function from the density line), or the
 * characteristic variables of the Euler flux Jacobian along each line, with
 * the eigenvectors at the mean of the two interface-adjacent states (at the
 * node's own state for node derivatives) and the path function the smallest
 * of the acoustic fields' left and right values.  Characteristic mode is
 * available to fdcgks_problem steps (1D and 2D, either flux precision), to
 * batches and to the step adjoint. */
enum { FDCGKS_RECON_CONSERVATIVE = 0, FDCGKS_RECON_CHARACTERISTIC = 1 };

typedef struct fdcgks_params {
  int32_t dim;            /* 1 or 2 */
  int32_t nx, ny;         /* primary nodes per axis (ny = 1 in 1D); 2D needs nx, ny >= 4 */
  int32_t bc;             /* FDCGKS_BC_*: 1D both ends (not NO_SLIP); 2D every side not set in `side` */
  int32_t dual_1d;        /* 1D: also advance the shifted copy (grid 1) */
  int32_t flux_variant;   /* FDCGKS_FLUX_* */
  int32_t flux_precision; /* FDCGKS_FP64 | FDCGKS_FP32_FLUX */
  int32_t grad_update;    /* FDCGKS_GRAD_* */
  int32_t geno_r;         /* exponent r of the GENO smoothness ratio, 1..8 (default 3) */
  int32_t recon_vars;     /* FDCGKS_RECON_* (default conservative) */
  int32_t flux_order;     /* 6 (default) or 8, see above */
  int32_t side[4];        /* 2D: FDCGKS_BC_* of the x-low, x-high, y-low, y-high sides, -1 = bc (default);
                             a periodic side needs a periodic opposite side */
  double x0, lx, y0, ly;  /* domain origin and lengths; 2D needs lx/nx == ly/ny */
  double gamma;           /* ratio of specific heats, > 1 and < 5/3 (2D) or < 3 (1D) */
  double mu;              /* dynamic viscosity; 0 = Euler */
  double prandtl;         /* Prandtl number (used when mu > 0) */
  double geno_C;          /* path-function constant C (20) */
  double geno_eps;        /* epsilon of the GENO smoothness ratio (1e-15) */
  double geno_eps_a;      /* epsilon of the low-order weights (1e-6) */
  double geno_d_central;  /* ideal weight of the central sub-stencil (8) */
  double geno_d_side;     /* ideal weight of the other two sub-stencils (1) */
  double tau_c1;          /* Euler collision time tau = c1 dt + c2 dt |p_l-p_r|/(p_l+p_r) */
  double tau_c2;          /*   (defaults c1 = 0, c2 = 1; with mu > 0 the first term is mu/p) */
} fdcgks_params;

typedef struct fdcgks_problem fdcgks_problem; /* opaque, owned by the library */

/* Fill *p with the defaults (2D, 64x64 on [0,1]^2, periodic, gamma 1.4, Euler,
 * (6-4) flux, FP64, GENO constants above). */
void fdcgks_default_params(fdcgks_params* p);

/* Validate *p, allocate the device planes on the current HIP device and bind
 * the problem to `hip_stream` (a hipStream_t; NULL = the null stream).  All
 * later work of the problem is enqueued on that stream.  *out receives the
 * handle; on error *out is NULL and nothing is allocated. */
fdcgks_status fdcgks_create(const fdcgks_params* p, void* hip_stream, fdcgks_problem** out);

/* Copy one grid's state in.  W, Wx must be non-NULL; Wy must be non-NULL in 2D
 * and is ignored in 1D.  Each holds ncomp planes of the grid's ny_g rows of
 * nx_g doubles (the layout above); a row starts every row_stride doubles
 * (0 = nx_g, dense; otherwise >= nx_g) and a plane every ny_g * row_stride.
 * on_device = 1: device pointers (read on the problem's stream, no host
 * synchronisation); 0: host pointers (synchronous).  Values with rho <= 0,
 * p <= 0 or NaN are accepted here and reported by the first step as
 * FDCGKS_ENONPHYS. */
fdcgks_status fdcgks_set_state(fdcgks_problem* pb, int32_t grid, const double* W, const double* Wx,
                               const double* Wy, int64_t row_stride, int32_t on_device);

/* Copy one grid's state out (same layout, row_stride and on_device rule as
 * set_state; with on_device = 0 the call waits for the stream). */
fdcgks_status fdcgks_get_state(const fdcgks_problem* pb, int32_t grid, double* W, double* Wx, double* Wy,
                               int64_t row_stride, int32_t on_device);

/* Every grid's state from point samples of the initial conservative field
 * on the half-spacing lattice (periodic problems; EINVAL with a bounded
 * side).  2D: S[ncomp][2 ny][2 nx], sample (c, ky, kx) at
 * (x0 + (kx+1) h/2, y0 + (ky+1) h/2): (even, even) are the primary nodes,
 * (odd, odd) the dual nodes, (odd, even) and (even, odd) the interface points
 * X and Y.  1D: S[ncomp][2 nx], even samples the primary line, odd samples the
 * shifted copy.  Nodal values are the samples; the averaged derivatives are
 * the Gauss differences of the samples at the node's two bounding interfaces
 * divided by h (Eq. define-averaged-gradient), with periodic wrap.
 * on_device as for set_state (a host array is staged through the library's
 * stage buffer). */
fdcgks_status fdcgks_set_state_from_samples(fdcgks_problem* pb, const double* S, int32_t on_device);

/* Diagnostics of the current state (synchronous): out[q] for q < ngrid*ncomp
 * is the sum of conserved component q % ncomp over the stored nodes of grid
 * q / ncomp (primary first); then the smallest rho and the smallest pressure
 * over all nodes.  out must hold ngrid*ncomp + 2 doubles (2D: 10; 1D: 5 or
 * 8).  Sums are formed in a fixed order, so repeated calls on one state agree
 * bit for bit. */
fdcgks_status fdcgks_diagnostics(fdcgks_problem* pb, double* out);

/* CFL time step of the current state (Sec. 5): dt = cfl h / max over all
 * nodes of (max(|U|,|V|) + c); with mu > 0 also dt <= cfl h^2 / (8 mu/rho_min).
 * Synchronous. */
fdcgks_status fdcgks_compute_dt(fdcgks_problem* pb, double cfl, double* dt_out);

/* Advance up to nsteps S2O4 steps.  dt > 0: fixed step; dt <= 0: CFL step
 * recomputed on the device before every step.  t_end > 0 clips the last step
 * so that t does not pass t_end and stops there.  *t_inout is the time before
 * and after; *steps_done (may be NULL) the number of steps taken.  On
 * FDCGKS_ENONPHYS the state is the one after the last good step and *t_inout,
 * *steps_done describe it. */
fdcgks_status fdcgks_step(fdcgks_problem* pb, double dt, double cfl, int32_t nsteps, double t_end,
                          double* t_inout, int32_t* steps_done);

/* fdcgks_step with a per-kernel device-time breakdown: a HIP event is
 * recorded on the problem's stream after every kernel, and kernel_ms[8]
 * receives the summed milliseconds between consecutive events for: halo fill,
 * interface sweep (stage 1), node sweep (1), assemble+update (1), interface
 * sweep (2), node sweep (2), assemble+update (2), step bookkeeping (CFL
 * reduction, dt, time advance).  Synchronous. */
fdcgks_status fdcgks_step_timed(fdcgks_problem* pb, double dt, double cfl, int32_t nsteps, double t_end,
                                double* t_inout, int32_t* steps_done, double* kernel_ms);

/* ---------------------------------------------------- allocation-free run
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the 1D run
 * of fdcgks_create + fdcgks_set_state + fdcgks_step + fdcgks_get_state in one
 * call that allocates nothing.  Every working buffer (state ping-pong, stage
 * buffers, interface and node results, step scalars) lives in a static device
 * array of the library, about 11.4 MB per device, held until the process
 * ends; the call itself does no hipMalloc, hipFree or other allocation.
 *   p       : a 1D problem (dim 1, ny 1), nx <= 2048; periodic, zero-gradient
 *             or reflecting ends, dual_1d for the shifted copy; the other
 *             fields as for fdcgks_create;
 *   state   : device memory of the current device, [lines][6][nx] doubles
 *             (lines = 2 with dual_1d, else 1; per line W[3] then Wx[3], each
 *             nx contiguous), read at the start and overwritten with the
 *             state after the last completed step;
 *   dt, cfl, nsteps, t_end, t_inout, steps_done: as for fdcgks_step.
 * Runs on hip_stream (0 = the null stream) and synchronizes it once, to
 * return t and the step count.  Results are bitwise those of the handle
 * path.  EINVAL for larger problems, 2D, NULL pointers or a state pointer
 * that is not device memory of the current device; ENONPHYS as fdcgks_step
 * (state = the last good step).  Messages: fdcgks_last_error(NULL).
 * Calls on one device share the array: calls that overlap in time on one
 * device (other threads, other streams) race and must be serialised by the
 * caller. */
fdcgks_status fdcgks_step1d_static(const fdcgks_params* p, double* state, double dt, double cfl, int32_t nsteps,
                                   double t_end, double* t_inout, int32_t* steps_done, void* hip_stream);

/* Free all device memory of the problem.  NULL is accepted. */
fdcgks_status fdcgks_destroy(fdcgks_problem* pb);

/* Message of the last failed call on this problem (or of the last failed
 * create when pb is NULL).  Valid until the next call on the same problem. */
const char* fdcgks_last_error(const fdcgks_problem* pb);

/* ------------------------------------------------------------ diagnostics
 * One stage without committing it, for stage-level comparison.  Stage 1
 * starts from the current state, stage 2 from the internal stage-1 buffers
 * left by the previous fdcgks_debug_stage(.., 1, ..) call, with the same dt.
 * Host outputs: out_state[grid][12][ny][nx] (2D; 1D: [grid][6][nx]; with
 * bounded axes the dual grid's planes have their own size, see above) holds
 * the stage result (W*, grad W* after stage 1; W^{n+1}, grad W^{n+1} after stage
 * 2); out_acc (stage 1 only, may be NULL) the accumulators
 * W + dt L + dt^2/6 L_t and the base gradient.  Grids not present are not
 * written. */
fdcgks_status fdcgks_debug_stage(fdcgks_problem* pb, int32_t stage, double dt, double* out_state,
                                 double* out_acc);

/* Per-interface and per-node intermediates of stage 1 at step dt from the
 * current state (2D only).  Host outputs, each plane ny*nx:
 *   edge_x, edge_y: [2 normals][25] planes for the interface families
 *     X(i,j) at (x0+(i+1)h, y0+(j+1/2)h) and Y(i,j) at (x0+(i+1/2)h, y0+(j+1)h);
 *     normal 0 = x, 1 = y; per normal: flux F[4], F_t[4], chi (path function
 *     of rho, min of left/right), blended interface values Wl[4], Wr[4],
 *     Wl_t[4], Wr_t[4] (Eq. W-model-2d);
 *   node_p, node_d: [16] planes: nodal x-flux F[4], F_t[4], y-flux G[4], G_t[4]. */
fdcgks_status fdcgks_debug_intermediates(fdcgks_problem* pb, double dt, double* edge_x, double* edge_y,
                                         double* node_p, double* node_d);

/* ------------------------------------------------------- launch options
 * FDCGKS_OPT_GRAPH = K in 0..64 (default 16): with K > 0, 2D fdcgks_step
 * replays K whole steps at a time (dt reduction, both stages, step end)
 * captured as one HIP graph per ping-pong parity, captured on first use on
 * a private stream and launched on the problem's stream; the last nsteps mod
 * K steps and K = 0 launch every kernel separately.
 * fdcgks_step_timed always launches separately (it times every kernel).
 * FDCGKS_OPT_TILE_EDGE / _NODE / _UPDATE: block shape of the interface
 * sweep, node sweep and update kernels as x | (y << 16); x in {32, 64, 128,
 * 256}, x*y a multiple of 64 and at most 256, y even for the interface
 * sweep (its two normals per point are paired thread rows).  Defaults:
 * 64 x 2 (interface), 64 x 1 (node), 128 x 1 (update), the autotuner's pick
 * on a 2048^2 Navier-Stokes problem.
 * The shape changes only the launch, never the arithmetic: results are
 * bitwise identical for every valid shape.
 * FDCGKS_OPT_FUSE_NODES (default 0): 1 makes 2D steps evaluate the nodal fluxes
 * inside the update kernel (per 64 x 4 tile plus a one-node halo, in LDS)
 * instead of a separate node sweep through a node buffer; the node and
 * update shapes then do not apply (bitwise the same results).  Periodic
 * problems with flux_order 6 only: bounded problems and the order-8 flux
 * (which reads nodal fluxes two nodes away) keep the separate sweep.  The
 * diagnostics and the step adjoint always use the separate sweep.
 * FDCGKS_OPT_FUSE_STAGE (default 2): 1 makes 2D steps run the node sweep and
 * then one kernel that marches up strips of node columns, evaluating each
 * row of interface points (reconstruction, gas-kinetic solver, blend of
 * Eq. W-model-2d) and assembling and updating the nodes as soon as their
 * interfaces exist; interface results stay in registers and LDS (no
 * interface buffer).  0 runs the separate interface sweep and update
 * through the interface buffer (the interface and update launch shapes then
 * apply).  2 chooses the fused kernel where its row chunks are tall, i.e.
 * ny * ceil(nx / 61) >= 128 * (compute units): 2048^2 and up on MI355X.
 * Bitwise the same results.  Periodic problems with flux_order 6 (the others
 * always take the separate sweeps); it takes precedence over
 * FDCGKS_OPT_FUSE_NODES.
 * FDCGKS_OPT_FUSED_ROWS (default 0): node rows per block of that kernel;
 * 0 chooses about two blocks per compute unit.
 * EINVAL for an unknown option or an invalid value. */
enum {
  FDCGKS_OPT_GRAPH = 0,
  FDCGKS_OPT_TILE_EDGE = 1,
  FDCGKS_OPT_TILE_NODE = 2,
  FDCGKS_OPT_TILE_UPDATE = 3,
  FDCGKS_OPT_FUSE_NODES = 4,
  FDCGKS_OPT_FUSE_STAGE = 5,
  FDCGKS_OPT_FUSED_ROWS = 6
};
fdcgks_status fdcgks_set_option(fdcgks_problem* pb, int32_t option, int64_t value);
fdcgks_status fdcgks_get_option(const fdcgks_problem* pb, int32_t option, int64_t* value);

/* Autotuner: times every valid candidate block shape of the three stage-1
 * kernels (reps launches each, HIP events on the problem's stream) on the
 * current state at its CFL 0.4 time step and keeps the fastest per kernel.
 * The state is not advanced (the stage scratch buffers are overwritten).
 * Synchronises the stream.  1D problems: nothing to tune, returns OK. */
fdcgks_status fdcgks_autotune(fdcgks_problem* pb, int32_t reps);

/* ---------------------------------------------------------------- adjoint
 * Vector-Jacobian product of one S2O4 step (Sec. 2.3 stages with the
 * interface and nodal solvers of Sec. 2, the compact flux of
 * Eq. fd-conservative-flux of order 6 or 8 and the GENO reconstructions of
 * Sec. 3) taken at
 * the current state with the time step dt held fixed (the CFL time step is
 * not differentiated).  lam_out[grid][12][ny][nx] is the adjoint of the step
 * output (W, Wx, Wy per grid, the get_state order); on return
 * lam_in[grid][12][ny][nx] = J^T lam_out, where J is the Jacobian of the
 * step map at the current state.  The state is not advanced (the step is
 * recomputed internally; the next-state buffer is used as scratch).
 * Non-smooth points take fixed one-sided derivatives: |x| has derivative 0
 * at 0 and min/max ties select the first argument.  2D problems (any sides:
 * the halo fill's ghost rules and the wall condition are differentiated like
 * the rest; either reconstruction, the characteristic frame included) with
 * FP64 fluxes only (EINVAL otherwise); ENONPHYS if the recomputed step is
 * non-physical.  With bounded
 * axes grid 1's planes have the dual grid's size (as fdcgks_get_state):
 * lam_out and lam_in hold grid 0's 12 planes, then grid 1's.
 * on_device: both arrays are device pointers (1) or host pointers (0).
 * The first call allocates an adjoint workspace of about 410 planes of
 * (nx + 16) x (ny + 6) doubles, kept until fdcgks_destroy.  Calls on one
 * problem must not overlap. */
fdcgks_status fdcgks_step_vjp(fdcgks_problem* pb, double dt, const double* lam_out, double* lam_in,
                              int32_t on_device);

/* ---------------------------------------------------------------- batches
 * Many independent 2D problems of different sizes advanced together (same
 * scheme constants, each member its own grid, mesh size, sides and CFL time
 * step): every launch covers every member, one launch per phase of a stage
 * (captured as HIP graphs by default) or one cooperative persistent launch
 * per stage (see fdcgks_batch_set_mode).  Same state layout and on_device
 * rule as the single-problem calls; the dual grid of a member with bounded
 * axes has one more column / row along them. */
typedef struct fdcgks_batch fdcgks_batch; /* opaque, owned by the library */

/* How a batched stage is launched.  PERSISTENT: one cooperative launch per
 * stage, sized to the co-resident grid, that walks the device work list in
 * three phases separated by grid barriers (CFL partials and halo; interface
 * and node sweeps; update).  PHASED: the same work list and device code as
 * one launch per phase (halo, interfaces, nodes, update), so that every
 * phase runs at its own occupancy.  GRAPH (default): the PHASED launches of
 * 16 steps captured as one HIP graph (per start parity and cfl, on first
 * use) and replayed; the last nsteps mod 16 steps launch separately.  All
 * give bitwise the same results. */
enum { FDCGKS_BATCH_PERSISTENT = 0, FDCGKS_BATCH_PHASED = 1, FDCGKS_BATCH_GRAPH = 2 };

/* params[count]: every member 2D (EINVAL otherwise); members may differ only
 * in nx, ny, x0, lx, y0, ly and their sides (bc, side[4]): the scheme
 * constants, the reconstruction variables, the flux order and the flux
 * precision are the batch's, and each member advances bit for bit like the
 * same problem alone.
 * Allocates all device memory on the current device. */
fdcgks_status fdcgks_batch_create(int32_t count, const fdcgks_params* params, void* hip_stream, fdcgks_batch** out);
fdcgks_status fdcgks_batch_set_state(fdcgks_batch* b, int32_t member, int32_t grid, const double* W,
                                     const double* Wx, const double* Wy, int32_t on_device);
fdcgks_status fdcgks_batch_get_state(const fdcgks_batch* b, int32_t member, int32_t grid, double* W, double* Wx,
                                     double* Wy, int32_t on_device);
/* Advance every member nsteps steps with its own CFL time step.  Optional
 * host outputs: t_out[count] (time since the batch was created), dt_out[count]
 * (last step), *steps_done.  On FDCGKS_ENONPHYS every member is left after the
 * last step all members completed. */
fdcgks_status fdcgks_batch_step(fdcgks_batch* b, double cfl, int32_t nsteps, double* t_out, double* dt_out,
                                int32_t* steps_done);
fdcgks_status fdcgks_batch_destroy(fdcgks_batch* b);
const char* fdcgks_batch_last_error(const fdcgks_batch* b);

/* Select FDCGKS_BATCH_PERSISTENT, FDCGKS_BATCH_PHASED or FDCGKS_BATCH_GRAPH
 * for later fdcgks_batch_step calls (EINVAL otherwise). */
fdcgks_status fdcgks_batch_set_mode(fdcgks_batch* b, int32_t mode);

#ifdef __cplusplus
}
#endif

#endif /* FDCGKS_H */
