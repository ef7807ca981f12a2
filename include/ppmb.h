/*
 * ppmb.h -- C ABI of the MI355X (gfx950) PPM + PPB library.
 *
 * The library advances the directionally split 3-D PPM gas-dynamics step
 * coupled to PPB multifluid advection of Woodward, Lin, Mao, Andrassy &
 * Herwig (arXiv 1810.13416):
 *   - Sec. 1: cell-interface values one order higher than the parabola;
 *     monotonicity constraints only where a 5-cell smoothness test fails;
 *     a hydrostatic base state subtracted out so that the sweeps can run in
 *     32-bit arithmetic; PPB moment-conserving advection of the entrained
 *     fluid fraction fv;
 *   - Sec. 3: gravity tapered to zero a few cells inside an impenetrable
 *     confining sphere inscribed in the cube;
 *   - Sec. 4: fv carried as its cell average and 9 lowest moments, all
 *     updated by 1-D passes; the pass stencil reaches 4 cells.
 *
 * Conventions (every entry point):
 *   - Returns ppmb_status; 0 (PPMB_OK) is success.  No C++ exception crosses
 *     the ABI.  ppmb_last_error() gives a text for the last failure of a
 *     context.
 *   - Host and device exchange arrays (set/get state, conserved, base) are
 *     dense x-fastest: element (k * ny + j) * nx + i of each field.
 *   - The library's device state is a pitched structure-of-arrays: field q
 *     of cell (i, j, k) sits at element q * fs + k * plane + j * px + i,
 *     with rows padded to px (a multiple of 64), plane = px * ny and a
 *     padded field stride fs; ppmb_state_layout() gives the numbers.
 *   - Host pointers are named host_*; device pointers dev_*.  The library
 *     never frees memory it did not allocate.
 *   - Calls that take a context enqueue work on the context's HIP stream and
 *     return without waiting, unless documented as synchronising.
 *     Asynchronous HIP errors surface at the next synchronising call.
 *   - A context is used by one host thread at a time.
 *
 * The 15 evolving fields, in order:
 *   0 rho'  1 m_x  2 m_y  3 m_z  4 E'       (conserved perturbations of the
 *          base state: rho' = rho - rho0, m = rho u, E' = E - p0/(gamma-1))
 *   5 f0  6 fx  7 fy  8 fz  9 fxx 10 fyy 11 fzz 12 fxy 13 fyz 14 fzx
 *          (fv as coefficients of the orthogonal basis 1, x, y, z, P2(x),
 *           P2(y), P2(z), xy, yz, zx on the unit cell, P2(s) = s^2 - 1/12)
 * Primitive exchange arrays (set/get state) hold instead
 *   0 rho' 1 u_x 2 u_y 3 u_z 4 p'  followed by the same 10 fv coefficients.
 */
#ifndef PPMB_H
#define PPMB_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PPMB_OK = 0,
    PPMB_ERR_INVALID = -1,      /* bad argument, shape or call order */
    PPMB_ERR_NOMEM = -2,        /* device allocation failed */
    PPMB_ERR_HIP = -3,          /* a HIP runtime call or kernel failed */
    PPMB_ERR_NONPHYSICAL = -4,  /* non-positive density or pressure, or NaN, found */
    PPMB_ERR_CFL = -5,          /* a step was given a dt above the checked Courant limit */
    PPMB_ERR_UNSUPPORTED = -6   /* a combination the library does not implement */
} ppmb_status;

typedef enum {
    PPMB_FP64 = 0,              /* state, sweeps and reductions in FP64 */
    PPMB_FP32 = 1               /* state and sweeps in FP32; base state
                                   integration, dt and totals in FP64, and
                                   an FP64 re-solve of Riemann problems whose
                                   FP32 iteration has not converged (Sec. 1:
                                   32-bit sweeps on perturbations) */
} ppmb_precision;

enum { PPMB_BC_PERIODIC = 0, PPMB_BC_REFLECT = 1 };
enum { PPMB_GRAV_NONE = 0, PPMB_GRAV_CONST = 1, PPMB_GRAV_RADIAL = 2 };
enum { PPMB_BASE_NONE = 0, PPMB_BASE_CONST = 1, PPMB_BASE_POLY_Z = 2, PPMB_BASE_POLY_R = 3 };
enum { PPMB_HEAT_NONE = 0, PPMB_HEAT_LAYER_Z = 1, PPMB_HEAT_BALL = 2 };
enum { PPMB_NFIELDS = 15 };

/* Grid and physics.  Cell (i, j, k) has centre origin + (index + 1/2) dx.
 *   bc[d]        boundary on both ends of axis d: periodic or reflecting
 *   sphere       1: cells whose centre lies at r >= sphere_r from the origin
 *                of coordinates are solid (Sec. 3 confining sphere); faces
 *                between fluid and solid cells are reflecting walls
 *   grav_kind    CONST: grav[0..2] is the acceleration vector.
 *                RADIAL: g = -grav[0] r_hat * (r/grav[1] for r < grav[1],
 *                else (grav[1]/r)^2), times a taper falling linearly from 1
 *                at r = grav[2] to 0 at r = grav[3] (Sec. 3)
 *   heat_kind    LAYER_Z: energy source heat[0] * h((z - heat[2]) / heat[1]);
 *                BALL: heat[0] * h(r / heat[1]); h = 1 below 1/2, smoothstep
 *                down to 0 at 1
 *   smooth_detect 1: the 5-cell smoothness test gates the constraints (the
 *                method); 0: constraints everywhere; 2: no constraints
 *                (the last two for comparison) */
typedef struct {
    int    n[3];
    double dx;
    double origin[3];
    int    bc[3];
    double gamma;
    int    sphere;
    double sphere_r;
    int    grav_kind;
    double grav[4];
    int    heat_kind;
    double heat[3];
    int    smooth_detect;
} ppmb_grid;

typedef struct ppmb_ctx ppmb_ctx;

/* Create a context for one grid on `hip_stream` (a hipStream_t; NULL = the
 * null stream).  Allocates the library's own device buffers: the FP64 base
 * state (2 fields), its copy in the working precision, reduction buffers and
 * counters.  The state itself is caller memory bound with
 * ppmb_bind_state().  Errors: INVALID for n < 1, dx <= 0, gamma <= 1 or an
 * unknown kind; NOMEM; HIP. */
ppmb_status ppmb_create(const ppmb_grid *grid, ppmb_precision prec, void *hip_stream,
                        ppmb_ctx **out);

/* Synchronise the stream, then free the library's buffers and the context. */
ppmb_status ppmb_destroy(ppmb_ctx *ctx);

/* Bytes the caller must provide per state buffer: 15 * fs * elem_size
 * summed over bricks (elem_size 8 for FP64, 4 for FP32). */
ppmb_status ppmb_state_bytes(const ppmb_ctx *ctx, size_t *bytes, size_t *elem_size);

/* Storage layout of brick `brick` (0 for a single grid) in a state buffer:
 * field q of cell (i, j, k) at element out[0] + q * out[1] + k * out[2]
 * + j * out[3] + i (offset, field stride fs, plane stride, row pitch px),
 * in elements of the working precision.  Padding elements are never read.
 * Not synchronising.  Errors: INVALID for a NULL argument or a brick out of
 * range. */
ppmb_status ppmb_state_layout(const ppmb_ctx *ctx, int brick, long long out[4]);

/* Bind two caller-owned device buffers of ppmb_state_bytes() each.  Passes
 * read one and write the other (ping-pong); ppmb_current_state() names the
 * one holding the latest state.  The caller keeps both alive until destroy
 * and must not touch them while work is queued.  Errors: INVALID for NULL
 * or identical pointers. */
ppmb_status ppmb_bind_state(ppmb_ctx *ctx, void *dev_buf_a, void *dev_buf_b);
ppmb_status ppmb_current_state(const ppmb_ctx *ctx, void **dev_state);

/* Hydrostatic base state (Sec. 1: the initial state is saved on the grid and
 * subtracted out).  kind NONE: no base (plain form, the state is the full
 * state).  CONST: rho0 = params[0], p0 = params[1].  POLY_Z / POLY_R:
 * piecewise polytrope in hydrostatic balance with the grid's gravity along z
 * (constant gravity) or r (radial gravity): rho0 = params[0] and
 * p0 = params[1] at s = params[2]; the density jumps by the factor params[4]
 * at continuous pressure at s = params[3]; tables reach s = params[5].
 * Integrated on the GPU in FP64 (RK4, 8 steps per cell width, segments split
 * at the jump and every kink of g), then written to the base fields.
 * Synchronising.  Call before ppmb_set_state. */
ppmb_status ppmb_set_base_state(ppmb_ctx *ctx, int kind, const double params[6]);

/* Gravity of every brick, after create (Sec. 3: gravity tapered to zero
 * before the confining sphere).  kind and params as grav_kind and grav of
 * ppmb_grid: NONE with nparams 0; CONST with nparams 3 (the acceleration
 * vector); RADIAL with nparams 4 (g0, rc, r1, r2: g = -g0 r_hat times
 * r/rc inside rc, (rc/r)^2 outside, times a taper from 1 at r1 to 0 at r2).
 * Acts on the passes enqueued after the call (the half-step sources of the
 * tracing and the momentum and energy sources of the update).  The base
 * state is not re-integrated: call ppmb_set_base_state again for a base in
 * balance with the new gravity.  Synchronises the stream (the brick table
 * is rewritten) and drops a captured step graph.  INVALID for an unknown
 * kind, a wrong nparams, a non-finite parameter, rc <= 0 or r2 <= r1. */
ppmb_status ppmb_set_gravity(ppmb_ctx *ctx, int kind, const double *params, int nparams);

/* Heating of every brick, after create (Sec. 2: the driving luminosity,
 * boosted in the paper's runs).  kind and params as heat_kind and heat of
 * ppmb_grid: NONE with nparams 0; LAYER_Z with nparams 3 (Q0, extent, z0:
 * energy source Q0 h((z - z0) / extent)); BALL with nparams 2 or 3 (Q0,
 * extent: Q0 h(r / extent); a third value is ignored).  The source is added
 * after the last pass of each step.  Synchronises the stream and drops a
 * captured step graph.  INVALID for an unknown kind, a wrong nparams, a
 * non-finite parameter or extent <= 0. */
ppmb_status ppmb_set_heating(ppmb_ctx *ctx, int kind, const double *params, int nparams);

/* Copy the FP64 base fields (rho0, p0; ncell each) to host memory.
 * Synchronising. */
ppmb_status ppmb_get_base(ppmb_ctx *ctx, double *host_rho0, double *host_p0);

/* Set the state from 15 FP64 host arrays of primitive perturbations
 * (rho', u_x, u_y, u_z, p', then the 10 fv coefficients), converted on the
 * GPU to the conserved perturbation fields of the working precision.
 * Synchronising (the host arrays may be reused on return). */
ppmb_status ppmb_set_state(ppmb_ctx *ctx, const double *const host_prim[15]);

/* Same, from 15 FP64 device arrays (ncell each). */
ppmb_status ppmb_set_state_device(ppmb_ctx *ctx, const double *const dev_prim[15]);

/* Set / read the z-planes k0 .. k0 + nk - 1 of brick 0 only, from / to 15
 * FP64 host arrays of nx * ny * nk primitive values each (dense, x
 * fastest, plane k0 first), so that a grid too large for one host copy of
 * its fields is filled and checked plane slab by plane slab.  A run sets
 * every plane before its first step.  Synchronising.  INVALID for planes
 * outside the grid or a NULL field. */
ppmb_status ppmb_set_state_planes(ppmb_ctx *ctx, int k0, int nk, const double *const host_prim[15]);
ppmb_status ppmb_get_state_planes(ppmb_ctx *ctx, int k0, int nk, double *const host_prim[15]);

/* Read the state back as 15 FP64 host arrays of primitive perturbations.
 * Synchronising. */
ppmb_status ppmb_get_state(ppmb_ctx *ctx, double *const host_prim[15]);

/* Conserved fields (the stored representation, widened to FP64) for
 * checkpoints; set_conserved rounds to the working precision.
 * Synchronising. */
ppmb_status ppmb_get_conserved(ppmb_ctx *ctx, double *const host_cons[15]);
ppmb_status ppmb_set_conserved(ppmb_ctx *ctx, const double *const host_cons[15]);

/* CFL time step dt = cfl * dx / max over fluid cells and axes of |u_d| + c,
 * computed in FP64 from the stored state.  Synchronising.  Errors:
 * NONPHYSICAL if a fluid cell has rho <= 0, p <= 0 or a NaN.
 *
 * Deferred errors.  The passes and the CFL reductions raise device flags
 * that the synchronising calls ppmb_compute_dt, ppmb_last_dt,
 * ppmb_brick_last_dt, ppmb_reduce_totals, ppmb_brick_totals,
 * ppmb_counters and ppmb_synchronize read (after finishing their own work,
 * so that their outputs are filled) and clear: NONPHYSICAL when a step
 * produced or started from a fluid cell with rho <= 0, p <= 0 or a NaN
 * (ppmb_step_auto keeps stepping on such a state until one of these calls),
 * CFL when the Courant check of ppmb_set_cfl_check failed. */
ppmb_status ppmb_compute_dt(ppmb_ctx *ctx, double cfl, double *dt_out);

/* One step of size dt: three 1-D passes, x,y,z on even steps and z,y,x on
 * odd steps, then the heating source.  Asynchronous. */
ppmb_status ppmb_step(ppmb_ctx *ctx, double dt);

/* Solid cells of the confining sphere (Sec. 3) keep their values, so the
 * passes leave out those farther than the stencil reach (4 cells) from a
 * fluid cell: a wave of pencils marches over the union of its pencils'
 * fluid intervals (plus 4 cells either side, read only), the x pass visits
 * only the 56-cell segments from the row's first fluid cell to its last.
 * This needs the solid cells to hold the same values in both state
 * buffers: the first pass after a state change by the library (set_state,
 * set_conserved, bind_state, set_base_state) writes every cell, and later
 * passes skip.  A caller that writes a bound buffer directly calls
 * ppmb_bind_state again.  on = 0 makes every pass write every cell (the
 * results are bitwise the same either way); on = 1 is the default.
 * Drops a captured step graph.  INVALID for a null context. */
ppmb_status ppmb_set_solid_skip(ppmb_ctx *ctx, int on);

/* Courant check of caller-given time steps (a failure detector for
 * ppmb_step and ppmb_pass; ppmb_step_auto takes its dt from the CFL
 * condition and is not checked).  With courant_max > 0, each ppmb_step and
 * ppmb_pass first reduces, on the device and in FP64, the largest signal
 * speed s = max over fluid cells and axes of |u_d| + c of the state it
 * starts from, and raises the CFL flag when dt > courant_max * dx / s; the
 * step is still taken, and the next synchronising call returns
 * PPMB_ERR_CFL (the caller restores a checkpoint and retries with a
 * smaller dt).  courant_max = 0 switches the check off.  The default is off,
 * or 1.0 when the environment variable PPMB_CHECK_CFL is 1 at create.
 * Asynchronous; INVALID for courant_max < 0 or not finite. */
ppmb_status ppmb_set_cfl_check(ppmb_ctx *ctx, double courant_max);

/* `nsteps` steps, each taking dt from the CFL condition of the state at its
 * start, computed on the device: no host synchronisation.  The dt of the
 * last step is readable with ppmb_last_dt().  Asynchronous. */
ppmb_status ppmb_step_auto(ppmb_ctx *ctx, double cfl, int nsteps);
ppmb_status ppmb_last_dt(ppmb_ctx *ctx, double *dt_out);   /* synchronising */

/* One 1-D pass along `axis` (0, 1, 2) with step dt; `heat` = 1 adds the
 * heating source for dt to the updated cells.  Does not advance the step
 * counter.  Asynchronous. */
ppmb_status ppmb_pass(ppmb_ctx *ctx, int axis, double dt, int heat);

/* Step counter (its parity selects the pass order); set it when resuming a
 * checkpoint. */
ppmb_status ppmb_get_nstep(const ppmb_ctx *ctx, long *nstep);
ppmb_status ppmb_set_nstep(ppmb_ctx *ctx, long nstep);

/* Conserved totals over fluid cells in FP64 with a fixed reduction tree
 * (bitwise reproducible): out = { mass, p_x, p_y, p_z, total energy (base
 * included), fv volume, min f0, max f0 }.  Synchronising. */
ppmb_status ppmb_reduce_totals(ppmb_ctx *ctx, double out[8]);

/* ---- shock dissipation (Sec. 1) ---------------------------------------
 *
 * In flows with shocks the paper adds a fully 3-D dissipation inside shocks;
 * its form is given in a reference that is not available, so this one is a
 * reading after the artificial dissipation of Colella & Woodward (1984,
 * Sec. 4): at the start of each step the undivided divergence of the cell
 * velocity, D = sum over d of (u_d(i + e_d) - u_d(i - e_d)) / 2 (neighbours
 * through the boundary conditions; a solid neighbour is a wall whose normal
 * velocity is minus the cell's own), computed in FP64; then in each of the
 * three passes, at every face between two fluid cells, the flux
 * k max(0, -(D_i + D_i+1) / 2) (U_i - U_i+1) is added to the five conserved
 * hydro perturbations U (rho', the three momenta, E').  It vanishes where
 * the flow does not converge and conserves mass, momentum and energy.
 * k = 0 (the default) switches it off and the passes run exactly as
 * without it; k = 0.1 is the customary value.  ppmb_pass takes the
 * divergence of its own input.  The library allocates one field of the
 * working precision per brick on the first call with k > 0.  Host-side
 * setting; drops a captured step graph.  INVALID for k < 0 or not finite;
 * NOMEM if the field cannot be allocated. */
ppmb_status ppmb_set_shock_dissipation(ppmb_ctx *ctx, double k);

/* Flattening near strong shocks (Colella & Woodward 1984, Sec. 4), the
 * customary companion of the shock dissipation; the paper does not name it,
 * so this is a reading with CW84's constants.  Before each pass, for every
 * cell and the pass axis d, from the full pressure p (base plus
 * perturbation) and the velocity u along d of the pass's input (neighbours
 * through the boundary conditions, a reflecting image's u flipped), FP64:
 * a cell is a shock candidate when |p(i+1) - p(i-1)| > 0.33 min(p(i+1),
 * p(i-1)) and u(i-1) - u(i+1) > 1e-10 (|u(i-1)| + |u(i+1)|); its raw
 * coefficient is then min(1, max(0, 10 (z - 0.75))) with z = (p(i+1) -
 * p(i-1)) / (p(i+2) - p(i-2)) (0 when that difference is 0), else 0; its
 * coefficient f is the larger of its own raw value and that of its
 * neighbour on the low-pressure side (i+1 when p(i+1) < p(i-1), i-1 when
 * p(i+1) > p(i-1), both when |p(i+1) - p(i-1)| <= 1e-10 (p(i+1) + p(i-1))).
 * The 1e-10 margins keep the decisions off values equal but for rounding;
 * CW84's tests are strict.  Each parabola's final edge values (after the
 * constraints) become f q + (1 - f) edge, q the cell average, for all five
 * interpolated variables.  on = 0 (the default) switches it off and the
 * passes run exactly as without it.  The library allocates one field of the
 * working precision per brick on the first call with on != 0.  Host-side
 * setting; drops a captured step graph.  INVALID for a null context; NOMEM
 * if the field cannot be allocated. */
ppmb_status ppmb_set_flattening(ppmb_ctx *ctx, int on);

/* ---- rotation and spherical averages (Sec. 1, Sec. 3) ------------------
 *
 * Spin-up (Sec. 3: a solid-body rotation is added to the flow gradually
 * over the first steps of a run; the frame stays inertial).  The increment
 * domega gives every fluid cell of every brick the velocity change
 * domega * (z-hat x x) = domega * (-y, x, 0), x the cell centre in grid
 * coordinates (the rotation axis is the z axis through the coordinate
 * origin), and keeps rho' and p' unchanged: m_x += rho du_x,
 * m_y += rho du_y, E' += m.du + rho |du|^2 / 2, evaluated in FP64 and
 * stored in the working precision.  Solid cells are not touched. */

/* Ramp: each step whose index (ppmb_get_nstep before the step) lies in
 * [0, nramp) ends, after its passes and heating, with an increment of
 * omega / nramp, so the rotation reaches omega after nramp steps.  omega = 0
 * or nramp = 0 switches it off.  Steps in the ramp are never HIP-graph
 * captured (ppmb_batch_step mode 1 launches them directly), and the step
 * after an increment takes its dt from a full CFL reduction.  INVALID for a
 * non-finite omega or nramp < 0.  Host-side setting only. */
ppmb_status ppmb_set_spinup(ppmb_ctx *ctx, double omega, long nramp);

/* Rotating frame (Sec. 3 names rotating coordinates as the next step of
 * these runs).  With omega != 0 the equations are those seen from axes
 * turning at omega about the z axis through the coordinate origin: every
 * step ends, after its passes and heating and before a spin-up increment,
 * with the Coriolis acceleration -2 omega z-hat x u = 2 omega (u_y, -u_x,
 * 0) and, with centrifugal != 0, the centrifugal acceleration
 * omega^2 (x, y, 0), applied over the step's dt as a split step: half the
 * centrifugal velocity change, the exact Coriolis rotation of (u_x, u_y)
 * by the angle -2 omega dt, the other half.  Density and pressure are
 * kept; m and E' are rebuilt, in FP64, and stored in the working
 * precision.  Solid cells are not touched.  The step after it takes its dt
 * from a full CFL reduction.  omega = 0 (the default) is the inertial
 * frame.  Host-side setting; drops a captured step graph.  INVALID for a
 * non-finite omega. */
ppmb_status ppmb_set_rotating_frame(ppmb_ctx *ctx, double omega, int centrifugal);

/* One increment domega now, on the current state of every brick.
 * Asynchronous; INVALID for a non-finite domega or unbound state. */
ppmb_status ppmb_spin_add(ppmb_ctx *ctx, double domega);

/* Spherical-shell sums of one brick (Sec. 1: averages on spherical
 * surfaces).  Shell k holds the fluid cells whose centre radius r (from the
 * coordinate origin, r^2 = (x^2 + y^2) + z^2 in FP64) has
 * (k dr)^2 <= r^2 < ((k+1) dr)^2; cells with r >= nbins dr are left out.
 * host_out[8 k + q] (nbins * 8 doubles, caller-owned host memory) is the
 * FP64 sum over shell k of dV times q = 0: 1 (volume), 1: rho, 2: f0,
 * 3: rho u_r, 4: rho u_r^2, 5: rho |u|^2, 6: rho (x u_y - y u_x) (angular
 * momentum about z), 7: f0^2, with u_r = x.u / r (0 at r = 0).  Averages
 * over a shell are ratios (f0 by volume: q2 / q0; rms velocity by mass:
 * sqrt(q5 / q1)).  The summation order is fixed, so the result is bitwise
 * reproducible.  The library keeps a workspace of up to 8 * nbins * 4161
 * doubles (per-block partial sums), grown on demand.  Synchronising.  INVALID for nbins outside
 * [1, 1024], dr <= 0 or not finite, a bad brick index or unbound state;
 * NOMEM if the workspace cannot be allocated. */
ppmb_status ppmb_shell_profile(ppmb_ctx *ctx, int brick, int nbins, double dr, double *host_out);

/* The same shell sums for callers that cannot allocate device memory (code
 * under HIP-graph capture, tight serving loops, hosts that forbid
 * allocation): no hipMalloc, hipFree or allocating library call.  The
 * block partials live in a static device workspace of 4 Mi doubles
 * (32 MiB) that every GPU the library runs on holds from its first context
 * until the process ends.  dev_out: caller-owned device memory of
 * 8 * nbins doubles, the same layout and bitwise the same values as
 * ppmb_shell_profile's host_out.  Asynchronous (the result is in dev_out
 * once the context's stream reaches it).  All calls on one GPU share the
 * one workspace: calls that overlap on one GPU (two streams, two threads)
 * race and must be ordered by the caller.  INVALID as for
 * ppmb_shell_profile, a NULL dev_out, or a grid whose block partials
 * (8 * nbins * (blocks + groups) doubles; at most 4161 * 8 * nbins for
 * large grids) exceed the workspace. */
ppmb_status ppmb_shell_profile_noalloc(ppmb_ctx *ctx, int brick, int nbins, double dr, double *dev_out);

/* Event counters since create: { fv limiter activations that changed a
 * profile by more than round-off, unsmooth (cell, variable) pairs
 * constrained, Riemann problems re-solved in FP64 (FP32) or not converged
 * (FP64), steps }.  Synchronising. */
ppmb_status ppmb_counters(ppmb_ctx *ctx, unsigned long long out[4]);

/* ---- Batched bricks ------------------------------------------------------
 * A batch advances many independent bricks of different sizes together
 * (each with its own grid, boundaries, base state and CFL time step): every
 * stage of a step is ONE kernel launch covering all bricks, through a table
 * mapping each block to its brick.  The single-grid calls above act on
 * brick 0 of a context; ppmb_create makes a batch of one.
 *
 * ppmb_batch_create: nbricks grids (ppmb_grid each); the library allocates
 * both state arenas (15 * sum of cells * elem_size bytes each).  Errors as
 * ppmb_create; INVALID for nbricks < 1. */
ppmb_status ppmb_batch_create(int nbricks, const ppmb_grid *grids, ppmb_precision prec,
                              void *hip_stream, ppmb_ctx **out);
ppmb_status ppmb_brick_count(const ppmb_ctx *ctx, int *nbricks);

/* Per-brick versions of set_base_state, get_base, set_state, get_state,
 * get_conserved, reduce_totals and last_dt; `brick` in [0, nbricks), else
 * INVALID.  Same semantics and synchronisation as the single-grid calls. */
ppmb_status ppmb_brick_set_base_state(ppmb_ctx *ctx, int brick, int kind, const double params[6]);
ppmb_status ppmb_brick_get_base(ppmb_ctx *ctx, int brick, double *host_rho0, double *host_p0);
ppmb_status ppmb_brick_set_state(ppmb_ctx *ctx, int brick, const double *const host_prim[15]);
ppmb_status ppmb_brick_get_state(ppmb_ctx *ctx, int brick, double *const host_prim[15]);
ppmb_status ppmb_brick_get_conserved(ppmb_ctx *ctx, int brick, double *const host_cons[15]);
ppmb_status ppmb_brick_totals(ppmb_ctx *ctx, int brick, double out[8]);
ppmb_status ppmb_brick_last_dt(ppmb_ctx *ctx, int brick, double *dt_out);

/* `nsteps` steps of every brick, each brick's dt from its own CFL condition
 * computed on the device (the brick-update model of Sec. 5: bricks advance
 * independently, each on its own dt).  mode 0: one launch per stage for all
 * bricks; 1: the same launches captured once (two steps: both pass orders)
 * into a HIP graph and replayed (recaptured if the arena, step parity, cfl
 * or mode changed); 2: one launch per stage and brick (for comparison);
 * 3: one launch per step of the persistent step kernel: resident waves take
 * work items in order (per brick: its dt from the previous step's maxima,
 * then the waves of its three passes) from a device counter, and an item of
 * a brick waits until the brick's pass counter shows its earlier stages
 * done, so the passes of different bricks overlap and no launch boundary
 * separates them; 4: mode 3 captured and replayed as in mode 1.  Modes 3
 * and 4 cover the plain passes (no shock dissipation or flattening, x pass
 * by its lanes-along-x kernel); otherwise they take mode 0's and mode 1's
 * launches.  A wait of the persistent kernel that exceeds a bounded time
 * (0.25 s) gives up; the next synchronising call then returns PPMB_ERR_HIP.
 * Modes 3 and 4 are switched off in this build (INVALID): the persistent
 * kernel's launches did not complete on the target GPU and the cause is not
 * yet known.  All
 * modes give bitwise identical states, dts and event counters.
 * Asynchronous.  Modes 1 and 4 need a stream other than the null stream
 * (graph capture). */
ppmb_status ppmb_batch_step(ppmb_ctx *ctx, double cfl, int nsteps, int mode);

/* Launch shape of the pass kernels: waves per block of the marching kernel
 * (y and z passes) and of the lanes-along-x kernel (x pass), each 1, 2 or 4.
 * Changes no result bit.  Synchronising. */
ppmb_status ppmb_set_pass_shape(ppmb_ctx *ctx, int march_waves, int x_waves);
ppmb_status ppmb_get_pass_shape(const ppmb_ctx *ctx, int *march_waves, int *x_waves);

/* Work per wave of the pass kernels: the marching kernel (y and z passes)
 * cuts each pencil into chunks of march_chunk cells, one wave per chunk
 * (0: one wave marches the whole pencil; else at least 16), and the x pass
 * gives each wave at least x_rows x-rows (1..64); x_rows = 0 runs the x
 * pass by the marching kernel instead (lanes across y, loads gathered from
 * 64 rows), which can suit short rows.  Shorter chunks and more rows even
 * out the waves' work when solid cells are skipped; every wave reads 4
 * cells beyond its chunk either side.  Changes no result bit.
 * Synchronising.  The default is chunks of 256 cells and 2 rows
 * (PPMB_X_MARCH=1 at create: x_rows 0). */
ppmb_status ppmb_set_pass_tiling(ppmb_ctx *ctx, int march_chunk, int x_rows);
ppmb_status ppmb_get_pass_tiling(const ppmb_ctx *ctx, int *march_chunk, int *x_rows);

/* Autotuner: times, on this context's bricks, `reps` passes per candidate
 * (after one untimed pass), reading the current state and writing the
 * spare arena (the state, step count and counters are left as they were):
 * first the marching kernel over the y and z passes for waves per block 1,
 * 2, 4 and chunks of 0 (whole pencils), 128, 256 cells; then the x pass by
 * the lanes-along-x kernel for waves per block 1, 2, 4 and at least 1, 2, 4
 * rows per wave, and by the marching kernel with the shape just chosen;
 * and keeps the fastest of each.  If cache_path is not NULL, a line keyed
 * by precision, brick count and total cells is read from it (no timing
 * when present) or appended to it.  out_shape receives {march_waves,
 * x_waves}; ppmb_get_pass_tiling gives the rest.  Synchronising. */
ppmb_status ppmb_autotune(ppmb_ctx *ctx, double cfl, int reps, const char *cache_path, int out_shape[2]);

/* Per-pass timing.  While enabled, every pass kernel is bracketed by HIP
 * events recorded on the context's stream (the kernel's own stream).
 * ppmb_profile_read() synchronises, returns per axis the number of timed
 * pass kernels and their summed duration in milliseconds, and clears the
 * record.  Errors: INVALID for NULL arguments; HIP. */
ppmb_status ppmb_profile_enable(ppmb_ctx *ctx, int enable);
ppmb_status ppmb_profile_read(ppmb_ctx *ctx, double ms[3], long count[3]);

ppmb_status ppmb_synchronize(ppmb_ctx *ctx);
const char *ppmb_status_string(ppmb_status s);
const char *ppmb_last_error(const ppmb_ctx *ctx);

/* ------------------------------------------------------------------ */
/* 2-D PPB advection under a rigid rotation: the slotted-disk test of  */
/* Fig. 3 (a gas filling a slotted circle, tracked by PPB on a uniform */
/* 2-D grid as it rotates about the grid centre).                      */
/* ------------------------------------------------------------------ */

/* nx x ny cells of width dx; cell (i, j) centred at origin + (i + 1/2,
 * j + 1/2) dx; periodic boundaries; velocity u = -omega (y - centre_y),
 * v = omega (x - centre_x). */
typedef struct {
    int n[2];
    double dx;
    double origin[2];
    double centre[2];
    double omega;
} ppmb_ppb2d_grid;

typedef struct ppmb_ppb2d ppmb_ppb2d;

/* Create a context with its two device buffers for the 6 fv moments of
 * each cell (f0, fx, fy, fxx, fyy, fxy in the basis 1, x, y, P2(x), P2(y),
 * xy of the unit cell).  Work goes to hip_stream.  Errors: INVALID for a
 * bad grid or precision, NOMEM, HIP. */
ppmb_status ppmb_ppb2d_create(const ppmb_ppb2d_grid *grid, ppmb_precision prec, void *hip_stream,
                              ppmb_ppb2d **out);
ppmb_status ppmb_ppb2d_destroy(ppmb_ppb2d *ctx);

/* Set / read the moments from / to 6 dense FP64 host arrays (nx * ny each,
 * x fastest); rounded to the working precision on set.  Synchronising. */
ppmb_status ppmb_ppb2d_set(ppmb_ppb2d *ctx, const double *const host_coef[6]);
ppmb_status ppmb_ppb2d_get(ppmb_ppb2d *ctx, double *const host_coef[6]);

/* nsteps steps of size dt: an x pass then a y pass on even steps (counted
 * by the context from 0), the reverse on odd steps; each pass moves every
 * pencil by the PPB transport of the 1-D pass (Sec. 1, Sec. 4) with the
 * face Courant numbers of the rotation.  Asynchronous.  Errors: INVALID
 * for dt <= 0 or |omega| dt / dx times the largest lever arm >= 1. */
ppmb_status ppmb_ppb2d_steps(ppmb_ppb2d *ctx, double dt, int nsteps);

/* Step counter (its parity selects the pass order). */
ppmb_status ppmb_ppb2d_get_nstep(const ppmb_ppb2d *ctx, long *nstep);
ppmb_status ppmb_ppb2d_set_nstep(ppmb_ppb2d *ctx, long nstep);

#ifdef __cplusplus
}
#endif

#endif /* PPMB_H */
