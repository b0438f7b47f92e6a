/*
 * mhd.h - C ABI of the MI355X (gfx950) ideal-MHD finite-volume step.
 *
 * One call of mhd_step advances the conserved state
 *     U = (rho, m_x, m_y, m_z, E, B_x, B_y, B_z, psi)
 * on a uniform Cartesian grid by one strong-stability-preserving
 * Runge-Kutta step of a Godunov-type finite-volume scheme.  The paper (section "Porting of
 * gPLUTO") lists the steps repeated in every Runge-Kutta stage: boundary
 * (ghost-zone) calculation, conservative -> primitive map, reconstruction of
 * interface values, Riemann fluxes, right-hand side; plus one
 * divergence-control algorithm, here GLM divergence cleaning (section
 * "Results for gPLUTO", strong-scaling runs).  The paper prints no
 * formulas; the operations follow the published methods it names or uses:
 *   - ghosts: 2 layers per active face (3 with WENO-Z), periodic or
 *     zero-gradient outflow;
 *   - reconstruction, component-wise in the primitive variables: piecewise
 *     linear, minmod or MC limited (van Leer 1979), or fifth-order WENO-Z
 *     (Borges et al. 2008; p = 1, eps = 1e-40 in FP64, 1e-30 in FP32), the
 *     scheme of the paper's benchmark runs (section "Results for gPLUTO");
 *   - GLM: Dedner et al. (2002) mixed GLM, exact (B_n, psi) interface
 *     solve, psi damped by exp(-alpha c_h dt / dh_min) once per step;
 *   - Riemann: HLL (Harten, Lax & van Leer 1983) with Davis wave-speed
 *     bounds, or HLLD (Miyoshi & Kusano 2005) with outer speeds
 *     min(u_L, u_R) - max(c_fL, c_fR) and max(u_L, u_R) + max(c_fL, c_fR),
 *     which keep its rotational waves inside the fan;
 *   - time: SSP-RK2 or SSP-RK3 (Shu & Osher 1988; RK3 is the benchmark
 *     integrator of the paper), dt and c_h fixed for the step;
 *   - CFL: dt = C / max_{cells,d} (|v_d| + c_f,d)/dx_d and
 *     c_h = max_{cells,d} (|v_d| + c_f,d), reduced in FP64;
 *   - divergence control by constrained transport instead of GLM (the
 *     paper's weak-scaling runs; Evans & Hawley 1988) when ct = 1 or 2: the
 *     field lives on the cell faces, each face's value is the normal field
 *     of its Riemann problem, faces advance by the discrete curl of the edge
 *     EMFs with each Runge-Kutta stage, and the cell field is the mean of
 *     each cell's two faces along each axis.  Edge EMFs: ct = 1 the
 *     arithmetic mean of the four face fluxes around the edge (Balsara &
 *     Spicer 1999); ct = 2 the upwind EMF of Londrillo & Del Zanna (2004),
 *     which the paper cites: the two-dimensional HLL average of the EMFs of
 *     the four minmod-reconstructed states at the edge plus one HLL
 *     dissipation term per transverse direction.
 * Magnetic pressure is |B|^2/2; ideal gas E = p/(gamma-1) + rho|v|^2/2 + |B|^2/2
 * (psi is not part of E).  No density or pressure floors: a non-physical
 * state is reported as MHD_ERR_NONPHYSICAL.
 *
 * Layout: every state array is one contiguous device buffer of shape
 * [9][nz][ny][nx] (x fastest), interior cells only; with constrained
 * transport [12][nz][ny][nx], components 9..11 the face field bx, by, bz on
 * each cell's lower x, y, z face and 5..7 the cell field (face means),
 * maintained by the library.  Element type of the
 * context (float for MHD_F32, double for MHD_F64), at least 16-byte
 * aligned.  Adjoint arrays (lambda) are always double with the same shape.
 * Inactive dimensions have n = 1.
 *
 * Ownership: the caller owns every state, adjoint and primitive buffer.
 * The library owns the context and its scratch (stage-1 buffer when the
 * caller passes none, the SSP-RK3 stage-2 buffer, the constrained-transport
 * EMF buffer and, with the mean EMF, face-flux buffer, reduction partials,
 * result and error words), all
 * allocated by mhd_init and freed by mhd_destroy; mhd_step,
 * mhd_step_adjoint and mhd_cfl_dt allocate nothing.
 *
 * Streams: all device work is enqueued on the context's HIP stream.  Calls
 * marked "async" return without waiting; calls marked "syncs" wait for the
 * stream.  Calls on one context must not overlap from several host
 * threads.
 *
 * Errors: every call returns an mhd_status.  Arguments are validated before
 * any device work is enqueued; on MHD_ERR_ARG nothing was enqueued.  HIP
 * failures give MHD_ERR_HIP with the text in mhd_last_error.  Kernels raise
 * a device flag on any cell with rho <= 0, p <= 0 or a non-finite value;
 * the next syncing call returns MHD_ERR_NONPHYSICAL and clears the flag.
 */
#ifndef MHD_H
#define MHD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mhd_ctx mhd_ctx; /* opaque */

typedef enum {
    MHD_OK = 0,
    MHD_ERR_ARG = -1,         /* invalid argument; nothing enqueued           */
    MHD_ERR_NO_DEVICE = -2,   /* no usable gfx950 device                      */
    MHD_ERR_HIP = -3,         /* a HIP runtime call failed                    */
    MHD_ERR_NONPHYSICAL = -4, /* rho <= 0, p <= 0 or non-finite state seen    */
    MHD_ERR_UNSUPPORTED = -5  /* valid but not implemented combination        */
} mhd_status;

enum { MHD_F32 = 0, MHD_F64 = 1 };       /* storage and bulk arithmetic */
enum { MHD_HLL = 0, MHD_HLLD = 1 };      /* Riemann solver              */
enum { MHD_MINMOD = 0, MHD_MC = 1, MHD_WENOZ = 2 }; /* reconstruction */
enum { MHD_PERIODIC = 0, MHD_OUTFLOW = 1 }; /* boundary per face        */
/* MHD_FLAG_ADJOINT: mhd_init also allocates the adjoint scratch (an FP64
 * stage cotangent, 9 doubles per cell); mhd_step_adjoint needs it.  The
 * adjoint covers the PLM reconstructions with SSP-RK2 and cell-centred B
 * only: with WENO-Z, SSP-RK3 or constrained transport mhd_init returns
 * MHD_ERR_UNSUPPORTED for this flag. */
enum { MHD_FLAG_ADJOINT = 1 };

typedef struct {
    int32_t ndim;      /* 1, 2 or 3; axes >= ndim must have n = 1            */
    int32_t dtype;     /* MHD_F32 or MHD_F64                                 */
    int32_t riemann;   /* MHD_HLL or MHD_HLLD                                */
    int32_t limiter;   /* MHD_MINMOD, MHD_MC (PLM) or MHD_WENOZ              */
    int64_t n[3];      /* interior cells nx, ny, nz; n >= 2 on active axes   */
    double lo[3];      /* domain lower corner                                */
    double hi[3];      /* domain upper corner; dx_d = (hi-lo)/n              */
    int32_t bc[3][2];  /* per axis, low and high face; periodic on both or none */
    int32_t glm;       /* 1: GLM cleaning on; 0: psi inert, B_n = (B_L+B_R)/2 */
    int32_t flags;     /* MHD_FLAG_* bits; other bits must be 0              */
    double gamma;      /* adiabatic index > 1                                */
    double cfl;        /* Courant number C in (0, 1]                         */
    double glm_alpha;  /* GLM damping parameter alpha >= 0                   */
    int32_t time_order; /* 2: SSP-RK2, 3: SSP-RK3                            */
    int32_t ct;        /* 1, 2: constrained transport (3D, periodic, glm = 0) */
                       /* with the mean (1) or upwind (2) edge EMF           */
} mhd_config;

/* Create a context for one grid on the current HIP device.
 * Paper: section 3.2 "Porting of gPLUTO" (the steps of a Runge-Kutta stage
 * and the choice of one divergence-control algorithm) and section 4.2
 * "Results for gPLUTO" (the benchmark scheme: WENO-Z, HLLD, RK3; constrained
 * transport in the weak-scaling and GLM cleaning in the strong-scaling
 * runs).  The config fixes the scheme at this call.
 * hip_stream is a hipStream_t (NULL = the null stream).  Allocates the
 * library scratch (the only allocation besides mhd_timing_start).
 * Returns MHD_ERR_ARG for an invalid config (bad ndim, n, bounds, dtype,
 * solver, limiter, time_order, ct not 0, 1 or 2, ct with glm = 1, mixed
 * periodic/outflow on one axis, gamma <= 1, cfl not in (0,1],
 * glm_alpha < 0), MHD_ERR_UNSUPPORTED for MHD_FLAG_ADJOINT with WENO-Z,
 * SSP-RK3 or ct = 1 or 2 and for ct = 1 or 2 on a grid that is not 3D and
 * periodic,
 * MHD_ERR_NO_DEVICE when no gfx950 device is current, MHD_ERR_HIP when an
 * allocation fails.  *out is NULL on failure. */
mhd_status mhd_init(const mhd_config *cfg, void *hip_stream, mhd_ctx **out);

/* Release the context and its scratch (syncs).  NULL is ignored.  The
 * caller's buffers are not touched. */
void mhd_destroy(mhd_ctx *ctx);

/* Change the stream later calls enqueue on (work already enqueued stays on
 * the old stream; the caller orders the two).  MHD_ERR_ARG for a NULL ctx. */
mhd_status mhd_set_stream(mhd_ctx *ctx, void *hip_stream);

/* Primitive -> conserved map (async): the inverse of the conservative ->
 * primitive mapping that section 3.2 "Porting of gPLUTO" lists among the
 * steps of a stage, used to set up a state.  V: device double
 * [9][nz][ny][nx] holding (rho, vx, vy, vz, p, Bx, By, Bz, psi), caller
 * owned, read only; U: device state of the context dtype, caller owned,
 * written.  E = p/(gamma-1) + rho|v|^2/2 + |B|^2/2, computed in FP64 and
 * rounded once to the state type.  With constrained transport V is
 * [12][nz][ny][nx] with the face field in 9..11 (its discrete divergence
 * is the caller's to make zero); the cell field of U, and the B in E, are
 * the face means, whatever V holds in 5..7.  MHD_ERR_ARG for NULL
 * buffers; V is not validated (a non-physical V shows at the next step). */
mhd_status mhd_prim_to_cons(mhd_ctx *ctx, const double *V, void *U);

/* CFL reduction of a state (syncs): the time step of the Runge-Kutta
 * integration of section 3.2 "Porting of gPLUTO" (the paper prints no
 * stability condition; this is the Courant condition on the fast
 * magnetosonic speed).  U: device state of the context dtype, caller owned,
 * read only.  out (host, 2 doubles): out[0] = C / max (|v_d|+c_f,d)/dx_d
 * (not clipped to any end time), out[1] = c_h = max (|v_d|+c_f,d), the
 * GLM speed for the next step.  Each cell's state is converted to FP64
 * before the speeds are formed.  The result is kept apart from the
 * reductions of the last mhd_step (mhd_step_info and mhd_get_sums still
 * return those).  Returns MHD_ERR_NONPHYSICAL if any cell is non-physical
 * (or a kernel flagged one since the last syncing call), MHD_ERR_ARG for
 * NULL buffers. */
mhd_status mhd_cfl_dt(mhd_ctx *ctx, const void *U, double out[2]);

/* One Runge-Kutta step (async): section 3.2 "Porting of gPLUTO" (per
 * stage: boundary calculation, conservative -> primitive map,
 * reconstruction of interface values, Riemann fluxes, right-hand side) with
 * the divergence control and benchmark scheme of section 4.2 "Results for
 * gPLUTO".  SSP-RK2 (time_order 2):
 *   U1     = Un + dt L(Un)
 *   U_next = (Un + U1 + dt L(U1)) / 2,  then psi <- psi * damp;
 * SSP-RK3 (time_order 3):
 *   U1     = Un + dt L(Un)
 *   U2     = 3/4 Un + 1/4 (U1 + dt L(U1))
 *   U_next = 1/3 Un + 2/3 (U2 + dt L(U2)),  then psi <- psi * damp;
 * with L the flux divergence built with the given c_h (U2 lives in library
 * scratch).  Un: device state, caller owned, read only; U_next: device
 * state, caller owned, written, must not alias Un.  U1_out (may be NULL)
 * receives the stage-1 state, which the adjoint reuses; otherwise library
 * scratch is used.  The step also reduces, on U_next, the CFL maxima and
 * the FP64 sums read back by mhd_step_info and mhd_get_sums.  With FP64
 * states every cell's speeds are formed in FP64; with FP32 states each
 * thread picks, by FP32 estimates, the cells of its column with the
 * largest speeds and reports their FP64 speeds, so the maxima are FP64
 * speeds of actual cells, within the estimate's rounding (~1e-6 relative)
 * of the all-FP64 maxima.  MHD_ERR_ARG (nothing enqueued) for NULL or
 * aliased buffers, dt not finite and > 0, c_h not finite and > 0 with
 * GLM, damp not in (0, 1].  A non-physical cell met by a kernel is
 * reported by the next syncing call. */
mhd_status mhd_step(mhd_ctx *ctx, const void *Un, void *U_next, void *U1_out, double dt,
                    double c_h, double damp);

/* Reductions of the last mhd_step output (syncs).  The paper defines no
 * diagnostics; these are the conserved totals of the conservation law whose
 * right-hand side section 3.2 "Porting of gPLUTO" computes, and the CFL
 * maxima of the next step.  out (host, 11 doubles):
 *   out[0] = C / max (|v_d|+c_f,d)/dx_d, out[1] = c_h (as mhd_cfl_dt),
 *   out[2..10] = FP64 sums over cells of U_q times the cell volume.
 * MHD_ERR_ARG if no step has run; MHD_ERR_NONPHYSICAL if a kernel saw a
 * non-physical cell since the last syncing call. */
mhd_status mhd_step_info(mhd_ctx *ctx, double out[11]);

/* FP64 conservation sums of the last mhd_step output (syncs): the conserved
 * totals of the conservation law of section 3.2 "Porting of gPLUTO"
 * (rho, m, E and B are constant on periodic grids up to rounding, psi
 * decays).  out (host, 9 doubles) = sum over cells of U_q times the cell
 * volume, q = rho, m_x, m_y, m_z, E, B_x, B_y, B_z, psi, accumulated in
 * FP64 in a fixed order (identical run to run).  The same values as
 * out[2..10] of mhd_step_info.  MHD_ERR_ARG for a NULL buffer or if no step
 * has run; MHD_ERR_NONPHYSICAL if a kernel saw a non-physical cell since
 * the last syncing call. */
mhd_status mhd_get_sums(mhd_ctx *ctx, double out[9]);

/* mhd_step for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  No
 * context: the config (validated as by mhd_init) is passed on each call,
 * and the reduction partials, result words and non-physical flag live in
 * a static device array of the library (about 1.4 MB per device, held until
 * the process ends).  Nothing is allocated (no hipMalloc, hipFree or
 * allocating library call); on the first call on a device (or at mhd_init
 * on it) the library looks up that device's copy of the array.
 * Same step, kernels and results as mhd_step (bit for bit), for SSP-RK2
 * (time_order 2) without constrained transport (MHD_ERR_UNSUPPORTED
 * otherwise: those need state-sized scratch) and flags = 0.  U1_out (the
 * stage-1 state) is required; Un, U_next, U1_out are distinct device
 * buffers of the config's dtype, caller owned.  Limit: the stage grid
 * must fit the static partials (16384 workgroups: 512^3 needs 8192);
 * larger grids get MHD_ERR_ARG before anything is enqueued.  info (host,
 * 11 doubles) may be NULL: then the call is async and capturable (the flag
 * is cleared by a kernel, not a memset); otherwise it syncs the stream and
 * returns in info what mhd_step_info would (dt of the next step, c_h, FP64
 * sums), or MHD_ERR_NONPHYSICAL if a kernel of this call saw a non-physical
 * cell.  Every call on a device shares that device's array, which keeps the
 * last call's contents: calls that overlap on one device (several streams
 * or host threads) race and must be serialised by the caller.  Errors carry
 * no text (there is no context for mhd_last_error). */
mhd_status mhd_step_noalloc(const mhd_config *cfg, void *hip_stream, const void *Un, void *U_next,
                            void *U1_out, double dt, double c_h, double damp, double info[11]);

/* Adjoint of mhd_step (async).  The paper has no adjoint: this is the
 * transpose of the linearisation of the Runge-Kutta step of section 3.2
 * "Porting of gPLUTO" as mhd_step computes it (PLM, HLL or HLLD, GLM,
 * SSP-RK2).  Given lam_next = dJ/dU_next (device double, caller owned, read
 * only), write lam_n = dJ/dUn (device double, caller owned) for the same
 * dt, c_h, damp, which are treated as constants (not differentiated):
 *   mu = D lam_next (psi times damp), lam1 = mu/2 + (dt/2) J_L(U1)^T mu,
 *   lam_n = mu/2 + lam1 + dt J_L(Un)^T lam1.
 * U1 is the stage-1 state of that step (from mhd_step's U1_out) or NULL to
 * recompute it into library scratch.  lam_n must not alias lam_next or a
 * state buffer.  The context needs MHD_FLAG_ADJOINT (else MHD_ERR_ARG).
 * Kinks (limiter switches, Riemann fan regions) take the branch the
 * forward step took; at a tie |a| = |b| != 0 the minmod derivative follows
 * the left difference; where a limiter argument is exactly zero the
 * derivative is the one a central difference sees (1/2 toward each zero
 * argument for minmod, 1 for MC).  Local derivative arithmetic is in the
 * state type; the per-cell gathering and the lambda combinations are FP64.
 * MHD_ERR_ARG (nothing enqueued) for NULL or aliased buffers and the dt,
 * c_h, damp conditions of mhd_step. */
mhd_status mhd_step_adjoint(mhd_ctx *ctx, const void *Un, const void *U1, const double *lam_next,
                            double *lam_n, double dt, double c_h, double damp);

/* Adjoint of mhd_prim_to_cons (async): lam_V = (dU/dV)^T lam_U, all device
 * double, caller owned, V the primitive state the forward map was applied
 * to (the transpose of the set-up map above; the paper has no adjoint).
 * MHD_ERR_ARG for NULL buffers or lam_V aliasing lam_U;
 * MHD_ERR_UNSUPPORTED on a constrained-transport context. */
mhd_status mhd_prim_to_cons_adjoint(mhd_ctx *ctx, const double *V, const double *lam_U,
                                    double *lam_V);

/* Kernel timing with HIP events on the context stream (measurement, not a
 * step of the method; section 3.1 "Profiling activity" profiles every
 * kernel of the port).  mhd_timing_start creates 4 events per step for up
 * to `capacity` (1 .. 2^20) later mhd_step calls (the only allocation
 * besides mhd_init, made here) and starts recording; each mhd_step then
 * records an event before its first stage kernel, before its last stage
 * kernel, after it and after the final reduction.  mhd_timing_stop (syncs)
 * writes to out (host, 4 doubles): out[0] = steps recorded, out[1..3] =
 * total milliseconds of the stage kernels before the last one (one with
 * SSP-RK2, two with SSP-RK3), the last stage kernel (which also reduces
 * the CFL maxima and sums) and the final reduction over those steps, then
 * frees the events.  Steps beyond capacity are not timed.  MHD_ERR_ARG for
 * a capacity out of range or a NULL buffer; MHD_ERR_HIP if event creation
 * fails. */
mhd_status mhd_timing_start(mhd_ctx *ctx, int32_t capacity);
mhd_status mhd_timing_stop(mhd_ctx *ctx, double out[4]);

/* Static text naming a status (never NULL, not to be freed). */
const char *mhd_status_string(mhd_status st);

/* Text of the last error on this context (never NULL; owned by the
 * context, valid until its next call or mhd_destroy). */
const char *mhd_last_error(const mhd_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* MHD_H */
