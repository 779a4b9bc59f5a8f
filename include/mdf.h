/*
 * mdf.h -- C ABI of the MI355X MDF-FDLBM library (libmdf.so).
 *
 * The library advances the multiple-distribution-function finite-difference
 * lattice Boltzmann method (Chen, Chai, Zhao & Shi) for the incompressible
 * Navier-Stokes equations written as the convection-diffusion system of
 * eq. 2.1.2, on a 2D grid, in FP64, on one AMD Instinct MI355X (gfx950).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - All arrays are FP64 and, unless a call says otherwise, DEVICE memory.
 *  - A field is ny*nx values, x fastest:  a[y*nx + x].
 *  - A distribution array is 10 fields, plane index alpha*5 + j with
 *    alpha = 0 (u equation), 1 (v equation) and the D2Q5 velocities
 *    c_j = c*{(0,0),(1,0),(0,1),(-1,0),(0,-1)} of eq. 3.1.0.
 *  - Periodic axes place nodes at x_i = i*L/N; wall axes put nodes on both
 *    walls, x_i = X(i/(N-1)).
 *  - The caller owns all device memory.  mdf_init carves the caller's
 *    workspace (at least mdf_workspace_size bytes, 256-byte aligned) and
 *    keeps using it until mdf_destroy; the caller keeps it alive that long.
 *  - Calls that take an mdf_ctx enqueue work on the context's HIP stream
 *    and return without waiting, except where a call says it synchronises.
 *  - No call throws or aborts.  Every call returns an mdf_status; a short
 *    description of the last failure is available from mdf_last_error.
 *    A call that returns an error leaves the context's state unchanged
 *    unless it says otherwise.
 */
#ifndef MDF_H
#define MDF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mdf_ctx mdf_ctx;
typedef struct mdf_batch mdf_batch;

typedef enum {
    MDF_OK = 0,
    MDF_EINVAL = -1,    /* a parameter or argument is out of range            */
    MDF_ESTATE = -2,    /* the context cannot do this now                      */
    MDF_EDEVICE = -3,   /* a HIP runtime call failed                           */
    MDF_EUNSTABLE = -4  /* diagnostics found a non-finite value in the state   */
} mdf_status;

typedef enum { MDF_BC_PERIODIC = 0, MDF_BC_WALL = 1 } mdf_bc;

/* Problem parameters (Sec. 2 and the set-ups of Sec. 4).  Host memory. */
typedef struct {
    int32_t nx, ny;          /* nodes per axis, 5..32768 (wall axes include the wall nodes)          */
    double  lx, ly;          /* domain lengths                                                     */
    double  nu;              /* kinematic viscosity nu = c_s^2/s (eq. 2.3.14); the consistency K
                                of the power law when pl_n != 1                                     */
    double  pl_n;            /* power-law index: 1 (Newtonian), 0.5 or 1.5                          */
    double  nu_min, nu_max;  /* clamp of the local power-law viscosity (ignored when pl_n == 1)     */
    double  cfl;             /* dt = cfl * dx_min / c (eq. 3.1)                                      */
    double  c;               /* lattice speed |c_j|                                                  */
    double  eta;             /* weight of the central part of the mixed scheme (eq. 2.2.12), [0,1]  */
    double  s_ratio;         /* s'/s: rate of the non-conserved, non-flux moments (Sec. 3.1)        */
    int32_t bc_x, bc_y;      /* mdf_bc per axis                                                      */
    double  lid_u;           /* tangential speed of the wall at y = ly (corners excluded)           */
    double  fx, fy;          /* uniform body force F_alpha (eq. 2.2.6)                               */
    const double* inv_dx_x;  /* HOST, nx values: 1/(X'(xi_i) dxi) of a mapped x axis, or NULL (uniform) */
    const double* inv_dx_y;  /* HOST, ny values, same for y, or NULL                                */
    double  dx_min;          /* smallest node spacing; required when either metric array is given */
    const double* force_x;   /* HOST, ny*nx values (x fastest) added to fx at each node: a steady body
                                force field F(x) (eq. 2.2.6, Secs. 4.1-4.2), or NULL (none)          */
    const double* force_y;   /* HOST, ny*nx values added to fy, or NULL                            */
    /* Time dependence of the body force.  0: steady.  1: F(x, t) = F(x) cos(force_omega t +
     * force_phase), F(x) the uniform part plus the field above, t = (steps taken) * dt; the
     * full step then carries the (dt^2/2) d_t F term of eq. 2.3.24 and the half step h F(t)
     * (eq. 2.3.25).  force_omega and force_phase must be finite.  Batches take only 0. */
    double  force_omega;     /* angular frequency of the force (time units of nu and dt)          */
    double  force_phase;     /* phase at t = 0                                                      */
    int32_t force_harmonic;  /* 0 or 1                                                              */
    /* HOST, 4 planes of ny*nx values (x fastest), or NULL: a general (non-separable) coordinate
     * transformation x = X(i, j), y = Y(i, j) of the node indices, given by its inverse Jacobian
     * in node units at every node: d i/dx, d i/dy, d j/dx, d j/dy.  Transport then follows the
     * chain rule, c_j . grad = U d/di + V d/dj with the contravariant components U = c_j . grad i
     * and V = c_j . grad j, each index derivative by the mixed scheme of eqs. 2.2.12-2.2.13
     * upwinded by its own component's sign (Sec. 1 names the coordinate transformation and the
     * trapezoidal cavity; the formulas are this library's reading).  Walls lie on the index lines
     * i = 0, nx-1 and j = 0, ny-1.  Excludes inv_dx_x / inv_dx_y and needs dx_min > 0; the
     * values must be finite with a non-zero Jacobian.  Runs on the tiled step (variant 0)
     * only; batches and the closure take no general mapping. */
    const double* metric;
    /* HOST, ny*nx values (x fastest), or NULL for R = 0: the mass source R of eq. 2.1.1 (the
     * alpha = 0 source of eq. 2.1.2), steady.  It enters the pressure of eq. 2.3.23, which on the
     * stored distributions phi = f + kappa Lambda~ (f - f^eq) becomes the plain sum plus
     * R (nu + kappa c_s^2)/2; the alpha = 0 equation itself is not carried (Remark 1).  Needs a
     * Newtonian fluid (pl_n = 1) and finite values; runs on the tiled step (variant 0) only;
     * batches take none. */
    const double* mass_source;
} mdf_params;

/* Bytes of device workspace a context for these parameters needs, or 0 if the
 * parameters are invalid.  Depends only on nx, ny and whether a force field
 * (force_x or force_y), a general mapping (metric) or a mass source is given. */
size_t mdf_workspace_size(const mdf_params* p);

/* Create a context and initialise the state f_hat = f^eq(u0, v0, p0) of
 * eq. 2.2.5 at every node (the initialisation of Sec. 4), then apply the wall
 * rule so that wall nodes carry the wall velocity.
 *   p          host parameters; metric arrays are copied, p may be freed after
 *   u0,v0,p0   DEVICE fields (ny*nx, x fastest) of velocity and pressure
 *   workspace  DEVICE memory of at least mdf_workspace_size(p) bytes, 256-byte aligned
 *   ws_bytes   its size
 *   hip_stream hipStream_t the context enqueues on (NULL = default stream)
 *   out        receives the context
 * Synchronises the stream before returning.  Returns MDF_EINVAL when nu <= 0,
 * cfl <= 0, c <= 0, eta outside [0,1], an axis has fewer than 5 or more than
 * 32768 nodes, pl_n is
 * not 1, 0.5 or 1.5, the power-law clamp is empty, metrics come without dx_min,
 * a metric, force or mass-source value is not finite, a mass source comes with
 * a power-law fluid, or the workspace is too small or misaligned.  The metric,
 * force and mass-source arrays are copied; p may be freed after. */
mdf_status mdf_init(const mdf_params* p, const double* u0, const double* v0, const double* p0,
                    void* workspace, size_t ws_bytes, void* hip_stream, mdf_ctx** out);

/* Advance n time steps of Sec. 2.2, Steps (1)-(4): collision at t (eqs. 2.2.14,
 * 2.2.15), half step (eq. 2.3.25), collision at t+h (eq. 2.2.16) and full step
 * (eq. 2.3.24), with the mixed difference of eqs. 2.2.12-2.2.13.  n >= 0. */
mdf_status mdf_step(mdf_ctx* ctx, int64_t n);

/* Velocity and pressure of the current state (eqs. 2.3.4 and 2.3.23, with the
 * run's mass source R, zero without one) into caller-owned DEVICE fields (ny*nx
 * each); any pointer may be NULL. */
mdf_status mdf_moments(mdf_ctx* ctx, double* u, double* v, double* p);

/* Local quantities from the first moment of the non-equilibrium part
 * (Sec. 2.4, eqs. 2.4.1-2.4.5).  Bit k of mask selects plane k of the list
 *   0 du/dx  1 du/dy  2 dv/dx  3 dv/dy  4 div u  5 Sxx  6 Sxy  7 Syy
 *   8 sigma_xx  9 sigma_xy  10 sigma_yy  11 Omega_xy  12 vorticity  13 nu
 * and the selected planes are written consecutively (in list order) to the
 * DEVICE array out, ny*nx values each.  mask must be non-zero and < 2^14. */
mdf_status mdf_derived(mdf_ctx* ctx, double* out, uint32_t mask);

/* Diagnostics of the current state into HOST out[8]: sum u, sum v,
 * KE = 1/2 sum |u|^2 dA, enstrophy = 1/2 sum omega^2 dA, max |u|, max |div u|
 * by central differences over non-wall nodes, number of non-finite state
 * values, sum dA (dA = node area).  Synchronises the stream.  Returns
 * MDF_EUNSTABLE (with out filled) when the state holds a non-finite value. */
mdf_status mdf_diagnostics(mdf_ctx* ctx, double out[8]);

/* Copy the state out to / in from a caller-owned DEVICE distribution array
 * (10*ny*nx values, layout above).  mdf_load replaces the state; the step
 * counter is kept. */
mdf_status mdf_save(mdf_ctx* ctx, double* f);
mdf_status mdf_load(mdf_ctx* ctx, const double* f);

/* Restart from the fields u0, v0, p0 (DEVICE, ny*nx doubles each, x fastest):
 * the state becomes f^eq(u0, v0, p0) at every node, as at mdf_init; the step
 * counter is kept.  Asynchronous on the context's stream. */
mdf_status mdf_set_fields(mdf_ctx* ctx, const double* u0, const double* v0, const double* p0);

/* Kernel selection for the time step: variant 0 = tiled step (two tiled
 * passes: Steps (1)-(3), then Step (4); any grid mapping and source),
 * 1 = fused single-pass strip kernel with one wave per strip (default for a
 * power-law fluid), 2 = fused single-pass strip kernel with one wave per
 * velocity component (default for a Newtonian fluid).
 * tile_w (columns per strip incl. the 8-column halo, one wave per 64; 64,
 * 128 or 256, variant 1 only), seg_h and prefetch (rows loaded ahead, 2 or 3)
 * apply to the fused
 * variants; 0 keeps the current value.  With a force field only variants 0
 * and 1 exist, variant 1 with tile_w 64 and prefetch 2 (the default then).  seg_h > 0 cuts every strip into
 * segments of seg_h rows; seg_h = -r (r = 1..4; -1 is the default) selects
 * the balanced partition over r rounds of waves on the device (one wave per
 * SIMD per round; a 128-lane strip takes two), with fewer rows in the
 * segments next to walls, whose rows cost more; seg_h < -4 is MDF_EINVAL.
 * Changing the variant or the shape rebuilds that partition (a short
 * synchronous upload on the context's stream).  Results agree to rounding
 * whatever the choice.  A general mapping or a mass source has variant 0 only
 * (MDF_EINVAL for any other). */
mdf_status mdf_set_kernel(mdf_ctx* ctx, int32_t variant, int32_t tile_w, int32_t seg_h, int32_t prefetch);

/* Scalings (0..10) of the measured extra per-row cost of segments next to
 * an x wall and next to a y wall in the balanced partition (1 = measured
 * costs, 0 = all rows alike); rebuilds the partition (synchronous). */
mdf_status mdf_set_partition_costs(mdf_ctx* ctx, double x_wall_scale, double y_wall_scale);

/* Autotuner for this context: times every fused kernel (variant 1 with
 * tile_w 64, 128 and 256, and variant 2 for a Newtonian fluid; only variant 1
 * with tile_w 64 and prefetch 2 under a force field; a general mapping or a
 * mass source has only variant 0, which it reports without timing), prefetch
 * depth (2, 3) and eight scalings (0.3..3.5) of the
 * wall-row cost factors of the one-round balanced partition over `steps`
 * steps of the run itself, times the three fastest again over 4 x `steps`
 * steps, restores the state and step count after each run (a spare state-sized
 * buffer of the workspace holds the copy), and keeps the fastest of the
 * second timing.  choice (host, may be NULL; 6 doubles) receives {variant,
 * prefetch, x-wall scale, y-wall scale, milliseconds per step, tile_w}.
 * Synchronises.  Results do not depend on the choice (to rounding). */
mdf_status mdf_autotune(mdf_ctx* ctx, int32_t steps, double* choice);

/* Host-only preview of the balanced partition the fused variant (1 or 2)
 * uses for these parameters with `slots` workgroups per round (the library
 * takes 4 waves per compute unit, so 4 * CUs * 64 / tile_w workgroups):
 * writes (strip, first row, end row) triples to out[3*i..3*i+2], strips
 * being the tile_w-8 column slices of the grid (tile_w 64, 128 or 256 for
 * variant 1; variant 2 always uses 64), and returns the number of segments,
 * or 0 for invalid input or when cap is too small.  No device work.  On a
 * grid with x walls, variant 1 at 128 or 256 lanes does not launch this
 * plan once the grid is at least 128 columns wide: it runs the 56 columns
 * next to each x wall as single-wave tasks, several to a workgroup, and
 * cuts only the columns between them into strips. */
int32_t mdf_plan_segments(const mdf_params* p, int32_t variant, int32_t tile_w, int32_t slots, int32_t* out,
                          int32_t cap);

double      mdf_dt(const mdf_ctx* ctx);          /* time step, or 0 for NULL       */
int64_t     mdf_steps(const mdf_ctx* ctx);       /* steps taken since mdf_init     */
const char* mdf_last_error(const mdf_ctx* ctx);  /* never NULL; "" when none       */
void        mdf_destroy(mdf_ctx* ctx);           /* synchronises; NULL is a no-op  */

/* ---------------------------------------------------------------------------
 * Learned coarse-grid closure (a project addition, not in the paper): a
 * four-layer periodic 3x3 convolutional network, channels 2-32-32-32-2, ReLU
 * after the first three layers, on BF16 matrix cores with FP32 accumulation.
 * Input x = in_scale*(u, v) per node; output (du, dv) = out_scale*y.
 * Parameters: one FP32 DEVICE vector of mdf_cnn_param_count() values, layer
 * by layer W[9][cin][cout] (tap t = 3*(dy+1) + (dx+1)) then b[cout].
 * Fields: DEVICE FP64 arrays [batch][2][h][w] (u plane then v plane, x
 * fastest).  The caller owns a DEVICE workspace (256-byte aligned,
 * mdf_cnn_workspace_size bytes) that keeps the activations of the last
 * forward call for the backward call.  Asynchronous on `hip_stream`. */

int32_t    mdf_cnn_param_count(void);
/* 0 unless batch >= 1, h >= 3, w a multiple of 32 and batch*h*w <= 2^26. */
size_t     mdf_cnn_workspace_size(int32_t batch, int32_t h, int32_t w);
mdf_status mdf_cnn_forward(void* ws, size_t ws_bytes, const float* params, int32_t batch, int32_t h, int32_t w,
                           const double* uv, double in_scale, double out_scale, double* duv, void* hip_stream);
/* The forward pass of mdf_cnn_forward for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): no workspace argument; the activations live in a fixed device
 * array of the library (about 10 MiB per GPU, held until the process ends),
 * so batch*h*w may not exceed MDF_CNN_NOALLOC_MAX_PIXELS (one 128 x 128
 * field); larger inputs are MDF_EINVAL.  Same arguments, rounding and results
 * as mdf_cnn_forward; calls no allocator.  Every call on a GPU shares that
 * GPU's array, so calls that overlap on one GPU (other streams, other host
 * threads) race; the array keeps the last call's contents, none of which a
 * call reads before writing it.  The array used is that of the device that
 * runs hip_stream (the current device for the null stream).  Asynchronous on
 * hip_stream. */
#define MDF_CNN_NOALLOC_MAX_PIXELS 16384
mdf_status mdf_cnn_forward_noalloc(const float* params, int32_t batch, int32_t h, int32_t w, const double* uv,
                                   double in_scale, double out_scale, double* duv, void* hip_stream);
/* Gradient of L = mean((y - target/out_scale)^2) over pixels and both
 * channels with respect to every parameter, into grad (DEVICE FP32, one
 * value per parameter), for the activations of the last forward call on ws;
 * loss (DEVICE double, may be NULL) receives L. */
mdf_status mdf_cnn_backward(void* ws, size_t ws_bytes, const float* params, int32_t batch, int32_t h, int32_t w,
                            const double* duv_target, double out_scale, float* grad, double* loss, void* hip_stream);
/* Copies (DEVICE; any pointer may be NULL) of layer `layer`'s (1..4) BF16
 * input activation ([P][8] for layer 1, [P][32] otherwise, P = batch*h*w
 * pixels, channels last) and FP32 pre-activation z ([P][32], [P][2] for
 * layer 4) from the last forward call, and of the loss gradient at z from
 * the last backward call, BF16 and FP32 ([P][32] each, channels beyond the
 * layer's outputs zero).  For checking each layer on its own. */
mdf_status mdf_cnn_layer_io(const void* ws, size_t ws_bytes, int32_t batch, int32_t h, int32_t w, int32_t layer,
                            uint16_t* in_bf16, float* z, uint16_t* g_bf16, float* g, void* hip_stream);
/* Adam step `step` (1, 2, ...) on n FP32 parameters with first/second moment
 * buffers m, v (DEVICE, zero before step 1). */
mdf_status mdf_cnn_adam(float* params, const float* grad, float* m, float* v, int32_t n, float lr, float beta1,
                        float beta2, float eps, int32_t step, void* hip_stream);
/* Correct the velocity of a periodic, uniform-grid run in place:
 * f_hat += f^eq(u + du, P) - f^eq(u, P) (eq. 2.2.5), so that the moments
 * become (u + du, v + dv) with P unchanged.  Guard: the correction is made
 * only if the corrected field's kinetic energy sum |u|^2/2 does not exceed
 * ke_ref and its largest central-difference divergence |du/dx + dv/dy| does
 * not exceed div_factor times that of the current field (both finite);
 * otherwise the state is left alone and *fell_back = 1.  du, dv: DEVICE
 * [ny][nx], or both NULL to only measure the current field.  *ke_out and
 * *div_out (host, may be NULL) receive the kinetic energy and divergence of
 * the field the call leaves.  Synchronises the context's stream. */
mdf_status mdf_closure_apply(mdf_ctx* ctx, const double* du, const double* dv, double ke_ref, double div_factor,
                             double* ke_out, double* div_out, int32_t* fell_back);

/* The same guarded correction without any host synchronisation, for a
 * rollout that keeps the device busy: mdf_closure_begin sets the reference
 * energy ke_ref (DEVICE, in the context's workspace) to the current field's
 * kinetic energy and zeroes the counters; each mdf_closure_apply_async
 * evaluates the guard on the device (corrected energy <= ke_ref and largest
 * divergence <= div_factor times the current field's, both finite), applies
 * the correction only if it passes, counts a fall-back if not, and sets
 * ke_ref to the energy of the field it leaves.  du, dv: DEVICE [ny][nx], not
 * NULL.  mdf_closure_stats synchronises and writes {ke_ref, fall-backs,
 * windows since mdf_closure_begin} to HOST out[3].  The diagnostics and the
 * synchronous mdf_closure_apply share the scratch these calls use, but not
 * their state.  Periodic uniform grids only (else MDF_EINVAL). */
mdf_status mdf_closure_begin(mdf_ctx* ctx);
mdf_status mdf_closure_apply_async(mdf_ctx* ctx, const double* du, const double* dv, double div_factor);
mdf_status mdf_closure_stats(mdf_ctx* ctx, double out[3]);

/* ---------------------------------------------------------------------------
 * Batches: many independent instances of the same method advanced together
 * (a project addition, not in the paper).  Each instance has its own grid
 * size, viscosity and therefore its own time step dt = CFL dx / c (eq. 3.1)
 * and relaxation rates (Sec. 2.2); one mdf_batch_step advances every instance
 * by one of its own steps with ONE kernel launch covering all instances.  All
 * instances must be periodic on both axes, on uniform grids, and share pl_n.
 *
 * The caller owns the workspace (device, 256-byte aligned, at least
 * mdf_batch_workspace_size bytes) and keeps it alive until
 * mdf_batch_destroy; it holds the per-instance constants, the launch plan,
 * two state buffers and a backup buffer for the autotuner.  The library
 * creates one private stream and two events per batch (for graph replay). */

/* Bytes of workspace for `count` instances ps[0..count-1]; 0 if invalid. */
size_t mdf_batch_workspace_size(const mdf_params* ps, int32_t count);

/* u0s[i], v0s[i], p0s[i]: host arrays of DEVICE pointers to instance i's
 * initial fields (ny_i*nx_i doubles, x fastest), read before return.
 * Synchronises.  On error *out is NULL and nothing needs freeing. */
mdf_status mdf_batch_init(const mdf_params* ps, int32_t count, const double* const* u0s, const double* const* v0s,
                          const double* const* p0s, void* workspace, size_t ws_bytes, void* hip_stream,
                          mdf_batch** out);

/* n steps of every instance, one launch per step, asynchronous on the
 * batch's stream. */
mdf_status mdf_batch_step(mdf_batch* b, int64_t n);

/* The same n steps replayed from a captured HIP graph (captured on first use
 * for this n and starting buffer, then reused).  The replay runs on the
 * batch's private stream, ordered after earlier work on the batch's stream and
 * before later work on it.  Results are identical to mdf_batch_step. */
mdf_status mdf_batch_step_graph(mdf_batch* b, int64_t n);

/* Kernel for the batch: variant 1 (one wave per strip; tile_w 64, 128 or 256
 * lanes per strip, one wave per 64) or 2 (one wave per velocity component;
 * tile_w 64), tile_w 0 meaning 64; prefetch 2 or 3 rows;
 * `rounds` (1..8) rounds of waves in the balanced partition.  Other values
 * are MDF_EINVAL.  Rebuilds the plan (synchronous). */
mdf_status mdf_batch_set_kernel(mdf_batch* b, int32_t variant, int32_t tile_w, int32_t prefetch, int32_t rounds);

/* Autotuner: times each candidate kernel (variant, tile_w, prefetch, rounds
 * 1..3) over `steps` steps on the batch itself, then the three fastest again
 * over 4 x `steps`, restores the state and step count after each run,
 * selects the fastest of the second timing and writes {variant, prefetch,
 * rounds, tile_w} to choice[0..3] (may be NULL).  Synchronises.  Results do
 * not depend on the choice (to rounding). */
mdf_status mdf_batch_autotune(mdf_batch* b, int32_t steps, int32_t* choice);

/* Instance i's moments (DEVICE planes of ny_i*nx_i doubles, NULL skips a
 * plane) and dense state copy (DEVICE, 10*ny_i*nx_i doubles, same order as
 * mdf_save); asynchronous on the batch's stream. */
mdf_status mdf_batch_moments(mdf_batch* b, int32_t i, double* u, double* v, double* p);
mdf_status mdf_batch_save(mdf_batch* b, int32_t i, double* f);
/* Instance i's local quantities of Sec. 2.4 (eqs. 2.4.1-2.4.5), planes and
 * mask exactly as mdf_derived (DEVICE out, ny_i*nx_i doubles per selected
 * plane); asynchronous on the batch's stream. */
mdf_status mdf_batch_derived(mdf_batch* b, int32_t i, double* out, uint32_t mask);
/* Instance i's diagnostics into HOST out[8], as mdf_diagnostics; synchronises
 * the batch's stream; MDF_EUNSTABLE (out filled) on a non-finite value. */
mdf_status mdf_batch_diagnostics(mdf_batch* b, int32_t i, double out[8]);

double      mdf_batch_dt(const mdf_batch* b, int32_t i);   /* instance time step, 0 if invalid */
int64_t     mdf_batch_steps(const mdf_batch* b);          /* steps since mdf_batch_init       */
int32_t     mdf_batch_workgroups(const mdf_batch* b);     /* workgroups of one step launch    */
const char* mdf_batch_last_error(const mdf_batch* b);     /* never NULL                       */
void        mdf_batch_destroy(mdf_batch* b);               /* synchronises; NULL is a no-op    */

/* ---------------------------------------------------------------------------
 * Von Neumann screen (Sec. 3.1): spectral radius of the growth matrix of one
 * time step (Steps (1)-(4), the mixed difference of eqs. 2.2.12-2.2.13),
 * linearised about the uniform state (u0, v0), for the Fourier modes
 * exp(i (theta_x x/dx + theta_y y/dy)) of a periodic uniform grid with the
 * spacings lx/nx, ly/ny of p and its nu, cfl, c, eta and s_ratio (Newtonian
 * only; walls, metrics and forces are not part of the analysis).  theta runs
 * over nk points per axis on (-pi, pi], theta_i = -pi + 2 pi (i + 1)/nk.
 * rho (HOST, nk*nk values, row iy then column ix; may be NULL) receives the
 * radius of each mode; worst (HOST, 3 values) the largest radius and its
 * (theta_x, theta_y).  A mode is stable when its radius is at most 1.  Host
 * computation only; MDF_EINVAL for invalid parameters or nk outside 1..4096. */
mdf_status mdf_stability(const mdf_params* p, double u0, double v0, int32_t nk, double* rho, double* worst);

/* ---------------------------------------------------------------------------
 * Measurement aid (not part of the method): a streaming copy of `bytes`
 * bytes (a multiple of 16; both DEVICE pointers 16-byte aligned, regions not
 * overlapping) with 16-byte loads and stores, asynchronous on hip_stream.  Its
 * rate is the practical HBM ceiling the step's bandwidth is compared with, and
 * its known traffic calibrates the hardware byte counters. */
mdf_status mdf_stream_copy(const void* src, void* dst, size_t bytes, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* MDF_H */
