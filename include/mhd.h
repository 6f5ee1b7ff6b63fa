/*
 * mhd.h -- C ABI of the MI355X (gfx950) ideal-MHD update step.
 *
 * The library advances the ideal-MHD equations (1)-(5) of Pang, Pen &
 * Perrone, "Magnetohydrodynamics on Heterogeneous architectures: a
 * performance comparison" (arXiv:1004.1680), section II, on a periodic 3D
 * grid with the scheme of section II.B: dimensionally split relaxing-TVD
 * fluid sweeps (first-order upwind half step, van-Leer-limited full step)
 * and constrained-transport advection of the face-centred field, applied in
 * the order x, y, z, z, y, x.  Every step of the computation runs in HIP
 * kernels on the device; the host only validates and enqueues.
 *
 * State layout.  8 fields, structure of arrays, field-major [f][k][j][i]
 * with x fastest (section III: one array per component):
 *   0 rho, 1 m_x, 2 m_y, 3 m_z, 4 e   at cell centres (e = total energy
 *   density p/(gamma-1) + rho v^2/2 + b^2/2, section II.A),
 *   5 b_x, 6 b_y, 7 b_z               b_d[c] = field through the LOW d-face
 *                                     of cell c (b normalised by sqrt(4 pi)).
 * The grid spacing is h = 1/nx on every axis.  Dimensions must be >= 8 and
 * multiples of 4 (section III.B, aligned DMA); gamma > 1.
 *
 * Precision.  MHD_F32 keeps the state and the sweeps in float; MHD_F64 in
 * double.  The CFL reduction, the diagnostics sums and the time are FP64 in
 * both tiers.
 *
 * Relaxation speed.  The fluid sweeps use one relaxation (freezing) speed
 * per step: the largest signal speed max_d |v_d| + c_fast found by the CFL
 * function (section II.B, Jin & Xin relaxation; section IV.A, one CFL call
 * per step).  mhd_cfl_dt sets it; mhd_set_relaxation_speed sets it
 * explicitly; mhd_set_state invalidates it.
 *
 * Errors.  Functions returning int give MHD_OK (0) or a negative code;
 * mhd_last_error() returns a thread-local message for the last failure.
 * A HIP runtime error makes the handle sticky-failed: every later call on it
 * returns MHD_ESTATE.  Kernels are asynchronous on the handle's stream;
 * their faults surface at the next synchronising call.  A handle is not
 * thread-safe; use one handle per thread or serialise the calls.
 *
 * Ownership.  The library owns the handle and its device buffers.  Host
 * arrays passed in are read or written synchronously and stay the caller's.
 * Device pointers passed in (mhd_*_device) stay the caller's and must be
 * valid device memory on the handle's device.
 */
#ifndef MHD_H
#define MHD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mhd_ctx mhd_ctx;

enum {
    MHD_OK = 0,
    MHD_EINVAL = -1,     /* bad argument (sizes, dims, gamma, dt, null) */
    MHD_ENOMEM = -2,     /* device allocation failed */
    MHD_EDEVICE = -3,    /* HIP runtime error (handle becomes sticky-failed) */
    MHD_ENONPHYS = -4,   /* rho <= 0, p < 0 or a non-finite value found */
    MHD_ESTATE = -5      /* handle failed earlier, or relaxation speed unset */
};

enum { MHD_F32 = 0, MHD_F64 = 1 };

/* Create a solver for an nx x ny x nz periodic grid (section II; grid of
 * section III), FP32 tier, on the default stream.  Returns NULL on failure
 * (message in mhd_last_error()).  The state is zero until mhd_set_state. */
mhd_ctx *mhd_create(int nx, int ny, int nz, double gamma);

/* As mhd_create, with precision tier prec (MHD_F32 / MHD_F64), a HIP stream
 * (hipStream_t passed as void*, NULL = default stream) on which every kernel
 * of the handle is enqueued, and optionally the two state buffers (the
 * ping-pong pair the operators read from and write to; each field lives in
 * one of them at a time).
 *
 * dev_buf_a, dev_buf_b: both NULL (the library allocates and frees them) or
 * both device memory of the current device, owned by the caller (for
 * instance from a caching allocator), each at least 8*nx*ny*nz elements of
 * the tier's type inside its allocation, 256-byte aligned, not overlapping;
 * they are zeroed here, hold the state between calls, and must outlive the
 * handle, which never frees them.  Read the state with mhd_get_state or
 * mhd_get_state_device, not from the buffers (which one holds a field
 * changes from operator to operator).  Violations of these conditions that
 * the runtime can see (one buffer NULL, host or managed memory, another
 * device, misalignment, an allocation too short, overlap) give NULL with
 * MHD_EINVAL in mhd_last_error.  The stream must outlive the handle. */
mhd_ctx *mhd_create_ex(int nx, int ny, int nz, double gamma, int prec,
                       void *hip_stream, void *dev_buf_a, void *dev_buf_b);

/* Free the handle and its device memory (synchronises its stream). */
void mhd_destroy(mhd_ctx *h);

/* Grid and tier of the handle: dims[3], precision; MHD_EINVAL on NULL. */
int mhd_info(const mhd_ctx *h, int dims[3], int *prec);

/* Copy a state in from host memory: n == 8*nx*ny*nz doubles in the layout
 * above, converted to the handle's precision.  Synchronous.  Resets the
 * time to 0 and invalidates the relaxation speed. */
int mhd_set_state(mhd_ctx *h, const double *host, size_t n);

/* Copy the state out to host memory as doubles (same layout).  Synchronous. */
int mhd_get_state(mhd_ctx *h, double *host, size_t n);

/* Device-to-device variants: src/dst hold n == 8*nx*ny*nz values of type
 * float (prec MHD_F32) or double (MHD_F64) in the layout above, in device
 * memory of the handle's device.  Enqueued on the handle's stream (no host
 * synchronisation).  set resets time and relaxation speed like
 * mhd_set_state. */
int mhd_set_state_device(mhd_ctx *h, const void *src, size_t n, int prec);
int mhd_get_state_device(mhd_ctx *h, void *dst, size_t n, int prec);

/* CFL condition (section II.B; the CFL function of section IV.A):
 * vmax = max over cells of max_d |v_d| + sqrt((gamma p + |Bbar|^2)/rho),
 * Bbar the cell-centred mean of the two face values, p = (gamma-1)(e -
 * m.m/(2 rho) - |Bbar|^2/2); dt = cfl * h / vmax (h = 1/nx).  FP64 on the
 * device; synchronous.  Sets the relaxation speed to vmax.  Returns
 * MHD_ENONPHYS (dt = 0) if any cell has rho <= 0, p < 0 or a non-finite
 * value; MHD_EINVAL if cfl <= 0 or vmax == 0. */
int mhd_cfl_dt(mhd_ctx *h, double cfl, double *dt_out);

/* Set / read the relaxation speed c of the fluid sweeps (c > 0). */
int mhd_set_relaxation_speed(mhd_ctx *h, double c);
int mhd_get_relaxation_speed(const mhd_ctx *h, double *c);

/* The two operators of a sweep along axis dim (0 x, 1 y, 2 z), each over a
 * time dt > 0 (section II.B): the relaxing-TVD fluid update of rho, m, e with
 * b frozen (equations (1)-(3), (6)), and the constrained-transport
 * advection-constraint update of b with v frozen (equation (4)).
 * Asynchronous.  The fluid operator needs a relaxation speed (MHD_ESTATE
 * if none is set). */
int mhd_fluid(mhd_ctx *h, int dim, double dt);
int mhd_magnetic(mhd_ctx *h, int dim, double dt);

/* One sweep (section II.B): dim 0,1,2 = fluid then magnetic along x, y, z;
 * dim 3,4,5 = magnetic then fluid along x, y, z.  dim 6 = dim 3 with the
 * CFL maximum of the resulting state found on the way (what the last
 * launch of a step does); the next mhd_step_auto then takes its dt from it
 * instead of a separate reduction.  dim 7 = the middle of a step, M_z then
 * dim 5 (M_z M_z F_z; one launch where MHD_TUNE_MIDDLE chooses it).
 * Asynchronous. */
int mhd_sweep(mhd_ctx *h, int dim, double dt);

/* Slope limiter of the second-order parts of both operators, a method
 * variant (the paper's is van Leer's, section II.B).  With a, b the halved
 * one-sided differences and a b > 0:
 *   MHD_LIMITER_VANLEER   2ab/(a+b)                          (default)
 *   MHD_LIMITER_MINMOD    sign(a) min(|a|, |b|)
 *   MHD_LIMITER_MC        sign(a) min(2|a|, 2|b|, |a+b|/2)
 *   MHD_LIMITER_SUPERBEE  sign(a) max(min(2|a|, |b|), min(|a|, 2|b|))
 * and 0 when a b <= 0.  Applies to the handle's operators, sweeps and steps
 * (fused reverse pairs included) from the next call on.  MHD_EINVAL for
 * another value.  Ensembles have their own setting (mhd_batch_set_limiter). */
enum { MHD_LIMITER_VANLEER = 0, MHD_LIMITER_MINMOD = 1, MHD_LIMITER_MC = 2, MHD_LIMITER_SUPERBEE = 3 };
int mhd_set_limiter(mhd_ctx *h, int limiter);
int mhd_get_limiter(const mhd_ctx *h, int *limiter);

/* Freezing (relaxation) speed of the fluid operator, a method variant
 * (section II.B requires only that it exceed the characteristic speeds of
 * the flux; the reading taken here is one number per step):
 *   MHD_FREEZE_STEP    the step's relaxation speed, the largest signal speed
 *                      found by the CFL function (default; see above)
 *   MHD_FREEZE_CELL    |v_n| + c_fast of each cell, c_fast = sqrt((gamma p +
 *                      |Bbar|^2)/rho), from the state of each stage (the old
 *                      state for the first, the half-step state for the
 *                      second)
 *   MHD_FREEZE_PENCIL  the largest of those along the pencil, per stage.
 * The variants need no relaxation speed to be set, run the reverse-half
 * pairs as two launches each, and come with van Leer's limiter only
 * (MHD_EINVAL otherwise, here and in mhd_set_limiter).  Applies from the
 * next call on.  Ensembles always use the step's speed. */
enum { MHD_FREEZE_STEP = 0, MHD_FREEZE_CELL = 1, MHD_FREEZE_PENCIL = 2 };
int mhd_set_freezing_speed(mhd_ctx *h, int mode);
int mhd_get_freezing_speed(const mhd_ctx *h, int *mode);

/* Full step of 2*dt (section II.B; section IV.A): sweeps x, y, z, then
 * z, y, x, i.e. F_x M_x F_y M_y F_z M_z M_z F_z M_y F_y M_x F_x, every
 * operator over dt.  Advances the time by 2*dt.  Asynchronous. */
int mhd_step(mhd_ctx *h, double dt);

/* CFL and full step with dt = cfl h / vmax kept on the device (no host
 * synchronisation; the form a HIP graph can capture).  A non-physical state
 * is recorded on the device and reported by the next mhd_status call (the
 * step then leaves the state unchanged). */
int mhd_step_auto(mhd_ctx *h, double cfl);

/* Synchronise the handle's stream; report a non-physical state recorded by
 * mhd_step_auto (MHD_ENONPHYS), then clear that record.  If steps_out is not
 * NULL it receives the number of mhd_step_auto steps that ran. */
int mhd_status(mhd_ctx *h, long long *steps_out);

/* Simulated time (sum of 2*dt over all steps, FP64).  Synchronous. */
int mhd_time(mhd_ctx *h, double *t);

/* Diagnostics, FP64 on the device, synchronous: out[0..7] = h^3 * sum over
 * cells of each field (conserved totals, section II.B), out[8] =
 * max_c |sum_d (b_d[c+d] - b_d[c])| / max |b| (= max |div b| h / max |b|,
 * equation (5)). */
int mhd_diag(mhd_ctx *h, double out[9]);

/* Restriction of a fine state onto a coarse grid whose sizes divide the fine
 * ones by one integer factor r (8 for a 1024^3 -> 128^3 coarsening): coarse
 * rho, m, e = mean over the r^3 fine cells; coarse b_d on a low d-face =
 * mean of the r^2 fine face values tiling it.  Totals are kept and the
 * coarse div b is the block mean of the fine one.  Both handles must be of
 * the same precision and device; enqueued on the coarse handle's stream
 * after the fine handle's stream is synchronised.  Resets the coarse time
 * and relaxation speed. */
int mhd_restrict(mhd_ctx *fine, mhd_ctx *coarse);

/* Launch shape of the y and z sweep kernels: each lane walks one pencil
 * along the sweep axis in chunks of `value` cells (value must divide the
 * axis length and be >= 8; 0 restores the built-in choice).  key: MHD_TUNE_
 * CHUNK_Y or MHD_TUNE_CHUNK_Z for the single operators, MHD_TUNE_PAIR_
 * CHUNK_Y or MHD_TUNE_PAIR_CHUNK_Z for the fused reverse-half pairs.
 * key MHD_TUNE_REVERSE: how the reverse-half pairs M_d F_d of a step and of
 * mhd_sweep(3..5) run: 1 = one fused launch per pair (the new faces stay
 * in registers; 9 launches per step), 2 = the two operators in turn (12
 * launches), 0 = the built-in choice (1 in FP32 with the van Leer or
 * minmod limiter, 2 otherwise: the fused MC and superbee kernels spill
 * registers); mhd_get_launch reports the resolved 1 or 2.
 * key MHD_TUNE_MIDDLE: how the middle of a step, M_z M_z F_z (the last
 * forward operator and the first reverse pair), runs: 1 = one launch (the
 * second magnetic window takes the first one's new faces and edge
 * velocities from registers; 8 launches per step), 2 = M_z and the reverse
 * pair (9), 0 = the built-in choice (1 for grids of 128^3 cells and more,
 * 2 below); mhd_get_launch reports 1 or 2.  It takes effect in FP32 with
 * fused reverse pairs and van Leer's limiter only.
 * MHD_TUNE_MIDDLE_CHUNK: its march chunk along z (rules of the chunks above).
 * key MHD_TUNE_ROW_GROUP: the x sweeps visit their row tiles in groups of
 * consecutive rows along y, one group per z in turn, so that the rows z +- 1
 * a tile reads were read by tiles a few positions earlier on the same XCD;
 * the value is the most rows in a group (0 = built-in, 64; a value of ny or
 * more gives the linear y-then-z order).  mhd_get_launch reports the rows of
 * a group as resolved (ny: linear order, also where the rows of a
 * workgroup do not divide ny).
 * key MHD_TUNE_WIDE_OFFSETS: 1 makes the y and z sweeps address memory with
 * 64-bit arithmetic per access, as they must for fields over 4 GiB; 0 (the
 * default) uses 32-bit byte offsets wherever they fit.
 * Results do not depend on any of these (the fused pair is bitwise the two
 * operators).  Launch-shape parameters, not part of the method. */
enum { MHD_TUNE_CHUNK_Y = 1, MHD_TUNE_CHUNK_Z = 2, MHD_TUNE_REVERSE = 3,
       MHD_TUNE_PAIR_CHUNK_Y = 4, MHD_TUNE_PAIR_CHUNK_Z = 5, MHD_TUNE_WIDE_OFFSETS = 6,
       MHD_TUNE_MIDDLE = 7, MHD_TUNE_MIDDLE_CHUNK = 8, MHD_TUNE_ROW_GROUP = 9 };
int mhd_set_launch(mhd_ctx *h, int key, int value);
int mhd_get_launch(const mhd_ctx *h, int key, int *value);

/* ------------------------------------------------------------------------
 * Batched ensembles of uneven periodic boxes.  Each box is an independent
 * grid advanced by the same method (section II) with its own CFL time step
 * and relaxation speed; a step is the per-box CFL (FP64, on the device) and
 * the 12 operators, each operator ONE persistent launch over the work items
 * (box, tile) of all boxes, then the per-box time advance.  A box evolves
 * bit for bit as it would in a single-grid handle.  Box dims follow the
 * single-grid rules.  Not thread-safe.
 * ------------------------------------------------------------------------ */
typedef struct mhd_batch mhd_batch;

/* dims: 3*nbox ints (nx, ny, nz of each box).  hip_stream may be NULL (the
 * batch then creates its own stream, needed for graph capture). */
mhd_batch *mhd_batch_create(int nbox, const int *dims, double gamma, int prec,
                            void *hip_stream);
void mhd_batch_destroy(mhd_batch *b);
int mhd_batch_info(const mhd_batch *b, int *nbox, long long *ncell);

/* State of one box (n == 8 * its cell count doubles, single-grid layout);
 * synchronous; set resets the box's time and records. */
int mhd_batch_set_state(mhd_batch *b, int box, const double *host, size_t n);
int mhd_batch_get_state(mhd_batch *b, int box, double *host, size_t n);

/* One step of every box with its own dt = cfl h / vmax (asynchronous). */
int mhd_batch_step_auto(mhd_batch *b, double cfl);

/* nsteps steps; use_graph != 0 captures one step in a HIP graph (once per
 * cfl value and launch shape) and replays it.  Asynchronous. */
int mhd_batch_run(mhd_batch *b, double cfl, int nsteps, int use_graph);

/* Synchronise; steps[b] / nonphys[b] (each may be NULL) receive the steps a
 * box completed and its record (0 none, 1 non-physical state, 2 zero
 * signal speed).  A box with a record is left unchanged by later steps
 * until this call clears the record; returns MHD_ENONPHYS if any box had
 * one. */
int mhd_batch_status(mhd_batch *b, long long *steps, int *nonphys);

/* Simulated time of every box (nbox doubles). */
int mhd_batch_time(mhd_batch *b, double *times);

/* Launch shape (results do not depend on it): persistent workgroups of the
 * x, y, z operator launches (multiples of 8), the target march chunk (each
 * box takes the largest divisor of its axis length <= target, >= 8), and
 * MHD_BATCH_REVERSE as MHD_TUNE_REVERSE of a single grid (1: each
 * reverse-half pair M_d F_d in one launch, 2: the two operators in turn,
 * 0: built-in, 1 in FP32 with the van Leer or minmod limiter, 2 otherwise),
 * the target march chunk of the
 * fused pairs (MHD_BATCH_PAIR_CHUNK, default 128), MHD_BATCH_WIDE_OFFSETS
 * as MHD_TUNE_WIDE_OFFSETS, and MHD_BATCH_MIDDLE as MHD_TUNE_MIDDLE (1: M_z
 * M_z F_z in one launch, on the fused pairs' work list; 2: M_z and the z
 * pair; 0: built-in, 1 where the boxes hold 128^3 cells or more on average,
 * in FP32 with fused pairs and van Leer's limiter).
 * Launch-shape parameters, not part of the method. */
enum { MHD_BATCH_GRID_X = 10, MHD_BATCH_GRID_Y = 11, MHD_BATCH_GRID_Z = 12,
       MHD_BATCH_CHUNK = 13, MHD_BATCH_REVERSE = 14, MHD_BATCH_WIDE_OFFSETS = 15,
       MHD_BATCH_PAIR_CHUNK = 16, MHD_BATCH_MIDDLE = 17 };
int mhd_batch_set_launch(mhd_batch *b, int key, int value);
int mhd_batch_get_launch(const mhd_batch *b, int key, int *value);

/* Slope limiter of every box's operators (MHD_LIMITER_*, as mhd_set_limiter;
 * van Leer's by default).  Synchronises the ensemble's stream and drops a
 * captured step graph (the next graph run captures again).  MHD_EINVAL for
 * another value. */
int mhd_batch_set_limiter(mhd_batch *b, int limiter);
int mhd_batch_get_limiter(const mhd_batch *b, int *limiter);

/* ------------------------------------------------------------------------
 * Learned closure of a coarse grid (an addition to the paper's method).
 * A 3-layer periodic 3x3x3 convolutional net, 8 -> 32 -> 32 -> 8 channels
 * with ReLU, BF16 weights and activations, FP32 accumulation on MFMA,
 * predicts the correction that takes one plain coarse step toward the
 * restricted fine solution.  Its 8 outputs o are projected so that the
 * correction keeps every conserved total and every cell's div b: fluid
 * delta_f = s_f (o_f - mean o_f), f < 5; field delta_b = discrete curl of
 * the edge potential (s_5 o_5, s_6 o_6, s_7 o_7) (A_x on x-edges etc.).
 * Network input: (u_f - in_mean_f) / in_std_f of the plain-stepped state.
 * Loss: mean over channels and cells of ((delta - target)/target_scale)^2.
 * Parameters: 41544 floats, per layer l = 1..3 the weights
 * W[27][cin][cout] (offset o = (dz+1)*9 + (dy+1)*3 + (dx+1)) then the bias
 * [cout].  Grid dimensions must be multiples of 32.  States and targets are
 * FP32 device arrays [8][nz][ny][nx] (the state layout).
 * ------------------------------------------------------------------------ */
typedef struct mhd_closure mhd_closure;
mhd_closure *mhd_closure_create(int nx, int ny, int nz, void *hip_stream);
void mhd_closure_destroy(mhd_closure *c);
int mhd_closure_set_params(mhd_closure *c, const float *params, size_t n);
int mhd_closure_get_params(mhd_closure *c, float *params, size_t n);
int mhd_closure_set_scales(mhd_closure *c, const float *in_mean, const float *in_std,
                           const float *out_scale, const float *target_scale);
/* correction of a plain-stepped state u (device, FP32) into delta (device) */
int mhd_closure_forward(mhd_closure *c, const float *u_dev, float *delta_dev);
/* loss against a target correction and the gradient of every parameter
 * (grad_host may be NULL; n = 41544); synchronous */
int mhd_closure_grad(mhd_closure *c, const float *u_dev, const float *target_dev,
                     double *loss, float *grad_host, size_t n);
/* forward, backward and one Adam step (beta 0.9, 0.999, eps 1e-8) on the
 * FP32 master parameters; loss (may be NULL) makes it synchronous */
int mhd_closure_train_step(mhd_closure *c, const float *u_dev, const float *target_dev,
                           float lr, double *loss);
/* One learned coarse step of an FP32 handle on the closure's stream: the
 * plain step (mhd_step_auto) then u += theta * delta with the largest theta
 * in {1, 1/2, 1/4, 1/8} for which no cell has rho <= 0, p < 0 (pressure
 * from the cell-centred field) or a non-finite value; if none qualifies the
 * plain step is kept.  A uniform theta keeps the conserved totals and div b
 * of the correction.  No host synchronisation.  Counters since creation
 * (synchronous reads): mhd_closure_fallbacks, steps whose correction was
 * dropped; mhd_closure_reduced, steps applied with theta < 1. */
int mhd_closure_step(mhd_closure *c, mhd_ctx *coarse, double cfl);
int mhd_closure_fallbacks(mhd_closure *c, int *count);
int mhd_closure_reduced(mhd_closure *c, int *count);
/* Training-set preparation on the closure's stream (device FP32 arrays in
 * the state layout, 8 * nx * ny * nz values each):
 * residual: target = u_ref - u_plain, the correction that takes the plain
 *   coarse step u_plain to the restricted fine state u_ref (asynchronous);
 * stats: FP64 per-field sums over the cells, out[40] = { sum u_f, sum u_f^2,
 *   sum |u_f|, sum |target_f|, sum r_f } with f = 0..7 fastest and r_f the
 *   roughness below (synchronous), from which the normalisation of
 *   mhd_closure_set_scales and mhd_closure_set_gate is formed. */
int mhd_closure_residual(mhd_closure *c, const float *u_ref_dev, const float *u_plain_dev,
                         float *target_dev);
int mhd_closure_stats(mhd_closure *c, const float *u_dev, const float *target_dev, double *out);
/* Roughness gate of the correction (off after create).  With mean
 * roughness R[8] > 0 (host): r_f(c) = sum over the three axes of
 * |u_f(c+a) - 2 u_f(c) + u_f(c-a)| on the network input u, g0(c) =
 * (1/8) sum_f r_f(c) / R_f, g(c) = max of g0 over c and its six face
 * neighbours, and the projection acts on g(c) o(c): the correction (and its
 * gradient) vanishes where the state is locally linear.  R = NULL turns the
 * gate off.  get_gate copies the gate of the last forward pass (device,
 * nx*ny*nz floats). */
int mhd_closure_set_gate(mhd_closure *c, const float *mean_roughness);
int mhd_closure_get_gate(mhd_closure *c, float *gate_dev);

/* Single periodic 3x3x3 convolution layers on MFMA (BF16 inputs rounded to
 * nearest even, FP32 accumulate), synchronous on `stream`: n[3] grid
 * (multiples of 32), (cin, cout) in {(8,32), (32,32), (32,8), (8,8)},
 * weights host FP32 [27][cin][cout] (rounded to BF16).
 * forward: x bf16 [cell][cin] -> y fp32 [cell][cout] (+ bias, may be NULL);
 * dgrad:   dy bf16 [cell][cout] -> dx fp32 [cell][cin];
 * wgrad:   xT bf16 [cin][cell], dyT bf16 [cout][cell] -> dw host [27][cin][cout],
 *          dbias host [cout] (may be NULL). */
int mhd_conv3d_forward(const int *n, int cin, int cout, const void *x, const float *w_host,
                       const float *bias_host, float *y, void *stream);
int mhd_conv3d_dgrad(const int *n, int cin, int cout, const void *dy, const float *w_host,
                     float *dx, void *stream);
int mhd_conv3d_wgrad(const int *n, int cin, int cout, const void *xT, const void *dyT,
                     float *dw_host, float *dbias_host, void *stream);

/* CFL time step of a state in the caller's device memory, allocating
 * nothing: for callers that cannot allocate (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  The same kernels
 * and result as mhd_cfl_dt, with the reduction's block partials, scalars and
 * flag in a fixed array of 49,200 bytes of each device's global memory, held
 * until the process ends, instead of a handle's buffers.
 * state_dev: 8*nx*ny*nz values of type float (prec MHD_F32) or double
 * (MHD_F64) in the state layout above; out_dev: 3 doubles of device memory
 * that receive dt = cfl h / vmax, vmax, and the record (0 none, 1 a cell
 * with rho <= 0, p < 0 or a non-finite value, 2 zero signal speed; dt =
 * vmax = 0 with a record).  Grid limits of mhd_create_ex (MHD_EINVAL beyond
 * them, and for gamma <= 1, cfl <= 0 or a null pointer).  Enqueued on
 * `stream` (hipStream_t as void*, NULL = default); read out_dev after the
 * stream.  All calls on one device share the array: calls that overlap in
 * time on one device (other streams, other threads) race, so serialise
 * them.  Both buffers stay the caller's. */
int mhd_cfl_dt_noalloc(const void *state_dev, int nx, int ny, int nz, int prec, double gamma,
                       double cfl, double *out_dev, void *stream);

/* Plain device-to-device copy of `bytes` bytes with 16-byte vector loads and
 * stores, enqueued on `stream` (hipStream_t as void*, NULL = default): the
 * streaming-bandwidth reference the benchmark reports beside the sweep
 * kernels (not part of the method).  bytes and both pointers must be
 * multiples of 16 and the ranges must not overlap (MHD_EINVAL); a launch
 * failure gives MHD_EDEVICE.  Both buffers stay the caller's. */
int mhd_stream_copy(const void *src, void *dst, size_t bytes, void *stream);

/* Thread-local message describing the last error (never NULL). */
const char *mhd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MHD_H */
