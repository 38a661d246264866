/*
 * srwcr.h -- C ABI of the MI355X (gfx950) implementation of the spatially
 * region-weighted correlation ratio (SRWCR) and its analytic gradient with
 * respect to cubic B-spline free-form-deformation (FFD) displacements,
 * after Gong et al., "Non-rigid image registration using spatially
 * region-weighted correlation ratio and GPU-acceleration" (arXiv 1804.05061).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Volumes are dense, x fastest: element (x, y, z) of an (nx, ny, nz) grid
 *    sits at index (z * ny + y) * nx + x.
 *  - "Device pointer" means memory allocated on the current HIP device (for
 *    example by PyTorch); the caller owns it, the library never frees it.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  The
 *    value, gradient and warp calls only enqueue work on it and return; results
 *    are valid once the stream reaches them.  No call here allocates device
 *    memory after srwcr_plan_create, and none synchronises the device except
 *    where stated.
 *  - Every function returns an srwcr_status; on failure nothing was enqueued,
 *    and srwcr_last_error() returns a thread-local message.
 *  - FFD displacements are float32 [3][ncz][ncy][ncx] (component 0 = x), in
 *    fixed-voxel units; T(x) = x + sum beta_l beta_m beta_n d (Sec. II, eqs 8
 *    and 17).  Stored node index = the paper's node index + 1, so
 *    nc = floor((N - 1) / delta) + 4 per axis.
 */
#ifndef SRWCR_H
#define SRWCR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SRWCR_OK = 0,
    SRWCR_E_INVALID_ARG = -1,   /* a size, count, role or dtype out of range, or a NULL pointer */
    SRWCR_E_DEGENERATE = -2,    /* a normalisation range with hi <= lo */
    SRWCR_E_WORKSPACE = -3,     /* workspace smaller than srwcr_workspace_bytes() */
    SRWCR_E_HIP = -4,           /* a HIP runtime call failed (message has the HIP error string) */
    SRWCR_E_UNSUPPORTED = -5,   /* a valid request this build does not handle */
    SRWCR_E_NONFINITE = -6,     /* NaN or Inf found where finite data is required */
    SRWCR_E_LINESEARCH = -7     /* register_lbfgs: the line search found no acceptable step */
} srwcr_status;

/* Which image plays the model image A and which the estimated image B of
 * Sec. II-A.  Table II of the paper finds the moving image as A best. */
typedef enum { SRWCR_MOVING_AS_A = 0, SRWCR_MOVING_AS_B = 1 } srwcr_role;

/* Storage type of a normalised intensity volume. */
typedef enum { SRWCR_F32 = 0, SRWCR_F16 = 1, SRWCR_BF16 = 2 } srwcr_dtype;

/* The problem statement of Sec. II: minimise D(F, M o T(.; Phi)) over Phi. */
typedef struct {
    int32_t fixed_dims[3];     /* (nx, ny, nz) of F, each >= 2 */
    int32_t moving_dims[3];    /* (mx, my, mz) of M, each >= 2 */
    int32_t n_bins;            /* L_eps + 1 intensity bins, 2..64 (the paper uses 32) */
    int32_t spatial_bins[3];   /* K cubic B-spline spatial bins per axis, each 4..64; all three 0:
                                  the regions are the FFD nodes (the paper's setting, Sec. II-C),
                                  K = n_c per axis, node j at (j - 1) ctrl_spacing */
    int32_t ctrl_spacing[3];   /* FFD control spacing delta in fixed voxels, each >= 1 */
    int32_t role;              /* srwcr_role */
    int32_t fixed_dtype;       /* srwcr_dtype of the normalised fixed volume */
    int32_t moving_dtype;      /* srwcr_dtype of the normalised moving volume */
} srwcr_problem;

typedef struct srwcr_plan srwcr_plan;

/* Number of FFD control nodes per axis: floor((N - 1) / delta) + 4 (eq 17). */
int srwcr_ctrl_dims(const srwcr_problem *prob, int32_t out_nc[3]);

/* Validate `prob` and build a plan: per-axis spatial-weight tables, FFD weight
 * tables and the launch geometry, uploaded once to the current device.  The
 * plan is immutable and may be shared by concurrent calls on different
 * streams provided each call has its own workspace.  Spatial bins: K nodes per
 * axis at spacing (N - 1) / (K - 3), node j at (j - 1) * spacing (eqs 7, 8),
 * or, with spatial_bins (0, 0, 0), the FFD nodes themselves.  Returns
 * SRWCR_E_INVALID_ARG for a bad problem and SRWCR_E_UNSUPPORTED when the
 * passes do not fit the device's LDS (more than 64 bins cannot occur). */
int srwcr_plan_create(const srwcr_problem *prob, srwcr_plan **out);
void srwcr_plan_destroy(srwcr_plan *plan);

/* Launch-shape knobs of a plan, for autotuning (the Python `tune()` times
 * candidates on the caller's data and caches the best per problem and
 * device).  0 keeps the default.  grad_item_voxels: target voxels of a
 * gradient-pass work item (default |F| / 600 clamped to 2048 .. 65536; items
 * are also bounded by the spatial cells and the LDS); value_workgroups:
 * persistent value-pass workgroups (default one per compute unit).  Results
 * do not depend on the knobs beyond FP summation order.  Returns
 * SRWCR_E_INVALID_ARG for negative values. */
typedef struct {
    int32_t grad_item_voxels;
    int32_t value_workgroups;
} srwcr_tuning;
int srwcr_plan_create_tuned(const srwcr_problem *prob, const srwcr_tuning *tuning, srwcr_plan **out);

/* Device workspace bytes srwcr_eval / srwcr_grad / srwcr_grad_fixed need
 * (moment slots in FP64, per-region tables, gradient accumulators, the warp
 * pass's per-voxel samples and the value pass's staging slots; 213 MB at
 * 256 x 256 x 128).  Callers allocate it once; its contents need no
 * initialisation and do not persist between calls. */
size_t srwcr_workspace_bytes(const srwcr_plan *plan);

/* a1 -- intensity normalisation of Sec. II.  out[i] = clamp(fl32(fl32(in[i]
 * - (float)lo) * (float)(L / (hi - lo))), 0, L), L = n_bins - 1, stored in
 * `out_dtype` (round to nearest even for F16 / BF16).  in: device float32[n];
 * out: device buffer of n elements of out_dtype.  Runs once per image pair. */
int srwcr_normalize(const float *in, int64_t n, double lo, double hi, int32_t n_bins,
                    void *out, int32_t out_dtype, void *stream);

/* Minimum and maximum of a device float32 volume (a helper for choosing the
 * normalisation range; synchronises `stream` and writes host doubles).
 * Returns SRWCR_E_NONFINITE when the volume holds NaN or Inf. */
int srwcr_minmax(const float *in, int64_t n, double *lo, double *hi, void *stream);

/* SRWCR value D (eq 9; a dissimilarity in [0, 1], 0 for a perfect functional
 * dependence).  fixed, moving: device volumes normalised to [0, L] in the
 * plan's dtypes; ffd: device float32 displacements; d_value: device double.
 * Steps: FFD evaluation, trilinear backward warping of M (coordinates clamped
 * to the grid; grids of different size mapped by y = (T + 1/2) M / N - 1/2),
 * second-order Parzen window (eq 5), cubic B-spline spatial weights (eq 7),
 * joint moments of the 3-D PDF (eq 3) and the per-region correlation ratios
 * (eqs 4, 9-12) finalised in FP64. */
int srwcr_eval(const srwcr_plan *plan, const void *fixed, const void *moving, const float *ffd,
               double *d_value, void *workspace, size_t workspace_bytes, void *stream);

/* Value and gradient dD/d(displacement) (eqs 15-21): d_value as srwcr_eval,
 * d_grad a device float32 array shaped like ffd.  The warped samples and
 * their image gradients are kept in the workspace between the passes. */
int srwcr_grad(const srwcr_plan *plan, const void *fixed, const void *moving, const float *ffd,
               double *d_value, float *d_grad, void *workspace, size_t workspace_bytes, void *stream);

/* srwcr_grad for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same passes and results, with the workspace taken from a static device array
 * of SRWCR_NOALLOC_SCRATCH_BYTES that the library holds on every device it
 * runs on until the process ends (its address is looked up once per device;
 * the call allocates nothing).  The plan must have been made on the current
 * device and need at most that much workspace (srwcr_workspace_bytes),
 * otherwise SRWCR_E_INVALID_ARG or SRWCR_E_WORKSPACE.  All calls on one device
 * share the array: calls that overlap in time on one device race and must be
 * serialised by the caller (one stream, or events).  The array keeps the last
 * call's contents; srwcr_grad clears what has to start at zero itself. */
#define SRWCR_NOALLOC_SCRATCH_BYTES (64u << 20)
int srwcr_grad_noalloc(const srwcr_plan *plan, const void *fixed, const void *moving, const float *ffd,
                       double *d_value, float *d_grad, void *stream);

/* Dense-displacement variants (a loss for learning-based registration): the
 * warp is T(x) = x + u(x) with u a device float32 field [3][nz][ny][nx] on the
 * fixed grid (fixed-voxel units), instead of the FFD of eq 17; everything
 * else is srwcr_eval / srwcr_grad.  srwcr_grad_dense writes d_grad, a device
 * float32 [3][nz][ny][nx] array, with dD/du(x) = dD/dM(x) dM/dy dy/dT, the
 * per-voxel factor of eq 16 (dT/du = 1); nothing is scattered.  The plan's
 * ctrl_spacing is unused by these calls. */
int srwcr_eval_dense(const srwcr_plan *plan, const void *fixed, const void *moving, const float *field,
                     double *d_value, void *workspace, size_t workspace_bytes, void *stream);
int srwcr_grad_dense(const srwcr_plan *plan, const void *fixed, const void *moving, const float *field,
                     double *d_value, float *d_grad, void *workspace, size_t workspace_bytes, void *stream);

/* dD/ds_F: the derivative of D with respect to the normalised fixed intensity
 * at every fixed voxel, written to d_grad_fixed, a device float32 volume of
 * the fixed dims [nz][ny][nx] (it makes the fixed image a differentiable
 * input too, e.g. a network's output).  The fixed image plays B when the
 * moving image is A (eq 19) and A otherwise (eq 21), with the one-sided
 * window derivatives of srwcr_grad; the derivative is with respect to the
 * stored normalised value, so a caller that normalised raw intensities with
 * srwcr_normalize multiplies by L / (hi - lo).  disp is the FFD (dense = 0)
 * or a dense field [3][nz][ny][nx] (dense = 1); d_value receives D. */
int srwcr_grad_fixed(const srwcr_plan *plan, const void *fixed, const void *moving, const float *disp, int32_t dense,
                     double *d_value, float *d_grad_fixed, void *workspace, size_t workspace_bytes, void *stream);

/* Batched value + gradient over up to SRWCR_MAX_BATCH independent problems
 * (e.g. the phases of a 4-D series times the levels of their pyramids): one
 * launch per pass covers every problem, so small problems share the device
 * instead of running one after another.  Each problem is computed exactly as
 * srwcr_grad computes it (Sec. II-D, eqs 15-21).
 *
 * srwcr_batch_create: plans[0..n-1] must share role and storage dtypes and
 * outlive the batch (their device tables are referenced, not copied).
 * srwcr_grad_batched: items[p] holds problem p's device pointers, with the
 * meaning of srwcr_grad's arguments; the workspace (srwcr_batch_workspace_bytes)
 * is the caller's.  The call only enqueues kernels on `stream`: no allocation,
 * no host synchronisation, no memset node, so it may be captured in a graph. */
#define SRWCR_MAX_BATCH 32
typedef struct srwcr_batch srwcr_batch;
typedef struct {
    const void *fixed;         /* device, normalised, the plan's fixed dtype */
    const void *moving;        /* device, normalised, the plan's moving dtype */
    const float *ffd;          /* device float32 [3][ncz][ncy][ncx] */
    double *d_value;           /* device double: D */
    float *d_grad;             /* device float32, layout of ffd: dD/d(displacement) */
} srwcr_batch_item;

int srwcr_batch_create(int32_t n, const srwcr_plan *const *plans, srwcr_batch **out);
void srwcr_batch_destroy(srwcr_batch *batch);
size_t srwcr_batch_workspace_bytes(const srwcr_batch *batch);
int srwcr_grad_batched(const srwcr_batch *batch, const srwcr_batch_item *items, void *workspace,
                       size_t workspace_bytes, void *stream);

/* RaPTOR, the patch-based correlation ratio that SRWCR reduces to with a
 * boxcar spatial distribution (eq 6), a linear window h(t) = max(0, 1 - |t|)
 * on the A-bins and frequency estimates of p_r(b) and sigma_r^2 (eqs 13, 14):
 *   RaPTOR = (1/N_p) sum_r (E_r[B^2] - sum_a p_r(a) mu_r(a)^2) / sigma_r^2,
 * p_r(a) = sum_{x in r} h(a - A(x)) / N_r, mu_r(a) its h-weighted mean of B,
 * E_r and sigma_r^2 = E_r[B^2] - E_r[B]^2 plain means over the N_r voxels of
 * patch r.  A and B, the roles, dtypes, warp (FFD or dense field) and the
 * intensity bins are the plan's.  A patch whose B variance is at most 1e-5 of
 * E_r[B^2] adds 0; an empty bin adds nothing.
 *
 * srwcr_patch: a half-open voxel box [x0, x1) x [y0, y1) x [z0, z1) on the
 * fixed grid; it is clipped to the grid, and a patch that the clip empties
 * still counts in N_p.  raptor_patches_create copies n (1 .. 2^24) host boxes
 * to the device for `plan` (which must outlive the set) and returns
 * SRWCR_E_INVALID_ARG for n out of range or NULL pointers, SRWCR_E_UNSUPPORTED
 * for a fixed grid of 2^31 voxels or more.
 *
 * raptor_eval writes RaPTOR to the device double d_value; raptor_grad also
 * writes d_grad (device float32): dRaPTOR/d(FFD displacement) in the layout
 * of srwcr_grad's d_grad when dense = 0, or dRaPTOR/du(x) [3][nz][ny][nx] for
 * a dense field (dense = 1, disp as in srwcr_grad_dense).  The derivative is
 * the exact derivative of eq 13 with the one-sided window derivative of
 * srwcr_grad; the paper states none.  The workspace (raptor_workspace_bytes,
 * 0 for a set made for another plan) is the caller's; the calls only enqueue
 * kernels on `stream` and allocate nothing. */
typedef struct {
    int32_t x0, y0, z0, x1, y1, z1;
} srwcr_patch;
typedef struct raptor_patches raptor_patches;

int raptor_patches_create(const srwcr_plan *plan, const srwcr_patch *patches, int32_t n, raptor_patches **out);
void raptor_patches_destroy(raptor_patches *patches);
size_t raptor_workspace_bytes(const srwcr_plan *plan, const raptor_patches *patches);
int raptor_eval(const srwcr_plan *plan, const raptor_patches *patches, const void *fixed, const void *moving,
                const float *disp, int32_t dense, double *d_value, void *workspace, size_t workspace_bytes,
                void *stream);
int raptor_grad(const srwcr_plan *plan, const raptor_patches *patches, const void *fixed, const void *moving,
                const float *disp, int32_t dense, double *d_value, float *d_grad, void *workspace,
                size_t workspace_bytes, void *stream);

/* Backward-warped moving volume on the fixed grid: out[x] = M(T(x)) with the
 * interpolation of srwcr_eval (Sec. II-F).  moving: normalised device volume in
 * the plan's moving dtype; out: device float32 volume of the fixed dims. */
int ffd_warp(const srwcr_plan *plan, const void *moving, const float *ffd, float *out, void *stream);

/* Options and report of register_lbfgs (Sec. II-F). */
typedef struct {
    int32_t levels;            /* pyramid levels, 1..3 (paper: 3) */
    int32_t max_iter[3];       /* per level, coarsest first (paper: 200, 200, 120) */
    int32_t history;           /* L-BFGS corrections m (paper: 5) */
    int32_t stall_window;      /* stop when D is stable over this many iterations (paper: 20) */
    double stall_tol;          /* relative stability threshold of D over the window */
    double bending_weight;     /* w_p of eq (1); 0 disables the bending-energy term */
} srwcr_lbfgs_opts;

typedef struct {
    int32_t iterations[3];     /* iterations run per level */
    int32_t evaluations[3];    /* value+gradient evaluations per level */
    double initial_value[3];   /* cost at the start of each level */
    double final_value[3];     /* cost at the end of each level */
    int32_t status[3];         /* srwcr_status per level */
    double seconds[3];         /* wall-clock seconds per level (plan, evaluations, optimiser) */
} srwcr_lbfgs_report;

/* Fill `opts` with the paper's settings (3 levels, 200/200/120, m = 5, 20). */
void srwcr_lbfgs_default_opts(srwcr_lbfgs_opts *opts);

/* Multi-resolution L-BFGS registration of Sec. II-F minimising eq (1).
 * fixed, moving: device float32 volumes already normalised to [0, L] (the
 * finest level); ffd_inout: host float32 displacements at the finest level,
 * read as the start and overwritten with the result.  Coarser levels use
 * half-resolution volumes (Gaussian sigma 1 voxel, then every other voxel) and
 * the same control spacing in level voxels; the start is carried down to the
 * coarsest level by keeping every second control node and halving it, and
 * displacements are carried up by doubling and B-spline subdivision.  The line
 * search is the backtracking Wolfe search of Sec. II-F, bracketed (see
 * srwcr_lbfgs_minimize).  Synchronous; allocates its own temporaries. */
int register_lbfgs(const srwcr_problem *prob, const float *fixed, const float *moving, float *ffd_inout,
                   const srwcr_lbfgs_opts *opts, srwcr_lbfgs_report *report, void *stream);

/* The optimiser of register_lbfgs on the host, for any cost: L-BFGS with
 * `history` corrections (two-loop recursion) and a backtracking line search
 * on the Armijo (c1 = 1e-4) and curvature (c2 = 0.9) conditions: the step
 * halves while no acceptable step is bracketed from above and grows by 2.1
 * while none is bracketed from below, then bisects the bracket (at most 40
 * trials; if none satisfies both conditions the best trial point is kept,
 * else SRWCR_E_LINESEARCH).  Stops after max_iter iterations or when the cost
 * varied by at most stall_tol |f| over the last stall_window iterations
 * (Sec. II-F).  fg(user, x, f, g) writes the cost and its gradient (n doubles)
 * at x and returns 0, or a non-zero status that stops the run and is
 * returned.  x (n doubles, host) is the start and receives the result;
 * iterations, evaluations and f_final may be NULL. */
typedef int (*srwcr_fg_fn)(void *user, const double *x, double *f, double *g);
int srwcr_lbfgs_minimize(int64_t n, double *x, srwcr_fg_fn fg, void *user, int32_t max_iter, int32_t history,
                         int32_t stall_window, double stall_tol, int32_t *iterations, int32_t *evaluations,
                         double *f_final);

/* Carry displacements from a pyramid level to the next finer one: u_f(x) =
 * 2 u_c(x / 2) represented exactly on the finer lattice by cubic B-spline
 * subdivision (fine node 2i = (c[i-1] + 6 c[i] + c[i+1]) / 8, node 2i + 1 =
 * (c[i] + c[i+1]) / 2, paper node indices; nodes outside the coarse lattice
 * count as 0).  Host arrays float32 [3][nc_z][nc_y][nc_x]. */
int srwcr_refine_ffd(const int32_t coarse_nc[3], const float *coarse, const int32_t fine_nc[3], float *fine);

/* Bending energy C_p of eq (1) (the constraint term, after Rueckert et al.):
 * the sum over control-node positions inside the fixed grid of
 * sum_e [u_xx^2 + u_yy^2 + u_zz^2 + 2 (u_xy^2 + u_xz^2 + u_yz^2)] of the FFD
 * displacement u.  Host arrays; `grad` (optional) receives dC_p/dd.
 * Returns -1 on invalid arguments. */
double srwcr_bending_energy(const srwcr_problem *prob, const float *ffd, float *grad);

/* ---- diagnostics (used by the test-suite; not needed for registration) ---- */

/* Run only the value pass and copy the raw joint moments of eq (3) summed over
 * b -- per region r and A-bin a: P = sum w h(a - A), S1 = sum w h(a - A) m1(B),
 * S2 = sum w h(a - A) m2(B) with m1, m2 the Parzen moments of B -- into the
 * device array d_moments, double [R][n_bins][3], R = Kx Ky Kz (x fastest). */
int srwcr_debug_moments(const srwcr_plan *plan, const void *fixed, const void *moving, const float *ffd,
                        double *d_moments, void *workspace, size_t workspace_bytes, void *stream);

/* Diagnostic: the warp pass alone (eq 17 and the backward warp of Sec. II-F),
 * then, per fixed voxel, the moving sample's lower Parzen bin
 * k = min(floor(s), L - 1) (eq 5; decided in FP64) into d_bin (int32, fixed
 * dims, x fastest) and its in-bin position s - k, rounded to FP32, into d_frac.
 * These are the bins the value and gradient passes use.  Device pointers,
 * caller-owned; asynchronous on `stream`; the workspace is the plan's
 * (srwcr_workspace_bytes).  Returns SRWCR_E_INVALID_ARG for NULL pointers and
 * SRWCR_E_WORKSPACE for a short workspace. */
int srwcr_debug_samples(const srwcr_plan *plan, const void *moving, const float *ffd, int32_t *d_bin,
                        float *d_frac, void *workspace, size_t workspace_bytes, void *stream);

/* Diagnostic of the bounds-checked debug build (a library compiled with
 * SRWCR_CHECK, see build.py): its kernels range-check the computed indices of
 * their scatters, atomics and voxel reads, skip an access that falls outside
 * its array and record the failed check as a bit of a device-wide word
 * (bit 0: warp-pass voxel, 1: value-pass block region, 2: moment slot, 3:
 * gradient-table slot, 4: gradient scratch, 5: node block, 6: gradient
 * accumulator, 7: gradient-pass voxel, 8: column value-pass voxel).
 * Synchronises the device, writes the word to *flags (host int32) and, if
 * `reset`, clears it.  Returns SRWCR_E_UNSUPPORTED in the normal build,
 * SRWCR_E_INVALID_ARG for a NULL flags. */
int srwcr_debug_check_flags(int32_t *flags, int32_t reset);

/* Launch geometry of a plan: number of work items and LDS bytes per workgroup
 * of the value and gradient passes.  Any output pointer may be NULL. */
int srwcr_plan_info(const srwcr_plan *plan, int32_t *n_items, int32_t *value_lds, int32_t *grad_lds);

/* Per-kernel timing of srwcr_grad with HIP events on the caller's stream.
 * srwcr_profile(plan, 1) starts a session (up to 4096 calls are recorded, the
 * first call creates the events), srwcr_profile(plan, 0) stops recording.
 * srwcr_profile_read synchronises the recorded events and returns the summed
 * milliseconds of the six phases -- zeroing (no kernel for a plan with a
 * staged value pass, whose warp pass clears the gradient accumulators), warp
 * pass, value pass, finalisation (with the merge of a staged value pass),
 * gradient pass, gradient output -- and the number of calls
 * recorded.  raptor_grad calls on the plan are recorded too, with the phases
 * zeroing, warp pass, patch sums, patch finalisation, per-voxel derivative,
 * chain rule (gradient pass and output).  enable = 2 records only the two
 * events around the value pass (patch sums for RaPTOR), enable = 3 only those
 * around the gradient pass (per-voxel derivative for RaPTOR), so that timing
 * one pass adds one event pair per call; the other phases then read 0.  Any
 * other mode is SRWCR_E_INVALID_ARG.  Read the results before changing the
 * mode.  Not thread-safe: profile one stream and
 * one kind of call at a time. */
int srwcr_profile(const srwcr_plan *plan, int32_t enable);
int srwcr_profile_read(const srwcr_plan *plan, double ms[6], int32_t *calls);

/* Thread-local description of the last failure on this thread. */
const char *srwcr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SRWCR_H */
