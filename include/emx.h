/*
 * emx.h - C ABI of the MI355X (gfx950) box-constrained Euclidean-median
 * library.
 *
 * Method: K. N. Chaudhury and K. R. Ramakrishnan, "A new ADMM algorithm for
 * the Euclidean median and its application to robust patch regression"
 * (arXiv:1501.03879).  The library computes, for many independent instances,
 *
 *     min over z in C = [lo, hi]^d of  sum_k w_k ||z - a_k||_2        (EM)
 *
 * by the variable-splitting ADMM of Section 2 (Algorithm 1, EM-ADMM): local
 * copies x_k updated by the closed-form prox of w_k/mu ||. - a_k|| (block
 * soft-thresholding, equation (closed-form)), the global z by the box
 * projection of the unweighted mean of x_k + y_k/mu (equation (updatez)),
 * and the multipliers by y_k += mu (x_k - z) (equation (updatey)).  The
 * penalty mu is called rho in this interface.  nlem_denoise applies it to
 * every pixel of an image as in Section 3 (Non-Local Euclidean Medians).
 *
 * Conventions shared by every call:
 *  - All array arguments are DEVICE pointers owned by the caller.  They must
 *    stay valid until the work queued on `stream` has finished.  The library
 *    never frees or retains them.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Every compute call only queues work on it and returns; kernel faults
 *    surface from em_sync or from the caller's own synchronisation.
 *    em_solve_batch(_ex) also runs shape classes on three internal streams
 *    of the handle, forked from `stream` and joined back into it by events,
 *    so its work is still ordered on `stream` as seen by the caller.
 *  - Graph capture: em_solve_batch(_ex), em_solve_plain(_ex), nlem_denoise,
 *    nlem_denoise_ex and nlm_denoise may be recorded into a HIP graph by
 *    stream capture after an earlier call of the same sizes on the same
 *    handle has sized its workspace: they then only
 *    launch kernels (work-queue heads are cleared by a kernel, not a memset)
 *    and neither allocate nor synchronise.  nlem_autotune and
 *    em_batch_autotune synchronise and cannot be captured; a batch plan with
 *    host_counts makes em_solve_batch(_ex) wait for its classification
 *    outside capture (em_batch_plan_t).
 *  - Argument errors are detected on the host before anything is queued and
 *    return EM_ERR_INVALID_ARG (nothing is written).  Problems inside one
 *    instance (no points, a bad weight or point) are reported per instance in
 *    em_stats_t.flags, never as a call error.
 *  - Starting point: y_k = 0 (Section 3) and z as documented per call; the
 *    starting z is used as given (Algorithm 1 does not project it).
 *  - Stopping (the paper leaves the criterion open): after iteration t,
 *        r_pri  = sqrt( sum_k ||x_k - z||^2 / (n d) )
 *        r_dual = sqrt( ||z^t - z^{t-1}||^2 / d ),
 *    stop when both are <= tol * D, where D = hi - lo for a finite box and
 *    max(1, max_k ||a_k||_inf) otherwise.  The primal residual is only
 *    evaluated on iterations that follow one with r_dual <= tol D (times a
 *    plan's arm factor >= 1; nlem_plan_t, em_batch_plan_t) and on the last
 *    allowed iteration, so a solve may end one iteration later than a solver
 *    that evaluates both every iteration (up to check_every iterations later
 *    under a plan that checks only every check_every-th iteration).  tol = 0 runs
 *    exactly max_iter iterations; max_iter = 0 returns the starting z.
 *  - Arithmetic is FP32 (image storage may be FP16, widened on load).
 */
#ifndef EMX_H
#define EMX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    EM_OK = 0,
    EM_ERR_INVALID_ARG = -1,   /* bad pointer, size, parameter or handle */
    EM_ERR_UNSUPPORTED = -2,   /* valid request outside the compiled limits */
    EM_ERR_OUT_OF_MEMORY = -3, /* workspace allocation failed */
    EM_ERR_HIP = -4            /* a HIP runtime call failed */
} em_status_t;

/* em_stats_t.flags bits */
enum {
    EM_CONVERGED = 1, /* stopped by the residual test */
    EM_MAXITER = 2,   /* stopped after max_iter iterations */
    EM_EMPTY = 4,     /* n = 0: z left as given */
    EM_BAD_INPUT = 8  /* negative/non-finite weight or non-finite point: z set to NaN */
};
/* Accelerated ADMM (EM_SOLVER_ADMM_FAST): flags >> EM_RESTART_SHIFT is the
 * number of restarts the solve took (capped at 2^23 - 1); the low byte holds
 * the bits above.  Other solvers leave the upper bits zero. */
#define EM_RESTART_SHIFT 8

/* Starting value of z for em_solve_batch / em_solve_plain. */
typedef enum {
    EM_INIT_GIVEN = 0, /* the caller's z (in/out) */
    EM_INIT_MAXW = 1,  /* the point of largest weight, lowest index on ties */
    EM_INIT_WMEAN = 2  /* the weighted mean sum_k w_k a_k / sum_k w_k, the analogue of the
                          NLM patch of Section 3 (the plain mean of the points when every
                          weight is zero); not projected, like the other starts */
} em_init_t;

/* Limits of the library. */
#define EM_MAX_D 64            /* largest dimension d per instance */
#define EM_MAX_N 512           /* largest point count n per instance */
#define EM_MAX_PATCH_RADIUS 3  /* nlem: patch side 2r+1 <= 7 (d <= 49) */
#define EM_MAX_WINDOW_RADIUS 10/* nlem: window side 2R+1 <= 21 (n <= 441) */
#define EM_NOALLOC_MAX_PIXELS (1 << 22) /* nlem_denoise_noalloc: largest H * W */

/*
 * One instance of a batch, in device memory (32 bytes).  Points a_k are
 * n x d float32 values, point-major, starting at a[a_off]; weights w_k are n
 * float32 at w[w_off]; z (d float32) lives at z[z_off].
 */
typedef struct {
    int64_t a_off;
    int64_t w_off;
    int64_t z_off;
    int32_t n;
    int32_t d;
} em_instance_t;

/* Per-instance (or per-pixel) result record, in device memory (16 bytes). */
typedef struct {
    int32_t iters;  /* iterations run */
    int32_t flags;  /* EM_* bits */
    float r_pri;    /* residuals of the last iteration (NaN if not evaluated, 0 if none ran) */
    float r_dual;
} em_stats_t;

typedef struct em_context *em_handle_t;

/*
 * Create a handle bound to HIP device `device` (it becomes current for the
 * calling thread).  The handle owns a small device workspace (work-queue
 * counters, instance class lists) that grows on demand and is released by
 * em_destroy.  One handle per host thread; a handle is not thread-safe, and
 * concurrent calls on one handle from different streams race on its
 * workspace.
 * Errors: INVALID_ARG for a NULL out-pointer or a bad device index;
 * OUT_OF_MEMORY; HIP.
 */
em_status_t em_create(em_handle_t *handle, int device);

/* Release a handle after synchronising its device.  NULL is accepted. */
em_status_t em_destroy(em_handle_t handle);

/*
 * em_solve_batch - solve B independent instances of (EM) with one persistent
 * kernel per shape class (Algorithm 1; the z-update mean is over the n points
 * of the instance, equation (updatez) with N = n).
 *   a, w, inst, z, stats: device pointers (stats may be NULL);
 *   inst[B] describes the instances (n in [0, EM_MAX_N], d in [1, EM_MAX_D]);
 *   lo <= hi (either may be infinite; lo = -inf and hi = +inf give the
 *   unconstrained median); rho > 0 finite is the penalty mu; max_iter >= 0;
 *   tol >= 0; init is an em_init_t.
 * Instances must not overlap in z.  n = 0 leaves z unchanged (EMPTY).
 * Errors: INVALID_ARG (NULL handle, NULL pointers with B > 0, B < 0, rho <= 0
 * or not finite, max_iter < 0, tol < 0 or NaN, lo > hi or NaN, bad init);
 * UNSUPPORTED when an instance exceeds the limits is NOT detected on the host
 * (the descriptors are device data): such instances get flags = EM_BAD_INPUT
 * and z = NaN.  HIP on launch failure.
 */
em_status_t em_solve_batch(em_handle_t handle, void *stream, int64_t B,
                           const float *a, const float *w, const em_instance_t *inst,
                           float lo, float hi, float rho, int32_t max_iter, float tol,
                           int32_t init, float *z, em_stats_t *stats);

/* Solver of em_solve_batch_ex. */
typedef enum {
    EM_SOLVER_ADMM = 0,          /* Algorithm 1, fixed penalty rho (as em_solve_batch) */
    EM_SOLVER_IRLS = 1,          /* IRLS on the smooth surrogate (EM_surrogate), parameter eps */
    EM_SOLVER_ADMM_ADAPTIVE = 2, /* Algorithm 1 with the penalty adapted by residual balancing */
    EM_SOLVER_ADMM_FAST = 3,     /* accelerated ADMM with restart (boxes; em_solve_batch_ex, em_solve_plain_ex) */
    EM_SOLVER_ADMM_WEIGHTED = 4  /* consensus ADMM with penalty rho w_k per constraint (a weighted-
                                    mean z-update; a different algorithm from Algorithm 1) */
} em_solver_t;

/* The convex set C of (EM) for em_solve_batch_ex. */
typedef enum {
    EM_SET_BOX = 0,  /* [lo, hi] per coordinate (Section 3 uses [0, 255]^d) */
    EM_SET_BALL = 1  /* {z : ||z - center|| <= radius}: projection scales z - center */
} em_set_t;

/* Options of em_solve_batch_ex (host memory; the box arrays are device memory). */
typedef struct {
    int32_t solver;        /* em_solver_t */
    int32_t init;          /* em_init_t */
    float lo, hi;          /* one interval for every coordinate (when box_lo is NULL) */
    const float *box_lo;   /* NULL, or per-coordinate lower bounds, device, indexed like z */
    const float *box_hi;   /* NULL, or per-coordinate upper bounds (both NULL or both set) */
    float rho;             /* ADMM penalty mu (the starting penalty for ADAPTIVE) */
    float eps;             /* IRLS surrogate parameter */
    int32_t max_iter;
    float tol;
    int32_t adapt_every;   /* ADAPTIVE: balance after every adapt_every-th iteration (>= 1) */
    float adapt_ratio;     /* ADAPTIVE: imbalance ratio that triggers a change (> 1, e.g. 10) */
    float adapt_factor;    /* ADAPTIVE: factor applied to rho (> 1, e.g. 2) */
    float fast_eta;        /* FAST: restart parameter eta in (0, 1) (0.999 in [Goldstein2012]) */
    int32_t set;           /* em_set_t: the convex set C */
    const float *ball_center; /* BALL: NULL (origin) or centres, device, indexed like z */
    const float *ball_radius; /* BALL: NULL (use radius) or one radius per instance, device */
    float radius;          /* BALL: the radius when ball_radius is NULL */
    int32_t points_f16;    /* nonzero: `a` holds the points as FP16 (binary16), widened to FP32
                              when staged; offsets count elements (em_solve_batch_ex only) */
} em_options_t;

/*
 * em_solve_batch_ex - em_solve_batch with a choice of solver and a general box.
 *   Box (set = EM_SET_BOX): [lo, hi] for every coordinate, or per
 *     coordinate: instance b, coordinate j uses [box_lo[z_off + j],
 *     box_hi[z_off + j]] (same layout as z).  An instance whose bounds have
 *     lo_j > hi_j or a NaN gets flags = EM_BAD_INPUT and z = NaN.  The
 *     tolerance scale D is the widest interval max_j (hi_j - lo_j) when
 *     finite and > 0, else max(1, max_k ||a_k||_inf).
 *   Ball (set = EM_SET_BALL; (EM) allows any closed convex C, and the ball
 *     has the closed-form projection center + (z - center) min(1, radius /
 *     ||z - center||)): centre ball_center[z_off + j] (origin when NULL),
 *     radius ball_radius[b] (or `radius`); a negative or NaN radius or a
 *     non-finite centre gives EM_BAD_INPUT; D = 2 radius when finite and
 *     > 0.  Solvers ADMM, WEIGHTED and IRLS (not ADAPTIVE); box_lo / box_hi
 *     must be NULL.
 *   EM_SOLVER_ADMM: Algorithm 1 exactly as em_solve_batch.
 *   EM_SOLVER_ADMM_ADAPTIVE: after every adapt_every-th iteration t that did
 *     not stop, with ||r|| = (sum_k ||x_k - z||^2)^(1/2) and
 *     ||s|| = rho (n ||z^t - z^{t-1}||^2)^(1/2) (residual balancing, the
 *     extension the paper's conclusion names; Boyd et al. 2011, 3.4.1):
 *     ||r|| > adapt_ratio ||s|| multiplies rho by adapt_factor,
 *     ||s|| > adapt_ratio ||r|| divides it; the multipliers y_k are kept.
 *     Both residuals are evaluated on those iterations.
 *   EM_SOLVER_IRLS: omega_k = w_k / (||z - a_k||^2 + eps)^(1/2),
 *     z' = P_C(sum_k omega_k a_k / sum_k omega_k) (majorise-minimise steps of
 *     the surrogate; the box projection is exact for its isotropic
 *     quadratic majoriser); stopped on r_dual alone (stats r_pri = 0); all
 *     weights zero: every point of C is a minimiser, z becomes the start
 *     projected onto C and the solve reports CONVERGED after one iteration.
 *   EM_SOLVER_ADMM_FAST: the accelerated ADMM with restart, as documented
 *     at em_solve_plain_ex (same iterates, both residuals tested every
 *     sweep, restarts counted in flags >> EM_RESTART_SHIFT), batched: 8
 *     coordinates per wave, up to 8 waves and 8 points per lane, its
 *     second n x d state in registers.  Boxes only.
 *   EM_SOLVER_ADMM_WEIGHTED: the consensus splitting of Section 2 with the
 *     penalty rho w_k on the constraint x_k = z of point k instead of one rho
 *     for all: x_k = prox with threshold w_k / (rho w_k) = 1 / rho at
 *     z - y_k / (rho w_k), z' = P_C(sum_k w_k (x_k + y_k / (rho w_k)) /
 *     sum_k w_k), y_k += rho w_k (x_k - z').  Same minimiser as Algorithm 1,
 *     other iterates; points of weight zero are left out (all weights zero:
 *     z' = P_C(z)); r_pri runs over the points of positive weight.
 * Other arguments, limits and per-instance rules as for em_solve_batch.
 * Errors: INVALID_ARG (NULL options, bad solver or init, rho <= 0 for ADMM,
 * eps <= 0 for IRLS, adapt_every < 1, adapt_ratio <= 1 or adapt_factor <= 1
 * for ADAPTIVE, one of box_lo / box_hi NULL, a bad set, a ball with box
 * arrays, fast_eta outside (0, 1) for FAST, and em_solve_batch's errors);
 * UNSUPPORTED for the ball with ADAPTIVE or FAST; HIP.
 */
em_status_t em_solve_batch_ex(em_handle_t handle, void *stream, int64_t B,
                              const float *a, const float *w, const em_instance_t *inst,
                              const em_options_t *opt, float *z, em_stats_t *stats);

/*
 * em_solve_plain_ex - the one-launch-per-instance path with options: solver
 * EM_SOLVER_ADMM (as em_solve_plain, with the general box) or
 * EM_SOLVER_ADMM_FAST, the accelerated ADMM the conclusion names
 * ([Goldstein2012], fast ADMM with restart for weakly convex problems) on the
 * same splitting, with predictors z_hat, y_hat (starting at z0 and 0):
 *   x_k = prox at z_hat - y_hat_k / rho, z = P_C(mean_k(x_k + y_hat_k / rho)),
 *   y_k = y_hat_k + rho (x_k - z),
 *   c = rho (sum_k ||x_k - z||^2 + n ||z - z_hat||^2);
 *   c < fast_eta (1 - 2^-16) c_prev: alpha' = (1 + sqrt(1 + 4 alpha^2)) / 2, beta =
 *     (alpha - 1) / alpha', z_hat = z + beta (z - z_prev),
 *     y_hat = y + beta (y - y_prev);
 *   otherwise restart: z_hat = z_prev, y_hat = y_prev, alpha = 1,
 *     c_prev = c_prev / fast_eta
 * (alpha = 1 and c_prev = +inf at the start; no decision is taken after the
 * last allowed sweep, and stats.flags >> EM_RESTART_SHIFT counts the
 * restarts).  The guard 1 - 2^-16 on the momentum test resolves the exact
 * ties of a stalled iterate (each sweep repeating c, then c against
 * fast_eta (c / fast_eta) after a restart) to the restart side, as exact
 * arithmetic does, in FP32 as in the FP64 oracle.  Residuals and stopping as for
 * em_solve_batch, evaluated every iteration.  Its momentum needs the previous
 * multipliers, a second n x d state, which this path keeps in device memory
 * (em_solve_batch_ex runs the same solver batched, the state in registers).
 * Other solvers and the ball return EM_ERR_UNSUPPORTED; arguments and errors
 * otherwise as em_solve_plain and em_solve_batch_ex (fast_eta must be in
 * (0, 1)).
 */
em_status_t em_solve_plain_ex(em_handle_t handle, void *stream, int64_t B,
                              const float *a, const float *w, const em_instance_t *inst,
                              const em_instance_t *inst_host, const em_options_t *opt, float *z,
                              em_stats_t *stats);

/*
 * em_solve_plain - the same computation as em_solve_batch with one kernel
 * launch per instance and the iterates kept in device memory: the simple
 * one-instance-per-launch baseline the batched solver is measured against.
 * Same arguments and errors; it additionally needs the descriptors on the
 * host, so `inst_host` (host memory, B entries, identical to `inst`) is
 * required.
 */
em_status_t em_solve_plain(em_handle_t handle, void *stream, int64_t B,
                           const float *a, const float *w, const em_instance_t *inst,
                           const em_instance_t *inst_host,
                           float lo, float hi, float rho, int32_t max_iter, float tol,
                           int32_t init, float *z, em_stats_t *stats);

/*
 * nlem_denoise - Non-Local Euclidean Medians (Section 3): for every pixel i of
 * the H x W image (row-major, FP32, or FP16 when img_is_f16 != 0):
 *   points  a_j = P_j, the (2r+1)^2 patch around pixel j (row-major; pixels
 *           beyond the image border by symmetric reflection, x[-1] = x[0]),
 *           for every pixel j of the (2R+1)^2 search window around i that is
 *           inside the image (the window is truncated at borders; j = i is
 *           included);
 *   weights w_ij = exp(-||P_i - P_j||^2 / h^2)  (not normalised, w_ii = 1);
 *   box     [lo, hi]^d (finite), z starts at the noisy patch P_i;
 *   output  out[i] = the centre coordinate of the solution patch
 *           (equation (L1regression) and the text after it).
 * r = patch_radius in [0, EM_MAX_PATCH_RADIUS], R = window_radius in
 * [0, EM_MAX_WINDOW_RADIUS], both < min(H, W); h_param > 0.
 * stats: NULL or H*W records.  `out` must not alias `img`.
 * Scheduling: in tolerance mode (tol > 0) the pixels of a shape group at
 * least four times as large as the resident grid are solved in longest-first
 * order (decreasing standard deviation of the noisy patch, which tracks the
 * iteration count for 7x7 patches; with smaller patches only groups below
 * sixteen times the resident grid are ordered); the environment variable
 * EMX_NLEM_ORDER=0 keeps raster order.  Each
 * workgroup takes a few consecutive queue positions per atomic when pixels
 * are cheap (small windows and patches); EMX_NLEM_CHUNK=k (1..64) fixes
 * that count.  Results do not depend on either.
 * Errors: INVALID_ARG (NULL handle/img/out, H or W < 1, radii out of range,
 * h_param <= 0, lo/hi not finite or lo > hi, rho <= 0, max_iter < 0,
 * tol < 0); UNSUPPORTED (radii above the compiled limits); HIP.
 */
em_status_t nlem_denoise(em_handle_t handle, void *stream, const void *img, int32_t img_is_f16,
                         int32_t H, int32_t W, int32_t patch_radius, int32_t window_radius,
                         float h_param, float lo, float hi, float rho, int32_t max_iter,
                         float tol, float *out, em_stats_t *stats);

/*
 * nlem_denoise_noalloc - nlem_denoise for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, semantics, kernels and
 * results as nlem_denoise (bit for bit), but the work-queue head and the
 * longest-first order scratch live in a static device array of the library
 * (256 + 5 * EM_NOALLOC_MAX_PIXELS + 4096 bytes, about 20 MiB), which every
 * GPU the library runs on holds until the process ends; the call makes no
 * hipMalloc, hipFree or other allocating call (em_kernel_timing does not
 * cover it).  The array is shared by every call on the same GPU and keeps
 * the last call's contents; the call clears what must start at zero with
 * kernels on `stream`.  Calls that overlap on one GPU (concurrent streams,
 * several handles or host threads) race on the array and give wrong
 * results: serialise them.
 * Errors: as nlem_denoise; UNSUPPORTED also when H * W > EM_NOALLOC_MAX_PIXELS
 * or the device index is 64 or more.
 */
em_status_t nlem_denoise_noalloc(em_handle_t handle, void *stream, const void *img, int32_t img_is_f16,
                                 int32_t H, int32_t W, int32_t patch_radius, int32_t window_radius,
                                 float h_param, float lo, float hi, float rho, int32_t max_iter,
                                 float tol, float *out, em_stats_t *stats);

/* One image of an nlem_denoise_multi call (host memory; pointers are device). */
typedef struct {
    const void *img;       /* H x W, FP32 or FP16 (per img_is_f16) */
    float *out;            /* H x W */
    em_stats_t *stats;     /* NULL or H*W */
    int32_t H, W;
    int32_t patch_radius, window_radius;
    float h_param;
    int32_t img_is_f16;
} nlem_image_t;

/*
 * nlem_denoise_multi - nlem_denoise for `count` images of different sizes and
 * radii, queued as one captured HIP graph (one persistent launch per shape
 * class, the classes running concurrently).  The graph is cached on the
 * handle and re-launched when the same image list (pointers, sizes, radii)
 * and parameters are passed again.  Per-image rules and errors as for
 * nlem_denoise; `images` is host memory with `count` entries.
 */
em_status_t nlem_denoise_multi(em_handle_t handle, void *stream, int32_t count,
                               const nlem_image_t *images, float lo, float hi, float rho,
                               int32_t max_iter, float tol);

/* Solver of nlem_denoise_ex. */
typedef enum {
    NLEM_SOLVER_ADMM = 0, /* EM-ADMM (Algorithm 1) on (EM), penalty rho */
    NLEM_SOLVER_IRLS = 1  /* IRLS on the smooth surrogate (EM_surrogate), parameter eps */
} nlem_solver_t;

/* Starting patch z^0 of nlem_denoise_ex (the two options of Section 3). */
typedef enum {
    NLEM_INIT_NOISY = 0, /* the noisy patch P_i */
    NLEM_INIT_NLM = 1    /* the Non-Local Means patch sum_j w_ij P_j / sum_j w_ij */
} nlem_init_t;

/* Options of nlem_denoise_ex (host memory). */
typedef struct {
    int32_t solver;   /* nlem_solver_t */
    int32_t init;     /* nlem_init_t */
    float lo, hi;     /* the box [lo, hi]^d, finite, lo <= hi */
    float rho;        /* ADMM penalty mu, finite > 0 (ignored by IRLS) */
    float eps;        /* IRLS surrogate parameter, finite > 0 (ignored by ADMM) */
    int32_t max_iter; /* >= 0 */
    float tol;        /* >= 0 */
} nlem_options_t;

/*
 * nlem_denoise_ex - nlem_denoise for `count` images (one persistent launch per
 * shape group, no graph) with a choice of solver and starting patch.
 *   ADMM: exactly nlem_denoise, started from opt->init's patch.
 *   IRLS: the iteratively reweighted least-squares method for the smooth
 *     surrogate sum_j w_ij (||P - P_j||^2 + eps)^(1/2) that Section 1 cites
 *     and Table 1 compares (the paper does not print its steps; they are the
 *     majorise-minimise steps of that surrogate over the box):
 *       omega_j = w_ij / (||z - P_j||^2 + eps)^(1/2),
 *       z'      = P_C( sum_j omega_j P_j / sum_j omega_j ),
 *     stopped when r_dual = sqrt(||z' - z||^2 / d) <= tol (hi - lo) (checked
 *     one iteration late, as the ADMM primal residual) or after max_iter
 *     iterations; stats report r_pri = 0.  eps is in squared intensity units
 *     (the paper uses 1e-6 with intensities in [0, 255]).
 *   init = NLEM_INIT_NLM with max_iter = 0 returns the NLM estimate.
 * Weights, window, border and output rules as for nlem_denoise; `images` and
 * `opt` are host memory.
 * Errors: INVALID_ARG (NULL handle/options, bad image list or image, bad
 * solver/init, eps <= 0 for IRLS, parameter errors of nlem_denoise);
 * UNSUPPORTED (radii above the limits); HIP.
 */
em_status_t nlem_denoise_ex(em_handle_t handle, void *stream, int32_t count,
                            const nlem_image_t *images, const nlem_options_t *opt);

/*
 * nlm_denoise - the Non-Local Means estimate that Table 1 compares NLEM with:
 * out[i] = sum_j w_ij g_j / sum_j w_ij over the same truncated search window
 * and weights as nlem_denoise (g_j the noisy pixel j, the centre of P_j).
 * Arguments and errors as for nlem_denoise (no solver parameters, no stats).
 */
em_status_t nlm_denoise(em_handle_t handle, void *stream, const void *img, int32_t img_is_f16,
                        int32_t H, int32_t W, int32_t patch_radius, int32_t window_radius,
                        float h_param, float *out);

/* Where the values of a plan come from. */
typedef enum {
    EM_PLAN_BUILTIN = 0,  /* the built-in table and rules */
    EM_PLAN_TUNED = 1,    /* measured by an autotune call on this handle */
    EM_PLAN_CACHE = 2,    /* loaded from the EMX_AUTOTUNE_CACHE file when the handle was created */
    EM_PLAN_SET = 3       /* given by the caller (nlem_plan_set, em_batch_plan_set) */
} em_plan_source_t;

/*
 * The schedule of the NLEM solve kernel for one shape (patch radius, window
 * class, solver, image storage): its tile shape and the schedule of its
 * persistent work queue.  Every choice gives a correct solve: waves changes
 * the summation order (results agree to FP32 rounding), chunk and order only
 * which workgroup solves which pixel when, and arm_factor and check_every
 * only on which iterations the primal residual is evaluated (a solve stops at
 * the first evaluated iteration with both residuals within tol D: at most one
 * iteration after an evaluation on every iteration would have stopped it with
 * check_every = 1, at most check_every iterations after it otherwise).
 */
typedef struct {
    int32_t waves;       /* coordinate waves per pixel (a compiled count, 1..4) */
    int32_t chunk;       /* queue positions per atomic pop, 1..64; 0 = the built-in size rule */
    int32_t order;       /* longest-first pixel order (tolerance mode): -1 = the built-in rule,
                            0 = off, 1 = on */
    float arm_factor;    /* the primal residual is evaluated on iterations that follow one with
                            r_dual <= arm_factor tol D, and on the last one; >= 1, 1 = built-in */
    int32_t check_every; /* ... and only on iterations t that are multiples of check_every
                            (1, 2, 4 or 8; 1 = built-in) */
    int32_t source;      /* em_plan_source_t; ignored by nlem_plan_set */
} nlem_plan_t;

/*
 * nlem_autotune - measure schedules for this image's shape, solver and
 * storage on `stream` (synchronously, `repeats` timed runs of each candidate
 * after one warm-up) and keep the fastest as the handle's plan: first every
 * compiled coordinate-wave count with the built-in queue rules, then, with
 * the best count, queue chunks 1, 2, 4 and 8, then (tolerance mode) the
 * queue order off and on, then (tolerance mode, EM-ADMM) arm factors 1.5, 2
 * and 3 and residual-check intervals 2, 4 and 8; a candidate after the wave
 * count replaces the plan only when it is more than 1% faster than the plan
 * kept so far, timed again right before it.  nlem_denoise, nlem_denoise_ex and nlem_denoise_multi
 * use the plan from then on (for a launch of several images, the plan of its
 * shape with FP16 storage when every image in it is FP16); the environment
 * variables EMX_NLEM_WC, EMX_NLEM_CHUNK and EMX_NLEM_ORDER still override.
 * When EMX_AUTOTUNE_CACHE names a file, the plan is appended to it and every
 * later em_create on the same architecture loads it.  The image's out and
 * stats are written by the trials (the last candidate's results).
 * chosen: NULL or receives the chosen coordinate-wave count.
 * Errors: as nlem_denoise_ex for one image, INVALID_ARG for repeats < 1; HIP.
 */
em_status_t nlem_autotune(em_handle_t handle, void *stream, const nlem_image_t *image,
                          const nlem_options_t *opt, int32_t repeats, int32_t *chosen);

/* The coordinate-wave count the handle uses for a shape and solver with FP32
 * storage (the plan's, else the built-in default; without a plan, a shape
 * group shorter than four rounds of the resident grid in tolerance mode runs
 * with the most waves compiled for the shape instead).  Errors: INVALID_ARG. */
em_status_t nlem_plan(em_handle_t handle, int32_t patch_radius, int32_t window_radius,
                      int32_t solver, int32_t *waves);

/* The whole plan of a shape, solver and storage (img_is_f16): the handle's
 * plan with its source, or the built-in values (waves = the default count,
 * chunk 0, order -1, arm_factor 1, check_every 1, source EM_PLAN_BUILTIN).
 * Errors: INVALID_ARG (NULL arguments, bad shape or solver). */
em_status_t nlem_plan_get(em_handle_t handle, int32_t patch_radius, int32_t window_radius,
                          int32_t solver, int32_t img_is_f16, nlem_plan_t *plan);

/* Set the handle's plan of a shape, solver and storage (source becomes
 * EM_PLAN_SET; not written to the cache file), or with plan = NULL return
 * it to the built-in values.  Errors: INVALID_ARG (bad shape or solver,
 * waves not compiled for the shape, chunk outside 0..64, order outside
 * -1..1, arm_factor not finite or below 1, check_every not 1, 2, 4 or 8). */
em_status_t nlem_plan_set(em_handle_t handle, int32_t patch_radius, int32_t window_radius,
                          int32_t solver, int32_t img_is_f16, const nlem_plan_t *plan);

/*
 * The schedule of the batched fixed-penalty EM-ADMM (em_solve_batch and
 * em_solve_batch_ex with EM_SOLVER_ADMM over a box, and the plain path,
 * which follows the same routing): for each of the 28 sliced classes (d in
 * (16, 64], n <= 448; class k = 7 (ceil(d / 13) - 2) + ceil(n / 64) - 1:
 * 13-coordinate slices over ceil(d / 13) waves, ceil(n / 64) points per lane)
 * whether its instances run there or in the generic classes (16-coordinate
 * slices over ceil(d / 16) waves, 1, 2 or 4 points per lane and one or two
 * point waves), and the arm factor and check interval of the primal residual
 * (as nlem_plan_t).  Far-outlier deferral is unaffected.
 */
typedef struct {
    uint64_t generic_classes;  /* bit k set: sliced class k is routed to the generic classes */
    float arm_factor;          /* >= 1, 1 = built-in */
    int32_t check_every;       /* 1, 2, 4 or 8; 1 = built-in */
    int32_t host_counts;       /* 1: the call reads the class counts back after classifying the
                                  batch (it then waits for the stream up to that point, so it is
                                  no longer asynchronous) and launches only the populated classes,
                                  largest work first over its streams, each grid no larger than
                                  its count; ignored while the stream is being captured; 0 =
                                  built-in (every class launched, nothing waited for) */
    int32_t source;            /* em_plan_source_t; ignored by em_batch_plan_set */
} em_batch_plan_t;

/*
 * em_batch_autotune - measure the batched fixed-penalty EM-ADMM on this batch
 * (arguments as em_solve_batch_ex; opt->solver must be EM_SOLVER_ADMM over a
 * box) and keep the fastest schedule as the handle's plan for its point
 * storage (opt->points_f16): after the built-in plan, each sliced class that
 * holds instances of the batch (largest first) is tried in the generic
 * classes, then arm factors 1.5, 2 and 3 and check intervals 2, 4 and 8
 * (tolerance mode), then host_counts; a change is kept when more than 1%
 * faster than the plan kept so far, timed again right before it.  `repeats` timed calls per candidate after one
 * warm-up, synchronously on `stream`; z and stats hold the last candidate's
 * results.  The plan is appended to the EMX_AUTOTUNE_CACHE file as for
 * nlem_autotune.  chosen: NULL or receives the plan.
 * Errors: as em_solve_batch_ex; INVALID_ARG for repeats < 1; UNSUPPORTED for
 * other solvers or sets; HIP.
 */
em_status_t em_batch_autotune(em_handle_t handle, void *stream, int64_t B, const float *a,
                              const float *w, const em_instance_t *inst, const em_options_t *opt,
                              float *z, em_stats_t *stats, int32_t repeats, em_batch_plan_t *chosen);

/* The batch plan for point storage points_f16 (the handle's, else the
 * built-in: no class routed, arm_factor 1, check_every 1, host_counts 0).
 * solver must be EM_SOLVER_ADMM.
 * Errors: INVALID_ARG. */
em_status_t em_batch_plan_get(em_handle_t handle, int32_t solver, int32_t points_f16,
                              em_batch_plan_t *plan);

/* Set the batch plan for point storage points_f16 (source EM_PLAN_SET), or
 * with plan = NULL return to the built-in one.  Errors: INVALID_ARG (solver
 * other than EM_SOLVER_ADMM, bits above the 28 classes, arm_factor not finite
 * or below 1, check_every not 1, 2, 4 or 8, host_counts not 0 or 1). */
em_status_t em_batch_plan_set(em_handle_t handle, int32_t solver, int32_t points_f16,
                              const em_batch_plan_t *plan);

/*
 * em_kernel_timing - for measurement tools: while enabled (enable != 0),
 * every NLEM solve launch of nlem_denoise, nlem_denoise_ex and nlm_denoise
 * (and of nlem_autotune's trials) is bracketed by two HIP events on its stream, so the solve kernel's own duration can be
 * read without the small kernels that precede it (the queue-order kernels,
 * or a reset of the queue head where the order is not used).  Not recorded: launches into a stream that is being captured, and
 * the multi-image graph.  Enabling or disabling discards unread timings.
 * em_kernel_timing_read - waits for the recorded events and returns the sum
 * of their durations (ms) and the number of launches, then clears them;
 * read at least every 4096 launches (the next timed launch fails with
 * UNSUPPORTED otherwise).  Errors: INVALID_ARG (NULL handle or outputs); HIP.
 */
em_status_t em_kernel_timing(em_handle_t handle, int32_t enable);
em_status_t em_kernel_timing_read(em_handle_t handle, double *total_ms, int64_t *launches);

/* Wait for the stream and report any asynchronous HIP error as EM_ERR_HIP. */
em_status_t em_sync(em_handle_t handle, void *stream);

/* Static description of a status code. */
const char *em_status_string(em_status_t status);

/* Text of the last error recorded on the handle ("" if none). */
const char *em_last_error(em_handle_t handle);

#ifdef __cplusplus
}
#endif

#endif /* EMX_H */
