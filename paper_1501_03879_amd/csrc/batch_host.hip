// Host side of the batched solvers: the device classification pre-pass, one
// persistent launch per shape class, and the plain one-launch-per-instance
// baseline (literal Algorithm 1 with the iterates in device memory).
#include <float.h>

#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <string>

#include "batch_kernel.hpp"

namespace emx {

int blocks_per_cu(em_context *ctx, const void *fn, int threads);
int ctx_num_cus(em_context *ctx);
em_status_t ctx_error(em_context *ctx, em_status_t st, const char *msg);
em_status_t ctx_hip_error(em_context *ctx, hipError_t e, const char *what);
unsigned int *ctx_counters(em_context *ctx, int n);
em_status_t ctx_reset_counters(em_context *ctx, hipStream_t s, unsigned int *c, int n);
void *ctx_workspace(em_context *ctx, size_t bytes, em_status_t *st);
void *ctx_plain_workspace(em_context *ctx, size_t bytes, em_status_t *st);
em_status_t ctx_side_streams(em_context *ctx, hipStream_t **side, hipEvent_t *fork, hipEvent_t **join);
BatchPlanView ctx_batch_plan(em_context *ctx, const em_options_t &o);
unsigned int *ctx_host_counts(em_context *ctx, int n);

// Classify: counts per class; empty / malformed instances finished here.
// Counts go through a per-block LDS histogram (one global atomic per block
// and class): a million instances over twenty counters would otherwise
// serialise on the hot ones.
__global__ __launch_bounds__(256) void batch_classify_count(const em_instance_t *inst, int64_t B, float *z,
                                                            em_stats_t *stats, unsigned int *counts, int mode,
                                                            uint64_t generic_mask) {
    __shared__ unsigned int hist[kNumAllClasses];
    for (int i = threadIdx.x; i < kNumAllClasses; i += blockDim.x) hist[i] = 0u;
    __syncthreads();
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B) {
        const em_instance_t e = inst[b];
        if (e.n == 0 && e.d >= 1 && e.d <= EM_MAX_D) {
            if (stats) stats[b] = em_stats_t{0, EM_EMPTY, 0.0f, 0.0f};
        } else if (e.n < 0 || e.n > EM_MAX_N || e.d < 1 || e.d > EM_MAX_D) {
            if (e.d >= 1 && e.d <= EM_MAX_D)
                for (int j = 0; j < e.d; ++j) z[e.z_off + j] = __builtin_nanf("");
            if (stats) stats[b] = em_stats_t{0, EM_BAD_INPUT, 0.0f, 0.0f};
        } else {
            atomicAdd(&hist[class_of(e.n, e.d, mode, generic_mask)], 1u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kNumAllClasses; i += blockDim.x)
        if (hist[i]) atomicAdd(&counts[i], hist[i]);
}

// Class counts only (sliced classes, nothing routed back), for the autotuner.
__global__ __launch_bounds__(256) void batch_classify_count_only(const em_instance_t *inst, int64_t B,
                                                                 unsigned int *counts) {
    __shared__ unsigned int hist[kNumAllClasses];
    for (int i = threadIdx.x; i < kNumAllClasses; i += blockDim.x) hist[i] = 0u;
    __syncthreads();
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B) {
        const em_instance_t e = inst[b];
        if (e.n > 0 && e.n <= EM_MAX_N && e.d >= 1 && e.d <= EM_MAX_D) atomicAdd(&hist[class_of(e.n, e.d, 1)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kNumAllClasses; i += blockDim.x)
        if (hist[i]) atomicAdd(&counts[i], hist[i]);
}

__global__ void batch_classify_scan(const unsigned int *counts, unsigned int *offsets) {
    if (threadIdx.x == 0) {
        unsigned int s = 0;
        for (int c = 0; c < kNumAllClasses; ++c) {
            offsets[c] = s;
            s += counts[c];
        }
        offsets[kNumAllClasses] = s;
    }
}

// Ranks within the block from LDS atomics, then one global atomic per
// (block, class) reserves the block's range of the class list.
__global__ __launch_bounds__(256) void batch_classify_scatter(const em_instance_t *inst, int64_t B,
                                                              const unsigned int *offsets, unsigned int *fill,
                                                              int32_t *list, int mode, uint64_t generic_mask) {
    __shared__ unsigned int lcnt[kNumAllClasses];
    __shared__ unsigned int lbase[kNumAllClasses];
    for (int i = threadIdx.x; i < kNumAllClasses; i += blockDim.x) lcnt[i] = 0u;
    __syncthreads();
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int c = -1;
    unsigned int rank = 0;
    if (b < B) {
        const em_instance_t e = inst[b];
        if (e.n > 0 && e.n <= EM_MAX_N && e.d >= 1 && e.d <= EM_MAX_D) {
            c = class_of(e.n, e.d, mode, generic_mask);
            rank = atomicAdd(&lcnt[c], 1u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kNumAllClasses; i += blockDim.x)
        lbase[i] = lcnt[i] ? atomicAdd(&fill[i], lcnt[i]) : 0u;
    __syncthreads();
    if (c >= 0) list[offsets[c] + lbase[c] + rank] = (int32_t)b;
}

// Far outliers: the fixed-penalty EM-ADMM over a box defers an instance whose
// largest |a| exceeds kOutlierK D sqrt(n) to kernels that carry the prox
// displacement e itself (ClassLaunch, batch_wide.hpp).  With g = e - a the
// computed primal residual has a floor of about 3e-4 tol (max |a| / D) /
// sqrt(n) (measured on the 91 of 1,048,576 point sets that ended at max_iter
// that way, max |a| / D from 2.9e4 to 7.5e5); below the bound it stays under
// 0.12 tol.  On the point-set workload 0.9% of the instances (1.3% of the
// work) are deferred.
constexpr float kOutlierK = 300.0f;

// The class kernels of a solver and set.
static const ClassKernel *class_table(const em_options_t &o) {
    const bool ball = o.set == EM_SET_BALL;
    return (o.solver == EM_SOLVER_IRLS) ? (ball ? batch_class_table_irls_ball() : batch_class_table_irls())
           : (o.solver == EM_SOLVER_ADMM_ADAPTIVE) ? batch_class_table_adapt()
           : (o.solver == EM_SOLVER_ADMM_WEIGHTED) ? (ball ? batch_class_table_wpen_ball() : batch_class_table_wpen())
                                                   : (ball ? batch_class_table_admm_ball() : batch_class_table_admm());
}

// Arguments of a class launch (queue fields and `single` left to the caller).
static ClassLaunch class_launch(const float *a, const float *w, const em_instance_t *inst, const em_options_t &o,
                                float *z, em_stats_t *stats, int c) {
    const bool ball = o.set == EM_SET_BALL;
    const bool vbox = ball || o.box_lo != nullptr;
    ClassLaunch L;
    memset(&L, 0, sizeof(L));
    L.a = a;
    L.w = w;
    L.inst = inst;
    L.z = z;
    L.stats = stats;
    L.box_lo = ball ? nullptr : o.box_lo;
    L.box_hi = ball ? nullptr : o.box_hi;
    L.ball_center = ball ? o.ball_center : nullptr;
    L.ball_radius = ball ? o.ball_radius : nullptr;
    L.radius = o.radius;
    L.lo = vbox ? 0.0f : o.lo;   // padded coordinates clamp to 0 when the box is per coordinate
    L.hi = vbox ? 0.0f : o.hi;
    L.mu = (o.solver == EM_SOLVER_IRLS) ? 1.0f : o.rho;
    L.tol = o.tol;
    L.arm = 1.0f;  // primal residual evaluated after an iteration with r_dual <= arm tol D (set by the caller)
    L.eps = o.eps;
    L.adapt_every = (o.solver == EM_SOLVER_ADMM_ADAPTIVE) ? o.adapt_every : 0;
    L.adapt_ratio2 = o.adapt_ratio * o.adapt_ratio;
    L.adapt_factor = o.adapt_factor;
    L.max_iter = o.max_iter;
    L.init = o.init;
    L.cls = c;
    L.a16 = o.points_f16 ? 1 : 0;
    L.single = -1;
    L.outlier = kOutlierK;
    L.fast_eta = o.fast_eta;
    return L;
}

// EMX_BATCH_WIDE=0 keeps every instance on the generic classes (for comparison).
static bool wide_disabled() {
    const char *e = getenv("EMX_BATCH_WIDE");
    return e && e[0] == '0' && e[1] == '\0';
}

// Largest point-coordinate count an instance of class c can have.
static int64_t class_capacity(int c) {
    if (c >= kFirstFastClass) {
        const int k = c - kFirstFastClass;
        return (int64_t)(64 << (k % 4)) * (8 << (k / 4));
    }
    if (c >= kNumClasses) {
        const int k = c - kNumClasses;
        return (int64_t)(64 * (1 + k % kWideMaxM)) * (kWideNJ * (kWideMinWC + k / kWideMaxM));
    }
    const ClassShape sh = class_shape(c);
    return (int64_t)(64 * sh.m * sh.wp) * (sh.ds * sh.wc);
}

// Class launch order: largest instances first, so that on a batch of one
// heavy shape its kernel is among the first four launched (one per stream)
// instead of queued behind the dispatches of empty classes; each class's
// counts are only known on the device.
static const int *class_launch_order() {
    static const std::array<int, kNumAllClasses> order = [] {
        std::array<int, kNumAllClasses> o{};
        for (int c = 0; c < kNumAllClasses; ++c) o[c] = c;
        std::stable_sort(o.begin(), o.end(),
                         [](int x, int y) { return class_capacity(x) > class_capacity(y); });
        return o;
    }();
    return order.data();
}

em_status_t batch_solve(em_context *ctx, hipStream_t s, int64_t B, const float *a, const float *w,
                        const em_instance_t *inst, const em_options_t &o, float *z, em_stats_t *stats) {
    // fixed-penalty EM-ADMM over a box: d > 16, n <= 448 go to the sliced
    // kernel, far-outlier instances to the deferred lists
    const int wide = (o.solver == EM_SOLVER_ADMM && o.set == EM_SET_BOX && !wide_disabled()) ? 1 : 0;
    const bool defer = o.solver == EM_SOLVER_ADMM && o.set == EM_SET_BOX;
    const bool fast = o.solver == EM_SOLVER_ADMM_FAST;   // its own classes (batch_fast.hpp)
    const int mode = fast ? 2 : wide;
    const BatchPlanView plan = ctx_batch_plan(ctx, o);   // routing and arm factor of a plan
    const uint64_t gmask = wide ? plan.generic_mask : 0;
    // workspace: list[B] int32, then (deferral) the deferred lists of B each
    em_status_t st;
    int32_t *list = static_cast<int32_t *>(
        ctx_workspace(ctx, (size_t)B * sizeof(int32_t) * (defer ? 1 + kDeferLists : 1), &st));
    if (!list) return st;
    // counters: [0, K) class counts, [K, 2K+1) offsets, [2K+1, 3K+1) fill, [3K+1, 4K+1) queue heads,
    // then the deferred lists' {0, count} pairs and queue heads
    constexpr int K = kNumAllClasses;
    constexpr int NC = 4 * K + 1 + 3 * kDeferLists;
    unsigned int *cnt = ctx_counters(ctx, NC);
    if (!cnt) return ctx_error(ctx, EM_ERR_UNSUPPORTED, "counter pool too small");
    unsigned int *counts = cnt, *offsets = cnt + K, *fill = cnt + 2 * K + 1, *heads = cnt + 3 * K + 1;
    unsigned int *defer_q = cnt + 4 * K + 1, *defer_heads = defer_q + 2 * kDeferLists;
    st = ctx_reset_counters(ctx, s, cnt, NC);
    if (st != EM_OK) return st;
    const unsigned nb = (unsigned)((B + 255) / 256);
    hipLaunchKernelGGL(batch_classify_count, dim3(nb), dim3(256), 0, s, inst, B, z, stats, counts, mode, gmask);
    hipStream_t *side;
    hipEvent_t fork, *join;
    st = ctx_side_streams(ctx, &side, &fork, &join);
    if (st != EM_OK) return st;
    // a plan with host_counts: the class counts come back to the host (the
    // call waits for the stream up to here), so that only populated classes
    // are launched; not while the stream is being captured
    const unsigned int *hc = nullptr;
    if (plan.host_counts) {
        hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
        hipError_t ce = hipStreamIsCapturing(s, &cst);
        if (ce != hipSuccess) return ctx_hip_error(ctx, ce, "hipStreamIsCapturing");
        unsigned int *hbuf = (cst == hipStreamCaptureStatusNone) ? ctx_host_counts(ctx, K) : nullptr;
        if (hbuf) {
            ce = hipMemcpyAsync(hbuf, counts, K * sizeof(unsigned int), hipMemcpyDeviceToHost, s);
            if (ce == hipSuccess) ce = hipEventRecord(fork, s);
            if (ce == hipSuccess) ce = hipEventSynchronize(fork);
            if (ce != hipSuccess) return ctx_hip_error(ctx, ce, "class counts to the host");
            hc = hbuf;
        }
    }
    hipLaunchKernelGGL(batch_classify_scan, dim3(1), dim3(64), 0, s, counts, offsets);
    hipLaunchKernelGGL(batch_classify_scatter, dim3(nb), dim3(256), 0, s, inst, B, offsets, fill, list, mode,
                       gmask);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return ctx_hip_error(ctx, e, "classify launch");
    const ClassKernel *tab = class_table(o);
    // The classes run concurrently on the caller's stream and the handle's
    // side streams (fork after the classification, join before returning), so
    // one class's tail overlaps the others' work.  The launched classes go to
    // the four streams in turn, largest shapes first; with the counts on the
    // host, only the populated ones, each to the stream with the least work
    // so far (largest estimated work first: instances x the class's largest
    // n d), with at most one workgroup per instance.
    e = hipEventRecord(fork, s);
    for (int i = 0; i < kSideStreams && e == hipSuccess; ++i) e = hipStreamWaitEvent(side[i], fork, 0);
    if (e != hipSuccess) return ctx_hip_error(ctx, e, "fork of the class streams");
    const ClassKernel *wtab = batch_wide_table();
    const ClassKernel *ftab = batch_fast_table();
    const int *order = class_launch_order();
    int hc_order[K];
    if (hc) {
        for (int c = 0; c < K; ++c) hc_order[c] = c;
        std::stable_sort(hc_order, hc_order + K, [&](int x, int y) {
            return (double)hc[x] * (double)class_capacity(x) > (double)hc[y] * (double)class_capacity(y);
        });
        order = hc_order;
    }
    double load[kSideStreams + 1] = {};
    int launched = 0;
    for (int oi = 0; oi < K; ++oi) {
        const int c = order[oi];
        if (hc && hc[c] == 0) continue;
        // (with sliced classes routed back by a plan, every generic class may receive instances)
        const bool skip = fast ? c < kFirstFastClass
                               : (c >= kFirstFastClass ||
                                  (c >= kNumClasses ? !wide || ((gmask >> (c - kNumClasses)) & 1u)
                                                    : (wide && gmask == 0 && class_unused_with_wide(c))));
        if (skip) continue;
        const ClassKernel &ck = (c >= kFirstFastClass) ? ftab[c - kFirstFastClass]
                                : (c >= kNumClasses)  ? wtab[c - kNumClasses]
                                                      : tab[c];
        int si = launched++ % (kSideStreams + 1);
        if (hc) {
            si = 0;
            for (int i = 1; i <= kSideStreams; ++i)
                if (load[i] < load[si]) si = i;
            load[si] += (double)hc[c] * (double)class_capacity(c);
        }
        hipStream_t cs = (si == 0) ? s : side[si - 1];
        ClassLaunch L = class_launch(a, w, inst, o, z, stats, c);
        L.arm = plan.arm;
        L.check_mask = plan.check - 1;
        L.list = list;
        L.offsets = offsets;
        L.counter = heads + c;
        if (defer) {
            L.defer_list = list + B;
            L.defer_stride = B;
            L.defer_q = defer_q;
        }
        const int64_t cap = (int64_t)ctx_num_cus(ctx) * blocks_per_cu(ctx, ck.fn, ck.threads);
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(hc ? (int64_t)hc[c] : B, cap));
        void *args[] = {&L};
        e = hipLaunchKernel(ck.fn, dim3(grid), dim3(ck.threads), args, 0, cs);
        if (e != hipSuccess) return ctx_hip_error(ctx, e, "batch class launch");
    }
    for (int i = 0; i < kSideStreams && e == hipSuccess; ++i) {
        e = hipEventRecord(join[i], side[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, join[i], 0);
    }
    if (e != hipSuccess) return ctx_hip_error(ctx, e, "join of the class streams");
    if (defer) {
        // the deferred far-outlier instances, after every class kernel (an empty
        // list costs one launch whose workgroups exit at once); the two lists
        // run concurrently, the second on a side stream joined back
        e = hipEventRecord(fork, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(side[0], fork, 0);
        if (e != hipSuccess) return ctx_hip_error(ctx, e, "fork of the deferred lists");
        const ClassKernel *dtab = batch_deferred_table();
        for (int k = 0; k < kDeferLists; ++k) {
            ClassLaunch L = class_launch(a, w, inst, o, z, stats, 0);
            L.arm = plan.arm;
            L.check_mask = plan.check - 1;
            L.list = list + (int64_t)(k + 1) * B;
            L.offsets = defer_q + 2 * k;
            L.counter = defer_heads + k;
            const int64_t cap = (int64_t)ctx_num_cus(ctx) * blocks_per_cu(ctx, dtab[k].fn, dtab[k].threads);
            const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(B, cap));
            void *args[] = {&L};
            e = hipLaunchKernel(dtab[k].fn, dim3(grid), dim3(dtab[k].threads), args, 0, k == 0 ? s : side[0]);
            if (e != hipSuccess) return ctx_hip_error(ctx, e, "deferred launch");
        }
        e = hipEventRecord(join[0], side[0]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, join[0], 0);
        if (e != hipSuccess) return ctx_hip_error(ctx, e, "join of the deferred lists");
    }
    return EM_OK;
}

// Instances per sliced class of the fixed-penalty EM-ADMM over a box (the
// classification of batch_solve with no class routed back, counts copied to
// the host; synchronous on s).  For the autotuner.
em_status_t batch_wide_counts(em_context *ctx, hipStream_t s, int64_t B, const em_instance_t *inst,
                              unsigned int (&wide_counts)[kNumWideClasses]) {
    unsigned int *cnt = ctx_counters(ctx, kNumAllClasses);
    if (!cnt) return ctx_error(ctx, EM_ERR_UNSUPPORTED, "counter pool too small");
    em_status_t st = ctx_reset_counters(ctx, s, cnt, kNumAllClasses);
    if (st != EM_OK) return st;
    const unsigned nb = (unsigned)((B + 255) / 256);
    hipLaunchKernelGGL(batch_classify_count_only, dim3(nb), dim3(256), 0, s, inst, B, cnt);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(wide_counts, cnt + kNumClasses, sizeof(wide_counts),
                                            hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return ctx_hip_error(ctx, e, "class counts");
    return EM_OK;
}

// ------------------------------------------------------------------ plain

// The plain path, one instance per launch:
//  * EM-ADMM: the batched solver's own class kernels, each launched as a
//    single workgroup on a single instance (no work queue, no other instance
//    on the chip), so batched / plain measures what batching and the
//    persistent queue add, with the same per-instance code.
//  * The accelerated ADMM (its momentum needs the previous multipliers, a
//    second n x d state): iterates in device memory, one 256-thread
//    workgroup per instance (plain_solve_kernel<true>); em_solve_batch_ex
//    runs it batched with the state in registers (batch_fast.hpp).
//   FAST = false: literal Algorithm 1 (thread per point for the prox and the
//     multiplier update, thread per coordinate for the mean), residuals
//     every iteration (not used by the library).
//   FAST = true: fast ADMM with restart ([Goldstein2012], weakly convex
//     case) on the same splitting: the prox and the mean use the predictors
//     z_hat, u_hat; after the update, c = mu (sum_k ||x_k - z||^2 +
//     n ||z - z_hat||^2) decides between momentum
//     (z_hat = z + beta (z - z_prev), u_hat = u + beta (u - u_prev),
//     beta = (alpha - 1) / alpha', alpha' = (1 + sqrt(1 + 4 alpha^2)) / 2) and
//     a restart (z_hat = z_prev, u_hat = u_prev, alpha = 1, c_prev /= eta)
//     (momentum while c < eta (1 - 2^-16) c_prev),
//     except after the last allowed sweep; the restart count goes to the
//     flags word.  u = y / mu throughout (mu is fixed).
constexpr int kMaxRestartCount = (1 << 23) - 1;

struct PlainArgs {
    const float *a;
    const float *w;
    const em_instance_t *inst;
    float *z;
    em_stats_t *stats;
    const float *box_lo;  // per-coordinate bounds (indexed like z) or null
    const float *box_hi;
    float *u;   // n*d scaled multipliers y/mu
    float *x;   // n*d local variables
    float *up;  // FAST: n*d previous u
    float *uh;  // FAST: n*d predictor u_hat
    float lo, hi, mu, tol, eta;
    int32_t max_iter, init;
    int64_t b;
};

__device__ __forceinline__ float block_sum256(float v, float *red) {
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
    for (int s2 = 128; s2 > 0; s2 >>= 1) {
        if (tid < s2) red[tid] += red[tid + s2];
        __syncthreads();
    }
    const float r = red[0];
    __syncthreads();
    return r;
}

template <bool FAST>
__global__ __launch_bounds__(256) void plain_solve_kernel(PlainArgs P) {
    __shared__ float zs[EM_MAX_D], zprev[EM_MAX_D], zh[EM_MAX_D], blo[EM_MAX_D], bhi[EM_MAX_D];
    __shared__ float red[256];
    __shared__ int flag;
    __shared__ float amax_s;
    const int tid = threadIdx.x;
    const em_instance_t e = P.inst[P.b];
    const int n = e.n, d = e.d;
    float *Z = P.z + e.z_off;
    if (n == 0 && d >= 1 && d <= EM_MAX_D) {
        if (tid == 0 && P.stats) P.stats[P.b] = em_stats_t{0, EM_EMPTY, 0.0f, 0.0f};
        return;
    }
    const float *A = P.a + e.a_off;
    const float *Wt = P.w + e.w_off;
    if (tid == 0) {
        flag = 0;
        amax_s = 0.0f;
    }
    __syncthreads();
    if (n < 0 || n > EM_MAX_N || d < 1 || d > EM_MAX_D) {
        if (tid == 0) flag = 1;
    } else {
        for (int i = tid; i < n * d; i += 256) {
            if (!(fabsf(A[i]) <= FLT_MAX)) flag = 1;
            atomicMax(reinterpret_cast<int *>(&amax_s), __float_as_int(fabsf(A[i])));
        }
        for (int k = tid; k < n; k += 256)
            if (!(Wt[k] >= 0.0f && Wt[k] <= FLT_MAX)) flag = 1;
    }
    __syncthreads();
    if (flag == 0 && P.init == EM_INIT_WMEAN) {
        // weighted mean, weights scaled by their largest value and points by 1/n
        // (equal weights when every weight is zero); thread j sums coordinate j
        if (tid == 0) {
            float wm = 0.0f;
            for (int k = 0; k < n; ++k) wm = fmaxf(wm, Wt[k]);
            red[0] = wm;
        }
        __syncthreads();
        const float wm = red[0];
        const bool uni = !(wm > 0.0f);
        const float inv_n = 1.0f / (float)n;
        if (tid < d) {
            float acc = 0.0f, cs = 0.0f;
            for (int k = 0; k < n; ++k) {
                const float c = (uni ? 1.0f : Wt[k] / wm) * inv_n;
                cs += c;
                acc = fmaf(c, A[k * d + tid], acc);
            }
            zs[tid] = acc / cs;
        }
        __syncthreads();
    }
    float wmax = 0.0f;
    if (flag == 0 && tid == 0) {
        int best = 0;
        if (P.init == EM_INIT_MAXW)
            for (int k = 1; k < n; ++k)
                if (Wt[k] > Wt[best]) best = k;
        for (int j = 0; j < d; ++j) {
            zs[j] = (P.init == EM_INIT_MAXW) ? A[best * d + j] : (P.init == EM_INIT_WMEAN) ? zs[j] : Z[j];
            blo[j] = P.box_lo ? P.box_lo[e.z_off + j] : P.lo;
            bhi[j] = P.box_lo ? P.box_hi[e.z_off + j] : P.hi;
            if (!(fabsf(zs[j]) <= FLT_MAX) || !(blo[j] <= bhi[j])) flag = 1;
            const float wj = bhi[j] - blo[j];
            if (!(wj <= wmax)) wmax = wj;
            zprev[j] = zs[j];
            zh[j] = zs[j];
        }
        red[0] = wmax;
    }
    __syncthreads();
    if (flag) {
        if (tid == 0) {
            if (d >= 1 && d <= EM_MAX_D)
                for (int j = 0; j < d; ++j) Z[j] = __builtin_nanf("");
            if (P.stats) P.stats[P.b] = em_stats_t{0, EM_BAD_INPUT, 0.0f, 0.0f};
        }
        return;
    }
    wmax = red[0];
    __syncthreads();
    const float Dscale = (wmax <= FLT_MAX && wmax > 0.0f) ? wmax : fmaxf(1.0f, amax_s);
    const float tau = P.tol * Dscale;
    for (int i = tid; i < n * d; i += 256) {
        P.u[i] = 0.0f;
        if constexpr (FAST) {
            P.up[i] = 0.0f;
            P.uh[i] = 0.0f;
        }
    }
    __syncthreads();
    const float *UH = FAST ? P.uh : P.u;   // the multipliers the prox and the mean use
    const float *ZH = FAST ? zh : zs;
    float alpha = 1.0f, c_prev = INFINITY;
    int iters = 0, flags = EM_MAXITER, restarts = 0;
    float rpri = 0.0f, rdual = 0.0f;
    for (int t = 1; t <= P.max_iter; ++t) {
        // x_k = prox_{w_k/mu}(z_hat - u_hat_k, a_k)
        for (int k = tid; k < n; k += 256) {
            const float lam = Wt[k] / P.mu;
            float nu2 = 0.0f;
            for (int j = 0; j < d; ++j) {
                const float dl = ZH[j] - UH[k * d + j] - A[k * d + j];
                nu2 = fmaf(dl, dl, nu2);
            }
            const float nu = sqrtf(nu2);
            const float sh = (nu <= lam) ? 1.0f : lam / nu;
            for (int j = 0; j < d; ++j) {
                const float v = ZH[j] - UH[k * d + j];
                P.x[k * d + j] = v - sh * (v - A[k * d + j]);
            }
        }
        __syncthreads();
        // z = P_C(mean_k(x_k + u_hat_k))
        float sdl = 0.0f, shl = 0.0f;
        for (int j = tid; j < d; j += 256) {
            float r = 0.0f;
            for (int k = 0; k < n; ++k) r += P.x[k * d + j] + UH[k * d + j];
            const float zn = clampf(r / (float)n, blo[j], bhi[j]);
            sdl = fmaf(zn - zs[j], zn - zs[j], sdl);
            shl = fmaf(zn - ZH[j], zn - ZH[j], shl);
            zprev[j] = zs[j];
            zs[j] = zn;
        }
        __syncthreads();
        // u_k = u_hat_k + x_k - z, primal residual
        float rp = 0.0f;
        for (int i = tid; i < n * d; i += 256) {
            const float dlt = P.x[i] - zs[i % d];
            const float un = UH[i] + dlt;
            if constexpr (FAST) P.up[i] = P.u[i];
            P.u[i] = un;
            rp = fmaf(dlt, dlt, rp);
        }
        const float sp = block_sum256(rp, red);
        const float sd = block_sum256(sdl, red);
        rpri = sqrtf(sp / ((float)n * (float)d));
        rdual = sqrtf(sd / (float)d);
        iters = t;
        if (tau > 0.0f && rpri <= tau && rdual <= tau) {
            flags = EM_CONVERGED;
            break;
        }
        if constexpr (FAST) {
            const float sh2 = block_sum256(shl, red);
            if (t == P.max_iter) break;   // no sweep follows: the decision would change nothing
            const float c = P.mu * (sp + (float)n * sh2);
            if (c < P.eta * (1.0f - 0x1p-16f) * c_prev) {   // guard: see batch_fast.hpp
                const float an = 0.5f * (1.0f + sqrtf(1.0f + 4.0f * alpha * alpha));
                const float beta = (alpha - 1.0f) / an;
                for (int j = tid; j < d; j += 256) zh[j] = zs[j] + beta * (zs[j] - zprev[j]);
                for (int i = tid; i < n * d; i += 256) P.uh[i] = P.u[i] + beta * (P.u[i] - P.up[i]);
                alpha = an;
                c_prev = c;
            } else {
                for (int j = tid; j < d; j += 256) zh[j] = zprev[j];
                for (int i = tid; i < n * d; i += 256) P.uh[i] = P.up[i];
                alpha = 1.0f;
                c_prev = c_prev / P.eta;
                ++restarts;
            }
            __syncthreads();
        }
    }
    if (tid < d) Z[tid] = zs[tid];
    if (tid == 0 && P.stats)
        P.stats[P.b] = em_stats_t{iters, flags | (FAST ? min(restarts, kMaxRestartCount) << EM_RESTART_SHIFT : 0),
                                  rpri, rdual};
}

// EM-ADMM one instance per launch through the class kernels; empty and
// malformed instances are finished by the classification kernel on that
// instance alone (EMPTY, or BAD_INPUT with z = NaN).
static em_status_t plain_admm(em_context *ctx, hipStream_t s, int64_t B, const float *a, const float *w,
                              const em_instance_t *inst, const em_instance_t *inst_host, const em_options_t &o,
                              float *z, em_stats_t *stats) {
    const bool wide = o.set == EM_SET_BOX && !wide_disabled();
    const BatchPlanView plan = ctx_batch_plan(ctx, o);   // the batched path's routing and arm factor
    const ClassKernel *tab = class_table(o);
    const ClassKernel *wtab = batch_wide_table();
    unsigned int *scratch = ctx_counters(ctx, kNumAllClasses);   // class counts of the finishing kernel
    if (!scratch) return ctx_error(ctx, EM_ERR_UNSUPPORTED, "counter pool too small");
    for (int64_t b = 0; b < B; ++b) {
        const em_instance_t &e = inst_host[b];
        if (e.n <= 0 || e.n > EM_MAX_N || e.d < 1 || e.d > EM_MAX_D) {
            hipLaunchKernelGGL(batch_classify_count, dim3(1), dim3(256), 0, s, inst + b, (int64_t)1, z,
                               stats ? stats + b : nullptr, scratch, 0, (uint64_t)0);
            continue;
        }
        const int c = class_of(e.n, e.d, wide, wide ? plan.generic_mask : 0);
        const ClassKernel &ck = (c >= kNumClasses) ? wtab[c - kNumClasses] : tab[c];
        ClassLaunch L = class_launch(a, w, inst, o, z, stats, c);
        L.arm = plan.arm;
        L.check_mask = plan.check - 1;
        L.single = b;
        void *args[] = {&L};
        const hipError_t err = hipLaunchKernel(ck.fn, dim3(1), dim3(ck.threads), args, 0, s);
        if (err != hipSuccess) return ctx_hip_error(ctx, err, "plain launch");
    }
    const hipError_t err = hipGetLastError();
    if (err != hipSuccess) return ctx_hip_error(ctx, err, "plain launch");
    return EM_OK;
}

em_status_t plain_solve(em_context *ctx, hipStream_t s, int64_t B, const float *a, const float *w,
                        const em_instance_t *inst, const em_instance_t *inst_host, const em_options_t &o,
                        float *z, em_stats_t *stats) {
    const bool fast = o.solver == EM_SOLVER_ADMM_FAST;
    if (!fast) return plain_admm(ctx, s, B, a, w, inst, inst_host, o, z, stats);
    int64_t maxnd = 1;
    for (int64_t b = 0; b < B; ++b) {
        const int64_t n = inst_host[b].n, d = inst_host[b].d;
        if (n > 0 && n <= EM_MAX_N && d >= 1 && d <= EM_MAX_D) maxnd = std::max(maxnd, n * d);
    }
    em_status_t st;
    const int64_t arrays = fast ? 4 : 2;
    float *ws = static_cast<float *>(ctx_plain_workspace(ctx, (size_t)(arrays * maxnd) * sizeof(float), &st));
    if (!ws) return st;
    PlainArgs P;
    memset(&P, 0, sizeof(P));
    P.a = a;
    P.w = w;
    P.inst = inst;
    P.z = z;
    P.stats = stats;
    P.box_lo = o.box_lo;
    P.box_hi = o.box_hi;
    P.u = ws;
    P.x = ws + maxnd;
    P.up = fast ? ws + 2 * maxnd : nullptr;
    P.uh = fast ? ws + 3 * maxnd : nullptr;
    P.lo = o.lo;
    P.hi = o.hi;
    P.mu = o.rho;
    P.tol = o.tol;
    P.eta = o.fast_eta;
    P.max_iter = o.max_iter;
    P.init = o.init;
    for (int64_t b = 0; b < B; ++b) {
        P.b = b;
        hipLaunchKernelGGL(plain_solve_kernel<true>, dim3(1), dim3(256), 0, s, P);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return ctx_hip_error(ctx, e, "plain launch");
    return EM_OK;
}

}  // namespace emx
