// Batched solvers over independent point sets of uneven size: EM-ADMM
// (Algorithm 1 of arXiv:1501.03879 for every instance, optionally with an
// adaptive penalty) and IRLS on the smooth surrogate (EM_surrogate).
//
//  * A device pre-pass sorts instances into shape classes (coordinate slice
//    DS, points per lane M, waves over coordinates WC, waves over points WP)
//    with a counting sort; empty and malformed instances are finished there.
//  * One persistent kernel per class pops instances from a work queue.  A
//    workgroup of WC x WP waves owns one instance: wave (cw, pw) holds
//    coordinates [cw DS, cw DS + DS) of points pw 64 M + l + 64 q.  Points
//    and the iteration state (g = e - a, see the NLEM kernel) stay in
//    registers for the whole solve; the points are read from HBM once,
//    coalesced, through an LDS staging buffer.
//  * ADMM iteration: pass 1 (delta = g + c, partial ||delta||^2), norms summed
//    over the WC coordinate waves in LDS, shrink factor, pass 2 (E += s delta,
//    g = s delta - a), wave reduce-scatter of E, sum over the WP point waves
//    in LDS, then z = clamp(z - E / n), c = 2 z - z_prev.
//  * Set C: a box (one interval for all coordinates, or per-coordinate
//    bounds read from device arrays indexed like z), or (SET = 1) the
//    Euclidean ball ||z - center|| <= radius, whose projection scales
//    z - center by min(1, radius / ||z - center||): one more sum over the
//    coordinates (rows, then the coordinate waves through LDS) per iteration.
//  * Adaptive penalty (residual balancing): on every k-th iteration both
//    residuals are evaluated; the next iteration compares them and may scale
//    mu by a factor.  The multipliers y are unchanged by that, so the scaled
//    state is rescaled: with tau = mu'/mu, the current delta = v - a becomes
//    delta / tau + (1 - 1/tau)(z - a), lambda = w / mu becomes lambda / tau,
//    the prox displacement sum E^t becomes E^t / tau and
//    c = v - e becomes c / tau + (1 - 1/tau) z.
//  * IRLS iteration: omega_k = w_k (||z - a_k||^2 + eps)^(-1/2), then
//    z' = P_C(sum_k omega_k a_k / sum_k omega_k), held relative to the
//    starting point projected onto C, o = P_C(z0) (points as o - a), so the
//    distance to a point at o keeps FP32 precision of its own size.
#pragma once

#include <float.h>
#include <hip/hip_fp16.h>

#include "em_device.hpp"
#include "batch_plan.hpp"
#include "emx_internal.hpp"

namespace emx {

// Last word of the buffer resources the staging builds (base, stride 0, a
// byte range): the gfx9 data-format field set to 32 bits, the other fields
// zero.  Raw buffer loads take their width from the instruction; the range
// makes a load past it return 0.
constexpr int kBufferRsrcWord3 = 0x00020000;

struct ClassShape {
    int ds, m, wc, wp;
};

// Class table (index = class id).  d <= 4 uses DS = 4; otherwise DS = 16
// with WC = ceil(d / 16).  M = ceil(n / 64) rounded up to 1, 2, 4 (8 for
// DS = 4); n in (256, 512] with DS = 16 uses two point waves (WP = 2).
constexpr int kNumClasses = 20;
__host__ __device__ constexpr ClassShape class_shape(int c) {
    return (c < 4) ? ClassShape{4, 1 << c, 1, 1}
                   : ClassShape{16, ((c - 4) % 4 == 3) ? 4 : (1 << ((c - 4) % 4)), 1 + (c - 4) / 4,
                                ((c - 4) % 4 == 3) ? 2 : 1};
}

__host__ __device__ inline int class_of(int n, int d) {
    if (d <= 4) {
        const int m = (n + 63) / 64;
        return (m <= 1) ? 0 : (m <= 2) ? 1 : (m <= 4) ? 2 : 3;
    }
    const int wc = (d + 15) / 16;
    const int m = (n + 63) / 64;
    const int k = (m <= 1) ? 0 : (m <= 2) ? 1 : (m <= 4) ? 2 : 3;
    return 4 + (wc - 1) * 4 + k;
}

// Classes of the sliced EM-ADMM kernel (batch_wide.hpp; fixed penalty over a
// box; shapes in batch_plan.hpp, where a batch plan numbers them too): d in
// (16, 64] and n <= 448 go to 13-coordinate slices over WC = ceil(d / 13) in
// [2, 5] waves with M = ceil(n / 64) in [1, 7] points per lane.  Their ids
// follow the kNumClasses classes above.
// Classes of the accelerated ADMM (batch_fast.hpp): 8-coordinate slices over
// WC in {1, 2, 4, 8} waves (the smallest with 8 WC >= d) and M in {1, 2, 4, 8}
// points per lane (the smallest with 64 M >= n); ids after the sliced ones.
constexpr int kNumFastClasses = 16;
constexpr int kFirstFastClass = kNumClasses + kNumWideClasses;
constexpr int kNumAllClasses = kFirstFastClass + kNumFastClasses;

__host__ __device__ constexpr int pow2_index(int v) { return v <= 1 ? 0 : v <= 2 ? 1 : v <= 4 ? 2 : 3; }

// mode 0: generic classes; 1: sliced classes where they apply (fixed-penalty
// EM-ADMM over a box), except those whose bit k = class - kNumClasses is set
// in generic_mask (a plan's routing); 2: the accelerated ADMM's classes
__host__ __device__ inline int class_of(int n, int d, int mode, uint64_t generic_mask = 0) {
    if (mode == 2) return kFirstFastClass + 4 * pow2_index((d + 7) / 8) + pow2_index((n + 63) / 64);
    if (mode == 1 && d > 16 && n <= 64 * kWideMaxM) {
        const int wc = (d + kWideNJ - 1) / kWideNJ;
        const int m = (n + 63) / 64;
        const int k = (wc - kWideMinWC) * kWideMaxM + (m - 1);
        if (!((generic_mask >> k) & 1u)) return kNumClasses + k;
    }
    return class_of(n, d);
}

// With the sliced classes in use, the classes above that only take d > 16 and
// n <= 256 never receive an instance.
__host__ __device__ constexpr bool class_unused_with_wide(int c) {
    return c >= 8 && c < kNumClasses && (c - 4) % 4 != 3;
}

// Kernel arguments of one class launch.
struct ClassLaunch {
    const float *a;               // points (FP32, or FP16 when a16)
    const float *w;
    const em_instance_t *inst;
    const int32_t *list;
    const unsigned int *offsets;  // class offsets into list (kNumClasses + 1)
    unsigned int *counter;        // work-queue head of this class
    float *z;
    em_stats_t *stats;
    const float *box_lo;          // per-coordinate bounds (indexed like z) or null
    const float *box_hi;
    const float *ball_center;     // SET = 1: centres (indexed like z) or null (origin)
    const float *ball_radius;     // SET = 1: radii (one per instance) or null (radius below)
    float radius;
    float lo, hi, mu, tol, arm;
    int32_t check_mask;           // primal residual only on iterations t with (t & check_mask) == 0 (or the last)
    float eps;                    // IRLS
    float adapt_ratio2;           // ADMM: (residual ratio)^2 that triggers a penalty change
    float adapt_factor;           // ADMM: penalty scale factor
    int32_t adapt_every;          // ADMM: 0 = fixed penalty
    int32_t max_iter, init, cls;
    int32_t a16;                  // points stored as FP16 (widened on staging)
    int64_t single;               // >= 0: solve only this instance (one workgroup, no queue)
    // Far outliers (fixed-penalty EM-ADMM over a box): an instance whose
    // largest |a| exceeds outlier * D * sqrt(n) is not solved by the class
    // kernel but appended to deferred list k (k = 0: d <= 16; 1: d > 16), at
    // defer_list + k * defer_stride, its count at defer_q[2 k + 1]
    // (defer_q[2 k] stays 0); null defer_q: no deferral
    float outlier;
    float fast_eta;               // accelerated ADMM: restart when c >= fast_eta (1 - 2^-16) c_prev
    int32_t *defer_list;
    int64_t defer_stride;
    unsigned int *defer_q;
};

// Append instance b to its deferred list (thread 0 of the workgroup).
__device__ __forceinline__ void defer_instance(const ClassLaunch &L, int b, int n, int d) {
    const int k = (d <= 16) ? 0 : 1;
    const unsigned int pos = atomicAdd(&L.defer_q[2 * k + 1], 1u);
    L.defer_list[k * L.defer_stride + pos] = b;
}

struct ClassKernel {
    const void *fn;
    int threads;
};

template <int DS, int M, int WC, int WP>
struct BatchShape {
    static constexpr int THREADS = 64 * WC * WP;
    static constexpr int H2 = RS<DS>::H2;
    static constexpr int STAGE = 64 * 65 + 1;  // one 64-point chunk, odd pitch <= 65
    static constexpr int XNB = WC * WP * M * 64;  // one buffer of per-wave norm partials
};

template <int DS, int M, int WC, int WP, int SOLVER, int SET>
__global__ __launch_bounds__(64 * WC * WP, 2) void batch_solve_kernel(ClassLaunch L) {
    constexpr bool IRLS = SOLVER == 1;
    constexpr bool BALL = SET == 1;
    constexpr bool ADAPT = SOLVER == 2;   // adaptive penalty (a separate kernel: it needs registers)
    constexpr bool WPEN = SOLVER == 4;    // penalty mu w_k per constraint (weighted-mean z-update)
    // SOLVER 5: EM-ADMM carrying the prox displacement e itself instead of
    // g = e - a (far-outlier instances deferred by SOLVER 0, see ClassLaunch)
    constexpr bool ES = SOLVER == 5;
    using S = BatchShape<DS, M, WC, WP>;
    using RSx = RS<DS>;
    constexpr int H2 = S::H2;
    __shared__ float stage[S::STAGE];
    // buffers 0/1 alternate by iteration; buffer 2 is the penalty-rescale exchange
    __shared__ float xn[(WC > 1) ? (ADAPT ? 3 : 2) * S::XNB : 1];
    // buffers 0/1 alternate by iteration; WPEN adds two for sum_k (x_k - c)
    __shared__ float xe[(WP > 1) ? (WPEN ? 4 : 2) * WP * WC * H2 * 4 : 1];
    __shared__ float xo[(WP > 1) ? 2 * WP : 1];
    __shared__ float xs[3 * WC * WP * 4];   // third slot: the test after armed iterations
    __shared__ float Epv[WC * H2 * 4 * WP];
    __shared__ float Bv[WC * WP * 2 * H2 * 4];   // box bounds, or the ball centre
    __shared__ float xb[BALL ? 2 * WC * WP : 1];  // ball: per-wave sums of squares
    __shared__ float cvec[WC * WP * DS];
    __shared__ float zvec[ADAPT ? WC * WP * DS : 1];
    __shared__ unsigned int item_s;
    __shared__ int flag_s[4];

    const int lane = threadIdx.x & 63;
    const int row = lane >> 4;
    const int wave = uniform_int(threadIdx.x >> 6);
    const int cw = wave % WC, pw = wave / WC;
    float *Ep_s = Epv + wave * H2 * 4;  // per wave: E^t in the reduced layout [slot][row]
    float *cv = cvec + wave * DS;       // per wave: c of the slice (ADMM), z - z0 (IRLS)
    float *zb = zvec + wave * DS;       // per wave: z of the slice, for a penalty rescale
    float *Bl_s = Bv + wave * 2 * H2 * 4;  // per wave: the box (ball: centre) in the reduced layout
    float *Bh_s = Bl_s + H2 * 4;
    // one instance per launch (L.single >= 0: the plain path) or the class's
    // work queue
    const bool one = L.single >= 0;
    const unsigned int cbeg = one ? 0u : L.offsets[L.cls];
    const unsigned int ccount = one ? 1u : L.offsets[L.cls + 1] - cbeg;
    // workgroups beyond the class's instance count would only find the queue
    // empty: they leave before the atomic, so an empty class costs its dispatch
    if (blockIdx.x >= ccount) return;
    unsigned int taken = 0;   // thread 0, single-instance mode: instances taken
    const bool vbox = L.box_lo != nullptr;

    for (;;) {
        if (threadIdx.x == 0) {
            item_s = one ? taken++ : atomicAdd(L.counter, 1u);
            flag_s[0] = 0;  // a point or weight is bad
            flag_s[1] = 0;  // max |a| (float bits, non-negative)
            flag_s[2] = 0;  // the starting z or the box is bad
            flag_s[3] = 0;  // widest box interval (float bits, non-negative)
        }
        __syncthreads();
        const unsigned int it = (unsigned int)uniform_int((int)item_s);
        if (it >= ccount) break;
        const int b = one ? (int)L.single : uniform_int(L.list[cbeg + it]);
        const em_instance_t e = L.inst[b];
        const int n = uniform_int(e.n), d = uniform_int(e.d);
        const float *A = L.a + e.a_off;
        const __half *A16 = reinterpret_cast<const __half *>(L.a) + e.a_off;
        auto aval = [&](int64_t i) -> float { return L.a16 ? __half2float(A16[i]) : A[i]; };
        const float *Wt = L.w + e.w_off;
        float *Z = L.z + e.z_off;
        const int pitch = d | 1;

        // ---- stage points into registers (coalesced via LDS), check them.
        // A chunk of 64 points is copied flat, at most KS values per thread,
        // by range-checked buffer loads (values past the instance read 0),
        // all of a chunk's loads in flight together; the weights of the
        // lane's points are loaded before the points.
        constexpr int NCH = M * WP;               // chunks, in the order (q, pc)
        constexpr int KS = (DS + WP - 1) / WP;    // 64 d <= 64 DS WC = KS x THREADS values
        const bool h16 = L.a16 != 0;
        const int tb = h16 ? 2 : 4;
        // (the descriptor is read into vector registers: its offset is made
        // uniform so that the buffer resources are scalar)
        const int64_t aoff = ((int64_t)uniform_int((int)(e.a_off >> 32)) << 32) |
                             (int64_t)(unsigned int)uniform_int((int)(e.a_off & 0xffffffff));
        const char *abase = h16 ? (const char *)(reinterpret_cast<const __half *>(L.a) + aoff)
                                : (const char *)(L.a + aoff);
        const float inv_d = 1.0f / (float)d;
        // (the thread index passed through an opaque move per instance: the
        // positions derived from it would otherwise be hoisted out of the
        // instance loop and hold KS registers each for the whole kernel)
        int tid;
        asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"((int)threadIdx.x));
        unsigned int raw[KS];
        // the chunk's values from its first one on: a resource per chunk (its
        // base and the rest of the instance as the range), the thread's
        // position as the vector offset, k x THREADS as the immediate one
        auto issue = [&](int c) {
            const int first = ((c % WP) * M + c / WP) * 64 * d;
            const int rest = max(0, n * d - first);
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<char *>(abase) + (int64_t)min(first, n * d) * tb, (short)0, rest * tb, kBufferRsrcWord3);
            if (h16) {
#pragma unroll
                for (int k = 0; k < KS; ++k)
                    raw[k] = __builtin_amdgcn_raw_buffer_load_b16(rs, tid * 2 + S::THREADS * 2 * k, 0, 0);
            } else {
#pragma unroll
                for (int k = 0; k < KS; ++k)
                    raw[k] = __builtin_amdgcn_raw_buffer_load_b32(rs, tid * 4 + S::THREADS * 4 * k, 0, 0);
            }
        };
        float na[M][DS];
        float lam[M];
        float wraw[M];
#pragma unroll
        for (int q = 0; q < M; ++q) wraw[q] = Wt[min(pw * M * 64 + q * 64 + lane, n - 1)];
        bool bad_l = false;
        float amax = 0.0f;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const int q = c / WP, pc = c % WP;
            issue(c);
            __syncthreads();   // the previous chunk has been read back
            // the whole chunk is staged: values past the instance read 0, so
            // the rows of absent points hold zeros
#pragma unroll
            for (int k = 0; k < KS; ++k) {
                if (tid < 64 * d - S::THREADS * k) {
                    const int i = tid + S::THREADS * k;
                    // row i / d by a float reciprocal: exact for i < 2^22
                    const int pp = (int)(((float)i + 0.5f) * inv_d);
                    const unsigned int bits = raw[k];
                    stage[pp * pitch + (i - pp * d)] =
                        h16 ? __half2float(__ushort_as_half((unsigned short)bits)) : __uint_as_float(bits);
                }
            }
            __syncthreads();
            if (pc == pw) {
                // (a NaN is caught by unordered compares of pairs, an
                // infinity by the running maximum, checked below)
#pragma unroll
                for (int jj = 0; jj < DS; jj += 2) {
                    const int j = cw * DS + jj;
                    const float v0 = (j < d) ? stage[lane * pitch + j] : 0.0f;
                    const float v1 = (jj + 1 < DS && j + 1 < d) ? stage[lane * pitch + j + 1] : 0.0f;
                    bad_l |= __builtin_isunordered(v0, v1);
                    amax = fmaxf(amax, fmaxf(fabsf(v0), fabsf(v1)));
                    na[q][jj] = -v0;
                    if (jj + 1 < DS) na[q][jj + 1] = -v1;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < M; ++q) {
            const int p = pw * M * 64 + q * 64 + lane;
            const float wv = (p < n) ? wraw[q] : 0.0f;
            bad_l |= !(wv >= 0.0f && wv <= FLT_MAX);
            lam[q] = (p < n) ? wv : -1.0f;  // weight for now (-1: no point); lambda below
        }
        bad_l |= !(amax <= FLT_MAX);   // an infinite point (NaN ones are flagged already)
        const float wamax = wave_max(amax);
        if (__any(bad_l) && lane == 0) flag_s[0] = 1;
        if (lane == 0) atomicMax(&flag_s[1], __float_as_int(wamax));  // non-negative floats order as ints
        // ---- MAXW init: largest weight, lowest index on ties
        int best = 0;
        if (L.init == EM_INIT_MAXW) {
            float wb = -1.0f;
            int pb = 0x7fffffff;
#pragma unroll
            for (int q = 0; q < M; ++q) {
                const int p = pw * M * 64 + q * 64 + lane;
                if (lam[q] > wb) {
                    wb = lam[q];
                    pb = p;
                }
            }
            const float wm = wave_max(wb);
            const float cand = (wb == wm) ? (float)pb : 3.0e38f;
            const float pmin = -wave_max(-cand);
            if constexpr (WP > 1) {
                if (lane == 0) {
                    xs[wave * 4 + 0] = wm;
                    xs[wave * 4 + 1] = pmin;
                }
                __syncthreads();
                float bw = -1.0f, bp = 3.0e38f;
                for (int v = 0; v < WP; ++v) {
                    const float wv = xs[(v * WC) * 4 + 0], pv = xs[(v * WC) * 4 + 1];
                    if (wv > bw || (wv == bw && pv < bp)) bw = wv, bp = pv;
                }
                best = uniform_int((int)bp);
            } else {
                best = uniform_int((int)pmin);
            }
            // no weight >= 0 at all leaves no candidate: the instance is bad
            // (NaN z below) and the clamp only keeps the read inside it
            best = min(max(best, 0), n - 1);
        }

        // ---- WMEAN init: sum_k w_k a_k / sum_k w_k, the weights scaled by their
        // largest value and the points by 1/n (no overflow); every weight zero:
        // equal weights
        float zw[H2];
        if (L.init == EM_INIT_WMEAN) {
            float wl = 0.0f;
#pragma unroll
            for (int q = 0; q < M; ++q) wl = fmaxf(wl, lam[q]);
            float wmx = wave_max(wl);
            if constexpr (WP > 1) {
                if (lane == 0) xs[wave * 4 + 2] = wmx;
                __syncthreads();
                wmx = xs[2];
#pragma unroll
                for (int v = 1; v < WP; ++v) wmx = fmaxf(wmx, xs[(v * WC) * 4 + 2]);
            }
            wmx = readfirstlane(wmx);
            const bool uni = !(wmx > 0.0f);
            const float sw = uni ? 0.0f : 1.0f / wmx;
            const float inv_n = 1.0f / (float)n;
            float cq[M];
            float cs = 0.0f;
#pragma unroll
            for (int q = 0; q < M; ++q) {
                cq[q] = (lam[q] >= 0.0f) ? (uni ? 1.0f : lam[q] * sw) * inv_n : 0.0f;
                cs += cq[q];
            }
            float acc[DS];
#pragma unroll
            for (int jj = 0; jj < DS; ++jj) {
                float ac = 0.0f;
#pragma unroll
                for (int q = 0; q < M; ++q) ac = fmaf(-cq[q], na[q][jj], ac);   // na = -a
                acc[jj] = ac;
            }
            reduce_scatter<DS>(acc, zw);
            float Cs = readfirstlane(wave_sum(cs));
            if constexpr (WP > 1) {
                float *XE = xe;   // buffer 0; the solve's first exchange uses buffer 1
                float *XO = xo;
                if (lane == 16 * row) {
#pragma unroll
                    for (int j = 0; j < H2; ++j) XE[((pw * WC + cw) * H2 + j) * 4 + row] = zw[j];
                }
                if (cw == 0 && lane == 0) XO[pw] = Cs;
                __syncthreads();
#pragma unroll
                for (int j = 0; j < H2; ++j) {
                    float sum = XE[(cw * H2 + j) * 4 + row];
#pragma unroll
                    for (int v = 1; v < WP; ++v) sum += XE[((v * WC + cw) * H2 + j) * 4 + row];
                    zw[j] = sum;
                }
                float os = XO[0];
#pragma unroll
                for (int v = 1; v < WP; ++v) os += XO[v];
                Cs = readfirstlane(os);
            }
            const float inv_c = 1.0f / Cs;
#pragma unroll
            for (int j = 0; j < H2; ++j) zw[j] *= inv_c;
        }

        // ---- starting z and the box in the reduced layout
        float zr[H2];
        bool zbad = false;
        float wid = 0.0f;
#pragma unroll
        for (int j = 0; j < H2; ++j) {
            const int cc = cw * DS + RSx::coord(row, j);
            const bool vj = RSx::valid(row, j) && cc < d;
            float zv = 0.0f, lv = BALL ? 0.0f : L.lo, hv = BALL ? 0.0f : L.hi;
            if (vj) {
                zv = (L.init == EM_INIT_MAXW) ? aval((int64_t)best * d + cc)
                     : (L.init == EM_INIT_WMEAN) ? zw[j] : Z[cc];
                if (BALL) {
                    if (L.ball_center) lv = L.ball_center[e.z_off + cc];
                } else if (vbox) {
                    lv = L.box_lo[e.z_off + cc];
                    hv = L.box_hi[e.z_off + cc];
                }
            }
            zbad |= vj && !(fabsf(zv) <= FLT_MAX);
            zbad |= vj && (BALL ? !(fabsf(lv) <= FLT_MAX) : !(lv <= hv));
            const float wj = hv - lv;
            if (vj && !(wj <= wid)) wid = wj;   // also takes inf
            zr[j] = zv;
            if (lane == 16 * row) {
                Bl_s[j * 4 + row] = lv;
                Bh_s[j * 4 + row] = hv;
            }
        }
        const float wwid = wave_max(wid);
        if (__any(zbad) && lane == 0) flag_s[2] = 1;
        if (lane == 0) atomicMax(&flag_s[3], __float_as_int(wwid));
        __syncthreads();
        const float rad = BALL ? (L.ball_radius ? readfirstlane(L.ball_radius[b]) : L.radius) : 0.0f;
        const bool bad_all = uniform(flag_s[0] != 0 || flag_s[2] != 0 || (BALL && !(rad >= 0.0f)));
        const float wmax = BALL ? 2.0f * rad : readfirstlane(__int_as_float(flag_s[3]));
        const float amax_all = readfirstlane(__int_as_float(flag_s[1]));
        const float Dscale = (wmax <= FLT_MAX && wmax > 0.0f) ? wmax : fmaxf(1.0f, amax_all);
        const float tau = L.tol * Dscale;
        const float tau2 = tau * tau;
        const float arm2 = (L.arm * tau) * (L.arm * tau);
        __syncthreads();  // flags are reset by the next pop
        if constexpr (SOLVER == 0 && !BALL) {
            if (L.defer_q != nullptr && !bad_all &&
                uniform(amax_all > L.outlier * Dscale * sqrtf((float)n))) {
                if (threadIdx.x == 0) defer_instance(L, b, n, d);
                continue;
            }
        }

        // Ball projection factor min(1, radius / ||m - center||) from the lane's
        // row partial sum of (m_j - center_j)^2 (identical on the row's lanes);
        // rows summed by readlanes, coordinate waves through LDS.
        auto ball_factor = [&](float s2row, int t) -> float {
            float S = readfirstlane((readlane(s2row, 0) + readlane(s2row, 16)) +
                                    (readlane(s2row, 32) + readlane(s2row, 48)));
            if constexpr (WC > 1) {
                float *XB = xb + (t & 1) * WC * WP;
                if (lane == 0) XB[pw * WC + cw] = S;
                __syncthreads();
                S = XB[pw * WC];
#pragma unroll
                for (int v = 1; v < WC; ++v) S += XB[pw * WC + v];
                S = readfirstlane(S);
            }
            return (S > rad * rad) ? rad / sqrtf(S) : 1.0f;
        };

        // c = z (ADMM); IRLS keeps its frame origin per slot (below)
        float z0[IRLS ? H2 : 1];
        if (lane == 16 * row) {
#pragma unroll
            for (int j = 0; j < H2; ++j) {
                Ep_s[j * 4 + row] = 0.0f;
                if (RSx::valid(row, j)) cv[RSx::coord(row, j)] = zr[j];  // 0 on padded coordinates
            }
        }
        if constexpr (IRLS) {
#pragma unroll
            for (int j = 0; j < H2; ++j) z0[j] = zr[j];
        }

        int iters = 0, flags = EM_MAXITER;
        float rp2 = 0.0f, rd2 = 0.0f;
        if (bad_all) {
            flags = EM_BAD_INPUT;
        } else if constexpr (IRLS) {
            // ---- frame origin o = P_C(z0): points as o - a, iterate z - o (the
            // distance to a point at o keeps FP32 precision of its own size;
            // projecting keeps |z - o| within the set's diameter when z0 is a
            // far point)
            {
                float fo = 1.0f;
                if constexpr (BALL) {
                    float s2 = 0.0f;
#pragma unroll
                    for (int j = 0; j < H2; ++j) {
                        const int cc = cw * DS + RSx::coord(row, j);
                        const bool vj = RSx::valid(row, j) && cc < d;
                        const float dv = z0[j] - Bl_s[j * 4 + row];
                        s2 += vj ? dv * dv : 0.0f;
                    }
                    fo = ball_factor(s2, 0);
                }
#pragma unroll
                for (int j = 0; j < H2; ++j) {
                    const float bl = Bl_s[j * 4 + row], bh = Bh_s[j * 4 + row];
                    const float o = BALL ? ((fo < 1.0f) ? bl + (z0[j] - bl) * fo : z0[j]) : clampf(z0[j], bl, bh);
                    zr[j] = z0[j] - o;   // the start relative to o
                    z0[j] = o;
                }
            }
            if (lane == 16 * row) {
#pragma unroll
                for (int j = 0; j < H2; ++j)
                    if (RSx::valid(row, j)) cv[RSx::coord(row, j)] = z0[j];
            }
#pragma unroll
            for (int jj = 0; jj < DS; ++jj) {
                const float cj = cv[jj];
#pragma unroll
                for (int q = 0; q < M; ++q) na[q][jj] += cj;
            }
            if (lane == 16 * row) {
#pragma unroll
                for (int j = 0; j < H2; ++j)
                    if (RSx::valid(row, j)) cv[RSx::coord(row, j)] = zr[j];
            }
#pragma unroll
            for (int q = 0; q < M; ++q) lam[q] = fmaxf(lam[q], 0.0f);   // the weights
            const float eps = L.eps;
            const float inv_d = 1.0f / (float)d;
            const int max_iter = L.max_iter;
            float rd_w = 0.0f;
            bool done = false;
            int t = 1;
            for (; t <= max_iter; ++t) {
                // ---- ||z - a_k||^2 (+ eps, counted once over the coordinate waves)
                float nrm[M];
#pragma unroll
                for (int q = 0; q < M; ++q) nrm[q] = (cw == 0) ? eps : 0.0f;
#pragma unroll
                for (int jj = 0; jj < DS; ++jj) {
                    const float cj = cv[jj];
#pragma unroll
                    for (int q = 0; q < M; ++q) {
                        const float dv = na[q][jj] + cj;
                        nrm[q] = fmaf(dv, dv, nrm[q]);
                    }
                }
                float rd_all = rd_w;
                if constexpr (WC > 1 || WP > 1) {
                    float *XS = xs + (t & 1) * WC * WP * 4;
                    if constexpr (WC > 1) {
                        float *X = xn + (t & 1) * S::XNB;
#pragma unroll
                        for (int q = 0; q < M; ++q) X[((pw * WC + cw) * M + q) * 64 + lane] = nrm[q];
                    }
                    if (lane == 0) XS[wave * 4] = rd_w;
                    __syncthreads();
                    if constexpr (WC > 1) {
                        float *X = xn + (t & 1) * S::XNB;
#pragma unroll
                        for (int q = 0; q < M; ++q) {
                            float sum = X[(pw * WC * M + q) * 64 + lane];
#pragma unroll
                            for (int v = 1; v < WC; ++v) sum += X[((pw * WC + v) * M + q) * 64 + lane];
                            nrm[q] = sum;
                        }
                    }
                    rd_all = 0.0f;
#pragma unroll
                    for (int v = 0; v < WC * WP; ++v) rd_all += XS[v * 4];
                    rd_all = readfirstlane(rd_all);
                }
                if (t > 1) {
                    rd2 = rd_all * inv_d;
                    if (uniform(tau2 > 0.0f && rd2 <= tau2)) {
                        flags = EM_CONVERGED;
                        iters = t - 1;
                        done = true;
                        break;
                    }
                }
                // ---- omega_k and the omega-weighted sums
                float om[M];
                float ol = 0.0f;
#pragma unroll
                for (int q = 0; q < M; ++q) {
                    om[q] = lam[q] * __builtin_amdgcn_rsqf(nrm[q]);
                    ol += om[q];
                }
                float acc[DS];
#pragma unroll
                for (int jj = 0; jj < DS; ++jj) {
                    float ac = 0.0f;
#pragma unroll
                    for (int q = 0; q < M; ++q) ac = fmaf(om[q], na[q][jj], ac);
                    acc[jj] = ac;
                }
                float E[H2];
                reduce_scatter<DS>(acc, E);   // sum_k omega_k (z0 - a_k)
                float Om = readfirstlane(wave_sum(ol));
                if constexpr (WP > 1) {
                    float *XE = xe + (t & 1) * WP * WC * H2 * 4;
                    float *XO = xo + (t & 1) * WP;
                    if (lane == 16 * row) {
#pragma unroll
                        for (int j = 0; j < H2; ++j) XE[((pw * WC + cw) * H2 + j) * 4 + row] = E[j];
                    }
                    if (cw == 0 && lane == 0) XO[pw] = Om;
                    __syncthreads();
#pragma unroll
                    for (int j = 0; j < H2; ++j) {
                        float sum = XE[(cw * H2 + j) * 4 + row];
#pragma unroll
                        for (int v = 1; v < WP; ++v) sum += XE[((v * WC + cw) * H2 + j) * 4 + row];
                        E[j] = sum;
                    }
                    float os = XO[0];
#pragma unroll
                    for (int v = 1; v < WP; ++v) os += XO[v];
                    Om = readfirstlane(os);
                }
                // all weights zero: every point of C is a minimiser; z' = P_C(z)
                const bool live = Om > 0.0f;
                const float inv_om = live ? 1.0f / Om : 0.0f;
                float fb = 1.0f;
                if constexpr (BALL) {
                    float s2 = 0.0f;
#pragma unroll
                    for (int j = 0; j < H2; ++j) {
                        const int cc = cw * DS + RSx::coord(row, j);
                        const bool vj = RSx::valid(row, j) && cc < d;
                        const float dv = (z0[j] - Bl_s[j * 4 + row]) + (live ? -E[j] * inv_om : zr[j]);
                        s2 += vj ? dv * dv : 0.0f;
                    }
                    fb = ball_factor(s2, t);
                }
                float rdx = 0.0f;
#pragma unroll
                for (int j = 0; j < H2; ++j) {
                    const int cc = cw * DS + RSx::coord(row, j);
                    const bool vj = RSx::valid(row, j) && cc < d;
                    // z' - z0 = P_C(z0 + raw) - z0, exact when the set is inactive
                    const float raw = live ? -E[j] * inv_om : zr[j];
                    float zn;
                    if constexpr (BALL) {
                        const float cn = Bl_s[j * 4 + row];
                        zn = (fb < 1.0f) ? (cn - z0[j]) + ((z0[j] - cn) + raw) * fb : raw;
                    } else {
                        const float zab = z0[j] + raw;
                        const float bl = Bl_s[j * 4 + row], bh = Bh_s[j * 4 + row];
                        zn = (zab < bl) ? bl - z0[j] : ((zab > bh) ? bh - z0[j] : raw);
                    }
                    zn = vj ? zn : zr[j];
                    const float dz = zn - zr[j];
                    rdx += dz * dz;
                    if (lane == 16 * row && RSx::valid(row, j)) cv[RSx::coord(row, j)] = zn;
                    zr[j] = zn;
                }
                const float rdw = readfirstlane((readlane(rdx, 0) + readlane(rdx, 16)) +
                                                (readlane(rdx, 32) + readlane(rdx, 48)));
                rd_w = (pw == 0) ? rdw : 0.0f;
                if (uniform(!live)) {   // all weights zero: done after the projection
                    float rd_all = rd_w;
                    if constexpr (WC > 1 || WP > 1) {
                        float *XS = xs + 2 * WC * WP * 4;   // third slot (unused by IRLS otherwise)
                        if (lane == 0) XS[wave * 4] = rd_w;
                        __syncthreads();
                        rd_all = 0.0f;
#pragma unroll
                        for (int v = 0; v < WC * WP; ++v) rd_all += XS[v * 4];
                        rd_all = readfirstlane(rd_all);
                    }
                    rd2 = rd_all * inv_d;
                    flags = EM_CONVERGED;
                    iters = t;
                    done = true;
                    break;
                }
            }
            if (!done) {
                iters = max_iter;
                if (max_iter >= 1) {
                    float rd_all = rd_w;
                    if constexpr (WC > 1 || WP > 1) {
                        float *XS = xs + (t & 1) * WC * WP * 4;
                        if (lane == 0) XS[wave * 4] = rd_w;
                        __syncthreads();
                        rd_all = 0.0f;
#pragma unroll
                        for (int v = 0; v < WC * WP; ++v) rd_all += XS[v * 4];
                        rd_all = readfirstlane(rd_all);
                    }
                    rd2 = rd_all * inv_d;
                    flags = (tau2 > 0.0f && rd2 <= tau2) ? EM_CONVERGED : EM_MAXITER;
                }
            }
#pragma unroll
            for (int j = 0; j < H2; ++j) zr[j] = z0[j] + zr[j];
        } else {
            float g[M][DS];
            float mu_c = L.mu;
            const float inv_mu0 = 1.0f / L.mu;
            // z-update divisor (1/n, or 1/sum of the weights for WPEN) and the
            // number of points the primal residual runs over
            float zdiv = 1.0f / (float)n;
            float fn = (float)n;
            float wq[M];   // WPEN: weights scaled by their largest value (the iterates do not change)
            if constexpr (WPEN) {
                float wl = 0.0f;
#pragma unroll
                for (int q = 0; q < M; ++q) wl = fmaxf(wl, lam[q]);
                float wmx = wave_max(wl);
                if constexpr (WP > 1) {
                    if (lane == 0) xs[wave * 4 + 0] = wmx;
                    __syncthreads();
                    wmx = xs[0];
#pragma unroll
                    for (int v = 1; v < WP; ++v) wmx = fmaxf(wmx, xs[(v * WC) * 4 + 0]);
                }
                wmx = readfirstlane(wmx);
                const float sc = (wmx > 0.0f) ? 1.0f / wmx : 0.0f;
                float ws = 0.0f, ne = 0.0f;
#pragma unroll
                for (int q = 0; q < M; ++q) {
                    const bool pos = lam[q] > 0.0f;   // a point of weight zero is left out
                    wq[q] = pos ? lam[q] * sc : 0.0f;
                    ws += wq[q];
                    ne += pos ? 1.0f : 0.0f;
                    lam[q] = pos ? inv_mu0 : 0.0f;    // threshold w_k / (mu w_k)
                }
                ws = wave_sum(ws);
                ne = wave_sum(ne);
                if constexpr (WP > 1) {
                    if (lane == 0) {
                        xs[wave * 4 + 1] = ws;
                        xs[wave * 4 + 2] = ne;
                    }
                    __syncthreads();
                    ws = xs[1];
                    ne = xs[2];
#pragma unroll
                    for (int v = 1; v < WP; ++v) {
                        ws += xs[(v * WC) * 4 + 1];
                        ne += xs[(v * WC) * 4 + 2];
                    }
                }
                ws = readfirstlane(ws);
                zdiv = (ws > 0.0f) ? 1.0f / ws : 0.0f;   // every weight zero: z' = P_C(z)
                fn = readfirstlane(ne);
            } else {
#pragma unroll
                for (int q = 0; q < M; ++q) {
                    lam[q] = (lam[q] >= 0.0f) ? lam[q] * inv_mu0 : 0.0f;
                    wq[q] = 1.0f;
                }
            }
#pragma unroll
            for (int q = 0; q < M; ++q)
#pragma unroll
                for (int jj = 0; jj < DS; ++jj) g[q][jj] = ES ? 0.0f : na[q][jj];
            const float inv_d = 1.0f / (float)d;
            const float inv_nd = (fn > 0.0f) ? 1.0f / (fn * (float)d) : 0.0f;
            const int max_iter = L.max_iter;
            const int every = ADAPT ? L.adapt_every : 0;
            float rd_w = 0.0f, rp_w = 0.0f;
            bool done = false;
            int t = 1;
            for (; t <= max_iter; ++t) {
                // ---- pass 1: delta = g + c, partial ||delta||^2
                float nrm[M];
#pragma unroll
                for (int q = 0; q < M; ++q) nrm[q] = kNu2Floor;
#pragma unroll
                for (int jj = 0; jj < DS; ++jj) {
                    const float cj = cv[jj];
#pragma unroll
                    for (int q = 0; q < M; ++q) {
                        if constexpr (ES) {
                            const float dl = (g[q][jj] + cj) + na[q][jj];
                            nrm[q] = fmaf(dl, dl, nrm[q]);
                        } else {
                            g[q][jj] += cj;
                            nrm[q] = fmaf(g[q][jj], g[q][jj], nrm[q]);
                        }
                    }
                }
                if constexpr (ES) {   // pass 2 recomputes delta (do not hold it across the exchange)
#pragma unroll
                    for (int q = 0; q < M; ++q)
#pragma unroll
                        for (int jj = 0; jj < DS; ++jj) asm volatile("" : "+v"(g[q][jj]));
                }
                float rd_all = rd_w;
                if constexpr (WC > 1 || WP > 1) {
                    float *XS = xs + (t & 1) * WC * WP * 4;
                    if constexpr (WC > 1) {
                        float *X = xn + (t & 1) * S::XNB;
#pragma unroll
                        for (int q = 0; q < M; ++q) X[((pw * WC + cw) * M + q) * 64 + lane] = nrm[q];
                    }
                    if (lane == 0) XS[wave * 4] = rd_w;
                    __syncthreads();
                    if constexpr (WC > 1) {
                        float *X = xn + (t & 1) * S::XNB;
#pragma unroll
                        for (int q = 0; q < M; ++q) {
                            float sum = X[(pw * WC * M + q) * 64 + lane];
#pragma unroll
                            for (int v = 1; v < WC; ++v) sum += X[((pw * WC + v) * M + q) * 64 + lane];
                            nrm[q] = sum;
                        }
                    }
                    rd_all = 0.0f;
#pragma unroll
                    for (int v = 0; v < WC * WP; ++v) rd_all += XS[v * 4];
                    rd_all = readfirstlane(rd_all);
                }
                // dual residual of iteration t-1 (all waves hold identical sums), which
                // arms this iteration; the stop test itself follows armed iterations
                if (t > 1) rd2 = rd_all * inv_d;
                // ---- adaptive penalty after a balancing iteration t-1: compare
                // ||r||^2 = n d rp2 with (ratio ||s||)^2 = ratio^2 mu^2 n d rd2
                if (ADAPT && t > 1 && (t - 1) % every == 0) {
                    const float m2 = mu_c * mu_c;
                    float tf = 1.0f;
                    if (rp2 > L.adapt_ratio2 * m2 * rd2)
                        tf = L.adapt_factor;
                    else if (m2 * rd2 > L.adapt_ratio2 * rp2)
                        tf = 1.0f / L.adapt_factor;
                    if (uniform(tf != 1.0f)) {
                        const float it_ = 1.0f / tf, omt = 1.0f - it_;
                        mu_c *= tf;
#pragma unroll
                        for (int q = 0; q < M; ++q) lam[q] *= it_;
                        // z of the slice to every lane; E^t and c rescaled
                        if (lane == 16 * row) {
#pragma unroll
                            for (int j = 0; j < H2; ++j) {
                                if (RSx::valid(row, j)) zb[RSx::coord(row, j)] = zr[j];
                                Ep_s[j * 4 + row] *= it_;
                            }
                        }
#pragma unroll
                        for (int q = 0; q < M; ++q) nrm[q] = kNu2Floor;
#pragma unroll
                        for (int jj = 0; jj < DS; ++jj) {
                            const float zj = zb[jj];
#pragma unroll
                            for (int q = 0; q < M; ++q) {
                                g[q][jj] = fmaf(g[q][jj], it_, omt * (na[q][jj] + zj));
                                nrm[q] = fmaf(g[q][jj], g[q][jj], nrm[q]);
                            }
                        }
                        if (lane == 16 * row) {
#pragma unroll
                            for (int j = 0; j < H2; ++j)
                                if (RSx::valid(row, j)) {
                                    const int k = RSx::coord(row, j);
                                    cv[k] = fmaf(cv[k], it_, omt * zr[j]);
                                }
                        }
                        if constexpr (WC > 1) {
                            float *X = xn + 2 * S::XNB;
#pragma unroll
                            for (int q = 0; q < M; ++q) X[((pw * WC + cw) * M + q) * 64 + lane] = nrm[q];
                            __syncthreads();
#pragma unroll
                            for (int q = 0; q < M; ++q) {
                                float sum = X[(pw * WC * M + q) * 64 + lane];
#pragma unroll
                                for (int v = 1; v < WC; ++v) sum += X[((pw * WC + v) * M + q) * 64 + lane];
                                nrm[q] = sum;
                            }
                        }
                    }
                }
                const bool armed = uniform((t == max_iter) ||
                                           (tau2 > 0.0f && t > 1 && rd2 <= arm2 && (t & L.check_mask) == 0) ||
                                           (ADAPT && t % every == 0));
                float s[M];
#pragma unroll
                for (int q = 0; q < M; ++q) s[q] = shrink(nrm[q], lam[q]);
                // ---- armed iterations: lane sums of ||x_k - c||^2, x_k = a_k + (1 - s) delta.
                // Absent points and padded coordinates give exactly 0 (g stays -a).
                float rp_lane = 0.0f;
                float Ys[H2];   // WPEN, armed: sum_k (x_k - c) in the reduced layout
                if (!ES && armed) {
                    float ysum[DS];   // WPEN: lane sums of x_k - c (points of weight zero give 0)
                    float rq[M];
#pragma unroll
                    for (int q = 0; q < M; ++q) rq[q] = 0.0f;
#pragma unroll
                    for (int jj = 0; jj < DS; ++jj) {
                        const float cj = cv[jj];
                        float ys = 0.0f;
#pragma unroll
                        for (int q = 0; q < M; ++q) {
                            const float y = fmaf(1.0f - s[q], g[q][jj], -(na[q][jj] + cj));
                            rq[q] = fmaf(y, y, rq[q]);
                            if constexpr (WPEN) ys += y;
                        }
                        ysum[jj] = ys;
                    }
#pragma unroll
                    for (int q = 0; q < M; ++q) rp_lane += rq[q];
                    if constexpr (WPEN) reduce_scatter<DS>(ysum, Ys);
                }
                // ---- pass 2: E = sum_k s delta (WPEN: sum_k w_k s delta), g = s delta - a
                float sw[M];
#pragma unroll
                for (int q = 0; q < M; ++q) sw[q] = WPEN ? s[q] * wq[q] : s[q];
                float acc[DS];
                if constexpr (ES) {
                    // delta = (e + c) - a again; e = s delta; armed: x_k - c = e - s delta
                    float rq[M];
#pragma unroll
                    for (int q = 0; q < M; ++q) rq[q] = 0.0f;
                    if (armed) {
#pragma unroll
                        for (int jj = 0; jj < DS; ++jj) {
                            const float cj = cv[jj];
                            float ac = 0.0f;
#pragma unroll
                            for (int q = 0; q < M; ++q) {
                                const float dl = (g[q][jj] + cj) + na[q][jj];
                                const float y = fmaf(-s[q], dl, g[q][jj]);
                                rq[q] = fmaf(y, y, rq[q]);
                                ac = fmaf(sw[q], dl, ac);
                                g[q][jj] = s[q] * dl;
                            }
                            acc[jj] = ac;
                        }
                    } else {
#pragma unroll
                        for (int jj = 0; jj < DS; ++jj) {
                            const float cj = cv[jj];
                            float ac = 0.0f;
#pragma unroll
                            for (int q = 0; q < M; ++q) {
                                const float dl = (g[q][jj] + cj) + na[q][jj];
                                ac = fmaf(sw[q], dl, ac);
                                g[q][jj] = s[q] * dl;
                            }
                            acc[jj] = ac;
                        }
                    }
#pragma unroll
                    for (int q = 0; q < M; ++q) rp_lane += rq[q];
                } else {
#pragma unroll
                    for (int jj = 0; jj < DS; ++jj) {
                        float ac = 0.0f;
#pragma unroll
                        for (int q = 0; q < M; ++q) {
                            const float dl = g[q][jj];
                            ac = fmaf(sw[q], dl, ac);
                            g[q][jj] = fmaf(s[q], dl, na[q][jj]);
                        }
                        acc[jj] = ac;
                    }
                }
#pragma unroll
                for (int q = 0; q < M; ++q)
#pragma unroll
                    for (int jj = 0; jj < DS; ++jj) asm volatile("" : "+v"(g[q][jj]));
                float E[H2];
                reduce_scatter<DS>(acc, E);
                if constexpr (WP > 1) {
                    float *XE = xe + (t & 1) * WP * WC * H2 * 4;
                    float *XY = xe + (2 + (t & 1)) * WP * WC * H2 * 4;
                    if (lane == 16 * row) {
#pragma unroll
                        for (int j = 0; j < H2; ++j) {
                            XE[((pw * WC + cw) * H2 + j) * 4 + row] = E[j];
                            if (WPEN && armed) XY[((pw * WC + cw) * H2 + j) * 4 + row] = Ys[j];
                        }
                    }
                    __syncthreads();
#pragma unroll
                    for (int j = 0; j < H2; ++j) {
                        float sum = 0.0f, ysm = 0.0f;
#pragma unroll
                        for (int v = 0; v < WP; ++v) {
                            sum += XE[((v * WC + cw) * H2 + j) * 4 + row];
                            if (WPEN && armed) ysm += XY[((v * WC + cw) * H2 + j) * 4 + row];
                        }
                        E[j] = sum;
                        if (WPEN && armed) Ys[j] = ysm;
                    }
                }
                float fb = 1.0f;
                if constexpr (BALL) {
                    float s2 = 0.0f;
#pragma unroll
                    for (int j = 0; j < H2; ++j) {
                        const int cc = cw * DS + RSx::coord(row, j);
                        const bool vj = RSx::valid(row, j) && cc < d;
                        const float dv = (zr[j] - E[j] * zdiv) - Bl_s[j * 4 + row];
                        s2 += vj ? dv * dv : 0.0f;
                    }
                    fb = ball_factor(s2, t);
                }
                float rdx = 0.0f, rpx = 0.0f;
#pragma unroll
                for (int j = 0; j < H2; ++j) {
                    const int cc = cw * DS + RSx::coord(row, j);
                    const bool vj = RSx::valid(row, j) && cc < d;
                    const int k = RSx::valid(row, j) ? RSx::coord(row, j) : 0;
                    const float zu = zr[j] - E[j] * zdiv;
                    const float zn = BALL ? ((fb < 1.0f) ? Bl_s[j * 4 + row] + (zu - Bl_s[j * 4 + row]) * fb : zu)
                                          : clampf(zu, Bl_s[j * 4 + row], Bh_s[j * 4 + row]);
                    const float dz = zn - zr[j];
                    const float cj = cv[k];
                    if (armed) {
                        // x_k - z' = (x_k - c) + (c - z'), sum_k (x_k - c) = E^t - E^{t+1}
                        // (WPEN: summed directly, E being weighted)
                        const float sxc = WPEN ? Ys[j] : (Ep_s[j * 4 + row] - E[j]);
                        const float cz = cj - zn;
                        rpx += vj ? (cz * (2.0f * sxc + fn * cz)) : 0.0f;
                    }
                    rdx += vj ? dz * dz : 0.0f;
                    if (lane == 16 * row) {
                        Ep_s[j * 4 + row] = E[j];
                        if (RSx::valid(row, j)) cv[k] = vj ? (2.0f * zn - zr[j]) : 0.0f;
                    }
                    zr[j] = vj ? zn : 0.0f;
                }
                // per-coordinate terms are counted once, by point-wave 0
                const float rdw = readfirstlane((readlane(rdx, 0) + readlane(rdx, 16)) +
                                                (readlane(rdx, 32) + readlane(rdx, 48)));
                rd_w = (pw == 0) ? rdw : 0.0f;
                if (armed) {
                    const float tot = readfirstlane(wave_sum(rp_lane));
                    const float px = readfirstlane((readlane(rpx, 0) + readlane(rpx, 16)) +
                                                   (readlane(rpx, 32) + readlane(rpx, 48)));
                    rp_w = tot + ((pw == 0) ? px : 0.0f);
                    // ---- stop test right after the armed iteration
                    float rd_all = rd_w, rp_all = rp_w;
                    if constexpr (WC > 1 || WP > 1) {
                        float *XS = xs + 2 * WC * WP * 4;
                        if (lane == 0) {
                            XS[wave * 4 + 0] = rd_w;
                            XS[wave * 4 + 1] = rp_w;
                        }
                        __syncthreads();
                        rd_all = 0.0f;
                        rp_all = 0.0f;
#pragma unroll
                        for (int v = 0; v < WC * WP; ++v) {
                            rd_all += XS[v * 4 + 0];
                            rp_all += XS[v * 4 + 1];
                        }
                        rd_all = readfirstlane(rd_all);
                        rp_all = readfirstlane(rp_all);
                    }
                    rd2 = rd_all * inv_d;
                    rp2 = fmaxf(rp_all, 0.0f) * inv_nd;
                    if (uniform(tau2 > 0.0f && rp2 <= tau2 && rd2 <= tau2)) {
                        flags = EM_CONVERGED;
                        iters = t;
                        done = true;
                        break;
                    }
                } else {
                    rp_w = 0.0f;
                }
            }
            if (!done) iters = max_iter;   // the last iteration was armed and tested
        }
        // ---- write z (point-wave 0 of each coordinate slice) and stats
        if (pw == 0 && lane == 16 * row) {
#pragma unroll
            for (int j = 0; j < H2; ++j) {
                const int cc = cw * DS + RSx::coord(row, j);
                if (RSx::valid(row, j) && cc < d) Z[cc] = bad_all ? __builtin_nanf("") : zr[j];
            }
        }
        if (wave == 0 && lane == 0 && L.stats != nullptr) {
            em_stats_t st;
            st.iters = bad_all ? 0 : iters;
            st.flags = flags;
            st.r_pri = (bad_all || IRLS) ? 0.0f : sqrtf(rp2);
            st.r_dual = bad_all ? 0.0f : sqrtf(rd2);
            L.stats[b] = st;
        }
    }
}

template <int C, int SOLVER, int SET>
constexpr ClassKernel class_kernel() {
    constexpr ClassShape s = class_shape(C);
    return ClassKernel{
        reinterpret_cast<const void *>(&batch_solve_kernel<s.ds, s.m, s.wc, s.wp, SOLVER, SET>),
        64 * s.wc * s.wp};
}

template <int SOLVER, int SET>
const ClassKernel *class_table_for() {
    static const ClassKernel t[kNumClasses] = {
        class_kernel<0, SOLVER, SET>(),  class_kernel<1, SOLVER, SET>(),  class_kernel<2, SOLVER, SET>(),
        class_kernel<3, SOLVER, SET>(),  class_kernel<4, SOLVER, SET>(),  class_kernel<5, SOLVER, SET>(),
        class_kernel<6, SOLVER, SET>(),  class_kernel<7, SOLVER, SET>(),  class_kernel<8, SOLVER, SET>(),
        class_kernel<9, SOLVER, SET>(),  class_kernel<10, SOLVER, SET>(), class_kernel<11, SOLVER, SET>(),
        class_kernel<12, SOLVER, SET>(), class_kernel<13, SOLVER, SET>(), class_kernel<14, SOLVER, SET>(),
        class_kernel<15, SOLVER, SET>(), class_kernel<16, SOLVER, SET>(), class_kernel<17, SOLVER, SET>(),
        class_kernel<18, SOLVER, SET>(), class_kernel<19, SOLVER, SET>(),
    };
    return t;
}

// Class kernel tables, one translation unit per (solver, set).
const ClassKernel *batch_class_table_admm();
const ClassKernel *batch_class_table_irls();
const ClassKernel *batch_class_table_adapt();
const ClassKernel *batch_class_table_admm_ball();
const ClassKernel *batch_class_table_irls_ball();
const ClassKernel *batch_class_table_wpen();
const ClassKernel *batch_class_table_wpen_ball();
const ClassKernel *batch_wide_table();   // kNumWideClasses entries
// The kernels that solve the deferred far-outlier lists 0 and 1 (fixed-penalty
// EM-ADMM over a box carrying e): d <= 16 (one 16-coordinate slice) and
// d <= 64 (four), both n <= 512 (2 x 4 points per lane).
constexpr int kDeferLists = 2;
const ClassKernel *batch_deferred_table();
const ClassKernel *batch_fast_table();   // kNumFastClasses entries

}  // namespace emx
