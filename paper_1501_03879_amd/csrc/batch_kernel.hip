// Batched EM-ADMM over independent point sets of uneven size (Algorithm 1 of
// arXiv:1501.03879 for every instance), and the plain one-launch-per-instance
// baseline.
//
// Batched solver
//  * A device pre-pass sorts instances into shape classes (coordinate slice
//    DS, points per lane M, waves over coordinates WC, waves over points WP)
//    with a counting sort; empty and malformed instances are finished there.
//  * One persistent kernel per class pops instances from a work queue.  A
//    workgroup of WC x WP waves owns one instance: wave (cw, pw) holds
//    coordinates [cw DS, cw DS + DS) of points pw 64 M + l + 64 q.  Points
//    and the iteration state (g = e - a, see the NLEM kernel) stay in
//    registers for the whole solve; the points are read from HBM once,
//    coalesced, through an LDS staging buffer.
//  * Per iteration: pass 1 (delta = g + c, partial ||delta||^2), norms summed
//    over the WC coordinate waves in LDS, shrink factor, pass 2 (E += s delta,
//    g = s delta - a), wave reduce-scatter of E, sum over the WP point waves
//    in LDS, then z = clamp(z - E / n), c = 2 z - z_prev.
#include <float.h>

#include <string>

#include "em_device.hpp"
#include "emx_internal.hpp"

namespace emx {

int blocks_per_cu(em_context *ctx, const void *fn, int threads);
int ctx_num_cus(em_context *ctx);
em_status_t ctx_error(em_context *ctx, em_status_t st, const std::string &msg);
em_status_t ctx_hip_error(em_context *ctx, hipError_t e, const char *what);
unsigned int *ctx_counters(em_context *ctx, int n);
em_status_t ctx_reset_counters(em_context *ctx, hipStream_t s, unsigned int *c, int n);
void *ctx_workspace(em_context *ctx, size_t bytes, em_status_t *st);
void *ctx_plain_workspace(em_context *ctx, size_t bytes, em_status_t *st);

// ------------------------------------------------------------------ classes

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

// Classify: counts per class; empty / malformed instances finished here.
__global__ void batch_classify_count(const em_instance_t *inst, int64_t B, float *z, em_stats_t *stats,
                                     unsigned int *counts) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const em_instance_t e = inst[b];
    if (e.n == 0 && e.d >= 1 && e.d <= EM_MAX_D) {
        if (stats) stats[b] = em_stats_t{0, EM_EMPTY, 0.0f, 0.0f};
        return;
    }
    if (e.n < 0 || e.n > EM_MAX_N || e.d < 1 || e.d > EM_MAX_D) {
        if (e.d >= 1 && e.d <= EM_MAX_D)
            for (int j = 0; j < e.d; ++j) z[e.z_off + j] = __builtin_nanf("");
        if (stats) stats[b] = em_stats_t{0, EM_BAD_INPUT, 0.0f, 0.0f};
        return;
    }
    atomicAdd(&counts[class_of(e.n, e.d)], 1u);
}

__global__ void batch_classify_scan(const unsigned int *counts, unsigned int *offsets) {
    if (threadIdx.x == 0) {
        unsigned int s = 0;
        for (int c = 0; c < kNumClasses; ++c) {
            offsets[c] = s;
            s += counts[c];
        }
        offsets[kNumClasses] = s;
    }
}

__global__ void batch_classify_scatter(const em_instance_t *inst, int64_t B, const unsigned int *offsets,
                                       unsigned int *fill, int32_t *list) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const em_instance_t e = inst[b];
    if (e.n <= 0 || e.n > EM_MAX_N || e.d < 1 || e.d > EM_MAX_D) return;
    const int c = class_of(e.n, e.d);
    const unsigned int k = atomicAdd(&fill[c], 1u);
    list[offsets[c] + k] = (int32_t)b;
}

// Kernel arguments of one class launch.
struct ClassLaunch {
    const float *a;
    const float *w;
    const em_instance_t *inst;
    const int32_t *list;
    const unsigned int *offsets;  // class offsets into list (kNumClasses + 1)
    unsigned int *counter;        // work-queue head of this class
    float *z;
    em_stats_t *stats;
    float lo, hi, mu, inv_mu, tol, arm;
    int32_t max_iter, init, cls;
};

template <int DS, int M, int WC, int WP>
struct BatchShape {
    static constexpr int THREADS = 64 * WC * WP;
    static constexpr int H2 = RS<DS>::H2;
    static constexpr int STAGE = 64 * 65 + 1;  // one 64-point chunk, odd pitch <= 65
};

template <int DS, int M, int WC, int WP>
__global__ __launch_bounds__(64 * WC * WP, 2) void batch_solve_kernel(ClassLaunch L) {
    using S = BatchShape<DS, M, WC, WP>;
    using RSx = RS<DS>;
    constexpr int H2 = S::H2;
    __shared__ float stage[S::STAGE];
    __shared__ float xn[(WC > 1) ? 2 * WC * WP * M * 64 : 1];
    __shared__ float xe[(WP > 1) ? 2 * WP * WC * H2 * 4 : 1];
    __shared__ float xs[2 * WC * WP * 4];
    __shared__ float zpE[WC * 2 * H2 * 4 * WP];
    __shared__ float cvec[WC * WP * DS];
    __shared__ unsigned int item_s;
    __shared__ int flag_s[4];

    const int lane = threadIdx.x & 63;
    const int row = lane >> 4;
    const int wave = uniform_int(threadIdx.x >> 6);
    const int cw = wave % WC, pw = wave / WC;
    float *zp_s = zpE + wave * 2 * H2 * 4;  // per wave: z^{t-1}, E^t in the reduced layout
    float *Ep_s = zp_s + H2 * 4;
    float *cv = cvec + wave * DS;           // per wave: c = 2 z^t - z^{t-1} of the slice
    const unsigned int cbeg = L.offsets[L.cls];
    const unsigned int ccount = L.offsets[L.cls + 1] - cbeg;

    for (;;) {
        if (threadIdx.x == 0) {
            item_s = atomicAdd(L.counter, 1u);
            flag_s[0] = 0;  // a point or weight is bad
            flag_s[1] = 0;  // max |a| (float bits, non-negative)
            flag_s[2] = 0;  // the starting z is bad
        }
        __syncthreads();
        const unsigned int it = (unsigned int)uniform_int((int)item_s);
        if (it >= ccount) break;
        const int b = uniform_int(L.list[cbeg + it]);
        const em_instance_t e = L.inst[b];
        const int n = uniform_int(e.n), d = uniform_int(e.d);
        const float *A = L.a + e.a_off;
        const float *Wt = L.w + e.w_off;
        float *Z = L.z + e.z_off;
        const int pitch = d | 1;

        // ---- stage points into registers (coalesced via LDS), check them
        float na[M][DS];
        float lam[M];
        bool bad_l = false;
        float amax = 0.0f;
#pragma unroll
        for (int q = 0; q < M; ++q) {
#pragma unroll
            for (int pc = 0; pc < WP; ++pc) {
                const int p0 = (pc * M + q) * 64;  // first point of this chunk
                const int cnt = max(0, min(64, n - p0));
                __syncthreads();
                for (int i = threadIdx.x; i < cnt * d; i += S::THREADS) {
                    const int pp = i / d, jj = i - (i / d) * d;
                    stage[pp * pitch + jj] = A[(int64_t)p0 * d + i];
                }
                __syncthreads();
                if (pc == pw) {
                    const int p = p0 + lane;
                    const bool vp = p < n;
#pragma unroll
                    for (int jj = 0; jj < DS; ++jj) {
                        const int j = cw * DS + jj;
                        const float v = (vp && j < d) ? stage[lane * pitch + j] : 0.0f;
                        bad_l |= !(fabsf(v) <= FLT_MAX);
                        amax = fmaxf(amax, fabsf(v));
                        na[q][jj] = -v;
                    }
                    const float wv = vp ? Wt[p] : 0.0f;
                    bad_l |= !(wv >= 0.0f && wv <= FLT_MAX);
                    lam[q] = vp ? wv : -1.0f;  // weight for now (-1: no point); lambda below
                }
            }
        }
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
        }
        __syncthreads();
        const bool bad = uniform(flag_s[0] != 0);
        const float Dscale = (__builtin_isfinite(L.lo) && __builtin_isfinite(L.hi) && L.hi > L.lo)
                                 ? (L.hi - L.lo)
                                 : fmaxf(1.0f, readfirstlane(__int_as_float(flag_s[1])));
        const float tau = L.tol * Dscale;
        const float tau2 = tau * tau;
        const float arm2 = (L.arm * tau) * (L.arm * tau);

        // ---- starting z in the reduced layout; c = z
        float zr[H2];
        bool zbad = false;
#pragma unroll
        for (int j = 0; j < H2; ++j) {
            const int cc = cw * DS + RSx::coord(row, j);
            const bool vj = RSx::valid(row, j) && cc < d;
            float zv = 0.0f;
            if (vj) zv = (L.init == EM_INIT_MAXW) ? A[(int64_t)best * d + cc] : Z[cc];
            zbad |= vj && !(fabsf(zv) <= FLT_MAX);
            zr[j] = zv;
            if (lane == 16 * row) {
                zp_s[j * 4 + row] = zv;
                Ep_s[j * 4 + row] = 0.0f;
                if (RSx::valid(row, j)) cv[RSx::coord(row, j)] = zv;  // 0 on padded coordinates
            }
        }
        if (__any(zbad) && lane == 0) flag_s[2] = 1;
        __syncthreads();
        const bool bad_all = uniform(bad || (flag_s[2] != 0));
        __syncthreads();  // flags are reset by the next pop

        int iters = 0, flags = EM_MAXITER;
        float rp2 = 0.0f, rd2 = 0.0f;
        if (bad_all) {
            flags = EM_BAD_INPUT;
        } else {
            float g[M][DS];
#pragma unroll
            for (int q = 0; q < M; ++q) {
                lam[q] = (lam[q] >= 0.0f) ? lam[q] * L.inv_mu : 0.0f;
#pragma unroll
                for (int jj = 0; jj < DS; ++jj) g[q][jj] = na[q][jj];
            }
            const float inv_n = 1.0f / (float)n;
            const float fn = (float)n;
            const float inv_d = 1.0f / (float)d;
            const float inv_nd = 1.0f / ((float)n * (float)d);
            const int max_iter = L.max_iter;
            float rd_w = 0.0f, rp_w = 0.0f;
            bool armed_last = false, done = false;
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
                        g[q][jj] += cj;
                        nrm[q] = fmaf(g[q][jj], g[q][jj], nrm[q]);
                    }
                }
                float rd_all = rd_w, rp_all = rp_w;
                if constexpr (WC > 1 || WP > 1) {
                    float *XS = xs + (t & 1) * WC * WP * 4;
                    if constexpr (WC > 1) {
                        float *X = xn + (t & 1) * WC * WP * M * 64;
#pragma unroll
                        for (int q = 0; q < M; ++q) X[((pw * WC + cw) * M + q) * 64 + lane] = nrm[q];
                    }
                    if (lane == 0) {
                        XS[wave * 4 + 0] = rd_w;
                        XS[wave * 4 + 1] = rp_w;
                    }
                    __syncthreads();
                    if constexpr (WC > 1) {
                        float *X = xn + (t & 1) * WC * WP * M * 64;
#pragma unroll
                        for (int q = 0; q < M; ++q) {
                            float sum = X[(pw * WC * M + q) * 64 + lane];
#pragma unroll
                            for (int v = 1; v < WC; ++v) sum += X[((pw * WC + v) * M + q) * 64 + lane];
                            nrm[q] = sum;
                        }
                    }
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
                // ---- stop test for iteration t-1 (all waves hold identical sums)
                if (t > 1) {
                    rd2 = rd_all * inv_d;
                    rp2 = fmaxf(rp_all, 0.0f) * inv_nd;
                    if (uniform(tau2 > 0.0f && armed_last && rp2 <= tau2 && rd2 <= tau2)) {
                        flags = EM_CONVERGED;
                        iters = t - 1;
                        done = true;
                        break;
                    }
                }
                const bool armed = uniform((t == max_iter) || (tau2 > 0.0f && t > 1 && rd2 <= arm2));
                float s[M];
#pragma unroll
                for (int q = 0; q < M; ++q) s[q] = shrink(nrm[q], lam[q]);
                // ---- armed iterations: lane sums of ||x_k - c||^2, x_k = a_k + (1 - s) delta.
                // Absent points and padded coordinates give exactly 0 (g stays -a).
                float rp_lane = 0.0f;
                if (armed) {
                    float rq[M];
#pragma unroll
                    for (int q = 0; q < M; ++q) rq[q] = 0.0f;
#pragma unroll
                    for (int jj = 0; jj < DS; ++jj) {
                        const float cj = cv[jj];
#pragma unroll
                        for (int q = 0; q < M; ++q) {
                            const float y = fmaf(1.0f - s[q], g[q][jj], -(na[q][jj] + cj));
                            rq[q] = fmaf(y, y, rq[q]);
                        }
                    }
#pragma unroll
                    for (int q = 0; q < M; ++q) rp_lane += rq[q];
                }
                // ---- pass 2: E = sum_k s delta, g = s delta - a
                float acc[DS];
#pragma unroll
                for (int jj = 0; jj < DS; ++jj) {
                    float ac = 0.0f;
#pragma unroll
                    for (int q = 0; q < M; ++q) {
                        const float dl = g[q][jj];
                        ac = fmaf(s[q], dl, ac);
                        g[q][jj] = fmaf(s[q], dl, na[q][jj]);
                    }
                    acc[jj] = ac;
                }
#pragma unroll
                for (int q = 0; q < M; ++q)
#pragma unroll
                    for (int jj = 0; jj < DS; ++jj) asm volatile("" : "+v"(g[q][jj]));
                float E[H2];
                reduce_scatter<DS>(acc, E);
                if constexpr (WP > 1) {
                    float *XE = xe + (t & 1) * WP * WC * H2 * 4;
                    if (lane == 16 * row) {
#pragma unroll
                        for (int j = 0; j < H2; ++j) XE[((pw * WC + cw) * H2 + j) * 4 + row] = E[j];
                    }
                    __syncthreads();
#pragma unroll
                    for (int j = 0; j < H2; ++j) {
                        float sum = 0.0f;
#pragma unroll
                        for (int v = 0; v < WP; ++v) sum += XE[((v * WC + cw) * H2 + j) * 4 + row];
                        E[j] = sum;
                    }
                }
                float rdx = 0.0f, rpx = 0.0f;
#pragma unroll
                for (int j = 0; j < H2; ++j) {
                    const int cc = cw * DS + RSx::coord(row, j);
                    const bool vj = RSx::valid(row, j) && cc < d;
                    const float zn = clampf(zr[j] - E[j] * inv_n, L.lo, L.hi);
                    const float dz = zn - zr[j];
                    const float zpj = zp_s[j * 4 + row];
                    if (armed) {
                        // x_k - z' = (x_k - c) + (c - z'), sum_k (x_k - c) = E^t - E^{t+1}
                        const float Epj = Ep_s[j * 4 + row];
                        const float cz = (2.0f * zr[j] - zpj) - zn;
                        rpx += vj ? (cz * (2.0f * (Epj - E[j]) + fn * cz)) : 0.0f;
                    }
                    rdx += vj ? dz * dz : 0.0f;
                    if (lane == 16 * row) {
                        zp_s[j * 4 + row] = zr[j];
                        Ep_s[j * 4 + row] = E[j];
                        if (RSx::valid(row, j)) cv[RSx::coord(row, j)] = vj ? (2.0f * zn - zr[j]) : 0.0f;
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
                } else {
                    rp_w = 0.0f;
                }
                armed_last = armed;
            }
            if (!done) {
                iters = max_iter;
                if (max_iter >= 1) {
                    float rd_all = rd_w, rp_all = rp_w;
                    if constexpr (WC > 1 || WP > 1) {
                        float *XS = xs + (t & 1) * WC * WP * 4;
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
                    flags = (tau2 > 0.0f && rp2 <= tau2 && rd2 <= tau2) ? EM_CONVERGED : EM_MAXITER;
                }
            }
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
            st.r_pri = bad_all ? 0.0f : sqrtf(rp2);
            st.r_dual = bad_all ? 0.0f : sqrtf(rd2);
            L.stats[b] = st;
        }
    }
}

struct ClassKernel {
    const void *fn;
    int threads;
};

template <int C>
constexpr ClassKernel class_kernel() {
    constexpr ClassShape s = class_shape(C);
    return ClassKernel{reinterpret_cast<const void *>(&batch_solve_kernel<s.ds, s.m, s.wc, s.wp>),
                       64 * s.wc * s.wp};
}

static const ClassKernel *class_table() {
    static const ClassKernel t[kNumClasses] = {
        class_kernel<0>(),  class_kernel<1>(),  class_kernel<2>(),  class_kernel<3>(),
        class_kernel<4>(),  class_kernel<5>(),  class_kernel<6>(),  class_kernel<7>(),
        class_kernel<8>(),  class_kernel<9>(),  class_kernel<10>(), class_kernel<11>(),
        class_kernel<12>(), class_kernel<13>(), class_kernel<14>(), class_kernel<15>(),
        class_kernel<16>(), class_kernel<17>(), class_kernel<18>(), class_kernel<19>(),
    };
    return t;
}

em_status_t batch_solve(em_context *ctx, hipStream_t s, int64_t B, const float *a, const float *w,
                        const em_instance_t *inst, float lo, float hi, float rho, int32_t max_iter,
                        float tol, int32_t init, float *z, em_stats_t *stats) {
    // workspace: list[B] int32
    em_status_t st;
    int32_t *list = static_cast<int32_t *>(ctx_workspace(ctx, (size_t)B * sizeof(int32_t), &st));
    if (!list) return st;
    // counters: [0, K) class counts, [K, 2K+1) offsets, [2K+1, 3K+1) fill, [3K+1, 4K+1) queue heads
    unsigned int *cnt = ctx_counters(ctx, 4 * kNumClasses + 1);
    if (!cnt) return ctx_error(ctx, EM_ERR_UNSUPPORTED, "counter pool too small");
    unsigned int *counts = cnt, *offsets = cnt + kNumClasses, *fill = cnt + 2 * kNumClasses + 1,
                 *heads = cnt + 3 * kNumClasses + 1;
    st = ctx_reset_counters(ctx, s, cnt, 4 * kNumClasses + 1);
    if (st != EM_OK) return st;
    const unsigned nb = (unsigned)((B + 255) / 256);
    hipLaunchKernelGGL(batch_classify_count, dim3(nb), dim3(256), 0, s, inst, B, z, stats, counts);
    hipLaunchKernelGGL(batch_classify_scan, dim3(1), dim3(64), 0, s, counts, offsets);
    hipLaunchKernelGGL(batch_classify_scatter, dim3(nb), dim3(256), 0, s, inst, B, offsets, fill, list);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return ctx_hip_error(ctx, e, "classify launch");
    const ClassKernel *tab = class_table();
    for (int c = 0; c < kNumClasses; ++c) {
        ClassLaunch L;
        L.a = a;
        L.w = w;
        L.inst = inst;
        L.list = list;
        L.offsets = offsets;
        L.counter = heads + c;
        L.z = z;
        L.stats = stats;
        L.lo = lo;
        L.hi = hi;
        L.mu = rho;
        L.inv_mu = 1.0f / rho;
        L.tol = tol;
        L.arm = 1.0f;  // primal residual evaluated after an iteration with r_dual <= tol D
        L.max_iter = max_iter;
        L.init = init;
        L.cls = c;
        const int64_t cap = (int64_t)ctx_num_cus(ctx) * blocks_per_cu(ctx, tab[c].fn, tab[c].threads);
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(B, cap));
        void *args[] = {&L};
        e = hipLaunchKernel(tab[c].fn, dim3(grid), dim3(tab[c].threads), args, 0, s);
        if (e != hipSuccess) return ctx_hip_error(ctx, e, "batch class launch");
    }
    return EM_OK;
}

// ------------------------------------------------------------------ plain

// One instance per launch, literal Algorithm 1 with the iterates in device
// memory: thread per point for the prox, thread per coordinate for the
// z-update, thread per point for the multiplier update, residuals every
// iteration.  The simple baseline for the batched solver.
struct PlainArgs {
    const float *a;
    const float *w;
    const em_instance_t *inst;
    float *z;
    em_stats_t *stats;
    float *u;  // n*d scaled multipliers y/mu
    float *x;  // n*d local variables
    float lo, hi, mu, tol;
    int32_t max_iter, init;
    int64_t b;
};

__global__ __launch_bounds__(256) void plain_solve_kernel(PlainArgs P) {
    __shared__ float zs[EM_MAX_D], zprev[EM_MAX_D];
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
    if (flag == 0 && tid == 0) {
        int best = 0;
        if (P.init == EM_INIT_MAXW)
            for (int k = 1; k < n; ++k)
                if (Wt[k] > Wt[best]) best = k;
        for (int j = 0; j < d; ++j) {
            zs[j] = (P.init == EM_INIT_MAXW) ? A[best * d + j] : Z[j];
            if (!(fabsf(zs[j]) <= FLT_MAX)) flag = 1;
        }
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
    const float Dscale = (__builtin_isfinite(P.lo) && __builtin_isfinite(P.hi) && P.hi > P.lo)
                             ? (P.hi - P.lo) : fmaxf(1.0f, amax_s);
    const float tau = P.tol * Dscale;
    for (int i = tid; i < n * d; i += 256) P.u[i] = 0.0f;
    __syncthreads();
    int iters = 0, flags = EM_MAXITER;
    float rpri = 0.0f, rdual = 0.0f;
    for (int t = 1; t <= P.max_iter; ++t) {
        // x_k = prox_{w_k/mu}(z - u_k, a_k)
        for (int k = tid; k < n; k += 256) {
            const float lam = Wt[k] / P.mu;
            float nu2 = 0.0f;
            for (int j = 0; j < d; ++j) {
                const float dl = zs[j] - P.u[k * d + j] - A[k * d + j];
                nu2 = fmaf(dl, dl, nu2);
            }
            const float nu = sqrtf(nu2);
            const float sh = (nu <= lam) ? 1.0f : lam / nu;
            for (int j = 0; j < d; ++j) {
                const float v = zs[j] - P.u[k * d + j];
                P.x[k * d + j] = v - sh * (v - A[k * d + j]);
            }
        }
        __syncthreads();
        // z = P_C(mean_k(x_k + u_k))
        for (int j = tid; j < d; j += 256) {
            float r = 0.0f;
            for (int k = 0; k < n; ++k) r += P.x[k * d + j] + P.u[k * d + j];
            zprev[j] = zs[j];
            zs[j] = clampf(r / (float)n, P.lo, P.hi);
        }
        __syncthreads();
        // u_k += x_k - z, primal residual
        float rp = 0.0f;
        for (int i = tid; i < n * d; i += 256) {
            const float dlt = P.x[i] - zs[i % d];
            P.u[i] += dlt;
            rp = fmaf(dlt, dlt, rp);
        }
        red[tid] = rp;
        __syncthreads();
        for (int s2 = 128; s2 > 0; s2 >>= 1) {
            if (tid < s2) red[tid] += red[tid + s2];
            __syncthreads();
        }
        float rd = 0.0f;
        for (int j = 0; j < d; ++j) rd += (zs[j] - zprev[j]) * (zs[j] - zprev[j]);
        rpri = sqrtf(red[0] / ((float)n * (float)d));
        rdual = sqrtf(rd / (float)d);
        iters = t;
        __syncthreads();
        if (tau > 0.0f && rpri <= tau && rdual <= tau) {
            flags = EM_CONVERGED;
            break;
        }
    }
    if (tid < d) Z[tid] = zs[tid];
    if (tid == 0 && P.stats) P.stats[P.b] = em_stats_t{iters, flags, rpri, rdual};
}

em_status_t plain_solve(em_context *ctx, hipStream_t s, int64_t B, const float *a, const float *w,
                        const em_instance_t *inst, const em_instance_t *inst_host, float lo, float hi,
                        float rho, int32_t max_iter, float tol, int32_t init, float *z, em_stats_t *stats) {
    int64_t maxnd = 1;
    for (int64_t b = 0; b < B; ++b) {
        const int64_t n = inst_host[b].n, d = inst_host[b].d;
        if (n > 0 && n <= EM_MAX_N && d >= 1 && d <= EM_MAX_D) maxnd = std::max(maxnd, n * d);
    }
    em_status_t st;
    float *ws = static_cast<float *>(ctx_plain_workspace(ctx, (size_t)(2 * maxnd) * sizeof(float), &st));
    if (!ws) return st;
    PlainArgs P;
    P.a = a;
    P.w = w;
    P.inst = inst;
    P.z = z;
    P.stats = stats;
    P.u = ws;
    P.x = ws + maxnd;
    P.lo = lo;
    P.hi = hi;
    P.mu = rho;
    P.tol = tol;
    P.max_iter = max_iter;
    P.init = init;
    for (int64_t b = 0; b < B; ++b) {
        P.b = b;
        hipLaunchKernelGGL(plain_solve_kernel, dim3(1), dim3(256), 0, s, P);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return ctx_hip_error(ctx, e, "plain launch");
    return EM_OK;
}

}  // namespace emx
