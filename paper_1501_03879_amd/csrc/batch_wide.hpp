// Batched EM-ADMM (Algorithm 1 of arXiv:1501.03879) for point sets of
// d in (16, 64] and n <= 448 with a fixed penalty over a box: one workgroup
// of WC waves per instance, the instance's coordinates cut into slices of NJ
// (wave cw owns coordinates [cw NJ, cw NJ + NJ)), its points into M per lane
// (lane l owns points l + 64 q, q < M).  Slices and point slots are sized to
// the instance (d = 49: 4 x 13 coordinates, n = 441: 7 x 64 slots), so the
// points and the iteration state fill the registers of four waves and two
// instances share a CU.
//
//  * Staging: 64 points at a time go through LDS (one row of d values per
//    load, coalesced; a chunk's loads all issued at once and the next
//    chunk's in flight while this one is read back), every lane then takes
//    its slice of its point.
//  * Iteration (same iterates as Algorithm 1; see the NLEM kernel for the
//    reduced form): with g = e - a per point coordinate and c = 2 z^t -
//    z^{t-1},
//      pass 1:  delta = g + c,  partial ||delta||^2 over the slice
//      the WC partials summed through LDS, s = min(1, lambda / nu)
//      pass 2:  E += s delta,  g = s delta - a
//      a full 64-lane reduce-scatter leaves E of one slice coordinate per
//      lane; that lane updates z = clamp(z - E / n, lo_j, hi_j) and hands
//      c to the wave through LDS.
//  * Stop: primal and dual residuals <= tol D, the primal one evaluated on
//    iterations after one whose dual residual was within tol D (and on the
//    last allowed one) and tested right after them.
#pragma once

#include <float.h>
#include <hip/hip_fp16.h>

#include "batch_kernel.hpp"

namespace emx {

template <int NJ, int M, int WC>
struct WideShape {
    static constexpr int THREADS = 64 * WC;
    static constexpr int STAGE = 64 * 65;       // 64 points x pitch (d | 1) <= 65
    static constexpr int XN = 2 * WC * M * 64;  // norm partials, two buffers by iteration parity
};

// Stage one instance's points (FP32 or FP16 storage, T) into registers: the
// workgroup's waves load whole rows of d values (wave cw rows cw + WC k of
// each 64-point chunk, one value per lane, coalesced), the loads of up to LA
// chunks in flight at once (all of them for WC >= 4), the next chunk issued
// as soon as one has been read back; chunk by chunk the rows go through LDS
// and every lane keeps its slice of its point as -a.  Rows past the instance
// read 0 (no branches, so nothing waits early); they are staged but never
// read back.
template <int NJ, int M, int WC, typename T>
__device__ __forceinline__ void stage_points(const T *A, int n, int d, int cw, int lane, int j0, float *stage,
                                             float (&na)[M][NJ], float &amax, bool &bad) {
    const int pitch = d | 1;
    if constexpr (WC == 1 && NJ <= 16) {
        // one wave and d <= NJ: a chunk's 64 d values are contiguous, so copy
        // them flat (element i = lane + 64 k, row i / d by a float reciprocal,
        // exact for i < 2^22) rather than one row of d <= 16 values per load
        const float inv_d = 1.0f / (float)d;
#pragma unroll
        for (int q = 0; q < M; ++q) {
            if (q > 0) __syncthreads();
            const int cnt = min(64, max(0, n - q * 64)) * d;   // values in the chunk
            T raw[NJ];
#pragma unroll
            for (int k = 0; k < NJ; ++k) {
                const int i = lane + 64 * k;
                raw[k] = A[(i < cnt) ? q * 64 * d + i : 0];
            }
#pragma unroll
            for (int k = 0; k < NJ; ++k) {
                const int i = lane + 64 * k;
                const int r = (int)(((float)i + 0.5f) * inv_d);
                if (i < cnt) stage[r * pitch + (i - r * d)] = (float)raw[k];
            }
            __syncthreads();
            const bool vp = q * 64 + lane < n;
#pragma unroll
            for (int jj = 0; jj < NJ; ++jj) {
                const int j = j0 + jj;
                const float v = (vp && j < d) ? stage[lane * pitch + j] : 0.0f;
                bad |= !(fabsf(v) <= FLT_MAX);
                amax = fmaxf(amax, fabsf(v));
                na[q][jj] = -v;
            }
        }
        return;
    }
    constexpr int RK = (64 + WC - 1) / WC;                 // rows per wave and chunk
    constexpr int LA0 = 112 / RK;                          // ~112 VGPRs of loads in flight
    constexpr int LA = LA0 < 1 ? 1 : (LA0 > M ? M : LA0);
    // One buffer load per row, range-checked against the instance: a row
    // costs one vector add for its offset, rows past the instance (and the
    // lanes past d of its last row) read 0, and lanes past d of the other
    // rows read values of the next row, which are not staged.
    constexpr int TB = (int)sizeof(T);
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(A), (short)0, n * d * TB, kBufferRsrcWord3);
    const int voff = lane * TB;
    T raw[LA][RK];
    auto issue = [&](int q) {
#pragma unroll
        for (int k = 0; k < RK; ++k) {
            const int off = voff + (q * 64 + cw + WC * k) * d * TB;
            if constexpr (TB == 4)
                raw[q % LA][k] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
            else
                raw[q % LA][k] = __ushort_as_half(__builtin_amdgcn_raw_buffer_load_b16(rs, off, 0, 0));
        }
    };
#pragma unroll
    for (int q = 0; q < LA; ++q) issue(q);
#pragma unroll
    for (int q = 0; q < M; ++q) {
        if (q > 0) __syncthreads();   // the previous chunk has been read back
#pragma unroll
        for (int k = 0; k < RK; ++k) {
            const int r = cw + WC * k;
            if (r < 64 && lane < d) stage[r * pitch + lane] = (float)raw[q % LA][k];
        }
        if (q + LA < M) issue(q + LA);
        __syncthreads();
        // (rows past the instance were staged as 0, so only coordinates past
        // d are masked; a NaN is caught by unordered compares of pairs, an
        // infinity by the running maximum, checked by the caller)
#pragma unroll
        for (int jj = 0; jj < NJ; jj += 2) {
            const int j = j0 + jj;
            const float v0 = (j < d) ? stage[lane * pitch + j] : 0.0f;
            const float v1 = (jj + 1 < NJ && j + 1 < d) ? stage[lane * pitch + j + 1] : 0.0f;
            bad |= __builtin_isunordered(v0, v1);
            amax = fmaxf(amax, fmaxf(fabsf(v0), fabsf(v1)));
            na[q][jj] = -v0;
            if (jj + 1 < NJ) na[q][jj + 1] = -v1;
        }
    }
}

// Per-instance set-up shared by the sliced kernels, between the queue pop and
// the solve: the weights (lam; -1 on empty slots), the lane's slices of its
// points as -a (na), the starting z and the bounds of the lane's coordinate,
// the checks that make an instance BAD_INPUT, and the tolerance scale D
// (flag_s cleared by the pop).  The starting z goes to the wave's broadcast
// slot cv[cidx] (slots of coordinates >= d get 0).
struct WideStart {
    float zr, blo, bhi;      // the owned coordinate's z^0 and bounds
    bool bad_all;            // the instance is BAD_INPUT
    float Dscale, amax_all;  // tolerance scale D and the largest |a|
};

template <int NJ, int M, int WC>
__device__ __forceinline__ WideStart wide_start(const ClassLaunch &L, const em_instance_t &e, int n, int d, int cw,
                                                int lane, bool holds, bool own, int j0, int cj, float *stage,
                                                int *flag_s, float *cv, int cidx, float (&lam)[M],
                                                float (&na)[M][NJ]) {
    const float *A = L.a + e.a_off;
    const __half *A16 = reinterpret_cast<const __half *>(L.a) + e.a_off;
    const float *Wt = L.w + e.w_off;
    const float *Z = L.z + e.z_off;
    const bool vbox = L.box_lo != nullptr;
    // ---- weights of the lane's points, and (largest-weight start) the
    // chosen point, before the points: their loads overlap the staging
    bool bad_l = false;
#pragma unroll
    for (int q = 0; q < M; ++q) {
        // unconditional loads (slots past n read weight 0, then drop it):
        // no branch, so all of them are in flight together
        const int p = q * 64 + lane;
        const float wr = Wt[min(p, n - 1)];
        const float wv = (p < n) ? wr : 0.0f;
        bad_l |= !(wv >= 0.0f && wv <= FLT_MAX);
        lam[q] = (p < n) ? wv : -1.0f;   // the weight for now (-1: no point)
    }
    float zr = 0.0f;
    if (L.init == EM_INIT_MAXW) {
        // the point of largest weight, lowest index on ties (every wave
        // holds all the weights, so no exchange is needed)
        float wb = -1.0f;
        int pb = 0x7fffffff;
#pragma unroll
        for (int q = 0; q < M; ++q)
            if (lam[q] > wb) wb = lam[q], pb = q * 64 + lane;
        const float wm = wave_max(wb);
        const float cand = (wb == wm) ? (float)pb : 3.0e38f;
        // (no weight >= 0 at all leaves no candidate: the instance is bad
        // and the clamp only keeps the read inside it)
        const int best = min(uniform_int((int)(-wave_max(-cand))), n - 1);
        if (own) zr = L.a16 ? __half2float(A16[(int64_t)best * d + cj]) : A[(int64_t)best * d + cj];
    } else if (L.init == EM_INIT_GIVEN) {
        if (own) zr = Z[cj];
    }
    float blo = L.lo, bhi = L.hi;
    if (own && vbox) {
        blo = L.box_lo[e.z_off + cj];
        bhi = L.box_hi[e.z_off + cj];
    }

    // ---- stage the points, 64 at a time through LDS: wave w copies rows
    // w, w + WC, ... of a chunk (one row of d values per load, all of a
    // chunk's loads issued together, the next chunk's loads in flight
    // while this one is read back); every lane then keeps its slice of
    // its point as -a
    float amax = 0.0f;
    if (L.a16)
        stage_points<NJ, M, WC>(A16, n, d, cw, lane, j0, stage, na, amax, bad_l);
    else
        stage_points<NJ, M, WC>(A, n, d, cw, lane, j0, stage, na, amax, bad_l);
    bad_l |= !(amax <= FLT_MAX);   // an infinite point (NaN ones are flagged already)
    const float wamax = wave_max(amax);
    if (__any(bad_l) && lane == 0) flag_s[0] = 1;
    if (lane == 0) atomicMax(&flag_s[1], __float_as_int(wamax));   // non-negative floats order as ints

    if (L.init == EM_INIT_WMEAN) {
        // sum_k w_k a_k / sum_k w_k, weights scaled by their largest value and
        // points by 1/n (no overflow); every weight zero: equal weights
        float wl = 0.0f;
#pragma unroll
        for (int q = 0; q < M; ++q) wl = fmaxf(wl, lam[q]);
        const float wmx = readfirstlane(wave_max(wl));
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
        float acc[NJ];
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) {
            float ac = 0.0f;
#pragma unroll
            for (int q = 0; q < M; ++q) ac = fmaf(-cq[q], na[q][jj], ac);   // na = -a
            acc[jj] = ac;
        }
        const float sum = reduce_scatter_full<NJ>(acc, lane, holds);
        const float Cs = readfirstlane(wave_sum(cs));
        if (own) zr = sum * (1.0f / Cs);
    }
    bool zbad = false;
    float wid = 0.0f;
    if (own) {
        zbad = !(fabsf(zr) <= FLT_MAX) || !(blo <= bhi);
        wid = bhi - blo;
        if (!(wid >= 0.0f)) wid = 0.0f;
    }
    const float wwid = wave_max(wid);
    if (__any(zbad) && lane == 0) flag_s[2] = 1;
    if (lane == 0) atomicMax(&flag_s[3], __float_as_int(wwid));
    cv[cidx] = zr;
    __syncthreads();
    WideStart r;
    r.zr = zr;
    r.blo = blo;
    r.bhi = bhi;
    r.bad_all = uniform(flag_s[0] != 0 || flag_s[2] != 0);
    const float wmax = readfirstlane(__int_as_float(flag_s[3]));
    r.amax_all = readfirstlane(__int_as_float(flag_s[1]));
    r.Dscale = (wmax <= FLT_MAX && wmax > 0.0f) ? wmax : fmaxf(1.0f, r.amax_all);
    return r;
}

// ES: carry the prox displacement e itself instead of g = e - a (as the
// generic kernel's SOLVER 5 for deferred far-outlier instances, see
// ClassLaunch): delta = (e + c) - a in both passes and x_k - c = e - s delta
// on armed iterations, 7 operations per point coordinate instead of 4,
// without the floor that a large |a| puts under the primal residual computed
// from g.  The class kernels use ES = false and defer such instances.
template <int NJ, int M, int WC, int WAVES_PER_SIMD, bool ES = false>
__global__ __launch_bounds__(64 * WC, WAVES_PER_SIMD) void batch_wide_kernel(ClassLaunch L) {
    using S = WideShape<NJ, M, WC>;
    using RSx = RSF<NJ>;
    __shared__ float stage[S::STAGE];
    __shared__ float xn[S::XN];
    __shared__ float sv[M * 64];       // shrink factors of the points, from the wave that took them
    // per-wave residual partials (two buffers + the armed test), then the
    // squared z steps of the owned coordinates by iteration parity
    __shared__ float xs[3 * WC * 4 + 128];
    float *dz2s = xs + 3 * WC * 4;
    __shared__ float cvec[WC * 128];   // per wave: c of the slice [0, NJ); private slots [64, 128)
    __shared__ unsigned int item_s;
    __shared__ int flag_s[4];

    const int lane = threadIdx.x & 63;
    const int cw = uniform_int(threadIdx.x >> 6);
    const bool holds = (RSx::mask() >> lane) & 1;   // lane holds a slice coordinate after the reduce-scatter
    const int myc = RSx::coord(lane);
    float *cv = cvec + cw * 128;
    const int cidx = holds ? myc : 64 + lane;
    // one instance per launch (L.single >= 0: the plain path) or the class's
    // work queue
    const bool one = L.single >= 0;
    const unsigned int cbeg = one ? 0u : L.offsets[L.cls];
    const unsigned int ccount = one ? 1u : L.offsets[L.cls + 1] - cbeg;
    // workgroups beyond the class's instance count would only find the queue
    // empty: they leave before the atomic, so an empty class costs its dispatch
    if (blockIdx.x >= ccount) return;
    unsigned int taken = 0;   // thread 0, single-instance mode: instances taken

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
        float *Z = L.z + e.z_off;
        const int j0 = cw * NJ;                  // first coordinate of the slice
        const int cj = j0 + myc;                 // the coordinate this lane owns after the reduce-scatter
        const bool own = holds && cj < d;

        float lam[M];
        float na[M][NJ];
        const WideStart st0 = wide_start<NJ, M, WC>(L, e, n, d, cw, lane, holds, own, j0, cj, stage, flag_s, cv,
                                                    cidx, lam, na);
        float zr = st0.zr;
        const float blo = st0.blo, bhi = st0.bhi;
        const bool bad_all = st0.bad_all;
        const float amax_all = st0.amax_all, Dscale = st0.Dscale;
        const float tau = L.tol * Dscale;
        const float tau2 = tau * tau;
        const float arm2 = (L.arm * tau) * (L.arm * tau);
        __syncthreads();   // flags are reset by the next pop
        if constexpr (!ES) {
            if (L.defer_q != nullptr && !bad_all &&
                uniform(amax_all > L.outlier * Dscale * sqrtf((float)n))) {
                if (threadIdx.x == 0) defer_instance(L, b, n, d);
                continue;
            }
        }

        int iters = 0, flags = EM_MAXITER;
        float rp2 = 0.0f, rd2 = 0.0f;
        if (bad_all) {
            flags = EM_BAD_INPUT;
        } else {
            const float inv_mu = 1.0f / L.mu;
#pragma unroll
            for (int q = 0; q < M; ++q) lam[q] = (lam[q] >= 0.0f) ? lam[q] * inv_mu : 0.0f;
            // wave cw takes the shrink factors of the lane's points [cw QS,
            // min((cw + 1) QS, M)): their lambdas, picked once per instance
            constexpr int QS = (M + WC - 1) / WC;
            float lq[QS];
#pragma unroll
            for (int qq = 0; qq < QS; ++qq) {
                float v = 0.0f;
#pragma unroll
                for (int q = 0; q < M; ++q) v = (q == cw * QS + qq) ? lam[q] : v;
                lq[qq] = v;
            }
            float g[M][NJ];
#pragma unroll
            for (int q = 0; q < M; ++q)
#pragma unroll
                for (int jj = 0; jj < NJ; ++jj) g[q][jj] = ES ? 0.0f : na[q][jj];
            const float inv_n = 1.0f / (float)n;
            const float fn = (float)n;
            const float inv_d = 1.0f / (float)d;
            const float inv_nd = 1.0f / (fn * (float)d);
            const int max_iter = L.max_iter;
            float zp = zr;      // z^{t-1}
            float Ep = 0.0f;    // E^t
            float rd_w = 0.0f, rp_w = 0.0f;
            bool done = false;
            for (int t = 1; t <= max_iter; ++t) {
                // ---- pass 1: delta = g + c, partial ||delta||^2
                float nrm[M];
#pragma unroll
                for (int q = 0; q < M; ++q) nrm[q] = kNu2Floor;
#pragma unroll
                for (int jj = 0; jj < NJ; ++jj) {
                    const float c = cv[jj];
#pragma unroll
                    for (int q = 0; q < M; ++q) {
                        if constexpr (ES) {
                            const float dl = (g[q][jj] + c) + na[q][jj];
                            nrm[q] = fmaf(dl, dl, nrm[q]);
                        } else {
                            g[q][jj] += c;
                            nrm[q] = fmaf(g[q][jj], g[q][jj], nrm[q]);
                        }
                    }
                }
                if constexpr (ES) {   // pass 2 recomputes delta (do not hold it across the exchange)
#pragma unroll
                    for (int q = 0; q < M; ++q)
#pragma unroll
                        for (int jj = 0; jj < NJ; ++jj) asm volatile("" : "+v"(g[q][jj]));
                }
                // ---- the slices' partials summed (in wave order, identical in
                // every wave), with the dual residual of iteration t-1
                bool arm_ok = false;
                float s[M];
                {
                    // wave cw adds up the partials of its share of the points
                    // (in wave order, as every wave would), takes their
                    // shrink factors and hands them to the other waves
                    // through LDS; the last wave also sums the squared z steps
                    // of iteration t-1 the coordinate owners left there
                    float *X = xn + (t & 1) * WC * M * 64;
                    float *XS = xs + (t & 1) * WC * 4;
#pragma unroll
                    for (int q = 0; q < M; ++q) X[(cw * M + q) * 64 + lane] = nrm[q];
                    __syncthreads();
                    if (cw == WC - 1 && t > 1) {
                        const float q2 = (lane < d) ? dz2s[((t - 1) & 1) * 64 + lane] : 0.0f;
                        const float tot = wave_sum(q2);
                        // (only the arming test needs it: the flag goes over)
                        if (lane == 0) reinterpret_cast<int *>(XS)[cw * 4 + 3] = (tot * inv_d <= arm2) ? 1 : 0;
                    }
#pragma unroll
                    for (int qq = 0; qq < QS; ++qq) {
                        const int q = cw * QS + qq;
                        if (q < M) {
                            float sum = X[q * 64 + lane];
#pragma unroll
                            for (int w = 1; w < WC; ++w) sum += X[(w * M + q) * 64 + lane];
                            sv[q * 64 + lane] = shrink(sum, lq[qq]);
                        }
                    }
                    __syncthreads();
#pragma unroll
                    for (int q = 0; q < M; ++q) s[q] = sv[q * 64 + lane];
                    if (t > 1) arm_ok = uniform_int(reinterpret_cast<const int *>(XS)[(WC - 1) * 4 + 3]) != 0;
                }
                // the dual residual of iteration t-1 (tested by the last
                // wave) arms the primal residual of this iteration
                const bool armed = (t == max_iter) || (tau2 > 0.0f && t > 1 && arm_ok && (t & L.check_mask) == 0);
                // ---- armed iterations: lane sums of ||x_k - c||^2 with
                // x_k = a_k + (1 - s) delta (absent points and padded
                // coordinates give exactly 0)
                float rp_lane = 0.0f;
                if (!ES && armed) {
                    float rq[M];
#pragma unroll
                    for (int q = 0; q < M; ++q) rq[q] = 0.0f;
#pragma unroll
                    for (int jj = 0; jj < NJ; ++jj) {
                        const float c = cv[jj];
#pragma unroll
                        for (int q = 0; q < M; ++q) {
                            const float y = fmaf(1.0f - s[q], g[q][jj], -(na[q][jj] + c));
                            rq[q] = fmaf(y, y, rq[q]);
                        }
                    }
#pragma unroll
                    for (int q = 0; q < M; ++q) rp_lane += rq[q];
                }
                // ---- pass 2: E = sum_k s delta, g = s delta - a (ES: delta again,
                // e = s delta, armed: lane sums of ||e - s delta||^2)
                float acc[NJ];
                if constexpr (ES) {
                    float rq[M];
#pragma unroll
                    for (int q = 0; q < M; ++q) rq[q] = 0.0f;
                    if (armed) {
#pragma unroll
                        for (int jj = 0; jj < NJ; ++jj) {
                            const float c = cv[jj];
                            float ac = 0.0f;
#pragma unroll
                            for (int q = 0; q < M; ++q) {
                                const float dl = (g[q][jj] + c) + na[q][jj];
                                const float y = fmaf(-s[q], dl, g[q][jj]);
                                rq[q] = fmaf(y, y, rq[q]);
                                ac = fmaf(s[q], dl, ac);
                                g[q][jj] = s[q] * dl;
                            }
                            acc[jj] = ac;
                        }
                    } else {
#pragma unroll
                        for (int jj = 0; jj < NJ; ++jj) {
                            const float c = cv[jj];
                            float ac = 0.0f;
#pragma unroll
                            for (int q = 0; q < M; ++q) {
                                const float dl = (g[q][jj] + c) + na[q][jj];
                                ac = fmaf(s[q], dl, ac);
                                g[q][jj] = s[q] * dl;
                            }
                            acc[jj] = ac;
                        }
                    }
#pragma unroll
                    for (int q = 0; q < M; ++q) rp_lane += rq[q];
                } else {
#pragma unroll
                    for (int jj = 0; jj < NJ; ++jj) {
                        float ac = 0.0f;
#pragma unroll
                        for (int q = 0; q < M; ++q) {
                            const float dl = g[q][jj];
                            ac = fmaf(s[q], dl, ac);
                            g[q][jj] = fmaf(s[q], dl, na[q][jj]);
                        }
                        acc[jj] = ac;
                    }
                }
                // keep the new state materialised here (not sunk past the reductions)
#pragma unroll
                for (int q = 0; q < M; ++q)
#pragma unroll
                    for (int jj = 0; jj < NJ; ++jj) asm volatile("" : "+v"(g[q][jj]));
                // ---- reduce-scatter; z-update of the owned coordinate
                const float Ev = reduce_scatter_full<NJ>(acc, lane, holds);
                const float zn = own ? clampf(fmaf(-Ev, inv_n, zr), blo, bhi) : 0.0f;
                const float dz = zn - zr;
                cv[cidx] = zn + dz;
                // (summed by the last wave after the next exchange; armed
                // iterations sum their own below)
                if (own) dz2s[(t & 1) * 64 + cj] = dz * dz;
                const float cz = (2.0f * zr - zp) - zn;   // c - z' (0 on lanes without a coordinate)
                zp = zr;
                zr = zn;
                if (armed) {
                    // sum_k ||x_k - z'||^2 = sum_k ||x_k - c||^2 + 2 (c - z') . sum_k (x_k - c)
                    // + n ||c - z'||^2, with sum_k (x_k - c) = E^t - E^{t+1}
                    const float rpx = own ? cz * fmaf(fn, cz, 2.0f * (Ep - Ev)) : 0.0f;
                    // this iteration's dual and primal lane sums in one
                    // reduction (the stages of one wave sum; the first total
                    // on lanes 0-31, the second on 32-63)
                    const float x2 = swap32_sum(dz * dz, rp_lane + rpx);
                    const float t2 = row_sum16(swap16_sum(x2, x2));
                    rd_w = readfirstlane(t2);
                    rp_w = readlane(t2, 32);
                    float rd_t = rd_w, rp_t = rp_w;
                    if constexpr (WC > 1) {
                        float *XS = xs + 2 * WC * 4;   // its own slot: armed iterations only
                        if (lane == 0) {
                            XS[cw * 4 + 0] = rd_w;
                            XS[cw * 4 + 1] = rp_w;
                        }
                        __syncthreads();
                        rd_t = XS[0];
                        rp_t = XS[1];
#pragma unroll
                        for (int w = 1; w < WC; ++w) {
                            rd_t += XS[w * 4 + 0];
                            rp_t += XS[w * 4 + 1];
                        }
                        rd_t = readfirstlane(rd_t);
                        rp_t = readfirstlane(rp_t);
                    }
                    rd2 = rd_t * inv_d;
                    rp2 = fmaxf(rp_t, 0.0f) * inv_nd;
                    if (uniform(tau2 > 0.0f && rp2 <= tau2 && rd2 <= tau2)) {
                        flags = EM_CONVERGED;
                        iters = t;
                        done = true;
                        break;
                    }
                }
                Ep = Ev;
            }
            if (!done) iters = max_iter;   // the last iteration was armed and tested
        }
        // ---- write z and the statistics
        if (own) Z[cj] = bad_all ? __builtin_nanf("") : zr;
        if (cw == 0 && lane == 0 && L.stats != nullptr) {
            em_stats_t st;
            st.iters = bad_all ? 0 : iters;
            st.flags = flags;
            st.r_pri = bad_all ? 0.0f : sqrtf(rp2);
            st.r_dual = bad_all ? 0.0f : sqrtf(rd2);
            L.stats[b] = st;
        }
    }
}

}  // namespace emx
