// Non-Local Euclidean Medians on gfx950: one persistent kernel that solves,
// for every pixel, the box-constrained Euclidean median of the patches of its
// search window with NLM weights (Section 3 of arXiv:1501.03879) by EM-ADMM
// (Algorithm 1).
//
// Mapping
//  * A workgroup of WC waves owns one pixel at a time (work queue, early
//    exit per pixel).  It stages the (2(R+r)+1)^2 image tile around the pixel
//    (symmetric reflection at the borders) into LDS once; every point a_j is
//    then read from that tile, never materialised.
//  * Wave w owns a fixed slice of the d = (2r+1)^2 patch coordinates; lane l
//    owns window positions p = l + 64 q, q < M (for R = 10: M = 7 consecutive
//    columns of one window row).  Per point and slice it keeps one state
//    value g = e - a in registers for the whole solve, where e is the prox
//    displacement s (v - a) of the last iteration.  Point values are read
//    from the tile along patch rows: with consecutive columns, coordinate
//    (r, c + 1) of point q is coordinate (r, c) of point q + 1, so each
//    further coordinate costs one LDS read per lane.
//  * Per iteration (exactly Algorithm 1, rewritten with the scaled multiplier
//    u_k = y_k / mu; c = 2 z^t - z^{t-1}):
//      delta = g + c = v_k - a_k             (v_k = z - u_k)
//      nu^2  = ||delta||^2                    (slices summed through LDS)
//      s     = min(lambda, nu) / nu           (closed-form prox, lambda = w/mu)
//      E    += s delta  (= sum_k e_k),  g = s delta - a
//      z'    = clamp(z - E / n, lo, hi)       (the unweighted mean of x_k + u_k)
//    so x_k = v_k - e_k and u_k' = z - z' - e_k are implicit.  The first
//    iteration's nu^2 equals ||P_i - P_j||^2 (z starts at P_i, u = 0), which
//    gives the NLM weights w_j = exp(-nu^2 / h^2) without a separate pass.
//  * Sums over points: in-lane, then a full permlane/DPP reduce-scatter across
//    the wave, after which one lane per slice coordinate holds E and keeps
//    z^t, z^{t-1}, E^t of that coordinate in registers; c is broadcast to the
//    other lanes through LDS for the next pass.
//  * Stopping: the primal residual is evaluated on iterations that follow one
//    with r_dual <= tol (hi - lo) ("armed") and the stop test is taken right
//    after them.
//  * Starting point (Section 3 compares two): the noisy patch P_i, or the
//    Non-Local Means patch sum_j w_j P_j / sum_j w_j, computed by a weights
//    pass before the loop; with zero iterations the output is then NLM.
//  * SOLVER = 1 runs IRLS on the smooth surrogate (EM_surrogate) instead:
//    omega_j = w_j / (||z - P_j||^2 + eps)^(1/2) and z' = P_C(sum_j omega_j
//    P_j / sum_j omega_j) (majorise-minimise; the box projection is exact for
//    the isotropic quadratic majoriser), 3 operations per point-coordinate.
#pragma once

#include <float.h>
#include <hip/hip_fp16.h>

#include "em_device.hpp"
#include "emx_internal.hpp"

namespace emx {

// Slices with at most this many point values per lane keep the points in
// registers (read from the LDS tile once per pixel).
#ifndef EMX_KEEP_POINTS
#define EMX_KEEP_POINTS 64
#endif
constexpr int kKeepPointsInRegs = EMX_KEEP_POINTS;

template <int M>
constexpr int rmax_for() {
    int r = 0;
    while ((2 * (r + 1) + 1) * (2 * (r + 1) + 1) <= 64 * M) ++r;
    return r;
}

template <int PR, int M, int WC>
struct NlemShape {
    static constexpr int PS = 2 * PR + 1;
    static constexpr int D = PS * PS;
    static constexpr int RMAX = rmax_for<M>();
    static constexpr int WSM = 2 * RMAX + 1;
    static constexpr int TW = 2 * (RMAX + PR) + 1;
    // Pitch = WSM + 32: after a full window row of WSM points the next row
    // continues on the next bank (mod 32), so 32 consecutive lanes reading
    // one patch coordinate of consecutive window points hit distinct banks.
    // (WSM + 64, conflict-free mod 64 as well, timed the same on MI355X.)
#ifndef EMX_TILE_PITCH_PAD
#define EMX_TILE_PITCH_PAD 32
#endif
    static constexpr int P = WSM + EMX_TILE_PITCH_PAD;
    static constexpr int TILE = TW * P;
    static constexpr int DS = (D + WC - 1) / WC;
    // Row mapping: each window row is cut into ceil(WS / M) runs of M
    // consecutive columns and lane l owns one run, so one base address plus
    // immediate offsets reaches all its points and consecutive points share
    // patch coordinates (one LDS read per coordinate instead of M).  The host
    // gives M = 4 to R = 7 (4 runs x 15 rows = 60 lanes) and M = 7 to R = 9
    // and 10 (3 runs x 19 or 21 rows); columns past the window in a last run
    // are masked slots.  Other windows would need a larger M for their runs
    // to fit 64 lanes, and the extra idle slots cost more than the loads
    // save (measured), so M = 2, 3, 5, 6 read the points slot by slot.
    static constexpr bool ROWMAP = (M == 4 || M == 7);
    // partial sums of ||delta||^2 from the WC waves (two buffers, by
    // iteration parity), then one shrink factor per point (M x 64)
    static constexpr int XN = (WC > 1) ? 2 * WC * M * 64 + M * 64 : 1;
    // shrink factors are taken by wave w for the lane's points
    // [w QS, min((w + 1) QS, M))
    static constexpr int QS = (M + WC - 1) / WC;
    static_assert(TW <= 64, "tile rows are staged one column per lane");
    static_assert(D <= 64, "one lane per patch coordinate sums the squared z steps");
};

// Totals of two per-lane values over the 64 lanes in one reduction (the
// stages of one wave sum): the first on lanes 0-31, the second on 32-63.
__device__ __forceinline__ float wave_sum2(float a, float b) {
    const float x = swap32_sum(a, b);   // lanes 0-31: a[l] + a[l + 32]; lanes 32-63: b
    return row_sum16(swap16_sum(x, x));
}

template <int PR, int M, int WC, int SW, int SOLVER>
__device__ __forceinline__ void nlem_wave(const NlemLaunch &L, float *tile, float *xn, float *xs,
                                          float *cvec, unsigned int *item_s) {
    constexpr bool IRLS = SOLVER == 1;
    using S = NlemShape<PR, M, WC>;
    constexpr int J0 = SW * S::DS;
    constexpr int NJ = (S::D - J0 < S::DS) ? (S::D - J0) : S::DS;
    using RSx = RSF<NJ>;
    constexpr int JC = (S::D - 1) / 2;  // centre coordinate

    const int lane = threadIdx.x & 63;
    // after the reduce-scatter this lane owns slice coordinate myc (if myv)
    const bool myv = (RSx::mask() >> lane) & 1;
    const int myc = RSx::coord(lane);
    const int myoff = myv ? ((J0 + myc) / S::PS) * S::P + ((J0 + myc) % S::PS) : 0;
    // per-wave c = 2 z^t - z^{t-1} of the slice, [0, NJ); lanes that own no
    // coordinate write to a private slot in [64, 128) instead
    float *cv = cvec + SW * 128;
    // squared z steps of the owned coordinates, by iteration parity (WC > 1)
    float *dz2s = xs + 3 * WC * 4;
    const int cidx = myv ? myc : 64 + lane;
    // points stay in registers when they fit (the compiler hoists the tile
    // reads); IRLS never changes g = -a, so it always keeps them
    constexpr bool kKeep = IRLS || M * NJ <= kKeepPointsInRegs;
    // tile offset of slice coordinate jj within a patch (folded after unrolling)
    auto poff = [](int jj) { return ((J0 + jj) / S::PS) * S::P + ((J0 + jj) % S::PS); };

    // The workgroup takes L.chunk consecutive queue positions per atomic: one
    // global counter serves every workgroup, and for cheap pixels (small
    // windows) its update rate, not the solves, would set the pace.
    unsigned int cbase = 0, cleft = 0;   // thread 0: the rest of the current chunk
    for (;;) {
        if (threadIdx.x == 0) {
            if (cleft == 0) {
                cbase = atomicAdd(L.counter, (unsigned int)L.chunk);
                cleft = (unsigned int)L.chunk;
            }
            *item_s = cbase++;
            --cleft;
        }
        __syncthreads();
        const int64_t qpos = (int64_t)(unsigned int)uniform_int((int)*item_s);
        if (qpos >= L.prefix[L.count]) break;
        const int64_t item = L.order ? (int64_t)uniform_int(L.order[qpos]) : qpos;
        int b = 0;
        while (b + 1 < L.count && item >= L.prefix[b + 1]) ++b;
        const NlemImageDesc I = L.img[b];
        const int pix = (int)(item - L.prefix[b]);
        const int H = I.H, W = I.W, R = I.R;
        const int iy = pix / W, ix = pix - (pix / W) * W;
        const int WSr = 2 * R + 1;
        const int TWr = 2 * (R + PR) + 1;
        const int LPR = (WSr + M - 1) / M;                       // runs per window row
        const int TWs = S::ROWMAP ? max(TWr, LPR * M + 2 * PR) : TWr;   // staged columns

        // ---- a1: stage the tile (rows iy-R-r .. iy+R+r), reflected at borders
        // (rows outside the reflection range are clamped; only window slots
        // outside the image read them).  Wave w loads rows w, w + WC, ...,
        // one column per lane (TW <= 64); the columns a last partial run
        // reaches past the window are staged too (finite values of masked
        // slots).
        // All of a wave's row loads are issued before the first is waited
        // on (reflected positions are always inside the image, so the loads
        // need no guard; rows past the tile re-read its last row).
        {
            constexpr int RPW = (S::TW + WC - 1) / WC;   // rows per wave, at most
            const int gx = reflect_idx(ix - R - PR + lane, W);
            float v[RPW];
            if (I.is_f16) {
                const __half *img = reinterpret_cast<const __half *>(I.img);
#pragma unroll
                for (int k = 0; k < RPW; ++k) {
                    const int64_t gy = reflect_idx(iy - R - PR + min(SW + WC * k, TWr - 1), H);
                    v[k] = __half2float(img[gy * W + gx]);
                }
            } else {
                const float *img = reinterpret_cast<const float *>(I.img);
#pragma unroll
                for (int k = 0; k < RPW; ++k) {
                    const int64_t gy = reflect_idx(iy - R - PR + min(SW + WC * k, TWr - 1), H);
                    v[k] = img[gy * W + gx];
                }
            }
#pragma unroll
            for (int k = 0; k < RPW; ++k) {
                const int ty = SW + WC * k;
                if (ty < TWr && lane < TWs) tile[ty * S::P + lane] = v[k];
            }
        }
        __syncthreads();

        // ---- points owned by this lane: window slot p -> tile offset of its patch
        const int y0 = max(iy - R, 0), y1 = min(iy + R, H - 1);
        const int x0 = max(ix - R, 0), x1 = min(ix + R, W - 1);
        const int n = (y1 - y0 + 1) * (x1 - x0 + 1);
        int base[S::ROWMAP ? 1 : M];
        float lam[M];
        if constexpr (S::ROWMAP) {
            // lane owns M consecutive columns of one window row
            const int wy = lane / LPR, wx0 = (lane - (lane / LPR) * LPR) * M;
            const bool rowok = lane < LPR * WSr && iy - R + wy >= 0 && iy - R + wy < H;
            base[0] = rowok ? (wy * S::P + wx0) : 0;
#pragma unroll
            for (int q = 0; q < M; ++q) {
                const int px = ix - R + wx0 + q;
                lam[q] = (rowok && wx0 + q < WSr && px >= 0 && px < W) ? 0.0f : -1.0f;
            }
        } else {
            const float inv_ws = 1.0f / (float)WSr;
#pragma unroll
            for (int q = 0; q < M; ++q) {
                const int p = lane + 64 * q;
                const int wy = (int)(((float)p + 0.5f) * inv_ws);
                const int wx = p - wy * WSr;
                const int py = iy - R + wy, px = ix - R + wx;
                const bool valid = (p < WSr * WSr) && py >= 0 && py < H && px >= 0 && px < W;
                base[q] = valid ? (wy * S::P + wx) : 0;
                lam[q] = valid ? 0.0f : -1.0f;
            }
        }
        // tile offset of point slot q (its patch's top-left corner)
        auto pbase = [&](int q) { return S::ROWMAP ? base[0] + q : base[q]; };
        // Stream of the values -a of slice coordinates jj = 0, 1, ... for the
        // lane's M points, loaded one coordinate ahead.  With the row mapping
        // the lane's points are consecutive window columns, so coordinate
        // (r, c + 1) of point q is coordinate (r, c) of point q + 1: moving
        // along a patch row loads one new value, a new row loads M.
        auto same_row = [](int jj) { return (J0 + jj) / S::PS == (J0 + jj + 1) / S::PS; };
        auto st_begin = [&](float (&win)[M]) {
#pragma unroll
            for (int q = 0; q < M; ++q) win[q] = -tile[pbase(q) + poff(0)];
        };
        auto st_prefetch = [&](int jj, float (&nx)[M]) {
            if (jj + 1 < NJ) {
                if (S::ROWMAP && same_row(jj)) {
                    nx[M - 1] = -tile[pbase(M - 1) + poff(jj + 1)];
                } else {
#pragma unroll
                    for (int q = 0; q < M; ++q) nx[q] = -tile[pbase(q) + poff(jj + 1)];
                }
            }
        };
        auto st_advance = [&](int jj, float (&win)[M], const float (&nx)[M]) {
            if (jj + 1 < NJ) {
                if (S::ROWMAP && same_row(jj)) {
#pragma unroll
                    for (int q = 0; q + 1 < M; ++q) win[q] = win[q + 1];
                    win[M - 1] = nx[M - 1];
                } else {
#pragma unroll
                    for (int q = 0; q < M; ++q) win[q] = nx[q];
                }
            }
        };

        // ---- a3: z = P_i (unprojected), u = 0  (so g = -a, c = z).  Lanes
        // without a coordinate hold z = clamp(0) and E = 0, a fixed point of
        // the z-update, so they need no masking below.
        float zr = myv ? tile[R * S::P + R + myoff] : clampf(0.0f, L.lo, L.hi);  // z^t
        const float pc = zr;                                                // P_i (own coordinate)
        float zp = zr;                                                      // z^{t-1}
        float Ep = 0.0f;                                                    // E^t
        cv[cidx] = zr;
        float g[M][NJ];
#pragma unroll
        for (int q = 0; q < M; ++q)
#pragma unroll
            for (int jj = 0; jj < NJ; ++jj) g[q][jj] = -tile[pbase(q) + poff(jj)];

        // sums of per-wave partials over the WC waves (identical in every wave)
        auto exchange = [&](float (&v)[M], float *X) {
            if constexpr (WC > 1) {
#pragma unroll
                for (int q = 0; q < M; ++q) X[(SW * M + q) * 64 + lane] = v[q];
                __syncthreads();
#pragma unroll
                for (int q = 0; q < M; ++q) {
                    float sum = X[q * 64 + lane];
#pragma unroll
                    for (int w = 1; w < WC; ++w) sum += X[(w * M + q) * 64 + lane];
                    v[q] = sum;
                }
            }
        };
        // a2: NLM weights w_j = exp(-||P_i - P_j||^2 / h^2) from the squared
        // distances (invalid window slots get 0); false if a distance is not finite
        auto weights_from = [&](const float (&nrm)[M], float (&wt)[M]) {
            bool nonfinite = false;
#pragma unroll
            for (int q = 0; q < M; ++q) {
                const bool valid = lam[q] >= 0.0f;   // -1 marks window slots outside the image
                nonfinite |= valid && !(nrm[q] <= FLT_MAX);
                wt[q] = valid ? exp2f(-nrm[q] * I.k_h) : 0.0f;
            }
            return !__any(nonfinite);
        };

        bool bad = false;
        float wt[M];           // IRLS: the NLM weights (ADMM keeps lam = w / mu)
        const bool pre = IRLS || L.init_nlm;
        if (pre) {
            // weights pass before the loop: ||P_i - P_j||^2 with c = P_i, g = -a
            float nrm[M];
#pragma unroll
            for (int q = 0; q < M; ++q) nrm[q] = kNu2Floor;
#pragma unroll
            for (int jj = 0; jj < NJ; ++jj) {
                const float cj = cv[jj];
#pragma unroll
                for (int q = 0; q < M; ++q) {
                    const float dv = g[q][jj] + cj;
                    nrm[q] = fmaf(dv, dv, nrm[q]);
                }
            }
            exchange(nrm, xn);   // buffer 0: the loop starts on buffer 1
            bad = !weights_from(nrm, wt);
            if constexpr (IRLS) {
                // IRLS works relative to the noisy patch: g = P_i - a and the
                // iterate is held as z - P_i, so the distance to the pixel's
                // own patch (which dominates the weights near the start, where
                // it is ~ eps^(1/2)) carries FP32 precision of its own size
                // rather than of the intensities.
#pragma unroll
                for (int jj = 0; jj < NJ; ++jj) {
                    const float cj = cv[jj];
#pragma unroll
                    for (int q = 0; q < M; ++q) g[q][jj] += cj;
                }
                zr = 0.0f;
                cv[cidx] = 0.0f;
            }
            if (!bad && L.init_nlm) {
                // z^0 = the NLM patch sum_j w_j P_j / sum_j w_j (a3, second option)
                float acc[NJ];
#pragma unroll
                for (int jj = 0; jj < NJ; ++jj) {
                    float ac = 0.0f;
#pragma unroll
                    for (int q = 0; q < M; ++q) ac = fmaf(wt[q], g[q][jj], ac);
                    acc[jj] = ac;
                }
                float wl = 0.0f;
#pragma unroll
                for (int q = 0; q < M; ++q) wl += wt[q];
                const float inv_ws = 1.0f / readfirstlane(wave_sum(wl));
                const float Ev = reduce_scatter_full<NJ>(acc, lane, myv);   // -sum_j w_j P_j
                if (myv) zr = -Ev * inv_ws;   // ADMM: the NLM patch; IRLS: it minus P_i
                zp = zr;
                cv[cidx] = zr;
            }
            if constexpr (!IRLS) {
#pragma unroll
                for (int q = 0; q < M; ++q) lam[q] = wt[q] * L.inv_mu;
            }
        }

        const float inv_n = 1.0f / (float)n;
        const float fn = (float)n;
        const float inv_d = 1.0f / (float)S::D;
        const float inv_nd = 1.0f / ((float)n * (float)S::D);
        const int max_iter = L.max_iter;
        const float tau2 = L.tau * L.tau;
        const float arm2 = L.tau_arm * L.tau_arm;

        int iters = 0, flags = EM_MAXITER;
        float rp2 = 0.0f, rd2 = 0.0f;  // mean squares of the last evaluated iteration
        float rd_w = 0.0f, rp_w = 0.0f;
        bool done = false;
        int t = 1;
        if constexpr (IRLS) {
            const float eps = L.eps;
            for (; t <= max_iter && !bad; ++t) {
                // ---- ||z - P_j||^2 (c = z; g = -a never changes)
                float nrm[M];   // + eps, counted once over the WC partial sums
#pragma unroll
                for (int q = 0; q < M; ++q) nrm[q] = (SW == 0) ? eps : 0.0f;
#pragma unroll
                for (int jj = 0; jj < NJ; ++jj) {
                    const float cj = cv[jj];
#pragma unroll
                    for (int q = 0; q < M; ++q) {
                        const float dv = g[q][jj] + cj;
                        nrm[q] = fmaf(dv, dv, nrm[q]);
                    }
                }
                float rd_all = rd_w;
                if constexpr (WC > 1) {
                    float *XS = xs + (t & 1) * WC * 4;
                    if (lane == 0) XS[SW * 4] = rd_w;
                    exchange(nrm, xn + (t & 1) * WC * M * 64);
                    rd_all = XS[0];
#pragma unroll
                    for (int w = 1; w < WC; ++w) rd_all += XS[w * 4];
                    rd_all = readfirstlane(rd_all);
                }
                // stop test for iteration t-1 (dual residual only)
                if (t > 1) {
                    rd2 = rd_all * inv_d;
                    if (uniform(tau2 > 0.0f && rd2 <= tau2)) {
                        flags = EM_CONVERGED;
                        iters = t - 1;
                        done = true;
                        break;
                    }
                }
                // ---- omega_j = w_j (||z - P_j||^2 + eps)^(-1/2); sum_j omega_j P_j
                float om[M];
                float ol = 0.0f;
#pragma unroll
                for (int q = 0; q < M; ++q) {
                    om[q] = wt[q] * __builtin_amdgcn_rsqf(nrm[q]);
                    ol += om[q];
                }
                float acc[NJ];
#pragma unroll
                for (int jj = 0; jj < NJ; ++jj) {
                    float ac = 0.0f;
#pragma unroll
                    for (int q = 0; q < M; ++q) ac = fmaf(om[q], g[q][jj], ac);
                    acc[jj] = ac;
                }
                const float Ev = reduce_scatter_full<NJ>(acc, lane, myv);   // -sum_j omega_j P_j
                const float inv_os = 1.0f / readfirstlane(wave_sum(ol));
                // z' - P_i = P_C(P_i + raw) - P_i, exact when the box is inactive
                const float raw = -Ev * inv_os;
                const float zab = pc + raw;
                const float zn = !myv ? zr : (zab < L.lo ? L.lo - pc : (zab > L.hi ? L.hi - pc : raw));
                const float dz = zn - zr;
                cv[cidx] = zn;
                rd_w = readfirstlane(wave_sum(dz * dz));
                zr = zn;
            }
        } else
        for (; t <= max_iter && !bad; ++t) {
            // Wave priority (several coordinate waves): a wave runs the first
            // half of an iteration (its own points: delta and the norm
            // partials) at the lowest priority and the rest, from the first
            // barrier on, at a higher one.  Several workgroups share each
            // SIMD (three for 7x7 patches and 21x21 windows); favouring the
            // waves past the barrier lets a workgroup reach its next barrier
            // sooner while the first halves of the others fill the issue
            // slots (2.375 -> 2.254 ms on the 256x256 image with that shape).
            if constexpr (WC > 1) __builtin_amdgcn_s_setprio(0);
            // Large slices read the points from the LDS tile every iteration;
            // without this the compiler hoists the loop-invariant tile reads
            // and keeps all M*NJ points live in registers.
            if constexpr (!kKeep) asm volatile("" ::: "memory");
            // ---- a4 (first half): delta = g + c, partial ||delta||^2
            float nrm[M];
#pragma unroll
            for (int q = 0; q < M; ++q) nrm[q] = kNu2Floor;
#pragma unroll
            for (int jj = 0; jj < NJ; ++jj) {
                const float cj = cv[jj];
#pragma unroll
                for (int q = 0; q < M; ++q) {
                    g[q][jj] += cj;
                    nrm[q] = fmaf(g[q][jj], g[q][jj], nrm[q]);
                }
            }
            float s[M];
            float rd_all = rd_w;
            bool arm_ok = false;   // WC > 1: iteration t-1's dual residual within the arm level
            if constexpr (WC > 1) {
                // The waves hold partial sums of ||delta||^2 over their
                // coordinate slices.  Wave SW adds up the partials of its
                // share of the lane's points, takes their shrink factors (on
                // the first iteration their weights too, a2) and hands them
                // to the other waves through LDS, so each point's factor is
                // computed once per workgroup rather than once per wave.  The
                // partials are added in wave order, as every wave would.
                constexpr int Q0 = (SW * S::QS < M) ? SW * S::QS : M;
                constexpr int QN = (M - Q0 < S::QS) ? (M - Q0) : S::QS;
                float *X = xn + (t & 1) * WC * M * 64;
                float *XS = xs + (t & 1) * WC * 4;
                float *SV = xn + 2 * WC * M * 64;
#pragma unroll
                for (int q = 0; q < M; ++q) X[(SW * M + q) * 64 + lane] = nrm[q];
                __syncthreads();
                __builtin_amdgcn_s_setprio(1);
                // the dual residual of iteration t-1: the last wave sums the
                // squared steps the coordinate owners left in LDS (coordinate
                // order), takes the arming test and hands its outcome over
                // with the shrink factors
                if constexpr (SW == WC - 1) {
                    if (t > 1) {
                        const float q2 = (lane < S::D) ? dz2s[((t - 1) & 1) * 64 + lane] : 0.0f;
                        const float tot = wave_sum(q2);
                        // (only the arming test needs it: the flag goes over)
                        if (lane == 0) reinterpret_cast<int *>(XS)[SW * 4 + 3] = (tot * inv_d <= arm2) ? 1 : 0;
                    }
                }
                float ns[QN > 0 ? QN : 1];
#pragma unroll
                for (int qq = 0; qq < QN; ++qq) {
                    ns[qq] = X[(Q0 + qq) * 64 + lane];
#pragma unroll
                    for (int w = 1; w < WC; ++w) ns[qq] += X[(w * M + Q0 + qq) * 64 + lane];
                }
                // (a branch of its own: folded into the iteration, the
                // exponentials would run on every iteration)
                const bool first = t == 1 && !pre;   // (uniform already: t and pre are)
                if (__builtin_expect(first, 0)) {
                    // ---- a2: NLM weights from the first iteration's
                    // distances (the noisy start: delta = P_i - P_j)
                    bool nonfinite = false;
#pragma unroll
                    for (int qq = 0; qq < QN; ++qq) {
                        const int q = Q0 + qq;
                        const bool valid = lam[q] >= 0.0f;   // -1: slot outside the image
                        nonfinite |= valid && !(ns[qq] <= FLT_MAX);
                        lam[q] = (valid ? exp2f(-ns[qq] * I.k_h) : 0.0f) * L.inv_mu;
                    }
                    if (lane == 0) XS[SW * 4 + 2] = __any(nonfinite) ? 1.0f : 0.0f;
                }
#pragma unroll
                for (int qq = 0; qq < QN; ++qq) SV[(Q0 + qq) * 64 + lane] = shrink(ns[qq], lam[Q0 + qq]);
                __syncthreads();
                if (first) {
                    float nf = XS[2];
#pragma unroll
                    for (int w = 1; w < WC; ++w) nf += XS[w * 4 + 2];
                    if (uniform(nf > 0.0f)) {
                        bad = true;
                        break;
                    }
                }
#pragma unroll
                for (int q = 0; q < M; ++q) s[q] = SV[q * 64 + lane];
                if (t > 1) arm_ok = uniform_int(reinterpret_cast<const int *>(XS)[(WC - 1) * 4 + 3]) != 0;
            } else {
                // ---- a2 (one wave holds whole points): the weights from the
                // first iteration's distances, unless the pre-pass made them
                if (t == 1 && !pre) {
                    float w1[M];
                    if (!weights_from(nrm, w1)) {
                        bad = true;
                        break;
                    }
#pragma unroll
                    for (int q = 0; q < M; ++q) lam[q] = w1[q] * L.inv_mu;
                }
#pragma unroll
                for (int q = 0; q < M; ++q) s[q] = shrink(nrm[q], lam[q]);
            }
            // the dual residual of iteration t-1 arms the primal residual of
            // this iteration (WC > 1: the last wave took the test)
            bool armed;
            if constexpr (WC > 1) {
                armed = (t == max_iter) || (tau2 > 0.0f && t > 1 && arm_ok && (t & L.check_mask) == 0);
            } else {
                if (t > 1) rd2 = rd_all * inv_d;
                armed = uniform((t == max_iter) ||
                                (tau2 > 0.0f && t > 1 && rd2 <= arm2 && (t & L.check_mask) == 0));
            }

            // ---- a8 (armed iterations only): lane sums of ||x_k - c||^2 with
            // x_k = v_k - e_k = a_k + (1 - s) delta, read-only on the state
            float rp_lane = 0.0f;
            if (armed) {
                float rq[M];
#pragma unroll
                for (int q = 0; q < M; ++q) rq[q] = 0.0f;
                float win[M], nx[M];
                st_begin(win);
#pragma unroll
                for (int jj = 0; jj < NJ; ++jj) {
                    const float cj = cv[jj];
                    st_prefetch(jj, nx);
#pragma unroll
                    for (int q = 0; q < M; ++q) {
                        const float y = fmaf(1.0f - s[q], g[q][jj], -(win[q] + cj));
                        rq[q] = fmaf(y, y, rq[q]);
                    }
                    st_advance(jj, win, nx);
                    if constexpr (!kKeep) __builtin_amdgcn_sched_barrier(0);
                }
                // Absent window slots need no mask: their s is 0 and their state
                // stays g = -a, so delta and -(-a + c) round identically, y = 0.
#pragma unroll
                for (int q = 0; q < M; ++q) rp_lane += rq[q];
            }
            // keep the two passes' tile reads separate (no values carried over)
            if constexpr (!kKeep) asm volatile("" ::: "memory");

            // ---- a4 (second half) + a5 partial sums: E = sum_k s delta, g = s delta - a
            // (tile reads streamed one coordinate ahead)
            float acc[NJ];
            {
                float win[M], nx[M];
                st_begin(win);
#pragma unroll
                for (int jj = 0; jj < NJ; ++jj) {
                    st_prefetch(jj, nx);
                    float ac = 0.0f;
#pragma unroll
                    for (int q = 0; q < M; ++q) {
                        const float d = g[q][jj];
                        ac = fmaf(s[q], d, ac);
                        g[q][jj] = fmaf(s[q], d, win[q]);
                    }
                    acc[jj] = ac;
                    st_advance(jj, win, nx);
                    if constexpr (!kKeep) __builtin_amdgcn_sched_barrier(0);
                }
            }
            // Materialise the new state here: otherwise the updates are sunk
            // past the reductions and delta and the points stay live meanwhile.
#pragma unroll
            for (int q = 0; q < M; ++q)
#pragma unroll
                for (int jj = 0; jj < NJ; ++jj) asm volatile("" : "+v"(g[q][jj]));
            // ---- a5: reduce over the wave; a6: z-update; a7 implicit in g and c
            const float Ev = reduce_scatter_full<NJ>(acc, lane, myv);
            const float zn = clampf(fmaf(-Ev, inv_n, zr), L.lo, L.hi);
            const float dz = zn - zr;
            cv[cidx] = zn + dz;
            if constexpr (WC > 1) {
                // (summed by the last wave after the next exchange; armed
                // iterations sum their own below)
                if (myv) dz2s[(t & 1) * 64 + J0 + myc] = dz * dz;
            } else {
                rd_w = readfirstlane(wave_sum(dz * dz));
            }
            const float cz = (2.0f * zr - zp) - zn;
            zp = zr;
            zr = zn;
            if (armed) {
                // ---- a8: sum_k ||x_k - z'||^2 from the lane sums of ||x_k - c||^2:
                // x_k - z' = (x_k - c) + (c - z') and sum_k (x_k - c) = E^t - E^{t+1};
                // the stop test is taken right away (one barrier for WC > 1)
                const float rpx = cz * fmaf(fn, cz, 2.0f * (Ep - Ev));
                if constexpr (WC > 1) {
                    // this iteration's dual and primal lane sums in one reduction
                    const float t2 = wave_sum2(dz * dz, rp_lane + rpx);
                    rd_w = readfirstlane(t2);
                    rp_w = readlane(t2, 32);
                } else {
                    rp_w = readfirstlane(wave_sum(rp_lane + rpx));
                }
                float rd_all = rd_w, rp_all = rp_w;
                if constexpr (WC > 1) {
                    float *XS = xs + 2 * WC * 4;   // its own slot: armed iterations only
                    if (lane == 0) {
                        XS[SW * 4 + 0] = rd_w;
                        XS[SW * 4 + 1] = rp_w;
                    }
                    __syncthreads();
                    rd_all = XS[0];
                    rp_all = XS[1];
#pragma unroll
                    for (int w = 1; w < WC; ++w) {
                        rd_all += XS[w * 4 + 0];
                        rp_all += XS[w * 4 + 1];
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
            }
            Ep = Ev;
        }

        if (!IRLS && !done && !bad) {
            iters = max_iter;   // the last iteration was armed and tested
        } else if (!done && !bad) {
            iters = max_iter;
            if (max_iter >= 1) {
                float rd_all = rd_w, rp_all = rp_w;
                if constexpr (WC > 1) {
                    float *XS = xs + (t & 1) * WC * 4;
                    if (lane == 0) {
                        XS[SW * 4 + 0] = rd_w;
                        XS[SW * 4 + 1] = rp_w;
                    }
                    __syncthreads();
                    rd_all = 0.0f;
                    rp_all = 0.0f;
#pragma unroll
                    for (int w = 0; w < WC; ++w) {
                        rd_all += XS[w * 4 + 0];
                        rp_all += XS[w * 4 + 1];
                    }
                    rd_all = readfirstlane(rd_all);
                    rp_all = readfirstlane(rp_all);
                }
                rd2 = rd_all * inv_d;
                rp2 = 0.0f;
                flags = (tau2 > 0.0f && rd2 <= tau2) ? EM_CONVERGED : EM_MAXITER;
            }
        }
        if (bad) {
            flags = EM_BAD_INPUT;
            iters = 0;
            rp2 = 0.0f;
            rd2 = 0.0f;
        }

        // ---- a9: the centre coordinate of the solution patch
        if constexpr (JC >= J0 && JC < J0 + NJ) {
            constexpr int lc = RSx::lane_of(JC - J0);
            if (lane == lc) I.out[pix] = bad ? __builtin_nanf("") : (IRLS ? pc + zr : zr);
        }
        if (SW == 0 && lane == 0 && I.stats != nullptr) {
            em_stats_t st;
            st.iters = iters;
            st.flags = flags;
            st.r_pri = sqrtf(rp2);
            st.r_dual = sqrtf(rd2);
            I.stats[pix] = st;
        }
    }
}

template <int PR, int M, int WC, int SW, int SOLVER>
__device__ __forceinline__ void nlem_dispatch(int wave, const NlemLaunch &L, float *tile, float *xn,
                                              float *xs, float *cvec, unsigned int *item_s) {
    if constexpr (SW + 1 == WC) {
        nlem_wave<PR, M, WC, SW, SOLVER>(L, tile, xn, xs, cvec, item_s);
    } else {
        if (wave == SW)
            nlem_wave<PR, M, WC, SW, SOLVER>(L, tile, xn, xs, cvec, item_s);
        else
            nlem_dispatch<PR, M, WC, SW + 1, SOLVER>(wave, L, tile, xn, xs, cvec, item_s);
    }
}

template <int PR, int M, int WC, int SOLVER = 0>
#ifndef EMX_NLEM_MIN_WAVES
#define EMX_NLEM_MIN_WAVES 2
#endif
__global__ __launch_bounds__(64 * WC, EMX_NLEM_MIN_WAVES) void nlem_solve_kernel(NlemLaunch L) {
    using S = NlemShape<PR, M, WC>;
    __shared__ float tile[S::TILE];
    __shared__ float xn[S::XN];
    __shared__ float xs[3 * WC * 4 + 128];   // residual partials; then the squared steps, two buffers
    __shared__ float cvec[WC * 128];
    __shared__ unsigned int item_s;
    const int wave = uniform_int(threadIdx.x >> 6);
    nlem_dispatch<PR, M, WC, 0, SOLVER>(wave, L, tile, xn, xs, cvec, &item_s);
}

}  // namespace emx
