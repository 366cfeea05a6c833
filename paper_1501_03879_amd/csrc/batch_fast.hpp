// Batched accelerated ADMM for the box-constrained Euclidean median: fast
// ADMM with restart ([Goldstein2012], the weakly convex case), the extension
// named in the conclusion of arXiv:1501.03879, on the splitting of
// Algorithm 1.  Same iterates as the one-launch-per-instance version
// (plain_solve_kernel<true>) and the oracle: predictors z_hat, u_hat
// (u = y / mu); x_k = prox of w_k/mu ||. - a_k|| at z_hat - u_hat_k;
// z = P_C(mean_k(x_k + u_hat_k)); u_k = u_hat_k + x_k - z; after the residual
// test, c = mu (sum_k ||x_k - z||^2 + n ||z - z_hat||^2) decides between
// momentum (alpha' = (1 + sqrt(1 + 4 alpha^2)) / 2, beta = (alpha - 1) /
// alpha', z_hat = z + beta (z - z_prev), u_hat = u + beta (u - u_prev)) while
// c < eta (1 - 2^-16) c_prev, and a restart (z_hat = z_prev, u_hat = u_prev,
// alpha = 1, c_prev /= eta); no decision after the last allowed sweep.  The
// guard factor puts the exact ties of a stalled iterate (each sweep repeating
// c, then c against eta (c / eta) after a restart) on the restart side, as
// exact arithmetic does, beyond the rounding of FP32.
//
// Reduced form.  With the prox displacement e_k = s_k delta_k of sweep t
// (delta_k = v_k - a_k, v_k the prox input), u_k = z_hat - z - e_k, so the
// next prox input is
//   momentum: v' = C' + (1 + beta) e - beta e_prev,
//   restart:  v' = C' + e_prev,
// with e = e^t, e_prev = e^{t-1} and a d-vector C':
//   momentum: C' = z_hat' - (1 + beta)(z_hat - z) + beta (z_hat_prev - z_prev),
//   restart:  C' = 2 z_prev - z_hat_prev.
// The first sweep has e = e_prev = 0 and C = z_hat = z^0.  The state is e,
// not e - a as in the plain kernels: |e_k| <= w_k / mu whatever the point, so
// x_k - z = (v - z) - e is formed from terms of the residual's own size.
// From e - a it cancels terms of size |a|, and the restart test c < eta c_prev
// (eta near 1) needs c to far better than 1e-3 on every sweep, which FP32
// then misses on point sets with far outliers.
// Per point coordinate and sweep: v (2 FMA), delta and ||delta||^2 (2), E
// (2), then with z known delta again, e, x - z and its square (5), and one
// move: 12 VALU against the plain iteration's 4; both residuals are tested on
// every sweep, as the oracle does.
//
// Layout: the sliced kernels' (batch_wide.hpp) with 8-coordinate slices, WC
// in {1, 2, 4, 8} waves and M in {1, 2, 4, 8} points per lane, so that e,
// e_prev and the points (3 x 8 M values per lane) stay in registers up to
// n = 512.
#pragma once

#include "batch_wide.hpp"

namespace emx {

constexpr int kFastNJ = 8;
constexpr int kMaxRestartCountBatch = (1 << 23) - 1;   // what the flags word above EM_RESTART_SHIFT holds

// Waves per SIMD the launch bound asks for: ~24 M VGPRs for e, e_prev and
// the points of M points, ~70 for the rest; M = 8 takes one wave (the
// accumulation registers then serve as spill space).
constexpr int fast_waves_per_simd(int m) { return m <= 1 ? 5 : m <= 2 ? 4 : m <= 4 ? 2 : 1; }

template <int M, int WC>
__global__ __launch_bounds__(64 * WC, fast_waves_per_simd(M)) void batch_fast_kernel(ClassLaunch L) {
    constexpr int NJ = kFastNJ;
    using S = WideShape<NJ, M, WC>;
    using RSx = RSF<NJ>;
    __shared__ float stage[S::STAGE];
    __shared__ float xn[S::XN];
    __shared__ float xs[2 * WC * 4];   // per-wave sums of the residual terms, two buffers
    __shared__ float cvec[WC * 128];   // per wave: C of the slice; private slots [64, 128)
    __shared__ float zvec[WC * 128];   // per wave: the new z of the slice (pass 3)
    __shared__ unsigned int item_s;
    __shared__ int flag_s[4];

    const int lane = threadIdx.x & 63;
    const int cw = uniform_int(threadIdx.x >> 6);
    const bool holds = (RSx::mask() >> lane) & 1;
    const int myc = RSx::coord(lane);
    float *cv = cvec + cw * 128;
    float *zv = zvec + cw * 128;
    const int cidx = holds ? myc : 64 + lane;
    const unsigned int cbeg = L.offsets[L.cls];
    const unsigned int ccount = L.offsets[L.cls + 1] - cbeg;
    // workgroups beyond the class's instance count would only find the queue
    // empty: they leave before the atomic, so an empty class costs its dispatch
    if (blockIdx.x >= ccount) return;

    for (;;) {
        if (threadIdx.x == 0) {
            item_s = atomicAdd(L.counter, 1u);
            flag_s[0] = 0;
            flag_s[1] = 0;
            flag_s[2] = 0;
            flag_s[3] = 0;
        }
        __syncthreads();
        const unsigned int it = (unsigned int)uniform_int((int)item_s);
        if (it >= ccount) break;
        const int b = uniform_int(L.list[cbeg + it]);
        const em_instance_t e = L.inst[b];
        const int n = uniform_int(e.n), d = uniform_int(e.d);
        float *Z = L.z + e.z_off;
        const int j0 = cw * NJ;
        const int cj = j0 + myc;
        const bool own = holds && cj < d;

        float lam[M];
        float na[M][NJ];
        const WideStart st0 = wide_start<NJ, M, WC>(L, e, n, d, cw, lane, holds, own, j0, cj, stage, flag_s, cv,
                                                    cidx, lam, na);
        const float z0 = st0.zr;
        const float blo = st0.blo, bhi = st0.bhi;
        const bool bad_all = st0.bad_all;
        const float tau = L.tol * st0.Dscale;
        const float tau2 = tau * tau;
        __syncthreads();   // flags are reset by the next pop

        int iters = 0, flags = EM_MAXITER, restarts = 0;
        float rp2 = 0.0f, rd2 = 0.0f;
        float zr = z0;   // z^t of the owned coordinate (0 on lanes without one)
        if (bad_all) {
            flags = EM_BAD_INPUT;
        } else {
            const float mu = L.mu;
            const float inv_mu = 1.0f / mu;
            float vld[M];   // 1 for slots holding a point (their x_k - z_hat enter the residual)
#pragma unroll
            for (int q = 0; q < M; ++q) {
                vld[q] = (lam[q] >= 0.0f) ? 1.0f : 0.0f;
                lam[q] = (lam[q] >= 0.0f) ? lam[q] * inv_mu : 0.0f;
            }
            float e[M][NJ], ep[M][NJ];   // e^{t-1}, e^{t-2}; e holds v during a sweep
#pragma unroll
            for (int q = 0; q < M; ++q)
#pragma unroll
                for (int jj = 0; jj < NJ; ++jj) {
                    e[q][jj] = 0.0f;
                    ep[q][jj] = 0.0f;
                }
            const float fn = (float)n;
            const float inv_n = 1.0f / fn;
            const float inv_d = 1.0f / (float)d;
            const float inv_nd = 1.0f / (fn * (float)d);
            // the owned coordinate's d-vector state (lanes without one hold 0)
            float Cr = z0;        // C of this sweep
            float zh = z0;        // z_hat^t
            float zhp = z0;       // z_hat^{t-1}
            float ae = 1.0f, ap = 0.0f;   // coefficients of e and e_prev in v
            float alpha = 1.0f, c_prev = INFINITY;
            const float eta_g = L.fast_eta * (1.0f - 0x1p-16f);
            const int max_iter = L.max_iter;
            bool done = false;
            for (int t = 1; t <= max_iter; ++t) {
                // ---- pass 1: v = C + a_e e + a_p e_prev, partial ||v - a||^2;
                // e_prev <- e, e <- v
                float nrm[M];
#pragma unroll
                for (int q = 0; q < M; ++q) nrm[q] = kNu2Floor;
#pragma unroll
                for (int jj = 0; jj < NJ; ++jj) {
                    const float c = cv[jj];
#pragma unroll
                    for (int q = 0; q < M; ++q) {
                        const float v = fmaf(ap, ep[q][jj], fmaf(ae, e[q][jj], c));
                        ep[q][jj] = e[q][jj];
                        e[q][jj] = v;
                        const float dl = v + na[q][jj];
                        nrm[q] = fmaf(dl, dl, nrm[q]);
                    }
                }
                if constexpr (WC > 1) {
                    float *X = xn + (t & 1) * WC * M * 64;
#pragma unroll
                    for (int q = 0; q < M; ++q) X[(cw * M + q) * 64 + lane] = nrm[q];
                    __syncthreads();
#pragma unroll
                    for (int q = 0; q < M; ++q) {
                        float sum = X[q * 64 + lane];
#pragma unroll
                        for (int w = 1; w < WC; ++w) sum += X[(w * M + q) * 64 + lane];
                        nrm[q] = sum;
                    }
                }
                float s[M];
#pragma unroll
                for (int q = 0; q < M; ++q) s[q] = shrink(nrm[q], lam[q]);
                // ---- pass 2: E = sum_k s (v - a)
                float acc[NJ];
#pragma unroll
                for (int jj = 0; jj < NJ; ++jj) {
                    float ac = 0.0f;
#pragma unroll
                    for (int q = 0; q < M; ++q) ac = fmaf(s[q], e[q][jj] + na[q][jj], ac);
                    acc[jj] = ac;
                }
                // ---- z = P_C(z_hat - E / n) on the owned coordinate, to the wave
                const float Ev = reduce_scatter_full<NJ>(acc, lane, holds);
                const float zn = own ? clampf(fmaf(-Ev, inv_n, zh), blo, bhi) : 0.0f;
                zv[cidx] = zn;
                // ---- pass 3: e <- s (v - a), lane sums of ||x_k - z||^2 with
                // x_k - z = (v - z) - e
                float rq[M];
#pragma unroll
                for (int q = 0; q < M; ++q) rq[q] = 0.0f;
#pragma unroll
                for (int jj = 0; jj < NJ; ++jj) {
                    const float zj = zv[jj];
#pragma unroll
                    for (int q = 0; q < M; ++q) {
                        const float v = e[q][jj];
                        const float en = s[q] * (v + na[q][jj]);
                        const float y = (v - zj) - en;
                        rq[q] = fmaf(y, y, rq[q]);
                        e[q][jj] = en;
                    }
                }
                float rpl = 0.0f;
#pragma unroll
                for (int q = 0; q < M; ++q) rpl = fmaf(vld[q], rq[q], rpl);
#pragma unroll
                for (int q = 0; q < M; ++q)
#pragma unroll
                    for (int jj = 0; jj < NJ; ++jj) {
                        asm volatile("" : "+v"(e[q][jj]));
                        asm volatile("" : "+v"(ep[q][jj]));
                    }
                // ---- the three residual sums of the workgroup
                const float dz = zn - zr;       // z^t - z^{t-1}
                const float dh = zh - zn;       // z_hat - z
                const float sp_l = rpl;
                float sd = readfirstlane(wave_sum(dz * dz));
                float sh = readfirstlane(wave_sum(dh * dh));
                float sp = readfirstlane(wave_sum(sp_l));
                if constexpr (WC > 1) {
                    float *XS = xs + (t & 1) * WC * 4;
                    if (lane == 0) {
                        XS[cw * 4 + 0] = sd;
                        XS[cw * 4 + 1] = sh;
                        XS[cw * 4 + 2] = sp;
                    }
                    __syncthreads();
                    sd = XS[0];
                    sh = XS[1];
                    sp = XS[2];
#pragma unroll
                    for (int w = 1; w < WC; ++w) {
                        sd += XS[w * 4 + 0];
                        sh += XS[w * 4 + 1];
                        sp += XS[w * 4 + 2];
                    }
                    sd = readfirstlane(sd);
                    sh = readfirstlane(sh);
                    sp = readfirstlane(sp);
                }
                rd2 = sd * inv_d;
                rp2 = fmaxf(sp, 0.0f) * inv_nd;
                iters = t;
                if (uniform(tau2 > 0.0f && rp2 <= tau2 && rd2 <= tau2)) {
                    flags = EM_CONVERGED;
                    zr = zn;
                    done = true;
                    break;
                }
                if (t == max_iter) {   // no sweep follows: the decision would change nothing
                    zr = zn;
                    break;
                }
                // ---- momentum or restart (the same decision in every wave)
                const float cval = mu * (fmaxf(sp, 0.0f) + fn * sh);
                float zh_next, C_next;
                if (uniform(cval < eta_g * c_prev)) {
                    const float an = 0.5f * (1.0f + sqrtf(1.0f + 4.0f * alpha * alpha));
                    const float beta = (alpha - 1.0f) / an;
                    zh_next = fmaf(beta, zn - zr, zn);
                    C_next = zh_next - (1.0f + beta) * (zh - zn) + beta * (zhp - zr);
                    ae = 1.0f + beta;
                    ap = -beta;
                    alpha = an;
                    c_prev = cval;
                } else {
                    zh_next = zr;
                    C_next = 2.0f * zr - zhp;
                    ae = 0.0f;
                    ap = 1.0f;
                    alpha = 1.0f;
                    c_prev = c_prev / L.fast_eta;
                    ++restarts;
                }
                if (!own) {
                    zh_next = 0.0f;
                    C_next = 0.0f;
                }
                zhp = zh;
                zh = zh_next;
                Cr = C_next;
                zr = zn;
                cv[cidx] = Cr;
            }
            (void)done;
        }
        // ---- z and the statistics (restarts in the flags word)
        if (own) Z[cj] = bad_all ? __builtin_nanf("") : zr;
        if (cw == 0 && lane == 0 && L.stats != nullptr) {
            em_stats_t st;
            st.iters = bad_all ? 0 : iters;
            st.flags = bad_all ? flags : (flags | (min(restarts, kMaxRestartCountBatch) << EM_RESTART_SHIFT));
            st.r_pri = bad_all ? 0.0f : sqrtf(rp2);
            st.r_dual = bad_all ? 0.0f : sqrtf(rd2);
            L.stats[b] = st;
        }
    }
}

}  // namespace emx
