// Longest-first order of the NLEM work queue.
//
// The persistent NLEM kernel pops pixels from a queue; a pixel whose solve
// needs many iterations and is popped late keeps a few workgroups busy after
// the rest of the chip has run dry.  The iteration count grows with the
// spread of the pixel's noisy patch (its standard deviation over the patch
// predicts log(iterations) with correlation 0.89 on the 256x256, sigma 20
// image with 7x7 patches), so the queue is ordered by decreasing patch
// standard deviation: a counting sort over kOrderBuckets buckets of
// std / (hi - lo).  The order only changes which workgroup solves a pixel
// and when; every pixel's arithmetic is the same.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "em_device.hpp"
#include "emx_internal.hpp"

namespace emx {

// counts [0, K), (unused) [K, 2K + 1), fill [2K + 1, 3K + 1)
static constexpr int kCnt = 3 * kOrderBuckets + 1;
// largest patch radius (the host rejects larger ones before any launch)
static constexpr int kOrderMaxPr = EM_MAX_PATCH_RADIUS;

// Zeroes the bucket counters and the NLEM launch's work-queue head (the
// launch that follows on the same stream needs no reset of its own).
__global__ void nlem_order_clear(NlemOrderArgs A) {
    for (int i = threadIdx.x; i < kCnt; i += blockDim.x) A.cnt[i] = 0u;
    if (threadIdx.x == 0) *A.L.counter = 0u;
}

// Sums of the values and of their squares over the PS x PS patch of pixel
// (iy, ix), reflected at the borders.  The loads are unrolled and all go out
// before the first is used; the sums run in row-major order.
template <int PS>
__device__ __forceinline__ void patch_sums(const NlemImageDesc &I, int iy, int ix, float &s1, float &s2) {
    constexpr int PR = PS / 2;
    int64_t ro[PS];
    int co[PS];
#pragma unroll
    for (int k = 0; k < PS; ++k) {
        ro[k] = (int64_t)reflect_idx(iy - PR + k, I.H) * I.W;
        co[k] = reflect_idx(ix - PR + k, I.W);
    }
    float v[PS * PS];
    if (I.is_f16) {
        const __half *f16 = static_cast<const __half *>(I.img);
#pragma unroll
        for (int k = 0; k < PS * PS; ++k) v[k] = __half2float(f16[ro[k / PS] + co[k % PS]]);
    } else {
        const float *f32 = static_cast<const float *>(I.img);
#pragma unroll
        for (int k = 0; k < PS * PS; ++k) v[k] = f32[ro[k / PS] + co[k % PS]];
    }
    s1 = 0.0f;
    s2 = 0.0f;
#pragma unroll
    for (int k = 0; k < PS * PS; ++k) {
        s1 += v[k];
        s2 = fmaf(v[k], v[k], s2);
    }
}

// Bucket of every pixel (stored) and the per-bucket counts.
template <int PS>
__device__ __forceinline__ void order_count(const NlemOrderArgs &A) {
    __shared__ unsigned int hist[kOrderBuckets];
    for (int i = threadIdx.x; i < kOrderBuckets; i += blockDim.x) hist[i] = 0u;
    __syncthreads();
    const NlemLaunch &L = A.L;
    const int64_t total = L.prefix[L.count];
    const float inv_d = 1.0f / (float)(PS * PS);
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        int b = 0;
        while (b + 1 < L.count && q >= L.prefix[b + 1]) ++b;
        const NlemImageDesc &I = L.img[b];
        const int pix = (int)(q - L.prefix[b]);
        const int iy = pix / I.W, ix = pix - (pix / I.W) * I.W;
        // one pass: the key only orders the queue, so the rounding of
        // E[v^2] - E[v]^2 in FP32 does not matter
        float s1, s2;
        patch_sums<PS>(I, iy, ix, s1, s2);
        const float m = s1 * inv_d;
        const float var = fmaxf(fmaf(-m, m, s2 * inv_d), 0.0f);
        const float key = sqrtf(var) * A.scale;   // std / (hi - lo) * 2K, in [0, K]
        const int bk = (key >= 0.0f) ? min((int)key, kOrderBuckets - 1) : kOrderBuckets - 1;  // NaN: first
        A.bucket[q] = (uint8_t)bk;
        atomicAdd(&hist[bk], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kOrderBuckets; i += blockDim.x)
        if (hist[i]) atomicAdd(&A.cnt[i], hist[i]);
}

__global__ __launch_bounds__(256) void nlem_order_count(NlemOrderArgs A) {
    static_assert(kOrderMaxPr == 3, "one case per patch radius");
    switch (A.pr) {
        case 0: order_count<1>(A); break;
        case 1: order_count<3>(A); break;
        case 2: order_count<5>(A); break;
        default: order_count<7>(A); break;
    }
}

// Every block first turns the bucket counts into offsets with the largest
// bucket first (an exclusive scan over the buckets in decreasing order, one
// bucket per thread, repeated by each block: cheaper than a launch of its
// own).  Then it takes 256 pixels at a time: ranks within the block come from
// LDS atomics, and one global atomic per (block, bucket) reserves the range.
__global__ __launch_bounds__(kOrderBuckets) void nlem_order_scatter(NlemOrderArgs A) {
    static_assert(kOrderBuckets == 256, "one bucket per thread of a 256-thread block");
    __shared__ unsigned int lcnt[kOrderBuckets];
    __shared__ unsigned int lbase[kOrderBuckets];
    __shared__ unsigned int offs[kOrderBuckets];
    const NlemLaunch &L = A.L;
    const int64_t total = L.prefix[L.count];
    unsigned int *fill = A.cnt + 2 * kOrderBuckets + 1;
    {
        const int i = threadIdx.x;             // position in decreasing bucket order
        const int k = kOrderBuckets - 1 - i;   // its bucket
        const unsigned int c = A.cnt[k];
        lcnt[i] = c;
        __syncthreads();
        for (int off = 1; off < kOrderBuckets; off <<= 1) {   // inclusive Hillis-Steele scan
            const unsigned int add = (i >= off) ? lcnt[i - off] : 0u;
            __syncthreads();
            lcnt[i] += add;
            __syncthreads();
        }
        offs[k] = lcnt[i] - c;
        __syncthreads();
    }
    for (int64_t q0 = (int64_t)blockIdx.x * blockDim.x; q0 < total; q0 += (int64_t)gridDim.x * blockDim.x) {
        for (int i = threadIdx.x; i < kOrderBuckets; i += blockDim.x) lcnt[i] = 0u;
        __syncthreads();
        const int64_t q = q0 + threadIdx.x;
        const bool valid = q < total;
        const int bk = valid ? A.bucket[q] : 0;
        const unsigned int rank = valid ? atomicAdd(&lcnt[bk], 1u) : 0u;
        __syncthreads();
        for (int i = threadIdx.x; i < kOrderBuckets; i += blockDim.x)
            lbase[i] = lcnt[i] ? atomicAdd(&fill[i], lcnt[i]) : 0u;
        __syncthreads();
        if (valid) A.order[offs[bk] + lbase[bk] + rank] = (int32_t)q;
        __syncthreads();   // lcnt and lbase are reused by the next chunk
    }
}

size_t nlem_order_bytes(int64_t total) {
    const size_t a = ((size_t)total * sizeof(int32_t) + 255) & ~(size_t)255;
    const size_t b = ((size_t)total + 255) & ~(size_t)255;
    return (a + b + (size_t)kCnt * sizeof(unsigned int) + 255) & ~(size_t)255;
}

NlemOrderArgs nlem_order_args(const NlemLaunch &L, int pr, float lo, float hi, void *ws) {
    NlemOrderArgs A;
    A.L = L;
    A.pr = pr;
    const float range = (hi > lo && hi - lo <= 3.0e38f) ? hi - lo : 1.0f;
    A.scale = (float)(2 * kOrderBuckets) / range;
    const int64_t total = L.prefix[L.count];
    char *p = static_cast<char *>(ws);
    A.order = reinterpret_cast<int32_t *>(p);
    p += ((size_t)total * sizeof(int32_t) + 255) & ~(size_t)255;
    A.bucket = reinterpret_cast<uint8_t *>(p);
    p += ((size_t)total + 255) & ~(size_t)255;
    A.cnt = reinterpret_cast<unsigned int *>(p);
    return A;
}

void nlem_order_kernels(const NlemOrderArgs &A, int num_cus, OrderKernel (&k)[kOrderKernels]) {
    const int64_t total = A.L.prefix[A.L.count];
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 4LL * num_cus));
    k[0] = OrderKernel{reinterpret_cast<const void *>(&nlem_order_clear), 1, 256};
    k[1] = OrderKernel{reinterpret_cast<const void *>(&nlem_order_count), grid, 256};
    k[2] = OrderKernel{reinterpret_cast<const void *>(&nlem_order_scatter), grid, kOrderBuckets};
}

}  // namespace emx
