// Structures shared by the host runtime and the kernels (not part of the ABI).
#pragma once

#include <stdint.h>

#include "../../include/emx.h"

namespace emx {

constexpr int kMaxImagesPerLaunch = 16;

constexpr int kSideStreams = 3;   // with the caller's stream: four concurrent class launches

// One image of a denoising launch (passed by value inside the kernel arguments).
struct NlemImageDesc {
    const void *img;      // H x W, FP32 or FP16
    float *out;           // H x W
    em_stats_t *stats;    // nullable, H x W
    int32_t H, W;
    int32_t R;            // window radius
    int32_t is_f16;
    float k_h;            // log2(e) / h^2: w = exp2(-dist^2 * k_h)
    int32_t pad_;
};

struct NlemLaunch {
    NlemImageDesc img[kMaxImagesPerLaunch];
    int64_t prefix[kMaxImagesPerLaunch + 1];  // pixel prefix sums
    int32_t count;
    int32_t max_iter;
    float inv_mu;
    float lo, hi;
    float tau;       // tol * (hi - lo); 0 = fixed iteration count
    float tau_arm;   // primal residual evaluated after an iteration with r_dual <= tau_arm
    int32_t check_mask;     // ... and only on iterations t with (t & check_mask) == 0 (or the last one)
    int32_t init_nlm;       // 1: start from the NLM patch instead of the noisy patch
    float eps;              // IRLS surrogate parameter
    unsigned int *counter;  // work-queue head, zeroed before the launch
    const int32_t *order;   // queue position -> pixel (prefix-based index); null: identity
    int32_t chunk;          // queue positions taken per atomic (>= 1)
};

// Longest-first queue order (nlem_order.hip): pixels by decreasing patch
// standard deviation, counting-sorted over kOrderBuckets buckets.
constexpr int kOrderBuckets = 256;

struct NlemOrderArgs {
    NlemLaunch L;          // the images (descriptors and pixel prefix sums)
    int32_t pr;            // patch radius
    float scale;           // 2 kOrderBuckets / (hi - lo)
    int32_t *order;        // [total] queue position -> pixel
    uint8_t *bucket;       // [total] bucket of each pixel
    unsigned int *cnt;     // counts, offsets and fill cursors (3 kOrderBuckets + 1)
};

struct OrderKernel {
    const void *fn;        // takes one NlemOrderArgs by value
    unsigned grid, block;
};

// Device bytes of the order scratch for `total` pixels.
size_t nlem_order_bytes(int64_t total);
// Arguments with the scratch laid out in `ws` (nlem_order_bytes(total) bytes).
NlemOrderArgs nlem_order_args(const NlemLaunch &L, int pr, float lo, float hi, void *ws);
// The kernels to run in order on one stream: clear, count, scatter.
constexpr int kOrderKernels = 3;
void nlem_order_kernels(const NlemOrderArgs &A, int num_cus, OrderKernel (&k)[kOrderKernels]);

}  // namespace emx
