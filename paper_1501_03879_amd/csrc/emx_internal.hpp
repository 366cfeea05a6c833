// Structures shared by the host runtime and the kernels (not part of the ABI).
#pragma once

#include <stdint.h>

#include "../../include/emx.h"

namespace emx {

constexpr int kMaxImagesPerLaunch = 16;

// Sliced classes of the batched fixed-penalty EM-ADMM (batch_wide.hpp): d in
// (16, 64] and n <= 448 in 13-coordinate slices over WC = ceil(d / 13) in
// [2, 5] waves, M = ceil(n / 64) in [1, 7] points per lane; sliced class
// k = 7 (WC - 2) + M - 1 (the bit of em_batch_plan_t.generic_classes).
constexpr int kWideNJ = 13;
constexpr int kWideMaxM = 7;
constexpr int kWideMinWC = 2, kWideMaxWC = 5;
constexpr int kNumWideClasses = (kWideMaxWC - kWideMinWC + 1) * kWideMaxM;

// The batch plan applied to one call (em_batch_plan_t without its source):
// sliced classes routed to the generic kernels, the arm factor and the
// residual-check interval.
struct BatchPlanView {
    uint64_t generic_mask;
    float arm;
    int check;        // residual-check interval (1, 2, 4 or 8)
    int host_counts;  // read the class counts back and launch only populated classes
};
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
