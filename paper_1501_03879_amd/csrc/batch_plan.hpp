// Batch-plan structures shared by the host runtime and the batched solver
// (not part of the ABI).
#pragma once

#include <stdint.h>

namespace emx {

// Sliced classes of the batched fixed-penalty EM-ADMM (batch_wide.hpp): d in
// (16, 64] and n <= 448 in 13-coordinate slices over WC = ceil(d / 13) in
// [2, 5] waves, M = ceil(n / 64) in [1, 7] points per lane; sliced class
// k = 7 (WC - 2) + M - 1 (the bit of em_batch_plan_t.generic_classes).
constexpr int kWideNJ = 13;
constexpr int kWideMaxM = 7;
constexpr int kWideMinWC = 2, kWideMaxWC = 5;
constexpr int kNumWideClasses = (kWideMaxWC - kWideMinWC + 1) * kWideMaxM;

// The batch plan applied to one call (em_batch_plan_t without its source):
// sliced classes routed to the generic kernels, the arm factor, the
// residual-check interval and the host-counts dispatch.
struct BatchPlanView {
    uint64_t generic_mask;
    float arm;
    int check;        // residual-check interval (1, 2, 4 or 8)
    int host_counts;  // read the class counts back and launch only populated classes
};

}  // namespace emx
