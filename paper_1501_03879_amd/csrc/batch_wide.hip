// Shape classes of the batched EM-ADMM for d in (16, 64] and n <= 448
// (fixed penalty, box): 13-coordinate slices, WC = ceil(d / 13) waves,
// M = ceil(n / 64) points per lane.
#include "batch_wide.hpp"

namespace emx {

// Waves per SIMD the launch bound asks for (its second argument): as many as
// the registers allow: ~26 M VGPRs for the state and points of M points of a
// 13-coordinate slice, 64 / WC for a chunk's staging loads, ~60 for the rest.
constexpr int wide_waves_per_simd(int m, int wc) {
    const int regs = 26 * m + 60 + 64 / wc;
    const int w = 512 / regs;
    return w > 6 ? 6 : (w < 2 ? 2 : w);
}

template <int C>
constexpr ClassKernel wide_kernel() {
    constexpr int wc = kWideMinWC + C / kWideMaxM;
    constexpr int m = 1 + C % kWideMaxM;
    return ClassKernel{
        reinterpret_cast<const void *>(&batch_wide_kernel<kWideNJ, m, wc, wide_waves_per_simd(m, wc)>), 64 * wc};
}

template <int... C>
const ClassKernel *wide_table(std::integer_sequence<int, C...>) {
    static const ClassKernel t[kNumWideClasses] = {wide_kernel<C>()...};
    return t;
}

const ClassKernel *batch_wide_table() { return wide_table(std::make_integer_sequence<int, kNumWideClasses>{}); }

// Kernels of the deferred far-outlier lists (EM-ADMM carrying e, generic
// shapes of batch_kernel.hpp: the carried state takes more registers than the
// sliced shapes have to spare).
const ClassKernel *batch_deferred_table() {
    static const ClassKernel t[kDeferLists] = {class_kernel<7, 5, 0>(), class_kernel<19, 5, 0>()};
    return t;
}

}  // namespace emx
