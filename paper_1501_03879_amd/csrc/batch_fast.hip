// Shape classes of the batched accelerated ADMM: 8-coordinate slices over WC
// in {1, 2, 4, 8} waves, M in {1, 2, 4, 8} points per lane.
#include "batch_fast.hpp"

namespace emx {

template <int C>
constexpr ClassKernel fast_kernel() {
    constexpr int wc = 1 << (C / 4);
    constexpr int m = 1 << (C % 4);
    return ClassKernel{reinterpret_cast<const void *>(&batch_fast_kernel<m, wc>), 64 * wc};
}

template <int... C>
const ClassKernel *fast_table(std::integer_sequence<int, C...>) {
    static const ClassKernel t[kNumFastClasses] = {fast_kernel<C>()...};
    return t;
}

const ClassKernel *batch_fast_table() { return fast_table(std::make_integer_sequence<int, kNumFastClasses>{}); }

}  // namespace emx
