// Compiled NLEM shapes for patch radius 0 (d = 1): EM-ADMM for every
// listed coordinate-wave count, IRLS for the default one.
#include "nlem_kernel.hpp"
#include "nlem_table.hpp"

namespace emx {

template <int PR, int M, int WC, int SOLVER>
static NlemKernelInfo info() {
    return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<PR, M, WC, SOLVER>), 64 * WC};
}

NlemKernelInfo nlem_kernels_pr0(int m, int wc, int solver) {
    if (solver == 0) {
        switch (m * 8 + wc) {
            case 9: return info<0, 1, 1, 0>();
            case 17: return info<0, 2, 1, 0>();
            case 25: return info<0, 3, 1, 0>();
            case 33: return info<0, 4, 1, 0>();
            case 41: return info<0, 5, 1, 0>();
            case 49: return info<0, 6, 1, 0>();
            case 57: return info<0, 7, 1, 0>();
        }
    } else if (solver == 1) {
        switch (m * 8 + wc) {
            case 9: return info<0, 1, 1, 1>();
            case 17: return info<0, 2, 1, 1>();
            case 25: return info<0, 3, 1, 1>();
            case 33: return info<0, 4, 1, 1>();
            case 41: return info<0, 5, 1, 1>();
            case 49: return info<0, 6, 1, 1>();
            case 57: return info<0, 7, 1, 1>();
        }
    }
    return NlemKernelInfo{nullptr, 0};
}

}  // namespace emx
