// Compiled NLEM shapes for patch radius 2 (d = 25): EM-ADMM for every
// listed coordinate-wave count, IRLS for the default one.
#include "nlem_kernel.hpp"
#include "nlem_table.hpp"

namespace emx {

template <int PR, int M, int WC, int SOLVER>
static NlemKernelInfo info() {
    return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<PR, M, WC, SOLVER>), 64 * WC};
}

NlemKernelInfo nlem_kernels_pr2(int m, int wc, int solver) {
    if (solver == 0) {
        switch (m * 8 + wc) {
            case 9: return info<2, 1, 1, 0>();
            case 10: return info<2, 1, 2, 0>();
            case 11: return info<2, 1, 3, 0>();
            case 17: return info<2, 2, 1, 0>();
            case 18: return info<2, 2, 2, 0>();
            case 19: return info<2, 2, 3, 0>();
            case 25: return info<2, 3, 1, 0>();
            case 26: return info<2, 3, 2, 0>();
            case 27: return info<2, 3, 3, 0>();
            case 33: return info<2, 4, 1, 0>();
            case 34: return info<2, 4, 2, 0>();
            case 35: return info<2, 4, 3, 0>();
            case 41: return info<2, 5, 1, 0>();
            case 42: return info<2, 5, 2, 0>();
            case 43: return info<2, 5, 3, 0>();
            case 49: return info<2, 6, 1, 0>();
            case 50: return info<2, 6, 2, 0>();
            case 51: return info<2, 6, 3, 0>();
            case 57: return info<2, 7, 1, 0>();
            case 58: return info<2, 7, 2, 0>();
            case 59: return info<2, 7, 3, 0>();
        }
    } else if (solver == 1) {
        switch (m * 8 + wc) {
            case 9: return info<2, 1, 1, 1>();
            case 17: return info<2, 2, 1, 1>();
            case 25: return info<2, 3, 1, 1>();
            case 34: return info<2, 4, 2, 1>();
            case 42: return info<2, 5, 2, 1>();
            case 50: return info<2, 6, 2, 1>();
            case 58: return info<2, 7, 2, 1>();
        }
    }
    return NlemKernelInfo{nullptr, 0};
}

}  // namespace emx
