// Compiled NLEM shapes for patch radius 3 (d = 49): EM-ADMM for every
// listed coordinate-wave count (one wave only at m = 1, where the 49
// coordinates of one point fit a wave's registers), IRLS for one count.
#include "nlem_kernel.hpp"
#include "nlem_table.hpp"

namespace emx {

template <int PR, int M, int WC, int SOLVER>
static NlemKernelInfo info() {
    return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<PR, M, WC, SOLVER>), 64 * WC};
}

NlemKernelInfo nlem_kernels_pr3(int m, int wc, int solver) {
    if (solver == 0) {
        switch (m * 8 + wc) {
            case 9: return info<3, 1, 1, 0>();
            case 10: return info<3, 1, 2, 0>();
            case 11: return info<3, 1, 3, 0>();
            case 12: return info<3, 1, 4, 0>();
            case 18: return info<3, 2, 2, 0>();
            case 19: return info<3, 2, 3, 0>();
            case 20: return info<3, 2, 4, 0>();
            case 26: return info<3, 3, 2, 0>();
            case 27: return info<3, 3, 3, 0>();
            case 28: return info<3, 3, 4, 0>();
            case 34: return info<3, 4, 2, 0>();
            case 35: return info<3, 4, 3, 0>();
            case 36: return info<3, 4, 4, 0>();
            case 42: return info<3, 5, 2, 0>();
            case 43: return info<3, 5, 3, 0>();
            case 44: return info<3, 5, 4, 0>();
            case 50: return info<3, 6, 2, 0>();
            case 51: return info<3, 6, 3, 0>();
            case 52: return info<3, 6, 4, 0>();
            case 58: return info<3, 7, 2, 0>();
            case 59: return info<3, 7, 3, 0>();
            case 60: return info<3, 7, 4, 0>();
        }
    } else if (solver == 1) {
        switch (m * 8 + wc) {
            case 10: return info<3, 1, 2, 1>();
            case 18: return info<3, 2, 2, 1>();
            case 26: return info<3, 3, 2, 1>();
            case 34: return info<3, 4, 2, 1>();
            case 44: return info<3, 5, 4, 1>();
            case 52: return info<3, 6, 4, 1>();
            case 60: return info<3, 7, 4, 1>();
        }
    }
    return NlemKernelInfo{nullptr, 0};
}

}  // namespace emx
