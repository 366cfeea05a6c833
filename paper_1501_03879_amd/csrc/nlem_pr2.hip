// Compiled NLEM shapes for patch radius 2 (d = 25).
#include "nlem_kernel.hpp"
#include "nlem_table.hpp"

namespace emx {

NlemKernelInfo nlem_kernels_pr2(int m, int wc) {
    switch (m * 8 + wc) {
        case 9: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<2, 1, 1>), 64};
        case 10: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<2, 1, 2>), 128};
        case 11: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<2, 1, 3>), 192};
        case 17: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<2, 2, 1>), 64};
        case 18: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<2, 2, 2>), 128};
        case 19: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<2, 2, 3>), 192};
        case 25: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<2, 3, 1>), 64};
        case 26: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<2, 3, 2>), 128};
        case 27: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<2, 3, 3>), 192};
        case 33: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<2, 4, 1>), 64};
        case 34: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<2, 4, 2>), 128};
        case 35: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<2, 4, 3>), 192};
        case 41: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<2, 5, 1>), 64};
        case 42: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<2, 5, 2>), 128};
        case 43: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<2, 5, 3>), 192};
        case 49: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<2, 6, 1>), 64};
        case 50: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<2, 6, 2>), 128};
        case 51: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<2, 6, 3>), 192};
        case 57: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<2, 7, 1>), 64};
        case 58: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<2, 7, 2>), 128};
        case 59: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<2, 7, 3>), 192};
        default: return NlemKernelInfo{nullptr, 0};
    }
}

}  // namespace emx
