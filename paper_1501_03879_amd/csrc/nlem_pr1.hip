// Compiled NLEM shapes for patch radius 1 (d = 9).
#include "nlem_kernel.hpp"
#include "nlem_table.hpp"

namespace emx {

NlemKernelInfo nlem_kernels_pr1(int m, int wc) {
    switch (m * 8 + wc) {
        case 9: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<1, 1, 1>), 64};
        case 17: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<1, 2, 1>), 64};
        case 25: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<1, 3, 1>), 64};
        case 33: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<1, 4, 1>), 64};
        case 41: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<1, 5, 1>), 64};
        case 49: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<1, 6, 1>), 64};
        case 57: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<1, 7, 1>), 64};
        default: return NlemKernelInfo{nullptr, 0};
    }
}

}  // namespace emx
