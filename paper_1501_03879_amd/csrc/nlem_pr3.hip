// Compiled NLEM shapes for patch radius 3 (d = 49).
#include "nlem_kernel.hpp"
#include "nlem_table.hpp"

namespace emx {

NlemKernelInfo nlem_kernels_pr3(int m, int wc) {
    switch (m * 8 + wc) {
        case 10: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<3, 1, 2>), 128};
        case 11: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<3, 1, 3>), 192};
        case 12: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<3, 1, 4>), 256};
        case 18: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<3, 2, 2>), 128};
        case 19: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<3, 2, 3>), 192};
        case 20: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<3, 2, 4>), 256};
        case 26: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<3, 3, 2>), 128};
        case 27: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<3, 3, 3>), 192};
        case 28: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<3, 3, 4>), 256};
        case 34: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<3, 4, 2>), 128};
        case 35: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<3, 4, 3>), 192};
        case 36: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<3, 4, 4>), 256};
        case 42: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<3, 5, 2>), 128};
        case 43: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<3, 5, 3>), 192};
        case 44: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<3, 5, 4>), 256};
        case 50: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<3, 6, 2>), 128};
        case 51: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<3, 6, 3>), 192};
        case 52: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<3, 6, 4>), 256};
        case 58: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<3, 7, 2>), 128};
        case 59: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<3, 7, 3>), 192};
        case 60: return NlemKernelInfo{reinterpret_cast<const void *>(&nlem_solve_kernel<3, 7, 4>), 256};
        default: return NlemKernelInfo{nullptr, 0};
    }
}

}  // namespace emx
