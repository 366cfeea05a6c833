// Table of compiled NLEM kernel shapes (one translation unit per patch radius).
#pragma once

namespace emx {

struct NlemKernelInfo {
    const void *fn;  // nullptr when the shape is not compiled
    int threads;
};

// m = points per lane (1..7), wc = waves per pixel over the patch coordinates,
// solver 0 = EM-ADMM (every compiled wc), 1 = IRLS (the default wc only)
NlemKernelInfo nlem_kernels_pr0(int m, int wc, int solver);
NlemKernelInfo nlem_kernels_pr1(int m, int wc, int solver);
NlemKernelInfo nlem_kernels_pr2(int m, int wc, int solver);
NlemKernelInfo nlem_kernels_pr3(int m, int wc, int solver);

// Default coordinate-wave count per (patch radius, points per lane), from
// timing the compiled candidates on MI355X (256x256 image, d = 49, n <= 441,
// tol 1e-4: 2 waves 3.09 ms, 3 waves 4.12 ms, 4 waves 3.02 ms per image;
// a 3-wave workgroup leaves wave slots of a CU unused).
inline int nlem_default_wc(int pr, int m) {
    if (pr <= 1) return 1;
    if (pr == 2) return (m <= 3) ? 1 : 2;
    return (m >= 5) ? 4 : 2;
}

inline NlemKernelInfo nlem_kernel(int pr, int m, int wc, int solver) {
    switch (pr) {
        case 0: return nlem_kernels_pr0(m, wc, solver);
        case 1: return nlem_kernels_pr1(m, wc, solver);
        case 2: return nlem_kernels_pr2(m, wc, solver);
        case 3: return nlem_kernels_pr3(m, wc, solver);
    }
    return NlemKernelInfo{nullptr, 0};
}

}  // namespace emx
