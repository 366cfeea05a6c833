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

// Default coordinate-wave count per (patch radius, points per lane, solver),
// from timing every compiled candidate on MI355X (480x640 image, sigma 20,
// h 200, tol 1e-4, window radius 2..10, longest-first queue; the 256x256
// d = 49, n <= 441 image: 2 waves 3.09 ms, 3 waves 4.12 ms, 4 waves 3.02 ms).
// EM-ADMM, patch radius 2: one wave (with the row mapping at R = 7 one wave
// took 3.95 ms against 4.42 for two); patch radius 3: one wave at m = 1
// (23.3 against 21.9 TFLOP/s at R = 3), two waves, three at m = 5 (35.0
// against 32.3), four at m = 7.  IRLS is compiled for one count per shape
// (the rule below).
inline int nlem_default_wc(int pr, int m, int solver = 0) {
    if (pr <= 1) return 1;
    if (solver == 1) return (pr == 2) ? ((m <= 3) ? 1 : 2) : ((m >= 5) ? 4 : 2);
    if (pr == 2) return 1;
    return (m == 7) ? 4 : (m == 5) ? 3 : (m == 1) ? 1 : 2;
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
