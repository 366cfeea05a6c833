/*
 * A C client of libemx: Non-Local Euclidean Medians (Section 3 of
 * arXiv:1501.03879) on a raw FP32 image through the C ABI of include/emx.h
 * alone, with the HIP runtime for device memory and a stream (no Python, no
 * torch).
 *
 *   nlem_client IN.f32 H W PATCH_RADIUS WINDOW_RADIUS H_PARAM LO HI RHO MAX_ITER TOL OUT.f32 [STATS.bin]
 *
 * IN.f32: H x W float32, row-major.  OUT.f32: the denoised H x W image.
 * STATS.bin: the H x W em_stats_t records.  Prints the mean iteration count.
 * Exit status: 0 on success, 1 usage, 2 I/O, 3 HIP error, 4 library error.
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include "emx.h"

#define HIP_OR(code, call)                                                        \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess) {                                                   \
            fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));            \
            return (code);                                                        \
        }                                                                         \
    } while (0)

#define EMX_OR(h, call)                                                           \
    do {                                                                          \
        em_status_t s_ = (call);                                                  \
        if (s_ != EM_OK) {                                                        \
            fprintf(stderr, "%s: %s %s\n", #call, em_status_string(s_),           \
                    (h) ? em_last_error(h) : "");                                 \
            return 4;                                                             \
        }                                                                         \
    } while (0)

static int read_all(const char *path, void *buf, size_t bytes) {
    FILE *f = fopen(path, "rb");
    if (!f) return 0;
    const size_t got = fread(buf, 1, bytes, f);
    fclose(f);
    return got == bytes;
}

static int write_all(const char *path, const void *buf, size_t bytes) {
    FILE *f = fopen(path, "wb");
    if (!f) return 0;
    const size_t put = fwrite(buf, 1, bytes, f);
    return (fclose(f) == 0) && put == bytes;
}

static int run(int argc, char **argv, float *img, float *out, em_stats_t *st, size_t npix) {
    const int H = atoi(argv[2]), W = atoi(argv[3]);
    const int pr = atoi(argv[4]), wr = atoi(argv[5]);
    const float hp = (float)atof(argv[6]), lo = (float)atof(argv[7]), hi = (float)atof(argv[8]);
    const float rho = (float)atof(argv[9]);
    const int max_iter = atoi(argv[10]);
    const float tol = (float)atof(argv[11]);
    if (!read_all(argv[1], img, npix * sizeof(float))) {
        fprintf(stderr, "cannot read %zu floats from %s\n", npix, argv[1]);
        return 2;
    }
    em_handle_t h = NULL;
    EMX_OR(h, em_create(&h, 0));
    void *dimg = NULL, *dout = NULL, *dst = NULL;
    hipStream_t s = NULL;
    HIP_OR(3, hipStreamCreate(&s));
    HIP_OR(3, hipMalloc(&dimg, npix * sizeof(float)));
    HIP_OR(3, hipMalloc(&dout, npix * sizeof(float)));
    HIP_OR(3, hipMalloc(&dst, npix * sizeof(em_stats_t)));
    HIP_OR(3, hipMemcpyAsync(dimg, img, npix * sizeof(float), hipMemcpyHostToDevice, s));
    EMX_OR(h, nlem_denoise(h, s, dimg, 0, H, W, pr, wr, hp, lo, hi, rho, max_iter, tol, (float *)dout,
                           (em_stats_t *)dst));
    EMX_OR(h, em_sync(h, s));
    HIP_OR(3, hipMemcpyAsync(out, dout, npix * sizeof(float), hipMemcpyDeviceToHost, s));
    HIP_OR(3, hipMemcpyAsync(st, dst, npix * sizeof(em_stats_t), hipMemcpyDeviceToHost, s));
    HIP_OR(3, hipStreamSynchronize(s));
    double iters = 0.0;
    for (size_t i = 0; i < npix; ++i) iters += st[i].iters;
    printf("nlem_client: %dx%d r=%d R=%d, mean iterations %.3f\n", H, W, pr, wr, iters / (double)npix);
    HIP_OR(3, hipFree(dimg));
    HIP_OR(3, hipFree(dout));
    HIP_OR(3, hipFree(dst));
    HIP_OR(3, hipStreamDestroy(s));
    EMX_OR(NULL, em_destroy(h));
    if (!write_all(argv[12], out, npix * sizeof(float))) return 2;
    if (argc > 13 && !write_all(argv[13], st, npix * sizeof(em_stats_t))) return 2;
    return 0;
}

int main(int argc, char **argv) {
    if (argc < 13) {
        fprintf(stderr,
                "usage: %s IN.f32 H W PATCH_RADIUS WINDOW_RADIUS H_PARAM LO HI RHO MAX_ITER TOL OUT.f32 "
                "[STATS.bin]\n", argv[0]);
        return 1;
    }
    const long H = atol(argv[2]), W = atol(argv[3]);
    if (H < 1 || W < 1 || H > 65536 || W > 65536) {
        fprintf(stderr, "bad image size\n");
        return 1;
    }
    const size_t npix = (size_t)H * (size_t)W;
    float *img = (float *)malloc(npix * sizeof(float));
    float *out = (float *)malloc(npix * sizeof(float));
    em_stats_t *st = (em_stats_t *)malloc(npix * sizeof(em_stats_t));
    int rc = 2;
    if (img && out && st) rc = run(argc, argv, img, out, st, npix);
    free(img);
    free(out);
    free(st);
    return rc;
}
