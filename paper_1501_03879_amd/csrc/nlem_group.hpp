// Host-side grouping of NLEM images into launches (plain C++, no HIP).
//
// Images that share the patch radius and the points per lane of their window
// run in one persistent launch.  A launch takes at most kMaxImagesPerLaunch
// images and fewer than 2^31 pixels in total: its work-queue positions and
// the longest-first order are 32-bit.
#pragma once

#include <stdint.h>

#include <vector>

#include "emx_internal.hpp"

namespace emx {

// Largest pixel count of one launch (exclusive bound).
constexpr int64_t kMaxPixelsPerLaunch = (int64_t)1 << 31;

// Points per lane M for a window radius (n = (2R+1)^2 <= 64 M): the
// smallest M, except R = 9, which takes M = 7 for the kernels' row mapping
// (3 runs of 7 columns x 19 rows; measured 4-5% faster than M = 6 slot by
// slot).  M = 4 (R = 7) and M = 7 (R = 9, 10) use the row mapping.
inline int points_per_lane(int R) {
    static const int kM[EM_MAX_WINDOW_RADIUS + 1] = {1, 1, 1, 1, 2, 2, 3, 4, 5, 7, 7};
    return kM[R];
}

struct NlemGroup {
    int pr, m;
    std::vector<int> images;
    int64_t pixels = 0;
};

// Groups in order of first appearance; an image joins the last open group of
// its shape that has room for it (count and pixels), else opens a new one.
// Every image must have H * W < 2^31 (checked by the caller).
inline std::vector<NlemGroup> group_images(int32_t count, const nlem_image_t *images) {
    std::vector<NlemGroup> groups;
    for (int i = 0; i < count; ++i) {
        const int pr = images[i].patch_radius, m = points_per_lane(images[i].window_radius);
        const int64_t px = (int64_t)images[i].H * images[i].W;
        NlemGroup *g = nullptr;
        for (auto &x : groups)
            if (x.pr == pr && x.m == m && (int)x.images.size() < kMaxImagesPerLaunch &&
                x.pixels + px < kMaxPixelsPerLaunch)
                g = &x;
        if (!g) {
            groups.push_back(NlemGroup{pr, m, {}, 0});
            g = &groups.back();
        }
        g->images.push_back(i);
        g->pixels += px;
    }
    return groups;
}

}  // namespace emx
