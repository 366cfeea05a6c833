"""CPU test of the host rule that groups NLEM images into launches
(paper_1501_03879_amd/csrc/nlem_group.hpp): at most 16 images per launch,
images of one (patch radius, points per lane) shape together, and fewer than
2^31 pixels per launch (the work-queue positions and the longest-first order
are 32-bit).  The header is compiled with g++ into a small driver; no GPU."""

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include "nlem_group.hpp"
int main(int argc, char **argv) {
    // argv: count, then (patch radius, window radius, H, W) per image
    const int count = atoi(argv[1]);
    std::vector<nlem_image_t> im(count);
    for (int i = 0; i < count; ++i) {
        im[i] = nlem_image_t{};
        im[i].patch_radius = atoi(argv[2 + 4 * i]);
        im[i].window_radius = atoi(argv[3 + 4 * i]);
        im[i].H = atoi(argv[4 + 4 * i]);
        im[i].W = atoi(argv[5 + 4 * i]);
    }
    for (const auto &g : emx::group_images(count, im.data())) {
        printf("%d %d %lld", g.pr, g.m, (long long)g.pixels);
        for (int i : g.images) printf(" %d", i);
        printf("\n");
    }
    return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("grouping")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_1501_03879_amd", "csrc"), str(src), "-o", str(exe)],
                   check=True)
    return str(exe)


def _groups(driver, images):
    args = [driver, str(len(images))] + [str(v) for im in images for v in im]
    out = subprocess.run(args, check=True, capture_output=True, text=True).stdout
    res = []
    for line in out.strip().splitlines():
        f = [int(v) for v in line.split()]
        res.append(dict(pr=f[0], m=f[1], pixels=f[2], images=f[3:]))
    return res


def test_sixteen_images_per_launch(driver):
    g = _groups(driver, [(3, 10, 64, 64)] * 17)
    assert [x["images"] for x in g] == [list(range(16)), [16]]


def test_shapes_grouped_apart(driver):
    # R = 9 and R = 10 share 7 points per lane; R = 5 has 2
    g = _groups(driver, [(3, 10, 32, 32), (2, 10, 32, 32), (3, 9, 16, 16), (3, 5, 8, 8), (2, 10, 4, 4)])
    assert [(x["pr"], x["m"], x["images"]) for x in g] == [(3, 7, [0, 2]), (2, 7, [1, 4]), (3, 2, [3])]
    assert g[0]["pixels"] == 32 * 32 + 16 * 16


def test_pixel_bound_of_a_launch(driver):
    big = 46340   # 46340^2 = 2,147,395,600 < 2^31; with a 400 x 400 image it is above
    g = _groups(driver, [(2, 5, 400, 400), (2, 5, big, big), (2, 5, 400, 400), (2, 5, big, big)])
    # the first big image cannot join the small one's launch; the second small
    # image joins the last launch with room (the first); the second big image
    # gets a launch of its own
    assert [x["images"] for x in g] == [[0, 2], [1], [3]]
    assert all(x["pixels"] < 2 ** 31 for x in g)
    half = 32768   # 2^30 pixels each: two of them make exactly 2^31, not allowed
    g = _groups(driver, [(1, 3, half, half)] * 3)
    assert [x["images"] for x in g] == [[0], [1], [2]]
    g = _groups(driver, [(1, 3, half, half - 1)] * 3)
    assert [x["images"] for x in g] == [[0, 1], [2]]
