"""The five workloads: four denoising setups and one batch of point sets.

Each denoising workload lists its noisy images (float32, H x W, row-major)
with the solver settings.  Sizes and parameters follow the paper's
experiments (Section 3: 256 x 256 and 512 x 512 grey images, S = 21 i.e.
window radius 10, k = 7 i.e. patch radius 3, h = 10 sigma, box [0, 255],
penalty mu about 1e-3) and the small / mixed / uneven variants described for
this library.  Penalties were frozen from oracle sweeps at tol 1e-4 (mean
iterations on 512-1024 sampled pixels): 1e-3 for sigma 20 (14.6 iterations
on the 256 x 256 image; 3e-4 and 3e-3 need 26.7 and 24.3), 3e-4 for the
mixed-noise image (24.2; 1e-3 needs 56.4).  Seeds are fixed; image and noise draw from separate
SeedSequence children.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .images import (add_gaussian_noise, add_impulses, gradient_shapes_image,
                     piecewise_smooth_image)
from .pointsets import make_pointset_batch


@dataclass
class NlemImage:
    noisy: np.ndarray          # float32 H x W
    clean: np.ndarray          # float64 H x W (for PSNR only)
    patch_radius: int
    window_radius: int
    sigma: float

    @property
    def h(self) -> float:
        return 10.0 * self.sigma


@dataclass
class NlemWorkload:
    name: str
    images: list = field(default_factory=list)   # list[NlemImage]
    lo: float = 0.0
    hi: float = 255.0
    mu: float = 1e-3
    max_iter: int = 200
    tol: float = 1e-4
    fp16_storage: bool = False

    @property
    def pixels(self) -> int:
        return int(sum(im.noisy.size for im in self.images))


def _rngs(seed: int, k: int):
    return [np.random.default_rng(c) for c in np.random.SeedSequence(seed).spawn(k)]


def nlem_small(seed: int = 101) -> NlemWorkload:
    """64x64 gradient+shapes image, sigma 20, r=2 (d=25), R=5 (n<=121), h=200,
    mu=1, exactly 50 iterations (tol 0)."""
    r_img, r_noise = _rngs(seed, 2)
    clean = gradient_shapes_image(r_img, 64, 64)
    noisy = add_gaussian_noise(r_noise, clean, 20.0).astype(np.float32)
    im = NlemImage(noisy=noisy, clean=clean, patch_radius=2, window_radius=5, sigma=20.0)
    return NlemWorkload(name="nlem-64x64-r2-R5-mu1-T50", images=[im], mu=1.0,
                        max_iter=50, tol=0.0)


def nlem_256(seed: int = 202, mu: float = 1e-3) -> NlemWorkload:
    """256x256 piecewise-smooth + texture bands, sigma 20, r=3 (d=49),
    R=10 (n<=441), h=200, tol 1e-4 (relative to 255), at most 200 iterations."""
    r_img, r_noise = _rngs(seed, 2)
    clean = piecewise_smooth_image(r_img, 256, 256)
    noisy = add_gaussian_noise(r_noise, clean, 20.0).astype(np.float32)
    im = NlemImage(noisy=noisy, clean=clean, patch_radius=3, window_radius=10, sigma=20.0)
    return NlemWorkload(name="nlem-256x256-r3-R10", images=[im], mu=mu)


def nlem_512_mixed(seed: int = 303, mu: float = 3e-4, fp16_storage: bool = False) -> NlemWorkload:
    """512x512, Gaussian sigma 30 then 10% salt-and-pepper impulses; d=49,
    n<=441, h=300; FP16 or FP32 image storage."""
    r_img, r_noise, r_imp = _rngs(seed, 3)
    clean = piecewise_smooth_image(r_img, 512, 512)
    noisy = add_impulses(r_imp, add_gaussian_noise(r_noise, clean, 30.0), 0.10).astype(np.float32)
    im = NlemImage(noisy=noisy, clean=clean, patch_radius=3, window_radius=10, sigma=30.0)
    return NlemWorkload(name="nlem-512x512-mixed-noise" + ("-fp16" if fp16_storage else "-fp32"),
                        images=[im], mu=mu, fp16_storage=fp16_storage)


MULTI_SIZES = ((96, 128), (240, 320), (480, 640), (768, 1024))   # (H, W)


def nlem_multi_image(seed: int = 404, count: int = 16, mu: float = 1e-3,
                     sizes=MULTI_SIZES) -> NlemWorkload:
    """``count`` images, size ~ U(sizes), window radius ~ U{5,7,10}, patch
    radius ~ U{2,3}, sigma 20, h = 10 sigma; solved together."""
    rngs = _rngs(seed, 1 + 2 * count)
    pick = rngs[0]
    ims = []
    for j in range(count):
        H, W = sizes[int(pick.integers(0, len(sizes)))]
        R = int(pick.choice([5, 7, 10]))
        r = int(pick.choice([2, 3]))
        clean = piecewise_smooth_image(rngs[1 + 2 * j], H, W)
        noisy = add_gaussian_noise(rngs[2 + 2 * j], clean, 20.0).astype(np.float32)
        ims.append(NlemImage(noisy=noisy, clean=clean, patch_radius=r, window_radius=R, sigma=20.0))
    return NlemWorkload(name=f"nlem-multi-{count}-images", images=ims, mu=mu)


# Penalty and limits for the point-set workload (mu from an oracle sweep over
# 1e-3 .. 1 on 2,048 instances: 0.5 needs the fewest iterations to tol 1e-4).
POINTSET_MU = 0.5
POINTSET_MAX_ITER = 1000
POINTSET_TOL = 1e-4


def pointset_workload(B: int = 1 << 20, seed: int = 505):
    """Uneven point sets: n ~ U{8..512}, d ~ U{2,3,16,49,64}, 20% Student-t
    (nu 1.5, scale 50) outliers, weights Exp(1), box [-3, 3]^d."""
    return make_pointset_batch(seed, B)


# ---- denoising-quality study (Table 1 and the PSNR-vs-iteration figure of
# Section 3, on synthetic stand-ins for the paper's four test images)

STUDY_SIGMAS = (10.0, 20.0, 40.0, 60.0, 80.0)


def study_images(seed: int = 606):
    """Four clean grey images standing in for the paper's test images (two of
    256 x 256 and two of 512 x 512, as House/Peppers and Lena/Barbara):
    name -> float64 array in [0, 255]."""
    rngs = _rngs(seed, 4)
    return {
        "shapes-256": gradient_shapes_image(rngs[0], 256, 256),
        "smooth-256": piecewise_smooth_image(rngs[1], 256, 256),
        "shapes-512": gradient_shapes_image(rngs[2], 512, 512),
        "smooth-512": piecewise_smooth_image(rngs[3], 512, 512),
    }


def study_noise(clean, sigma: float, realization: int, seed: int = 707) -> np.ndarray:
    """One noise realization of g = f + sigma xi (float32), seeded by
    (seed, sigma, realization)."""
    rng = np.random.default_rng([seed, int(round(sigma * 10)), realization])
    return add_gaussian_noise(rng, clean, sigma).astype(np.float32)
