"""Synthetic grey images in [0, 255] and the paper's noise model.

The paper's test images are not available, so these generators stand in for
them with the same sizes (256 x 256, 512 x 512) and intensity range.  Noise
follows the model of Section 3: g = f + sigma * xi with xi iid N(0, 1), not
clipped afterwards.  Impulse noise (pixels forced to 0 or 255) is an extra
corruption used for the robustness workload.

Every generator takes a ``numpy.random.Generator`` so callers decide seeding.
"""

from __future__ import annotations

import numpy as np


def gradient_shapes_image(rng: np.random.Generator, H: int, W: int,
                          n_rect: int = 8, n_disk: int = 8,
                          size_lo: int = 4, size_hi: int = 16) -> np.ndarray:
    """Linear gradient background with axis-aligned rectangles and disks.

    Background: 255 * (alpha * x / (W - 1) + (1 - alpha) * y / (H - 1)) with
    alpha ~ U[0, 1].  Then ``n_rect`` rectangles (width and height ~ U{size_lo..
    size_hi}) and ``n_disk`` disks (diameter ~ U{size_lo..size_hi}) with
    intensities ~ U[0, 255] are painted in a random order.  Returns float64.
    """
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    alpha = rng.uniform(0.0, 1.0)
    img = 255.0 * (alpha * x / max(W - 1, 1) + (1.0 - alpha) * y / max(H - 1, 1))
    kinds = np.array([0] * n_rect + [1] * n_disk)
    rng.shuffle(kinds)
    for kind in kinds:
        val = rng.uniform(0.0, 255.0)
        if kind == 0:
            h = int(rng.integers(size_lo, size_hi + 1))
            w = int(rng.integers(size_lo, size_hi + 1))
            y0 = int(rng.integers(0, H))
            x0 = int(rng.integers(0, W))
            img[y0:y0 + h, x0:x0 + w] = val
        else:
            diam = int(rng.integers(size_lo, size_hi + 1))
            cy = rng.uniform(0, H)
            cx = rng.uniform(0, W)
            mask = (y - cy) ** 2 + (x - cx) ** 2 <= (diam / 2.0) ** 2
            img[mask] = val
    return img


def piecewise_smooth_image(rng: np.random.Generator, H: int, W: int,
                           n_cells: int = 12, n_bands: int = 4) -> np.ndarray:
    """Voronoi cells of affine ramps plus sinusoidal texture bands, clipped.

    * ``n_cells`` Voronoi cells with uniform random sites; cell value
      c0 + m * (cos(t) * x / (W - 1) + sin(t) * y / (H - 1)) with
      c0 ~ U[30, 225], t ~ U[0, 2 pi), m ~ U[0, 60 / sqrt(2)] (so the ramp
      changes by at most 60 grey levels across the image).
    * ``n_bands`` horizontal bands, each H/8 rows high, placed in distinct
      eighths of the image, carrying A * sin(2 pi (x cos(phi) + y sin(phi)) / p
      + psi) with p ~ U[4, 32] px, A ~ U[20, 50], phi ~ U[0, pi),
      psi ~ U[0, 2 pi).
    * Clipped to [0, 255].  Returns float64.
    """
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    sy = rng.uniform(0, H, n_cells)
    sx = rng.uniform(0, W, n_cells)
    d2 = (y[None] - sy[:, None, None]) ** 2 + (x[None] - sx[:, None, None]) ** 2
    cell = np.argmin(d2, axis=0)
    c0 = rng.uniform(30.0, 225.0, n_cells)
    t = rng.uniform(0.0, 2 * np.pi, n_cells)
    m = rng.uniform(0.0, 60.0 / np.sqrt(2.0), n_cells)
    xn = x / max(W - 1, 1)
    yn = y / max(H - 1, 1)
    img = c0[cell] + m[cell] * (np.cos(t)[cell] * xn + np.sin(t)[cell] * yn)
    band_h = max(H // 8, 1)
    slots = rng.choice(8, size=min(n_bands, 8), replace=False)
    for s in slots:
        p = rng.uniform(4.0, 32.0)
        A = rng.uniform(20.0, 50.0)
        phi = rng.uniform(0.0, np.pi)
        psi = rng.uniform(0.0, 2 * np.pi)
        r0 = int(s) * band_h
        r1 = min(r0 + band_h, H)
        yy = y[r0:r1]
        xx = x[r0:r1]
        img[r0:r1] += A * np.sin(2 * np.pi * (xx * np.cos(phi) + yy * np.sin(phi)) / p + psi)
    return np.clip(img, 0.0, 255.0)


def add_gaussian_noise(rng: np.random.Generator, img: np.ndarray, sigma: float) -> np.ndarray:
    """g = f + sigma * xi, xi iid N(0, 1); no clipping (Section 3 noise model)."""
    return img + sigma * rng.standard_normal(img.shape)


def add_impulses(rng: np.random.Generator, img: np.ndarray, prob: float,
                 lo: float = 0.0, hi: float = 255.0) -> np.ndarray:
    """Salt-and-pepper: each pixel independently w.p. ``prob`` set to lo or hi (1/2 each)."""
    out = img.copy()
    hit = rng.uniform(size=img.shape) < prob
    salt = rng.uniform(size=img.shape) < 0.5
    out[hit & salt] = hi
    out[hit & ~salt] = lo
    return out


def psnr(estimate: np.ndarray, clean: np.ndarray, peak: float = 255.0) -> float:
    """Peak signal-to-noise ratio 10 log10(peak^2 / MSE) in dB (the quality
    measure of the paper's denoising table); an evaluation metric, not part of
    any denoiser."""
    err = np.asarray(estimate, np.float64) - np.asarray(clean, np.float64)
    return float(10.0 * np.log10(peak * peak / np.mean(err * err)))
