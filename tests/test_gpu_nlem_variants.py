"""Every compiled coordinate-wave count of the NLEM kernel (the autotuner may
pick any of them) against the FP64 oracle: EMX_NLEM_WC forces the variant.
Bar as for the other NLEM tests: 1e-4 of the intensity range per pixel,
fixed iteration count, and in tolerance mode the GPU's per-pixel counts fed
back to the oracle."""

import numpy as np
import pytest

import oracle
import synth
from helpers import rel_errors, report, run_nlem

pytestmark = pytest.mark.gpu
D = 255.0
# (patch radius, window radius) -> compiled coordinate-wave counts
# (points per lane M = 7, 2, 1, 4, 7, 5, 3, 5: the waves share each lane's
# points for the shrink factors in every split, including waves with none)
VARIANTS = [(3, 10, (2, 3, 4)), (3, 5, (2, 3, 4)), (3, 3, (1, 2, 3, 4)), (2, 7, (1, 2, 3)), (2, 10, (1, 2, 3)),
            (3, 8, (2, 3, 4)), (3, 6, (2, 3, 4)), (2, 8, (1, 2, 3))]


def _img(seed, H, W, sigma=25.0):
    rng = np.random.default_rng(seed)
    return synth.add_gaussian_noise(rng, synth.piecewise_smooth_image(rng, H, W), sigma).astype(np.float32)


@pytest.mark.parametrize("pr,wr,wcs", VARIANTS)
def test_every_wave_count_fixed_iterations(pr, wr, wcs, monkeypatch):
    img = _img(10 * pr + wr, 27, 31)
    ref = oracle.nlem(img, pr, wr, 250.0, 0, 255, 1e-3, 7, 0.0)
    for wc in wcs:
        monkeypatch.setenv("EMX_NLEM_WC", str(wc))
        got, st = run_nlem(img, pr, wr, 250.0, 1e-3, 7, 0.0)
        e, r = rel_errors(got, ref["out"], D)
        report(f"nlem r{pr} R{wr} {wc} coordinate waves T7", e, r)
        assert e <= 1e-4 and np.all(st["iters"] == 7)


@pytest.mark.parametrize("wc", [2, 3, 4])
def test_every_wave_count_tolerance_mode(wc, monkeypatch):
    img = _img(99, 33, 29, sigma=20.0)
    monkeypatch.setenv("EMX_NLEM_WC", str(wc))
    got, st = run_nlem(img, 3, 10, 200.0, 1e-3, 200, 1e-4)
    ref = oracle.nlem(img, 3, 10, 200.0, 0, 255, 1e-3, 200, 0.0, max_iter_each=st["iters"])
    e, r = rel_errors(got, ref["out"], D)
    report(f"nlem r3 R10 {wc} coordinate waves tol 1e-4 (mean iters {st['iters'].mean():.1f})", e, r)
    assert e <= 1e-4
