"""Pins of the oracle's NLEM pipeline (Section 3: patches, search window,
NLM weights, patch regression by the constrained EM, centre pixel).

Patches are rebuilt here with numpy's symmetric padding (a library routine)
and the weights by direct enumeration of the truncated window.
"""

import numpy as np

import synth


def _patch(img, pr, iy, ix):
    P = np.pad(img.astype(np.float64), pr, mode="symmetric")
    return P[iy:iy + 2 * pr + 1, ix:ix + 2 * pr + 1].reshape(-1)


def _window(img, pr, wr, iy, ix):
    H, W = img.shape
    pts, slots = [], []
    for dy in range(-wr, wr + 1):
        for dx in range(-wr, wr + 1):
            jy, jx = iy + dy, ix + dx
            if 0 <= jy < H and 0 <= jx < W:
                pts.append(_patch(img, pr, jy, jx))
                slots.append((dy + wr) * (2 * wr + 1) + dx + wr)
    return np.array(pts), np.array(slots)


def _img(seed=0, H=17, W=13):
    rng = np.random.default_rng(seed)
    return synth.add_gaussian_noise(rng, synth.piecewise_smooth_image(rng, H, W), 20.0).astype(np.float32)


def test_zero_iterations_returns_noisy_patch(orc):
    """z starts at the noisy patch P_i (Section 3 initialisation) and the
    output is its centre coordinate, the noisy pixel itself."""
    img = _img()
    H, W = img.shape
    for pr in (1, 2, 3):
        r = orc.nlem(img, pr, 2, 200.0, 0, 255, 1e-3, 0, 0.0, want_z=True)
        np.testing.assert_array_equal(r["out"], img.reshape(-1).astype(np.float64))
        for i in (0, 5, W - 1, W * (H // 2) + 3, H * W - 1):
            np.testing.assert_array_equal(r["z"][i], _patch(img, pr, i // W, i % W))


def test_weights_brute_force(orc):
    """w_ij = exp(-||P_i - P_j||^2 / h^2) over the window truncated to the
    image; slots outside the image are marked -1; w_ii = 1; w_ij = w_ji."""
    img = _img(1)
    H, W = img.shape
    pr, wr, h = 2, 3, 150.0
    r = orc.nlem(img, pr, wr, h, 0, 255, 1e-3, 0, 0.0, want_weights=True)
    Wt = r["weights"]
    nmax = (2 * wr + 1) ** 2
    for i in range(H * W):
        iy, ix = divmod(i, W)
        pts, slots = _window(img, pr, wr, iy, ix)
        Pi = _patch(img, pr, iy, ix)
        expect = np.full(nmax, -1.0)
        expect[slots] = np.exp(-np.sum((pts - Pi[None]) ** 2, axis=1) / h ** 2)
        np.testing.assert_allclose(Wt[i], expect, rtol=1e-13, atol=0)
        assert Wt[i][nmax // 2] == 1.0
    # symmetry: slot of j in i's window mirrors slot of i in j's window
    for i in range(0, H * W, 7):
        iy, ix = divmod(i, W)
        for dy in range(-wr, wr + 1):
            for dx in range(-wr, wr + 1):
                jy, jx = iy + dy, ix + dx
                if 0 <= jy < H and 0 <= jx < W:
                    a = Wt[i][(dy + wr) * (2 * wr + 1) + dx + wr]
                    b = Wt[jy * W + jx][(-dy + wr) * (2 * wr + 1) - dx + wr]
                    assert a == b


def test_pixel_is_em_of_window_patches(orc):
    """(L1regression) is (EM) on the window's patches: each NLEM pixel equals
    the centre coordinate of the EM solve over the brute-force points and
    weights, for interior, edge and corner pixels."""
    img = _img(2, 15, 16)
    H, W = img.shape
    pr, wr, h, mu, T = 2, 4, 200.0, 1e-2, 13
    pix = np.array([0, W - 1, 3 * W + 7, (H - 1) * W + 2, 7 * W + 8])
    r = orc.nlem(img, pr, wr, h, 0, 255, mu, T, 0.0, pix=pix, want_z=True)
    d = (2 * pr + 1) ** 2
    for q, i in enumerate(pix):
        iy, ix = divmod(int(i), W)
        pts, _ = _window(img, pr, wr, iy, ix)
        Pi = _patch(img, pr, iy, ix)
        w = np.exp(-np.sum((pts - Pi[None]) ** 2, axis=1) / h ** 2)
        one = orc.em_solve(pts, w, mu, 0, 255, Pi, max_iter=T)
        # weights here are summed pairwise by numpy, so allow a few ulps
        np.testing.assert_allclose(r["z"][q], one["z"], rtol=1e-12, atol=0)
        assert r["out"][q] == r["z"][q][(d - 1) // 2]


def test_constant_image_is_fixed(orc):
    """A constant image: every patch is the same point, so every EM is that
    point and the denoised image is the constant."""
    img = np.full((12, 11), 87.0, dtype=np.float32)
    r = orc.nlem(img, 3, 4, 200.0, 0, 255, 1e-3, 30, 1e-4)
    np.testing.assert_allclose(r["out"], 87.0, atol=1e-12)


def test_box_clamps_output(orc):
    """The box is imposed by the z-update: after one iteration every output
    is inside [lo, hi], even when the noisy image is not."""
    img = _img(3) * 1.5 - 60.0
    r = orc.nlem(img, 1, 2, 300.0, 0, 255, 1e-2, 1, 0.0)
    assert r["out"].min() >= 0.0 and r["out"].max() <= 255.0
    assert img.min() < 0 or img.max() > 255
