"""Pins of the oracle's IRLS solver (the surrogate (EM_surrogate) minimised by
majorise-minimise, over the box) and of its Non-Local Means estimate and NLM
starting patch (Section 3: the NLM baseline of Table 1 and the two starting
points the text compares).

The IRLS steps are not printed in the paper; the pins therefore check what
any correct minimiser of the surrogate must satisfy (monotone descent of an
MM scheme, stationarity / KKT conditions, scipy's bounded quasi-Newton
optimum, the 1-D clamp property, the epsilon -> 0 limit) rather than a
transcription of the update.
"""

import numpy as np
import pytest
from scipy.optimize import minimize, minimize_scalar
from scipy.signal import convolve2d

import synth


def _surrogate_grad(a, w, eps, z):
    diff = z[None, :] - a
    q = np.sum(diff * diff, axis=1)
    return np.sum((w / np.sqrt(q + eps))[:, None] * diff, axis=0)


def _instance(seed, n, d, scale=3.0):
    rng = np.random.default_rng(seed)
    a = rng.normal(size=(n, d)) * scale
    w = rng.uniform(0.2, 2.0, size=n)
    return a, w


def test_irls_mm_descent(orc):
    """Majorise-minimise: the surrogate never increases along the iterates,
    with and without the box."""
    for seed, (n, d, eps, lo, hi) in enumerate([(9, 2, 1e-6, -np.inf, np.inf), (30, 5, 1e-2, -1.0, 2.0),
                                                (50, 49, 1e-6, -2.0, 1.5), (7, 1, 0.5, 0.3, 4.0)]):
        a, w = _instance(seed, n, d)
        z = a[0].copy() + 0.37
        f_prev = orc.surrogate_objective(a, w, eps, z)
        for _ in range(40):
            z = orc.irls_solve(a, w, eps, lo, hi, z, max_iter=1)["z"]
            f = orc.surrogate_objective(a, w, eps, z)
            assert f <= f_prev * (1 + 1e-14) + 1e-300
            f_prev = f
        assert np.all(z >= lo) and np.all(z <= hi)


def test_irls_stationary_unconstrained(orc):
    """Unconstrained fixed point: the surrogate's gradient
    sum_k w_k (z - a_k) / (||z - a_k||^2 + eps)^(1/2) vanishes."""
    for seed, (n, d, eps) in enumerate([(12, 3, 1e-2), (40, 7, 1e-4), (200, 2, 1.0)]):
        a, w = _instance(10 + seed, n, d)
        r = orc.irls_solve(a, w, eps, -np.inf, np.inf, a.mean(0), max_iter=20000, tol=1e-15)
        g = _surrogate_grad(a, w, eps, r["z"])
        assert np.linalg.norm(g) <= 1e-8 * np.sum(w)


def test_irls_kkt_box(orc):
    """Over a box the minimiser satisfies the KKT conditions: zero gradient on
    free coordinates, gradient >= 0 at lo and <= 0 at hi."""
    a, w = _instance(21, 25, 6)
    lo, hi = -0.4, 0.5
    r = orc.irls_solve(a, w, 1e-3, lo, hi, np.zeros(6), max_iter=20000, tol=1e-15)
    z = r["z"]
    g = _surrogate_grad(a, w, 1e-3, z)
    scale = np.sum(w)
    for j in range(6):
        if z[j] <= lo:
            assert g[j] >= -1e-9 * scale
        elif z[j] >= hi:
            assert g[j] <= 1e-9 * scale
        else:
            assert abs(g[j]) <= 1e-8 * scale
    assert np.any((z <= lo) | (z >= hi)), "the test box should bind some coordinate"


def test_irls_matches_scipy_bounded(orc):
    """The surrogate is strictly convex, so its box minimiser is unique: IRLS
    agrees with scipy's L-BFGS-B on it (objective and point)."""
    a, w = _instance(33, 60, 4, scale=2.0)
    eps, lo, hi = 1e-2, -0.6, 0.8
    f = lambda z: np.sum(w * np.sqrt(np.sum((z[None, :] - a) ** 2, 1) + eps))
    ref = minimize(f, np.zeros(4), jac=lambda z: _surrogate_grad(a, w, eps, z), method="L-BFGS-B",
                   bounds=[(lo, hi)] * 4, options=dict(ftol=1e-15, gtol=1e-12, maxiter=10000))
    r = orc.irls_solve(a, w, eps, lo, hi, np.zeros(4), max_iter=20000, tol=1e-15)
    assert orc.surrogate_objective(a, w, eps, r["z"]) <= ref.fun + 1e-9
    np.testing.assert_allclose(r["z"], ref.x, atol=1e-5)


def test_irls_1d_is_clamp_of_unconstrained(orc):
    """In one dimension the minimiser of a convex function over [lo, hi] is the
    unconstrained minimiser clamped; the unconstrained one is found by a
    bracketing scalar search."""
    a, w = _instance(44, 11, 1)
    eps = 0.05
    f = lambda t: np.sum(w * np.sqrt((t - a[:, 0]) ** 2 + eps))
    t_star = minimize_scalar(f, bracket=(-5, 0, 5), tol=1e-12).x
    for lo, hi in [(-10, 10), (t_star + 0.5, t_star + 2), (t_star - 3, t_star - 0.25)]:
        r = orc.irls_solve(a, w, eps, lo, hi, [lo], max_iter=5000, tol=1e-15)
        assert abs(r["z"][0] - np.clip(t_star, lo, hi)) <= 1e-6


def test_irls_small_eps_approaches_em_median(orc):
    """As eps -> 0 the surrogate's minimiser tends to the Euclidean median
    computed by EM-ADMM (points in general position)."""
    a, w = _instance(55, 15, 3)
    em = orc.em_solve(a, w, 0.5, -np.inf, np.inf, a.mean(0), max_iter=20000, tol=1e-13)
    for eps, tol in [(1e-4, 1e-2), (1e-8, 1e-4)]:
        r = orc.irls_solve(a, w, eps, -np.inf, np.inf, a.mean(0), max_iter=200000, tol=1e-15)
        assert np.linalg.norm(r["z"] - em["z"]) <= tol


def test_irls_worked_example_three_points(orc):
    """d = 1, points 0, 1, 5, unit weights: the surrogate's minimiser lies
    within eps^(3/2) of the median 1 (its derivative at 1 is -15 eps / 32 up
    to O(eps^2) and its curvature there about eps^(-1/2))."""
    a = np.array([[0.0], [1.0], [5.0]])
    for eps in (1e-2, 1e-4, 1e-6):
        r = orc.irls_solve(a, [1, 1, 1], eps, 0.0, 10.0, [3.0], max_iter=100000, tol=1e-15)
        assert abs(r["z"][0] - 1.0) <= eps ** 1.5


def test_irls_flags(orc):
    """n = 0 -> EMPTY; eps <= 0 or a bad weight -> BAD_INPUT (z = NaN); all
    weights zero -> CONVERGED after one iteration with the start projected
    onto C (unchanged when it lies in C; clamped per coordinate otherwise)."""
    assert orc.irls_solve(np.zeros((0, 2)), np.zeros(0), 1e-6, 0, 1, [0.5, 0.5])["flags"] == orc.EMPTY
    r = orc.irls_solve(np.ones((3, 2)), [1, 1, 1], 0.0, 0, 1, [0.5, 0.5])
    assert r["flags"] == orc.BAD_INPUT and np.all(np.isnan(r["z"]))
    r = orc.irls_solve(np.ones((3, 2)), [1, -1, 1], 1e-6, 0, 1, [0.5, 0.5])
    assert r["flags"] == orc.BAD_INPUT
    r = orc.irls_solve(np.ones((3, 2)), [0, 0, 0], 1e-6, 0, 1, [0.25, 0.5], max_iter=9, tol=1e-3)
    assert r["flags"] == orc.CONVERGED and r["iters"] == 1
    np.testing.assert_array_equal(r["z"], [0.25, 0.5])
    r = orc.irls_solve(np.ones((3, 2)), [0, 0, 0], 1e-6, 0, 1, [-0.25, 1.5], max_iter=9, tol=1e-3)
    assert r["flags"] == orc.CONVERGED and r["iters"] == 1
    np.testing.assert_array_equal(r["z"], [0.0, 1.0])
    r = orc.irls_solve_ball(np.ones((3, 2)), [0, 0, 0], 1e-6, [1.0, 1.0], 2.0, [4.0, 5.0], max_iter=9)
    assert r["iters"] == 1
    np.testing.assert_allclose(r["z"], [2.2, 2.6], rtol=0, atol=1e-14)


# ---- Non-Local Means -------------------------------------------------------

def _img(seed=0, H=19, W=14, sigma=20.0):
    rng = np.random.default_rng(seed)
    return synth.add_gaussian_noise(rng, synth.piecewise_smooth_image(rng, H, W), sigma).astype(np.float32)


def test_nlm_infinite_h_is_window_mean(orc):
    """h -> infinity makes every weight 1: NLM is the mean of the noisy pixels
    of the truncated window, i.e. a box filter with zero padding divided by
    the in-image count (scipy's 2-D convolution)."""
    img = _img()
    for wr in (1, 3, 5):
        k = np.ones((2 * wr + 1, 2 * wr + 1))
        ref = convolve2d(img.astype(np.float64), k, mode="same") / convolve2d(np.ones(img.shape), k, mode="same")
        r = orc.nlm(img, 2, wr, 1e12)
        np.testing.assert_allclose(r["out"].reshape(img.shape), ref, rtol=1e-12, atol=1e-9)


def test_nlm_tiny_h_is_identity(orc):
    """h -> 0 leaves only the self-weight w_ii = 1 (noisy patches are distinct),
    so NLM returns the noisy image."""
    img = _img(1)
    r = orc.nlm(img, 1, 3, 1e-3)
    np.testing.assert_array_equal(r["out"], img.reshape(-1).astype(np.float64))


def test_nlm_constant_image(orc):
    img = np.full((9, 11), 37.5, np.float32)
    r = orc.nlm(img, 3, 4, 50.0, want_z=True)
    np.testing.assert_allclose(r["out"], 37.5, rtol=0, atol=1e-12)
    np.testing.assert_allclose(r["z"], 37.5, rtol=0, atol=1e-12)


def test_nlm_patch_and_transpose_equivariance(orc):
    """The NLM patch is a convex combination of window patches (inside their
    range); transposing the image transposes the NLM and NLEM results
    (non-square image, so a swapped row/column index cannot pass)."""
    img = _img(2, 15, 11)
    r = orc.nlm(img, 2, 3, 200.0, want_z=True)
    assert np.all(r["z"] >= img.min() - 1e-9) and np.all(r["z"] <= img.max() + 1e-9)
    rt = orc.nlm(np.ascontiguousarray(img.T), 2, 3, 200.0)
    np.testing.assert_allclose(rt["out"].reshape(img.T.shape), r["out"].reshape(img.shape).T,
                               rtol=1e-12)
    for solver in (orc.SOLVER_ADMM, orc.SOLVER_IRLS):
        a = orc.nlem(img, 2, 3, 200.0, 0, 255, 1e-3, 5, 0.0, solver=solver, init=orc.NLEM_INIT_NLM)
        b = orc.nlem(np.ascontiguousarray(img.T), 2, 3, 200.0, 0, 255, 1e-3, 5, 0.0, solver=solver,
                     init=orc.NLEM_INIT_NLM)
        np.testing.assert_allclose(b["out"].reshape(img.T.shape), a["out"].reshape(img.shape).T,
                                   rtol=1e-10)


def test_nlm_init_zero_iterations_is_nlm(orc):
    """NLEM started from the NLM patch with zero iterations returns NLM, for
    both solvers; one iteration from it moves the estimate."""
    img = _img(3)
    ref = orc.nlm(img, 2, 3, 150.0)["out"]
    for solver in (orc.SOLVER_ADMM, orc.SOLVER_IRLS):
        r = orc.nlem(img, 2, 3, 150.0, 0, 255, 1e-3, 0, 0.0, solver=solver, init=orc.NLEM_INIT_NLM)
        np.testing.assert_array_equal(r["out"], ref)
        r1 = orc.nlem(img, 2, 3, 150.0, 0, 255, 1e-3, 1, 0.0, solver=solver, init=orc.NLEM_INIT_NLM)
        assert np.max(np.abs(r1["out"] - ref)) > 1e-6


def test_nlem_irls_equals_irls_on_materialised_window(orc):
    """NLEM with the IRLS solver equals irls_solve on the window's patches
    (rebuilt with numpy's symmetric padding) and brute-force weights."""
    img = _img(4, 12, 10)
    pr, wr, h, eps = 1, 2, 120.0, 1e-6
    pix = [0, 7, 55, 119]
    r = orc.nlem(img, pr, wr, h, 0, 255, 1e-3, 6, 0.0, pix=pix, want_z=True, solver=orc.SOLVER_IRLS,
                 eps=eps)
    P = np.pad(img.astype(np.float64), pr, mode="symmetric")
    H, W = img.shape
    for q, i in enumerate(pix):
        iy, ix = divmod(i, W)
        pts = np.array([P[y:y + 3, x:x + 3].reshape(-1) for y in range(max(iy - wr, 0), min(iy + wr, H - 1) + 1)
                        for x in range(max(ix - wr, 0), min(ix + wr, W - 1) + 1)])
        Pi = P[iy:iy + 3, ix:ix + 3].reshape(-1)
        wts = np.exp(-np.sum((pts - Pi) ** 2, 1) / h ** 2)
        ref = orc.irls_solve(pts, wts, eps, 0, 255, Pi, max_iter=6)
        np.testing.assert_allclose(r["z"][q], ref["z"], rtol=1e-12, atol=1e-9)


def test_psnr_helper_closed_form():
    """PSNR = 10 log10(255^2 / MSE): a uniform error of e gives 20 log10(255/e)."""
    clean = np.zeros((8, 8))
    for e in (1.0, 5.0, 25.5):
        assert synth.psnr(clean + e, clean) == pytest.approx(20 * np.log10(255.0 / e), rel=1e-12)
