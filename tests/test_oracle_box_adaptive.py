"""Pins of the oracle's general box (per-coordinate bounds, the box C of
(EM) with one interval per coordinate), of the adaptive penalty (residual
balancing, the first extension the conclusion names) and of the batched
IRLS entry.

Pins: the KKT / normal-cone certificate of the box-constrained minimiser,
coordinate-wise translation equivariance (a swapped coordinate index of the
bounds fails it), the 1-D clamp property, agreement of the adaptive and
fixed-penalty solvers at the (unique) minimiser, factor = 1 reducing to the
fixed penalty exactly, and the adaptive rule moving a badly scaled penalty in
the right direction.  The weighted-mean start of the batch (the counterpart of
the NLM patch) is pinned by closed-form means and by reaching the same
minimiser as the largest-weight start.  The weighted-mean variant of the
ADMM (penalty mu w_k per constraint) is pinned by three hand-worked
iterations, its reduction to Algorithm 1 under equal weights, the
replication, zero-weight and scaling invariances that distinguish it, and
convergence to the same minimiser.
"""

import numpy as np

import synth


def _certificate(a, w, z, lo, hi, tol):
    """0 in grad F(z) + N_C(z) for the box prod_j [lo_j, hi_j] (points at z
    contribute subgradients of norm <= their weight)."""
    dist = np.linalg.norm(a - z[None], axis=1)
    K0 = dist <= 1e-6
    W0 = w[K0].sum()
    g = ((w[~K0] / dist[~K0])[:, None] * (z[None] - a[~K0])).sum(axis=0)
    q = g.copy()
    at_lo = z <= lo + 1e-12
    at_hi = z >= hi - 1e-12
    q[at_lo] = np.minimum(g[at_lo], 0.0)
    q[at_hi] = np.maximum(g[at_hi], 0.0)
    return np.linalg.norm(q) <= W0 + tol * w.sum()


def test_per_coordinate_box_certificate(orc):
    rng = np.random.default_rng(70)
    bound_hits = 0
    for _ in range(12):
        n, d = int(rng.integers(4, 20)), int(rng.integers(2, 6))
        a = rng.normal(size=(n, d)) * 2
        w = rng.uniform(0.1, 2.0, size=n)
        lo = rng.uniform(-1.5, 0.0, size=d)
        hi = lo + rng.uniform(0.2, 1.5, size=d)
        r = orc.em_solve(a, w, 0.5, lo, hi, a[0], max_iter=60000, tol=1e-13)
        z = r["z"]
        assert np.all(z >= lo) and np.all(z <= hi)
        assert _certificate(a, w, z, lo, hi, 1e-5)
        bound_hits += int(np.sum((z <= lo) | (z >= hi)))
        ri = orc.irls_solve(a, w, 1e-10, lo, hi, a[0], max_iter=200000, tol=1e-15)
        assert np.all(ri["z"] >= lo) and np.all(ri["z"] <= hi)
        assert np.linalg.norm(ri["z"] - z) <= 1e-3
    assert bound_hits > 5, "the boxes should bind some coordinates"


def test_per_coordinate_box_translation_equivariance(orc):
    """Shifting the points and the bounds by a vector t shifts the minimiser
    by t (with a different shift per coordinate)."""
    rng = np.random.default_rng(71)
    n, d = 17, 4
    a = rng.normal(size=(n, d))
    w = rng.uniform(0.2, 1.0, size=n)
    lo = np.array([-0.3, -2.0, 0.1, -0.6])
    hi = np.array([0.4, -0.5, 1.0, 0.6])
    t = np.array([5.0, -3.0, 11.0, 0.25])
    r0 = orc.em_solve(a, w, 0.5, lo, hi, a[0], max_iter=40000, tol=1e-13)
    r1 = orc.em_solve(a + t, w, 0.5, lo + t, hi + t, a[0] + t, max_iter=40000, tol=1e-13)
    np.testing.assert_allclose(r1["z"], r0["z"] + t, atol=1e-8)


def test_one_dimension_per_coordinate_equals_scalar_clamp(orc):
    """d = 1: the box minimiser is the weighted median clamped to [lo, hi]."""
    rng = np.random.default_rng(72)
    a = rng.normal(size=(9, 1)) * 3
    w = rng.uniform(0.5, 1.5, size=9)
    order = np.argsort(a[:, 0])
    cw = np.cumsum(w[order])
    med = a[order[np.searchsorted(cw, cw[-1] / 2)], 0]
    for lo, hi in [(-10.0, 10.0), (med + 0.3, med + 1.0), (med - 2.0, med - 0.1)]:
        r = orc.em_solve(a, w, 0.3, np.array([lo]), np.array([hi]), [lo], max_iter=20000, tol=1e-13)
        assert abs(r["z"][0] - np.clip(med, lo, hi)) <= 1e-8


def test_invalid_per_coordinate_box_is_bad_input(orc):
    a = np.ones((3, 2))
    r = orc.em_solve(a, [1, 1, 1], 1.0, [0.0, 1.0], [1.0, 0.5], [0.5, 0.5])
    assert r["flags"] == orc.BAD_INPUT and np.all(np.isnan(r["z"]))
    r = orc.irls_solve(a, [1, 1, 1], 1e-6, [0.0, np.nan], [1.0, 1.0], [0.5, 0.5])
    assert r["flags"] == orc.BAD_INPUT


def test_tolerance_scale_per_coordinate(orc):
    """D = the widest coordinate interval: with tol chosen between the
    residuals measured against D and against a narrower width, the solve
    stops exactly as the rule says."""
    rng = np.random.default_rng(73)
    a = rng.normal(size=(20, 3))
    w = np.ones(20)
    lo = np.array([-1.0, -1.0, -1.0])
    hi = np.array([1.0, 3.0, 0.0])     # widths 2, 4, 1: D = 4
    r = orc.em_solve(a, w, 0.5, lo, hi, a[0], max_iter=500, tol=1e-4)
    assert r["flags"] == orc.CONVERGED
    assert r["r_pri"] <= 4e-4 and r["r_dual"] <= 4e-4
    ref = orc.em_solve(a, w, 0.5, lo, hi, a[0], max_iter=r["iters"] - 1, tol=0.0)
    assert ref["r_pri"] > 4e-4 or ref["r_dual"] > 4e-4


def test_adaptive_penalty_reaches_the_same_minimiser(orc):
    rng = np.random.default_rng(74)
    for seed in range(6):
        n, d = int(rng.integers(5, 60)), int(rng.integers(2, 10))
        a = rng.normal(size=(n, d)) * 2
        w = rng.uniform(0.1, 1.0, size=n)
        fixed = orc.em_solve(a, w, 0.5, -1.0, 1.0, a[0], max_iter=100000, tol=1e-12)
        for mu0 in (1e-4, 0.5, 1e3):
            ad = orc.em_solve(a, w, mu0, -1.0, 1.0, a[0], max_iter=100000, tol=1e-12, adapt_every=1)
            assert ad["flags"] == orc.CONVERGED
            np.testing.assert_allclose(ad["z"], fixed["z"], atol=1e-7)


def test_adaptive_factor_one_is_the_fixed_penalty(orc):
    rng = np.random.default_rng(75)
    a = rng.normal(size=(30, 5))
    w = rng.uniform(0.2, 1.0, size=30)
    f = orc.em_solve(a, w, 0.05, -1.0, 1.0, a[3], max_iter=37)
    g = orc.em_solve(a, w, 0.05, -1.0, 1.0, a[3], max_iter=37, adapt_every=1, adapt_factor=1.0)
    np.testing.assert_array_equal(f["z"], g["z"])
    np.testing.assert_array_equal(f["y"], g["y"])
    assert g["mu"] == 0.05


def test_adaptive_penalty_moves_towards_balance_and_saves_iterations(orc):
    """A penalty far too small lets the primal residual dominate: mu grows and
    the adaptive solver converges where the fixed one stalls.  A penalty far
    too large lets the dual residual dominate: mu shrinks, and the adaptive
    solve still ends at the minimiser (the fixed one stops early on tiny steps
    there, which the residual test cannot tell from convergence)."""
    rng = np.random.default_rng(76)
    a = rng.normal(size=(200, 16)) * 2
    w = rng.uniform(0.2, 1.0, size=200)
    ref = orc.em_solve(a, w, 0.3, -3.0, 3.0, a[0], max_iter=100000, tol=1e-13)
    fixed = orc.em_solve(a, w, 1e-5, -3.0, 3.0, a[0], max_iter=3000, tol=1e-5)
    ad = orc.em_solve(a, w, 1e-5, -3.0, 3.0, a[0], max_iter=3000, tol=1e-5, adapt_every=1)
    assert fixed["flags"] == orc.MAXITER and ad["flags"] == orc.CONVERGED
    assert ad["mu"] > 1e-5 and ad["iters"] * 10 < fixed["iters"]
    ad = orc.em_solve(a, w, 1e4, -3.0, 3.0, a[0], max_iter=3000, tol=1e-9, adapt_every=1)
    assert ad["flags"] == orc.CONVERGED and ad["mu"] < 1e4
    assert np.linalg.norm(ad["z"] - ref["z"]) <= 1e-6


def test_batch_ex_matches_single_solves(orc):
    """The batched entry (IRLS, adaptive ADMM, per-coordinate boxes) equals
    the single-instance solvers on every instance."""
    b = synth.pointsets.make_pointset_batch(9, 24, n_lo=1, n_hi=40, d_choices=(1, 3, 7))
    rng = np.random.default_rng(77)
    blo = rng.uniform(-2.0, -0.5, size=b.z_size).astype(np.float32)
    bhi = (blo + rng.uniform(0.5, 3.0, size=b.z_size)).astype(np.float32)
    for kw in (dict(solver=orc.SOLVER_IRLS, eps=1e-4), dict(solver=orc.SOLVER_ADMM, adapt_every=2)):
        res = orc.em_batch(b, 0.3, 200, 1e-6, init=orc.INIT_MAXW, box_lo=blo, box_hi=bhi, **kw)
        for i in range(b.B):
            e = b.inst[i]
            n, d = int(e["n"]), int(e["d"])
            if n == 0:
                continue
            a = b.a[e["a_off"]:e["a_off"] + n * d].reshape(n, d).astype(np.float64)
            w = b.w[e["w_off"]:e["w_off"] + n].astype(np.float64)
            lo = blo[e["z_off"]:e["z_off"] + d].astype(np.float64)
            hi = bhi[e["z_off"]:e["z_off"] + d].astype(np.float64)
            z0 = a[int(np.argmax(w))]
            if kw["solver"] == orc.SOLVER_IRLS:
                ref = orc.irls_solve(a, w, 1e-4, lo, hi, z0, max_iter=200, tol=1e-6)
            else:
                ref = orc.em_solve(a, w, 0.3, lo, hi, z0, max_iter=200, tol=1e-6, adapt_every=2)
                assert res["mu"][i] == ref["mu"]
            np.testing.assert_array_equal(res["z"][e["z_off"]:e["z_off"] + d], ref["z"])
            assert res["iters"][i] == ref["iters"] and res["flags"][i] == ref["flags"]


# ---- accelerated ADMM (fast ADMM with restart) ------------------------------

def test_fast_admm_first_two_iterations_are_plain_admm(orc):
    """alpha starts at 1, so the first momentum weight (alpha - 1)/alpha' is 0:
    iterations 1 and 2 equal Algorithm 1 exactly; the third differs."""
    rng = np.random.default_rng(80)
    a = rng.normal(size=(40, 6)) * 2
    w = rng.uniform(0.2, 1.0, size=40)
    for T in (1, 2):
        f = orc.em_solve(a, w, 0.7, -1.0, 1.5, a[2], max_iter=T)
        g = orc.em_solve_fast(a, w, 0.7, -1.0, 1.5, a[2], max_iter=T)
        np.testing.assert_array_equal(f["z"], g["z"])
        assert f["r_pri"] == g["r_pri"] and f["r_dual"] == g["r_dual"]
    f = orc.em_solve(a, w, 0.7, -1.0, 1.5, a[2], max_iter=3)
    g = orc.em_solve_fast(a, w, 0.7, -1.0, 1.5, a[2], max_iter=3)
    assert np.max(np.abs(f["z"] - g["z"])) > 1e-9


def test_fast_admm_reaches_the_minimiser(orc):
    """Same (unique) minimiser as Algorithm 1, with its box certificate, for
    penalties over four decades (restarts happen on some)."""
    rng = np.random.default_rng(81)
    restarts = 0
    for _ in range(6):
        n, d = int(rng.integers(5, 80)), int(rng.integers(2, 12))
        a = rng.normal(size=(n, d)) * 2
        w = rng.uniform(0.1, 1.0, size=n)
        lo = rng.uniform(-1.5, -0.2, size=d)
        hi = lo + rng.uniform(0.5, 2.5, size=d)
        ref = orc.em_solve(a, w, 0.5, lo, hi, a[0], max_iter=200000, tol=1e-13)
        for mu in (1e-2, 0.5, 10.0):
            g = orc.em_solve_fast(a, w, mu, lo, hi, a[0], max_iter=200000, tol=1e-13)
            assert g["flags"] == orc.CONVERGED
            np.testing.assert_allclose(g["z"], ref["z"], atol=1e-7)
            assert _certificate(a, w, g["z"], lo, hi, 1e-5)
            restarts += g["restarts"]
    assert restarts > 0


def test_fast_admm_fewer_iterations_with_a_large_penalty(orc):
    """The reason for acceleration: with a penalty too large for the data the
    plain iteration is slow, the accelerated one several times faster."""
    rng = np.random.default_rng(82)
    a = rng.normal(size=(200, 16)) * 2
    w = rng.uniform(0.2, 1.0, size=200)
    f = orc.em_solve(a, w, 10.0, -3.0, 3.0, a[0], max_iter=5000, tol=1e-6)
    g = orc.em_solve_fast(a, w, 10.0, -3.0, 3.0, a[0], max_iter=5000, tol=1e-6)
    assert f["flags"] == g["flags"] == orc.CONVERGED
    assert g["iters"] * 4 < f["iters"]


# ---- the Euclidean ball as the constraint set -----------------------------------

def _ball_certificate(a, w, z, center, radius, tol):
    """0 in grad F(z) + N_C(z) for the ball: inside, the (sub)gradient
    vanishes; on the sphere, -grad F(z) = lam (z - center) with lam >= 0."""
    dist = np.linalg.norm(a - z[None], axis=1)
    K0 = dist <= 1e-6
    W0 = w[K0].sum()
    g = ((w[~K0] / dist[~K0])[:, None] * (z[None] - a[~K0])).sum(axis=0)
    u = z - center
    if np.linalg.norm(u) >= radius * (1 - 1e-9):
        un = u / np.linalg.norm(u)
        lam = max(0.0, -float(g @ un))   # best multiplier of the normal cone
        q = g + lam * un
    else:
        q = g
    return np.linalg.norm(q) <= W0 + tol * w.sum()


def test_ball_certificate_and_scipy(orc):
    from scipy.optimize import minimize
    rng = np.random.default_rng(90)
    on_sphere = 0
    for _ in range(8):
        n, d = int(rng.integers(5, 30)), int(rng.integers(2, 6))
        a = rng.normal(size=(n, d)) * 2 + 1.5
        w = rng.uniform(0.1, 1.0, size=n)
        c = rng.normal(size=d) * 0.3
        r = float(rng.uniform(0.3, 1.5))
        res = orc.em_solve_ball(a, w, 0.5, c, r, c, max_iter=60000, tol=1e-13)
        z = res["z"]
        assert np.linalg.norm(z - c) <= r * (1 + 1e-12)
        assert _ball_certificate(a, w, z, c, r, 1e-5)
        on_sphere += int(np.linalg.norm(z - c) >= r * (1 - 1e-9))
        f = lambda t: np.sum(w * np.linalg.norm(a - t[None], axis=1))
        ref = minimize(f, c, method="SLSQP",
                       constraints=[dict(type="ineq", fun=lambda t: r * r - np.sum((t - c) ** 2))],
                       options=dict(ftol=1e-14, maxiter=2000))
        assert orc.em_objective(a, w, z) <= ref.fun + 1e-7 * max(1.0, ref.fun)
    assert on_sphere >= 4, "the balls should bind"


def test_ball_in_one_dimension_is_the_interval(orc):
    """d = 1: the ball [c - r, c + r] is a box; both sets give the same solve."""
    rng = np.random.default_rng(91)
    a = rng.normal(size=(15, 1)) * 2
    w = rng.uniform(0.2, 1.0, size=15)
    for c, r in [(0.0, 0.5), (1.2, 0.3), (-3.0, 10.0)]:
        zb = orc.em_solve_ball(a, w, 0.4, [c], r, [c], max_iter=300)["z"]
        zx = orc.em_solve(a, w, 0.4, c - r, c + r, [c], max_iter=300)["z"]
        np.testing.assert_allclose(zb, zx, rtol=0, atol=1e-12)
        ib = orc.irls_solve_ball(a, w, 1e-3, [c], r, [c], max_iter=50)["z"]
        ix = orc.irls_solve(a, w, 1e-3, c - r, c + r, [c], max_iter=50)["z"]
        np.testing.assert_allclose(ib, ix, rtol=0, atol=1e-12)


def test_ball_rotation_equivariance(orc):
    """The ball (unlike a box) is invariant under rotations about its centre:
    rotating the points rotates the minimiser (ADMM and IRLS)."""
    rng = np.random.default_rng(92)
    n, d = 20, 4
    a = rng.normal(size=(n, d)) * 2 + 1.0
    w = rng.uniform(0.2, 1.0, size=n)
    c = np.array([0.3, -0.2, 0.1, 0.0])
    Q, _ = np.linalg.qr(rng.normal(size=(d, d)))
    ar = (a - c) @ Q.T + c
    r0 = orc.em_solve_ball(a, w, 0.5, c, 0.8, c, max_iter=40000, tol=1e-13)["z"]
    r1 = orc.em_solve_ball(ar, w, 0.5, c, 0.8, c, max_iter=40000, tol=1e-13)["z"]
    np.testing.assert_allclose(r1, (r0 - c) @ Q.T + c, atol=1e-8)
    i0 = orc.irls_solve_ball(a, w, 1e-4, c, 0.8, c, max_iter=5000, tol=1e-15)["z"]
    i1 = orc.irls_solve_ball(ar, w, 1e-4, c, 0.8, c, max_iter=5000, tol=1e-15)["z"]
    np.testing.assert_allclose(i1, (i0 - c) @ Q.T + c, atol=1e-8)


def test_ball_containing_the_median_changes_nothing_and_bad_radius(orc):
    rng = np.random.default_rng(93)
    a = rng.normal(size=(25, 3))
    w = rng.uniform(0.2, 1.0, size=25)
    free = orc.em_solve(a, w, 0.5, -np.inf, np.inf, a[0], max_iter=40000, tol=1e-13)["z"]
    big = orc.em_solve_ball(a, w, 0.5, np.zeros(3), 1e3, a[0], max_iter=40000, tol=1e-13)["z"]
    np.testing.assert_allclose(big, free, atol=1e-9)
    r = orc.em_solve_ball(a, w, 0.5, np.zeros(3), -1.0, a[0])
    assert r["flags"] == orc.BAD_INPUT and np.all(np.isnan(r["z"]))


# ------------------------------------------------------------ weighted-mean start

def _wmean_batch():
    """Instances whose weighted means have closed forms:
    1-D {0, 2, 7} equal weights -> 3; 1-D {0, 4} weights (1, 3) -> 3;
    a triangle (0,0), (4,0), (0,4) with weights (1, 1, 2) -> (1, 2);
    one nonzero weight -> that point; every weight zero -> the plain mean."""
    pts = [np.array([[0.0], [2.0], [7.0]]), np.array([[0.0], [4.0]]),
           np.array([[0.0, 0.0], [4.0, 0.0], [0.0, 4.0]]),
           np.array([[1.0, -2.0, 3.0], [5.0, 6.0, -7.0], [9.0, 1.0, 2.0]]),
           np.array([[1.0, 2.0], [3.0, 8.0], [-4.0, 5.0], [8.0, -3.0]])]
    wts = [np.ones(3), np.array([1.0, 3.0]), np.array([1.0, 1.0, 2.0]),
           np.array([0.0, 2.5, 0.0]), np.zeros(4)]
    want = [[3.0], [3.0], [1.0, 2.0], [5.0, 6.0, -7.0], [2.0, 3.0]]
    return synth.pointsets.pack_instances(pts, wts, -100.0, 100.0), want


def test_wmean_start_closed_forms(orc):
    """max_iter = 0 returns the start unchanged: the weighted mean (exactly
    representable here), not projected."""
    b, want = _wmean_batch()
    r = orc.em_batch(b, 1.0, 0, 0.0, init=orc.INIT_WMEAN)
    for i, wv in enumerate(want):
        e = b.inst[i]
        np.testing.assert_allclose(r["z"][e["z_off"]:e["z_off"] + e["d"]], wv, rtol=0, atol=1e-12)
    # unprojected: a box that excludes the mean leaves it in place at max_iter 0
    b2 = synth.pointsets.pack_instances([np.array([[0.0], [2.0], [7.0]])], [np.ones(3)], 5.0, 6.0)
    r2 = orc.em_batch(b2, 1.0, 0, 0.0, init=orc.INIT_WMEAN)
    assert r2["z"][0] == 3.0
    r3 = orc.em_batch(b2, 1.0, 1, 0.0, init=orc.INIT_WMEAN)
    assert 5.0 <= r3["z"][0] <= 6.0


def test_wmean_start_same_minimiser(orc):
    """The minimiser does not depend on the start: WMEAN and MAXW starts reach
    the same point (strictly convex instances, many iterations)."""
    b = synth.make_pointset_batch(21, 12, n_lo=5, n_hi=40, d_choices=(2, 3, 7))
    ra = orc.em_batch(b, 0.5, 4000, 0.0, init=orc.INIT_WMEAN)
    rb = orc.em_batch(b, 0.5, 4000, 0.0, init=orc.INIT_MAXW)
    np.testing.assert_allclose(ra["z"], rb["z"], rtol=0, atol=1e-6 * (b.hi - b.lo))
    ri = orc.em_batch(b, 0.5, 400, 0.0, init=orc.INIT_WMEAN, solver=orc.SOLVER_IRLS, eps=1e-10)
    np.testing.assert_allclose(ri["z"], rb["z"], rtol=0, atol=1e-4 * (b.hi - b.lo))


# ------------------------------------------------ weighted-mean ADMM variant

def test_wpen_hand_worked_iterations(orc):
    """d = 1, points 0, 1, 5 with weights 1, 2, 1, mu = 1 (penalties mu_k = 1, 2,
    1, thresholds w_k / mu_k = 1), C = [0, 10], z = 3, y = 0, worked by hand:
    t=1: v = 3, v - a = (3, 2, -2), x = v - sign = (2, 2, 4),
         z = (1*2 + 2*2 + 1*4) / 4 = 5/2, y = mu_k (x - z) = (-1/2, -1, 3/2);
    t=2: y/mu_k = (-1/2, -1/2, 3/2), v = (3, 3, 1), v - a = (3, 2, -4),
         x = (2, 2, 2), z = (1.5 + 2*1.5 + 3.5) / 4 = 2, y unchanged (x = z);
    t=3: v = (5/2, 5/2, 1/2), x = (3/2, 3/2, 3/2), z = (1 + 2 + 3) / 4 = 3/2.
    Algorithm 1 (one penalty) gives z = 7/3 at t = 1 on the same data.  The
    iterates reach the weighted median 1."""
    a = [0.0, 1.0, 5.0]
    for t, zt in ((1, 2.5), (2, 2.0), (3, 1.5)):
        r = orc.em_solve_wpen(a, [1, 2, 1], 1.0, 0.0, 10.0, [3.0], max_iter=t)
        assert abs(r["z"][0] - zt) <= 1e-15, (t, r["z"])
    assert abs(orc.em_solve(np.array(a)[:, None], [1, 2, 1], 1.0, 0.0, 10.0, [3.0], max_iter=1)["z"][0]
               - 7 / 3) <= 1e-15
    r = orc.em_solve_wpen(a, [1, 2, 1], 1.0, 0.0, 10.0, [3.0], max_iter=2000, tol=1e-14)
    assert abs(r["z"][0] - 1.0) <= 1e-9 and r["flags"] == 1


def test_wpen_equal_weights_is_algorithm_1(orc):
    """Equal weights c: penalties mu c for every constraint, thresholds 1/mu,
    an unweighted mean: exactly Algorithm 1 with penalty mu c."""
    rng = np.random.default_rng(81)
    for c in (1.0, 0.37, 5.0):
        a = rng.normal(size=(9, 3))
        z0 = rng.normal(size=3)
        for T in (1, 7, 40):
            r = orc.em_solve_wpen(a, np.full(9, c), 0.8, -1.0, 1.0, z0, max_iter=T)
            s = orc.em_solve(a, np.full(9, c), 0.8 * c, -1.0, 1.0, z0, max_iter=T)
            np.testing.assert_allclose(r["z"], s["z"], rtol=0, atol=1e-12)


def test_wpen_invariances(orc):
    """Properties of the variant that Algorithm 1 does not have: a point of
    weight 2 is two copies of weight 1 (same penalties and thresholds); a
    point of weight 0 changes nothing, wherever it lies; scaling every weight
    leaves the iterates unchanged."""
    rng = np.random.default_rng(82)
    a = rng.normal(size=(6, 4))
    w = rng.uniform(0.2, 2.0, size=6)
    w[2] = 2.0
    z0 = rng.normal(size=4)
    lo, hi = -0.7, 0.9
    for T in (1, 5, 60):
        base = orc.em_solve_wpen(a, w, 0.6, lo, hi, z0, max_iter=T)["z"]
        w2 = w.copy()
        w2[2] = 1.0
        rep = orc.em_solve_wpen(np.vstack([a, a[2:3]]), np.append(w2, 1.0), 0.6, lo, hi, z0, max_iter=T)["z"]
        np.testing.assert_allclose(rep, base, rtol=0, atol=1e-12)
        far = orc.em_solve_wpen(np.vstack([a, [[1e6, -3e5, 7.0, 0.0]]]), np.append(w, 0.0), 0.6, lo, hi, z0,
                                max_iter=T)["z"]
        np.testing.assert_array_equal(far, base)
        sc = orc.em_solve_wpen(a, 7.5 * w, 0.6, lo, hi, z0, max_iter=T)["z"]
        np.testing.assert_allclose(sc, base, rtol=0, atol=1e-12)
    # Algorithm 1 is not replication-invariant (thresholds w_k / mu differ)
    s1 = orc.em_solve(a, w, 0.6, lo, hi, z0, max_iter=5)["z"]
    s2 = orc.em_solve(np.vstack([a, a[2:3]]), np.append(w2, 1.0), 0.6, lo, hi, z0, max_iter=5)["z"]
    assert np.max(np.abs(s1 - s2)) > 1e-6


def test_wpen_converges_to_the_minimiser(orc):
    """Same problem (EM), another algorithm: the limit satisfies the box
    optimality certificate and equals Algorithm 1's limit; over a ball it
    equals Algorithm 1's limit too.  Every weight zero: the start projected."""
    rng = np.random.default_rng(83)
    for _ in range(8):
        n, d = int(rng.integers(3, 15)), int(rng.integers(1, 5))
        a = rng.normal(size=(n, d)) * 2
        w = rng.uniform(0.1, 2.0, size=n)
        lo = rng.uniform(-2, 0, size=d)
        hi = lo + rng.uniform(0.5, 3, size=d)
        r = orc.em_solve_wpen(a, w, 1.0, lo, hi, a[0], max_iter=40000, tol=1e-13)
        assert _certificate(a, w, r["z"], lo, hi, 1e-6)
        s = orc.em_solve(a, w, 1.0, lo, hi, a[0], max_iter=40000, tol=1e-13)
        np.testing.assert_allclose(r["z"], s["z"], rtol=0, atol=1e-6)
        rb = orc.em_solve_wpen(a, w, 1.0, None, None, a[0], max_iter=40000, tol=1e-13, center=lo, radius=1.0)
        sb = orc.em_solve_ball(a, w, 1.0, lo, 1.0, a[0], max_iter=40000, tol=1e-13)
        np.testing.assert_allclose(rb["z"], sb["z"], rtol=0, atol=1e-6)
    r = orc.em_solve_wpen(np.ones((3, 2)), np.zeros(3), 1.0, 0.0, 1.0, [-0.5, 2.0], max_iter=4)
    np.testing.assert_array_equal(r["z"], [0.0, 1.0])
    assert r["r_pri"] == 0.0
