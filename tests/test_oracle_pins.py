"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these tests re-implements the oracle's formulas: each checks an
output against an optimality condition, a theorem, a textbook special case,
brute-force minimisation, or a hand-worked example.  Section and equation
names refer to Chaudhury & Ramakrishnan, arXiv:1501.03879.
"""

import numpy as np
import pytest
from scipy.optimize import minimize

INF = float("inf")


def objective(z, a, w):
    """(EM): sum_k w_k ||z - a_k||_2."""
    return float(np.sum(w * np.linalg.norm(a - z[None, :], axis=1)))


# ---------------------------------------------------------------- prox (P1)

def test_prox_optimality_condition(orc):
    """(prox)-(closed-form): x* minimises lambda||x-u|| + 1/2||x-v||^2 iff
    v - x* lies in lambda * subdifferential of ||. - u|| at x*: equal to
    lambda (x*-u)/||x*-u|| when x* != u, any vector of norm <= lambda at u."""
    rng = np.random.default_rng(0)
    for _ in range(300):
        d = int(rng.integers(1, 9))
        v = rng.normal(size=d) * rng.uniform(0.1, 10)
        u = rng.normal(size=d) * rng.uniform(0.1, 10)
        lam = rng.uniform(0, 3) * np.linalg.norm(v - u) * rng.uniform(0.2, 1.5)
        x = orc.prox(v, u, lam)
        g = v - x
        if np.linalg.norm(x - u) > 1e-12:
            expect = lam * (x - u) / np.linalg.norm(x - u)
            np.testing.assert_allclose(g, expect, rtol=1e-9, atol=1e-9)
        else:
            assert np.linalg.norm(g) <= lam * (1 + 1e-12) + 1e-12


def test_prox_limits_and_moreau(orc):
    """lambda = 0 gives v and lambda -> inf gives u (text after
    (closed-form)); Moreau decomposition (MD): v = Psi_f(v) + Psi_f*(v) with
    Psi_f*(v) the projection of v - u onto the ball of radius lambda
    (proxfstar), computed here as the textbook ball projection."""
    rng = np.random.default_rng(1)
    for _ in range(200):
        d = int(rng.integers(1, 7))
        v, u = rng.normal(size=d) * 5, rng.normal(size=d) * 5
        np.testing.assert_allclose(orc.prox(v, u, 0.0), v, rtol=0, atol=0)
        np.testing.assert_allclose(orc.prox(v, u, 1e300), u, rtol=0, atol=0)
        lam = rng.uniform(0, 2 * np.linalg.norm(v - u))
        t = v - u
        nt = np.linalg.norm(t)
        ball = t if nt <= lam else t * (lam / nt)
        np.testing.assert_allclose(orc.prox(v, u, lam) + ball, v, rtol=1e-12, atol=1e-12)


def test_prox_brute_force(orc):
    """(defprox) as a minimisation solved numerically from several starts."""
    rng = np.random.default_rng(2)
    for _ in range(40):
        d = int(rng.integers(1, 5))
        v, u = rng.normal(size=d) * 3, rng.normal(size=d) * 3
        lam = rng.uniform(0.0, 2.0) * np.linalg.norm(v - u)

        def F(x):
            return lam * np.linalg.norm(x - u) + 0.5 * np.sum((x - v) ** 2)

        best = min((minimize(F, s, method="Nelder-Mead",
                             options=dict(xatol=1e-11, fatol=1e-14, maxiter=40000))
                    for s in (v, u, 0.5 * (u + v), rng.normal(size=d))), key=lambda r: r.fun)
        x = orc.prox(v, u, lam)
        assert F(x) <= best.fun + 1e-10
        # strong convexity (modulus 1): ||x - x_bf||^2 / 2 <= F(x_bf) - F(x)
        assert np.linalg.norm(x - best.x) <= np.sqrt(2 * max(best.fun - F(x), 0) + 1e-16) + 1e-6


# ------------------------------------------------- one iteration (P2, P3, P4)

def _one_step(orc, a, w, mu, lo, hi, z, y):
    r = orc.em_solve(a, w, mu, lo, hi, z, y0=y, max_iter=1)
    return r["x"], r["z"], r["y"]


def test_one_iteration_is_the_gauss_seidel_argmins(orc):
    """Each sub-step of Algorithm 1 checked against its defining problem:
    x_k solves (updatex) (minimised numerically, not by the closed form);
    z solves the box-constrained least squares above (updatez) (minimised with
    L-BFGS-B over the box); and the multipliers satisfy the ADMM dual
    relation -(y_k^{t+1} + mu (z^{t+1} - z^t)) in the subdifferential of f_k at
    x_k^{t+1}, which follows from (updatex) and (updatey)."""
    rng = np.random.default_rng(3)
    for trial in range(12):
        n, d = int(rng.integers(1, 6)), int(rng.integers(1, 4))
        a = rng.normal(size=(n, d)) * 2
        w = rng.uniform(0.1, 2.0, size=n)
        mu = rng.uniform(0.3, 3.0)
        lo, hi = -0.7, 1.1
        # the starting z may lie outside C: Algorithm 1 never projects it
        z = rng.uniform(lo - 1.0, hi + 1.0, size=d)
        y = rng.normal(size=(n, d))
        x, z1, y1 = _one_step(orc, a, w, mu, lo, hi, z, y)
        for k in range(n):
            def Fx(xx):
                return (w[k] * np.linalg.norm(xx - a[k]) + (xx - z) @ y[k]
                        + 0.5 * mu * np.sum((xx - z) ** 2))
            bf = min((minimize(Fx, s, method="Nelder-Mead",
                               options=dict(xatol=1e-12, fatol=1e-15, maxiter=40000))
                      for s in (z, a[k], z - y[k] / mu)), key=lambda r: r.fun)
            assert Fx(x[k]) <= bf.fun + 1e-10
        def Fz(zz):
            return 0.5 * mu * np.sum((zz[None, :] - x - y / mu) ** 2)
        bz = minimize(Fz, np.zeros(d), method="L-BFGS-B", bounds=[(lo, hi)] * d,
                      options=dict(ftol=1e-15, gtol=1e-12))
        assert Fz(z1) <= bz.fun + 1e-10
        np.testing.assert_allclose(z1, bz.x, atol=1e-6)
        for k in range(n):
            g = -(y1[k] + mu * (z1 - z))
            if np.linalg.norm(x[k] - a[k]) > 1e-12:
                np.testing.assert_allclose(g, w[k] * (x[k] - a[k]) / np.linalg.norm(x[k] - a[k]),
                                           rtol=1e-8, atol=1e-9)
            else:
                assert np.linalg.norm(g) <= w[k] * (1 + 1e-9) + 1e-9


def test_multiplier_sum_invariant(orc):
    """With C = R^d the z-update makes sum_k (x_k - z) = -sum_k y_k / mu, so
    (updatey) gives sum_k y_k = 0 after every iteration; with a box, sum_k y_k
    = mu n (z0 - z) is in the negative normal cone of the box at z."""
    rng = np.random.default_rng(4)
    n, d = 7, 3
    a = rng.normal(size=(n, d)) * 4
    w = rng.uniform(0.2, 1.5, size=n)
    for T in (1, 2, 5, 17):
        r = orc.em_solve(a, w, 0.8, -INF, INF, a[0] + 0.3, max_iter=T)
        np.testing.assert_allclose(r["y"].sum(axis=0), 0.0, atol=1e-10)
    lo, hi = -0.5, 0.5
    for T in (1, 3, 9):
        r = orc.em_solve(a, w, 0.8, lo, hi, np.zeros(d), max_iter=T)
        s = r["y"].sum(axis=0)
        z = r["z"]
        for j in range(d):
            if lo < z[j] < hi:
                assert abs(s[j]) < 1e-9
            elif z[j] == lo:
                assert s[j] <= 1e-9
            else:
                assert s[j] >= -1e-9


def test_worked_example_first_iteration(orc):
    """Hand-worked first iteration of Algorithm 1 for d = 1, points 0, 1, 5,
    unit weights, mu = 1 (lambda = 1), C = [0, 10], z = 3, y = 0:
    v_k = 3, v - a = (3, 2, -2), all of length > 1, so x = v - (v-a)/|v-a|
    = (2, 2, 4); r = 8, z = 8/3; y = x - z = (-2/3, -2/3, 4/3).  Later the
    iterates reach the median 1 (the minimiser of |z| + |z-1| + |z-5|)."""
    a = np.array([[0.0], [1.0], [5.0]])
    r = orc.em_solve(a, [1, 1, 1], 1.0, 0.0, 10.0, [3.0], max_iter=1)
    np.testing.assert_allclose(r["x"].ravel(), [2, 2, 4], rtol=0, atol=1e-15)
    np.testing.assert_allclose(r["z"], [8 / 3], rtol=1e-15)
    np.testing.assert_allclose(r["y"].ravel(), [-2 / 3, -2 / 3, 4 / 3], rtol=1e-14)
    r = orc.em_solve(a, [1, 1, 1], 1.0, 0.0, 10.0, [3.0], max_iter=400)
    np.testing.assert_allclose(r["z"], [1.0], atol=1e-9)


def test_worked_example_iterations_two_to_six(orc):
    """The same example continued by hand.  With y = (-2/3, -2/3, 4/3) after
    t = 1 and z = 8/3: v = z - y = (10/3, 10/3, 4/3), v - a = (10/3, 7/3, -11/3),
    all longer than 1, so x = v - sign(v - a) = (7/3, 7/3, 7/3) and z = (7 + 0)/3
    = 7/3; x = z, so y is unchanged.  Each later step repeats this with z lower
    by 1/3 (x = z - 1/3 per point): z = 2, 5/3, 4/3, and at t = 6,
    v = (2, 2, 0), v - a = (2, 1, -5): the middle point sits exactly at the tie
    |v - a| = lambda, where both prox branches give x_2 = 1, so z = 1.  The
    primal residual x - z is exactly 0 for t = 2..6 while z still moves: a
    stopping rule on the primal residual alone would stop at t = 2."""
    a = np.array([[0.0], [1.0], [5.0]])
    for t, zt in ((2, 7 / 3), (3, 2.0), (4, 5 / 3), (5, 4 / 3), (6, 1.0)):
        r = orc.em_solve(a, [1, 1, 1], 1.0, 0.0, 10.0, [3.0], max_iter=t)
        assert abs(r["z"][0] - zt) <= 1e-14, (t, r["z"])
        np.testing.assert_allclose(r["y"].ravel(), [-2 / 3, -2 / 3, 4 / 3], rtol=0, atol=1e-14)
        assert r["r_pri"] <= 1e-15
        assert abs(r["r_dual"] - 1 / 3) <= 1e-14
    # tol = 1e-3 (tol D = 0.01): the dual residual keeps the solve going past t = 2
    r = orc.em_solve(a, [1, 1, 1], 1.0, 0.0, 10.0, [3.0], max_iter=400, tol=1e-3)
    assert r["iters"] > 6 and abs(r["z"][0] - 1.0) <= 0.05


def test_worked_example_iterations_seven_to_twelve(orc):
    """The same example past the tie.  From t = 7 on the middle point is
    within lambda = 1 of v (so x_2 = a_2 = 1) and the outer two are not
    (x_1 = v_1 - 1, x_3 = v_3 + 1).  With v_k = z - y_k that gives
      x_1 + y_1 = z - 1,  x_2 + y_2 = 1 + y_2,  x_3 + y_3 = z + 1,
      z' = (2 z + 1 + y_2) / 3,   y_2' = y_2 + 1 - z',
      y_1' = z - 1 - z',          y_3' = z + 1 - z',
    a two-variable recursion worked out by hand, started from z = 1,
    y = (-2/3, -2/3, 4/3) after t = 6: z = 7/9, 19/27, 61/81, 211/243,
    721/729, 2347/2187: the iterates oscillate towards the median 1, and the
    primal residual is no longer zero (x_2 = 1 differs from z').  The branch
    conditions are checked along the way in exact arithmetic."""
    from fractions import Fraction as Fr
    a = np.array([[0.0], [1.0], [5.0]])
    z, y = Fr(1), [Fr(-2, 3), Fr(-2, 3), Fr(4, 3)]
    for t in range(7, 13):
        v = [z - yk for yk in y]
        assert abs(v[0] - 0) > 1 and abs(v[1] - 1) <= 1 and abs(v[2] - 5) > 1
        zn = (2 * z + 1 + y[1]) / 3
        x = [v[0] - 1, Fr(1), v[2] + 1]
        y = [z - 1 - zn, y[1] + 1 - zn, z + 1 - zn]
        z = zn
        r = orc.em_solve(a, [1, 1, 1], 1.0, 0.0, 10.0, [3.0], max_iter=t)
        assert abs(r["z"][0] - float(z)) <= 1e-14, (t, r["z"][0], z)
        np.testing.assert_allclose(r["y"].ravel(), [float(q) for q in y], rtol=0, atol=1e-13)
        rp = np.sqrt(sum(float(xk - z) ** 2 for xk in x) / 3)
        assert abs(r["r_pri"] - rp) <= 1e-14
    assert z == Fr(2347, 2187)


# --------------------------------------------------- converged solutions

def _solve(orc, a, w, lo=-INF, hi=INF, mu=None, z0=None, iters=20000):
    a = np.asarray(a, float)
    if mu is None:
        mu = float(np.sum(w)) / max(np.std(a) * np.sqrt(a.shape[1]), 1e-3) / len(w)
    z0 = a.mean(axis=0) if z0 is None else z0
    return orc.em_solve(a, w, mu, lo, hi, z0, max_iter=iters, tol=1e-13)


def test_single_point_is_its_projection(orc):
    """(EM) with n = 1: the objective is w ||z - a_1||, minimised over the box
    at the projection of a_1 (radial objective)."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        d = int(rng.integers(1, 6))
        a = rng.normal(size=(1, d)) * 3
        r = _solve(orc, a, [rng.uniform(0.1, 3)], -1.0, 1.0, mu=0.5, z0=np.zeros(d))
        np.testing.assert_allclose(r["z"], np.clip(a[0], -1, 1), atol=1e-8)


def test_scalar_weighted_median(orc):
    """d = 1: the minimiser of sum w_k |z - a_k| is the weighted median (sort;
    first point where the cumulative weight reaches half the total), and the
    box solution is its clamp (a convex 1-D function)."""
    rng = np.random.default_rng(6)
    for _ in range(25):
        n = int(rng.integers(2, 30))
        a = rng.normal(size=n) * 10
        w = rng.uniform(0.1, 2.0, size=n)
        order = np.argsort(a)
        cw = np.cumsum(w[order])
        med = a[order][np.searchsorted(cw, 0.5 * cw[-1])]
        lo, hi = (-INF, INF) if rng.uniform() < 0.5 else (-2.0, 2.0)
        r = _solve(orc, a[:, None], w, lo, hi, mu=float(w.sum()) / n / 5, iters=50000)
        zc = np.clip(med, lo, hi)
        f = lambda t: float(np.sum(w * np.abs(t - a)))
        assert f(r["z"][0]) <= f(zc) + 1e-7 * (1 + f(zc))
        np.testing.assert_allclose(r["z"][0], zc, atol=1e-5)


def test_odd_collinear_equal_weights_middle_point(orc):
    """Points on one line with equal weights: the EM is the middle point."""
    rng = np.random.default_rng(7)
    for _ in range(10):
        d = int(rng.integers(2, 6))
        n = 2 * int(rng.integers(1, 6)) + 1
        base, direc = rng.normal(size=d), rng.normal(size=d)
        t = np.sort(rng.normal(size=n) * 5)
        a = base[None] + t[:, None] * direc[None]
        r = _solve(orc, a, np.ones(n), iters=60000)
        np.testing.assert_allclose(r["z"], a[n // 2], atol=1e-5 * (1 + np.abs(a).max()))


def test_centrally_symmetric_set_centre(orc):
    """Pairs c +/- p_j with pairwise-equal weights: the centre has zero
    gradient (terms cancel pairwise) and is the unique minimiser."""
    rng = np.random.default_rng(8)
    for _ in range(10):
        d = int(rng.integers(2, 5))
        m = int(rng.integers(2, 6))
        c = rng.normal(size=d)
        p = rng.normal(size=(m, d)) * 3
        w = rng.uniform(0.2, 2.0, size=m)
        a = np.concatenate([c + p, c - p])
        r = _solve(orc, a, np.concatenate([w, w]), -20.0, 20.0, iters=60000)
        np.testing.assert_allclose(r["z"], c, atol=1e-6)


def test_2d_brute_force_grid(orc):
    """d = 2: the ADMM result is no worse than the best point of a fine grid
    over the box, up to the grid's Lipschitz slack sum(w) * step / sqrt(2)."""
    rng = np.random.default_rng(9)
    for _ in range(6):
        n = int(rng.integers(3, 12))
        a = rng.normal(size=(n, 2)) * 2
        w = rng.uniform(0.1, 2.0, size=n)
        lo, hi = -1.0, 0.8
        r = _solve(orc, a, w, lo, hi, iters=60000)
        g = np.linspace(lo, hi, 601)
        X, Y = np.meshgrid(g, g)
        F = sum(wk * np.hypot(X - ak[0], Y - ak[1]) for ak, wk in zip(a, w))
        step = g[1] - g[0]
        f = objective(r["z"], a, w)
        assert f <= F.min() + 1e-9
        assert f >= F.min() - w.sum() * step / np.sqrt(2)


def test_box_normal_cone_certificate(orc):
    """Optimality over the box: 0 in grad F(z) + N_C(z).  With K0 the points
    within delta of z and W0 their weight, the gradient g of the other terms
    may be cancelled by the K0 subgradients (norm <= W0) and the normal cone
    (free sign at an active bound).  The leftover q must have norm <= W0."""
    rng = np.random.default_rng(10)
    for _ in range(15):
        n, d = int(rng.integers(3, 15)), int(rng.integers(2, 5))
        a = rng.normal(size=(n, d)) * 2 + 1.0
        w = rng.uniform(0.1, 2.0, size=n)
        lo, hi = -0.5, 1.5
        r = _solve(orc, a, w, lo, hi, iters=80000)
        z = r["z"]
        dist = np.linalg.norm(a - z[None], axis=1)
        K0 = dist <= 1e-6
        W0 = w[K0].sum()
        g = ((w[~K0] / dist[~K0])[:, None] * (z[None] - a[~K0])).sum(axis=0)
        q = g.copy()
        at_lo = z <= lo + 1e-12
        at_hi = z >= hi - 1e-12
        q[at_lo] = np.minimum(g[at_lo], 0.0)
        q[at_hi] = np.maximum(g[at_hi], 0.0)
        assert np.linalg.norm(q) <= W0 + 1e-5 * w.sum()


def _weiszfeld(a, w, iters=200000):
    """Weiszfeld's fixed point x <- sum(w_k a_k / ||x - a_k||) / sum(w_k / ||x - a_k||)."""
    x = np.average(a, axis=0, weights=w)
    for _ in range(iters):
        dist = np.linalg.norm(a - x[None], axis=1)
        c = w / dist
        xn = (c[:, None] * a).sum(axis=0) / c.sum()
        if np.linalg.norm(xn - x) < 1e-15 * (1 + np.linalg.norm(x)):
            return xn
        x = xn
    return x


def test_weiszfeld_agreement(orc):
    """Unconstrained, non-degenerate data: agrees with Weiszfeld's algorithm
    (the classical method the paper cites) to 1e-7."""
    rng = np.random.default_rng(11)
    for _ in range(10):
        n, d = int(rng.integers(5, 40)), int(rng.integers(2, 8))
        a = rng.normal(size=(n, d)) * 3
        w = rng.uniform(0.2, 2.0, size=n)
        ref = _weiszfeld(a, w)
        r = _solve(orc, a, w, iters=100000)
        np.testing.assert_allclose(r["z"], ref, atol=1e-7 * (1 + np.abs(ref).max()))


def test_projection_of_unconstrained_median(orc):
    """When the unconstrained median lies in the box the box changes nothing;
    in general the box solution is at least as good as projecting the
    unconstrained median, and strictly better on the three-point example
    (-1,0), (1,0), (0,1): projecting the Fermat point (0, 1/sqrt(3)) onto a
    box that cuts it off is not optimal in general, so the projection claim in
    the introduction holds only in special cases (n = 1, d = 1, median in C).
    With the cube C = [0.5, 10]^2 the same three points show it: the box
    solution beats the projected Fermat point by more than 0.02."""
    rng = np.random.default_rng(12)
    for _ in range(8):
        n, d = int(rng.integers(4, 20)), int(rng.integers(2, 5))
        a = rng.normal(size=(n, d))
        w = rng.uniform(0.2, 2.0, size=n)
        em = _weiszfeld(a, w)
        r = _solve(orc, a, w, -10.0, 10.0, iters=80000)
        np.testing.assert_allclose(r["z"], em, atol=1e-6)
        lo, hi = -0.1, 0.1
        rc = _solve(orc, a, w, lo, hi, iters=80000)
        assert objective(rc["z"], a, w) <= objective(np.clip(em, lo, hi), a, w) + 1e-9
    a = np.array([[-1.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
    w = np.ones(3)
    fermat = np.array([0.0, 1.0 / np.sqrt(3.0)])
    rc = _solve(orc, a, w, 0.5, 10.0, iters=80000)
    proj = np.clip(fermat, 0.5, 10.0)
    assert objective(rc["z"], a, w) < objective(proj, a, w) - 0.02
    g = np.linspace(0.5, 1.5, 1001)
    X, Y = np.meshgrid(g, g)
    F = sum(np.hypot(X - ak[0], Y - ak[1]) for ak in a)
    assert objective(rc["z"], a, w) <= F.min() + 1e-9


def test_invariances(orc):
    """Algorithm 1 commutes with translating (a, box, z0), permuting points,
    scaling (w, mu) jointly (lambda = w/mu and y/mu unchanged) and scaling
    (a, box, z0) by s with mu -> mu/s (iterates scale by s)."""
    rng = np.random.default_rng(13)
    n, d, T = 9, 3, 23
    a = rng.normal(size=(n, d)) * 2
    w = rng.uniform(0.1, 2.0, size=n)
    mu, lo, hi = 0.7, -1.0, 1.3
    z0 = rng.uniform(lo, hi, size=d)
    base = orc.em_solve(a, w, mu, lo, hi, z0, max_iter=T)["z"]
    t = 3.25
    r = orc.em_solve(a + t, w, mu, lo + t, hi + t, z0 + t, max_iter=T)["z"]
    np.testing.assert_allclose(r - t, base, atol=1e-12)
    perm = rng.permutation(n)
    r = orc.em_solve(a[perm], w[perm], mu, lo, hi, z0, max_iter=T)["z"]
    np.testing.assert_allclose(r, base, atol=1e-12)
    r = orc.em_solve(a, 4.0 * w, 4.0 * mu, lo, hi, z0, max_iter=T)["z"]
    np.testing.assert_allclose(r, base, atol=1e-12)
    s = 8.0
    r = orc.em_solve(s * a, w, mu / s, s * lo, s * hi, s * z0, max_iter=T)["z"]
    np.testing.assert_allclose(r / s, base, atol=1e-12)


def test_fixed_point(orc):
    """(z*, y_k* = -w_k (z* - a_k)/||z* - a_k||) with z* the unconstrained
    median (so sum y* = 0) and z* interior is left unchanged by one iteration."""
    rng = np.random.default_rng(14)
    n, d = 11, 4
    a = rng.normal(size=(n, d))
    w = rng.uniform(0.2, 2.0, size=n)
    zs = _weiszfeld(a, w)
    u = (zs[None] - a) / np.linalg.norm(zs[None] - a, axis=1)[:, None]
    ys = -w[:, None] * u
    for mu in (0.05, 1.0, 20.0):
        r = orc.em_solve(a, w, mu, -5.0, 5.0, zs, y0=ys, max_iter=1)
        np.testing.assert_allclose(r["z"], zs, atol=1e-12)
        np.testing.assert_allclose(r["y"], ys, atol=1e-10)


def test_convergence_for_any_penalty(orc):
    """2-block ADMM converges for every mu > 0: objective reaches the optimum
    (Weiszfeld) for penalties over four decades."""
    rng = np.random.default_rng(15)
    n, d = 25, 3
    a = rng.normal(size=(n, d)) * 5
    w = rng.uniform(0.2, 2.0, size=n)
    fstar = objective(_weiszfeld(a, w), a, w)
    for mu in (0.01, 0.1, 1.0, 10.0):
        r = orc.em_solve(a, w, mu, -INF, INF, a[0], max_iter=200000, tol=1e-12)
        assert objective(r["z"], a, w) <= fstar * (1 + 1e-9)


# --------------------------------------------------- stopping rule and flags

def test_stopping_rule_and_scale(orc):
    """tol > 0: stops at the first iteration where both residuals are below
    tol * D, D = hi - lo for a finite box, else max(1, max |a|)."""
    rng = np.random.default_rng(16)
    a = rng.normal(size=(30, 4)) * 20
    w = rng.uniform(0.2, 2.0, size=30)
    for lo, hi, D in ((-100.0, 100.0, 200.0), (-INF, INF, float(np.abs(a).max()))):
        r = orc.em_solve(a, w, 0.05, lo, hi, a[0], max_iter=5000, tol=1e-5)
        assert r["flags"] == orc.CONVERGED
        assert r["r_pri"] <= 1e-5 * D and r["r_dual"] <= 1e-5 * D
        prev = orc.em_solve(a, w, 0.05, lo, hi, a[0], max_iter=r["iters"] - 1)
        assert prev["r_pri"] > 1e-5 * D or prev["r_dual"] > 1e-5 * D
        full = orc.em_solve(a, w, 0.05, lo, hi, a[0], max_iter=r["iters"])
        np.testing.assert_array_equal(full["z"], r["z"])
        # the residuals are the RMS of x_k - z and of z - z_prev
        np.testing.assert_allclose(r["r_pri"], np.sqrt(np.mean((full["x"] - full["z"]) ** 2)),
                                   rtol=1e-12)
        np.testing.assert_allclose(r["r_dual"], np.sqrt(np.mean((full["z"] - prev["z"]) ** 2)),
                                   rtol=1e-12)


def test_flags_and_degenerate_cases(orc):
    z0 = np.array([1.0, 2.0])
    r = orc.em_solve(np.zeros((0, 2)), np.zeros(0), 1.0, 0, 10, z0, max_iter=10)
    assert r["flags"] == orc.EMPTY and np.array_equal(r["z"], z0)
    r = orc.em_solve(np.ones((3, 2)), [1, -1, 1], 1.0, 0, 10, z0, max_iter=10)
    assert r["flags"] == orc.BAD_INPUT and np.all(np.isnan(r["z"]))
    r = orc.em_solve(np.array([[1, np.inf], [0, 0]]), [1, 1], 1.0, 0, 10, z0, max_iter=10)
    assert r["flags"] == orc.BAD_INPUT
    r = orc.em_solve(np.ones((3, 2)), [1, 1, 1], 1.0, 0, 10, [20.0, -5.0], max_iter=0)
    assert r["iters"] == 0 and np.array_equal(r["z"], [20.0, -5.0])
    # all weights zero: lambda = 0, x_k = v, so z stays in C and nothing moves
    r = orc.em_solve(np.random.default_rng(0).normal(size=(5, 2)), np.zeros(5), 1.0, -1, 1,
                     [0.25, -0.5], max_iter=7)
    np.testing.assert_allclose(r["z"], [0.25, -0.5], atol=1e-15)


# ------------------------------------------------------------ batch wrapper

def test_batch_matches_single(orc):
    import synth
    b = synth.make_pointset_batch(7, 40, n_lo=1, n_hi=30, d_choices=(1, 2, 5))
    res = orc.em_batch(b, 0.3, 60, 0.0, init=orc.INIT_MAXW)
    for i in range(b.B):
        a = b.points(i).astype(np.float64)
        w = b.weights(i).astype(np.float64)
        k = int(np.argmax(w))
        one = orc.em_solve(a, w, 0.3, b.lo, b.hi, a[k], max_iter=60)
        e = b.inst[i]
        np.testing.assert_array_equal(res["z"][e["z_off"]:e["z_off"] + e["d"]], one["z"])
