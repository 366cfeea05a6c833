"""Exact, hand-worked pins of the accelerated ADMM in the oracle (fast ADMM
with restart, [Goldstein2012], the extension the paper's conclusion names).

The momentum weights come from the textbook Nesterov sequence alone:
alpha_1 = 1, alpha_{k+1} = (1 + sqrt(1 + 4 alpha_k^2)) / 2, and the weight
applied after sweep k is beta_k = (alpha_k - 1) / alpha_{k+1} (so beta_1 = 0,
beta_2 = (phi - 1) / alpha_3 with phi the golden ratio).  Everything else is
worked out by hand below for d = 1, where the prox of (closed-form) is
x = a when |v - a| <= lambda and v - lambda sign(v - a) otherwise.

A mistake in the momentum weight (alpha / alpha' instead of
(alpha - 1) / alpha', an index shifted by one), in which iterate is
extrapolated (z_hat from z0 instead of the previous z, y_hat left at y), or in
the restart (z_hat, y_hat taken from the current instead of the previous
iterate) changes at least one of the values pinned here.
"""

import math

import pytest

ETA = 0.999


def nesterov_betas(k):
    """beta_1 .. beta_k of the textbook sequence."""
    alpha = [1.0]
    for _ in range(k):
        alpha.append((1.0 + math.sqrt(1.0 + 4.0 * alpha[-1] ** 2)) / 2.0)
    return [(alpha[i] - 1.0) / alpha[i + 1] for i in range(k)]


def test_nesterov_sequence_textbook_values():
    """alpha_2 = (1 + sqrt 5) / 2 (the golden ratio), so beta_1 = 0 and
    beta_2 = (phi - 1) / alpha_3 with alpha_3 = (1 + sqrt(7 + 2 sqrt 5)) / 2."""
    b = nesterov_betas(3)
    phi = (1 + math.sqrt(5)) / 2
    a3 = (1 + math.sqrt(7 + 2 * math.sqrt(5))) / 2
    assert b[0] == 0.0
    assert abs(b[1] - (phi - 1) / a3) <= 1e-15
    assert 0.28 < b[1] < 0.29 and 0.43 < b[2] < 0.44


def _run(orc, a, lam_w, mu, z0, T, lo=-10.0, hi=10.0):
    return orc.em_solve_fast([[p] for p in a], lam_w, mu, lo, hi, [z0], max_iter=T, tol=0.0, eta=ETA)


def test_momentum_sweeps_three_and_four_exact(orc):
    """Points 1, 3, 5, weights 2, mu = 1 (lambda = 2), z0 = 4, box [-10, 10].

    t = 1 (z_hat = 4, y_hat = 0): v - a = (3, 1, -1), so x = (2, 3, 5),
      z1 = 10/3, y1 = x - z1 = (-4/3, -1/3, 5/3); c1 = 42/9 + 3 (2/3)^2 = 6.
      c_prev = inf: momentum with beta_1 = 0, so z_hat = z1, y_hat = y1.
    From t = 2 on, the middle point stays within lambda of v and the outer two
    do not, so x = (z_hat - y_hat_1 - 2, 3, z_hat - y_hat_3 + 2) and
      z = (2 z_hat + 3 + y_hat_2) / 3,   y = y_hat + x - z
      (y_1 = z_hat - 2 - z, y_2 = y_hat_2 + 3 - z, y_3 = z_hat + 2 - z).
    t = 2: z2 = (20/3 + 3 - 1/3) / 3 = 28/9, y2 = (-16/9, -4/9, 20/9);
      c2 = 42/81 + 3 (2/9)^2 = 2/3 < eta c1: momentum with beta_2,
      z_hat = 28/9 - 2 beta_2 / 9, y_hat_2 = -4/9 - beta_2 / 9.
    t = 3: z3 = (79 - 5 beta_2) / 27,  y3_2 = (-10 + 2 beta_2) / 27;
      c3 ~ 0.155 < eta c2: momentum with beta_3.
    t = 4: z_hat = z3 + beta_3 (z3 - z2), y_hat_2 = y3_2 + beta_3 (y3_2 + 4/9),
      z4 = (229 - 8 beta_2 - 8 beta_3 (1 + beta_2)) / 81.
    z3 needs the y extrapolation (y2 != y1) as well as the z one."""
    b = nesterov_betas(4)
    b2, b3 = b[1], b[2]
    for T, want in ((1, 10 / 3), (2, 28 / 9), (3, (79 - 5 * b2) / 27),
                    (4, (229 - 8 * b2 - 8 * b3 * (1 + b2)) / 81)):
        r = _run(orc, [1.0, 3.0, 5.0], [2.0, 2.0, 2.0], 1.0, 4.0, T)
        assert abs(r["z"][0] - want) <= 1e-14, (T, r["z"][0], want)
        assert r["restarts"] == 0
        assert abs(r["r_dual"] - abs(want - _run(orc, [1.0, 3.0, 5.0], [2.0] * 3, 1.0, 4.0, T - 1)["z"][0])) <= 1e-14


def test_restart_returns_to_the_previous_iterate_exact(orc):
    """Same instance.  After t = 5 the progress measure c5 (~0.10010) is not
    below eta c4 (~0.09999): restart (counted when a sixth sweep is allowed;
    no decision follows the last allowed sweep).  The next sweep then starts from the previous
    iterate, z_hat = z4 and y_hat = y4 (not z5, y5), with the same branch
    pattern, so z6 = (2 z4 + 3 + y4_2) / 3 where
      y4_2 = y_hat4_2 + 3 - z4,  y_hat4_2 = (-10 + 2 beta_2 + 2 beta_3 (1 + beta_2)) / 27."""
    b = nesterov_betas(5)
    b2, b3 = b[1], b[2]
    z4 = (229 - 8 * b2 - 8 * b3 * (1 + b2)) / 81
    yh4 = (-10 + 2 * b2 + 2 * b3 * (1 + b2)) / 27
    y4 = yh4 + 3 - z4
    assert _run(orc, [1.0, 3.0, 5.0], [2.0, 2.0, 2.0], 1.0, 4.0, 5)["restarts"] == 0
    r6 = _run(orc, [1.0, 3.0, 5.0], [2.0, 2.0, 2.0], 1.0, 4.0, 6)
    assert r6["restarts"] == 1
    assert abs(r6["z"][0] - (2 * z4 + 3 + y4) / 3) <= 1e-14, r6["z"][0]


def test_restart_on_the_appendix_example(orc):
    """The worked example of Algorithm 1 (points 0, 1, 5, unit weights, mu = 1,
    box [0, 10], z0 = 3).  Sweeps 1 and 2 are Algorithm 1's (z = 8/3, 7/3;
    y = (-2/3, -2/3, 4/3) after both, since x = z at t = 2), with c1 = 3 and
    c2 = 3 (1/3)^2 = 1/3 < eta c1, so z_hat = 7/3 - beta_2 / 3, y_hat = y2.
    t = 3: v = z_hat - y = (3 - beta_2/3, 3 - beta_2/3, 1 - beta_2/3) is
    farther than 1 from every point, x = v -/+ 1 = 2 - beta_2/3 each, so
    z3 = 2 - beta_2 / 3 and c3 = 3 (1/3)^2 = 1/3 = c2 > eta c2: restart,
    z_hat = z2 = 7/3, y_hat = y2.  t = 4 is then Algorithm 1's third sweep
    from (7/3, y2): z4 = 2 exactly (with momentum it would be
    about 1.39)."""
    b2 = nesterov_betas(2)[1]
    a, w = [0.0, 1.0, 5.0], [1.0, 1.0, 1.0]
    for T, want in ((1, 8 / 3), (2, 7 / 3), (3, 2 - b2 / 3)):
        r = _run(orc, a, w, 1.0, 3.0, T, lo=0.0, hi=10.0)
        assert abs(r["z"][0] - want) <= 1e-14, (T, r["z"][0])
        assert r["restarts"] == 0, (T, r["restarts"])
    r = _run(orc, a, w, 1.0, 3.0, 4, lo=0.0, hi=10.0)
    assert abs(r["z"][0] - 2.0) <= 1e-14, r["z"][0]
    assert r["restarts"] == 1


@pytest.mark.parametrize("eta", [0.5, 0.999])
def test_restart_threshold_scales_with_eta(orc, eta):
    """c3 = c2 exactly on the appendix example, so the restart after t = 3
    happens for any eta < 1 (seen with max_iter = 4: no decision follows the
    last allowed sweep, which has nothing after it)."""
    for T, rs in ((3, 0), (4, 1)):
        r = orc.em_solve_fast([[0.0], [1.0], [5.0]], [1.0, 1.0, 1.0], 1.0, 0.0, 10.0, [3.0],
                              max_iter=T, tol=0.0, eta=eta)
        assert r["restarts"] == rs


def test_stalled_iterate_exact_tie_goes_to_restart(orc):
    """Points 5 and 6 with weights 1e6 (lambda = 1e6, every prox returns its
    own point), mu = 1, box [0, 1], z0 = 1.  Every sweep has x = a and z = 1
    (the mean of x + y_hat is above 1), so c = (5 - 1)^2 + (6 - 1)^2 = 41 on
    every sweep while y drifts by a - 1.  With eta' = eta (1 - 2^-16):
      t = 1: c = 41 < eta' inf: momentum (beta_1 = 0), c_prev = 41.
      t = 2: 41 >= eta' 41: restart (margin 1e-3), c_prev = 41 / eta.
      t = 3: 41 against eta' (41 / eta) = 41 (1 - 2^-16): the exact tie of
        the unguarded test, now 1.5e-5 on the restart side: restart,
        c_prev = 41 / eta^2 (z_hat, y_hat from the start of sweep 3).
      t = 4: 41 < eta' 41 / eta^2: momentum (margin 1e-3), c_prev = 41.
      t = 5: as t = 2: restart.
    Restarts after T sweeps (decisions 1 .. T - 1): 0, 1, 2, 2, 3 for
    T = 2 .. 6.  The batch entry's tie count sees the t = 3 decision with a
    band of 2e-5 and none with the default 2e-6; the decisions worked out by
    hand for the other instances of this file (sweeps 1 .. 3) count nothing."""
    import numpy as np
    from synth.pointsets import pack_instances
    pts = [np.array([[5.0], [6.0]], np.float32), np.array([[1.0], [3.0], [5.0]], np.float32),
           np.array([[0.0], [1.0], [5.0]], np.float32)]
    ws = [np.array([1e6, 1e6], np.float32), np.full(3, 2.0, np.float32), np.ones(3, np.float32)]
    b = pack_instances(pts, ws, 0.0, 1.0)
    lo = np.array([0.0, -10.0, 0.0], np.float32)
    hi = np.array([1.0, 10.0, 10.0], np.float32)
    z0 = np.array([1.0, 4.0, 3.0])

    def run(T, band=2e-6):
        return orc.em_batch(b, 1.0, T, 0.0, init=orc.INIT_GIVEN, z0=z0, solver=orc.SOLVER_FAST_ADMM,
                            box_lo=lo, box_hi=hi, tie_band=band)

    for T, rs in ((2, 0), (3, 1), (4, 2), (5, 2), (6, 3)):
        r = run(T)
        assert r["z"][0] == 1.0 and r["restarts"][0] == rs, (T, r["restarts"])
        assert r["ties"][0] == 0
        if T <= 4:
            assert r["ties"][1] == 0 and r["ties"][2] == 0, (T, r["ties"])
    assert run(4, 2e-5)["ties"][0] == 1
    assert run(3, 2e-5)["ties"][0] == 0
    assert run(6, 1.0)["ties"][0] == 4   # decisions 2 .. 5 (t = 1 compares with an infinite c_prev)
