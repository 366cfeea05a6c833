"""FP64 CPU oracle for EM-ADMM, IRLS on the smooth surrogate, NLEM and NLM
(ctypes shim over em_oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg may use this package; the product path never
does.  It shares no code with the GPU library.

Parity pins: every function here is checked in ``tests/test_oracle_pins.py``
against closed forms, optimality conditions and brute force (see each
test's docstring for the passage it follows).
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "em_oracle.c")
_LIB = os.path.join(_HERE, "libemoracle.so")

CONVERGED, MAXITER, EMPTY, BAD_INPUT = 1, 2, 4, 8
INIT_GIVEN, INIT_MAXW, INIT_WMEAN = 0, 1, 2
SOLVER_ADMM, SOLVER_IRLS, SOLVER_FAST_ADMM, SOLVER_WPEN = 0, 1, 3, 4
NLEM_INIT_NOISY, NLEM_INIT_NLM = 0, 1


def build(force: bool = True) -> str:
    """Compile em_oracle.c with gcc -O2 (no fast-math) and OpenMP."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-fno-fast-math", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = C.CDLL(_LIB)
        dp, fp, i64p, i32p = (C.POINTER(C.c_double), C.POINTER(C.c_float),
                              C.POINTER(C.c_int64), C.POINTER(C.c_int32))
        lib.oracle_prox.argtypes = [C.c_int64, dp, dp, C.c_double, dp]
        lib.oracle_prox.restype = None
        lib.oracle_em_solve.argtypes = [C.c_int64, C.c_int64, dp, dp, C.c_double, C.c_double,
                                        C.c_double, dp, dp, dp, C.c_int64, C.c_double,
                                        i64p, dp, dp]
        lib.oracle_em_solve.restype = C.c_int
        lib.oracle_em_solve_ex.argtypes = [C.c_int64, C.c_int64, dp, dp, C.c_double, dp, dp, dp, dp,
                                           dp, C.c_int64, C.c_double, C.c_int64, C.c_double,
                                           C.c_double, i64p, dp, dp, dp]
        lib.oracle_em_solve_ex.restype = C.c_int
        lib.oracle_em_solve_wpen.argtypes = [C.c_int64, C.c_int64, dp, dp, C.c_double, dp, dp, dp,
                                             C.c_int64, C.c_double, i64p, dp, dp]
        lib.oracle_em_solve_wpen.restype = C.c_int
        lib.oracle_em_solve_wpen_ball.argtypes = [C.c_int64, C.c_int64, dp, dp, C.c_double, dp,
                                                  C.c_double, dp, C.c_int64, C.c_double, i64p, dp, dp]
        lib.oracle_em_solve_wpen_ball.restype = C.c_int
        lib.oracle_em_solve_fast.argtypes = [C.c_int64, C.c_int64, dp, dp, C.c_double, dp, dp, dp,
                                             C.c_int64, C.c_double, C.c_double, i64p, dp, dp, i64p]
        lib.oracle_em_solve_fast.restype = C.c_int
        lib.oracle_irls_solve_ex.argtypes = [C.c_int64, C.c_int64, dp, dp, C.c_double, dp, dp, dp,
                                             C.c_int64, C.c_double, i64p, dp, dp]
        lib.oracle_irls_solve_ex.restype = C.c_int
        lib.oracle_em_solve_ball.argtypes = [C.c_int64, C.c_int64, dp, dp, C.c_double, dp, C.c_double,
                                             dp, dp, dp, C.c_int64, C.c_double, C.c_int64, C.c_double,
                                             C.c_double, i64p, dp, dp, dp]
        lib.oracle_em_solve_ball.restype = C.c_int
        lib.oracle_irls_solve_ball.argtypes = [C.c_int64, C.c_int64, dp, dp, C.c_double, dp, C.c_double,
                                               dp, C.c_int64, C.c_double, i64p, dp, dp]
        lib.oracle_irls_solve_ball.restype = C.c_int
        lib.oracle_em_batch_ex.argtypes = [C.c_int64, fp, fp, i64p, i64p, i64p, i32p, i32p, C.c_int,
                                           C.c_double, C.c_double, C.c_double, C.c_double, fp, fp, fp, fp,
                                           C.c_int64, i32p, C.c_double, C.c_int, C.c_int64,
                                           C.c_double, C.c_double, dp, i32p, i32p, dp, dp, dp, C.c_double,
                                           i32p, C.c_int, C.c_double, i32p]
        lib.oracle_em_batch_ex.restype = C.c_int
        lib.oracle_em_batch.argtypes = [C.c_int64, fp, fp, i64p, i64p, i64p, i32p, i32p,
                                        C.c_double, C.c_double, C.c_double, C.c_int64, i32p,
                                        C.c_double, C.c_int, dp, i32p, i32p, dp, dp, C.c_int]
        lib.oracle_em_batch.restype = C.c_int
        lib.oracle_nlem.argtypes = [C.c_int64, C.c_int64, fp, C.c_int64, C.c_int64, C.c_double,
                                    C.c_double, C.c_double, C.c_double, C.c_int64, i32p,
                                    C.c_double, C.c_int64, i64p, dp, dp, dp, i32p, i32p, dp, dp,
                                    C.c_int]
        lib.oracle_nlem.restype = C.c_int
        lib.oracle_nlem_ex.argtypes = [C.c_int64, C.c_int64, fp, C.c_int64, C.c_int64,
                                       C.c_double, C.c_double, C.c_double, C.c_int, C.c_int,
                                       C.c_double, C.c_double, C.c_int64, i32p, C.c_double,
                                       C.c_int64, i64p, dp, dp, dp, i32p, i32p, dp, dp, C.c_int]
        lib.oracle_nlem_ex.restype = C.c_int
        lib.oracle_irls_solve.argtypes = [C.c_int64, C.c_int64, dp, dp, C.c_double, C.c_double,
                                          C.c_double, dp, C.c_int64, C.c_double, i64p, dp, dp]
        lib.oracle_irls_solve.restype = C.c_int
        lib.oracle_em_objective.argtypes = [C.c_int64, C.c_int64, dp, dp, dp]
        lib.oracle_em_objective.restype = C.c_double
        lib.oracle_surrogate_objective.argtypes = [C.c_int64, C.c_int64, dp, dp, C.c_double, dp]
        lib.oracle_surrogate_objective.restype = C.c_double
        lib.oracle_max_threads.argtypes = []
        lib.oracle_max_threads.restype = C.c_int
        _lib = lib
    return _lib


def _p(arr, ctype):
    if arr is None:
        return None
    return arr.ctypes.data_as(C.POINTER(ctype))


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def prox(v, u, lam: float) -> np.ndarray:
    """Closed-form prox Psi_lambda(v, u) of lambda * ||x - u|| (equation closed-form)."""
    v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
    out = np.empty_like(v)
    _load().oracle_prox(v.size, _p(v, C.c_double), _p(u, C.c_double), float(lam),
                        _p(out, C.c_double))
    return out


def _box(lo, hi, d):
    lv = np.ascontiguousarray(np.broadcast_to(np.asarray(lo, np.float64), (d,)), dtype=np.float64)
    hv = np.ascontiguousarray(np.broadcast_to(np.asarray(hi, np.float64), (d,)), dtype=np.float64)
    return lv, hv


def em_solve(a, w, mu: float, lo, hi, z0, y0=None, max_iter: int = 100, tol: float = 0.0,
             adapt_every: int = 0, adapt_ratio: float = 10.0, adapt_factor: float = 2.0) -> dict:
    """One instance of Algorithm 1 in FP64 over the box [lo, hi] (scalars or
    per-coordinate arrays), optionally with the adaptive penalty; returns z,
    y, x, iters, residuals, flags and the final penalty mu."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a.reshape(-1, 1)
    n, d = a.shape
    w = np.ascontiguousarray(w, dtype=np.float64).reshape(-1)
    assert w.size == n
    z = np.array(z0, dtype=np.float64).reshape(-1).copy()
    assert z.size == d
    y = np.zeros((n, d)) if y0 is None else np.array(y0, dtype=np.float64).reshape(n, d).copy()
    x = np.zeros((n, d))
    lv, hv = _box(lo, hi, d)
    it = C.c_int64(0)
    rp = C.c_double(0.0)
    rd = C.c_double(0.0)
    mf = C.c_double(0.0)
    f = _load().oracle_em_solve_ex(n, d, _p(a, C.c_double), _p(w, C.c_double), float(mu),
                                   _p(lv, C.c_double), _p(hv, C.c_double), _p(z, C.c_double),
                                   _p(y, C.c_double), _p(x, C.c_double), int(max_iter), float(tol),
                                   int(adapt_every), float(adapt_ratio), float(adapt_factor),
                                   C.byref(it), C.byref(rp), C.byref(rd), C.byref(mf))
    return dict(z=z, y=y, x=x, iters=int(it.value), r_pri=rp.value, r_dual=rd.value, flags=int(f),
                mu=mf.value)


def em_solve_ball(a, w, mu: float, center, radius: float, z0, max_iter: int = 100,
                  tol: float = 0.0, adapt_every: int = 0, adapt_ratio: float = 10.0,
                  adapt_factor: float = 2.0) -> dict:
    """Algorithm 1 in FP64 over the ball ||z - center|| <= radius."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a.reshape(-1, 1)
    n, d = a.shape
    w = np.ascontiguousarray(w, dtype=np.float64).reshape(-1)
    z = np.array(z0, dtype=np.float64).reshape(-1).copy()
    cen = np.ascontiguousarray(np.broadcast_to(np.asarray(center, np.float64), (d,)), dtype=np.float64)
    y = np.zeros((n, d))
    x = np.zeros((n, d))
    it = C.c_int64(0)
    rp = C.c_double(0.0)
    rd = C.c_double(0.0)
    mf = C.c_double(0.0)
    f = _load().oracle_em_solve_ball(n, d, _p(a, C.c_double), _p(w, C.c_double), float(mu),
                                     _p(cen, C.c_double), float(radius), _p(z, C.c_double),
                                     _p(y, C.c_double), _p(x, C.c_double), int(max_iter), float(tol),
                                     int(adapt_every), float(adapt_ratio), float(adapt_factor),
                                     C.byref(it), C.byref(rp), C.byref(rd), C.byref(mf))
    return dict(z=z, y=y, x=x, iters=int(it.value), r_pri=rp.value, r_dual=rd.value, flags=int(f),
                mu=mf.value)


def irls_solve_ball(a, w, eps: float, center, radius: float, z0, max_iter: int = 100,
                    tol: float = 0.0) -> dict:
    """IRLS on the surrogate in FP64 over the ball ||z - center|| <= radius."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a.reshape(-1, 1)
    n, d = a.shape
    w = np.ascontiguousarray(w, dtype=np.float64).reshape(-1)
    z = np.array(z0, dtype=np.float64).reshape(-1).copy()
    cen = np.ascontiguousarray(np.broadcast_to(np.asarray(center, np.float64), (d,)), dtype=np.float64)
    it = C.c_int64(0)
    rp = C.c_double(0.0)
    rd = C.c_double(0.0)
    f = _load().oracle_irls_solve_ball(n, d, _p(a, C.c_double), _p(w, C.c_double), float(eps),
                                       _p(cen, C.c_double), float(radius), _p(z, C.c_double),
                                       int(max_iter), float(tol), C.byref(it), C.byref(rp), C.byref(rd))
    return dict(z=z, iters=int(it.value), r_dual=rd.value, flags=int(f))


def em_solve_wpen(a, w, mu: float, lo, hi, z0, max_iter: int = 100, tol: float = 0.0,
                  center=None, radius=None) -> dict:
    """The weighted-mean variant of the consensus ADMM (penalty mu w_k on the
    constraint of point k) in FP64, over the box [lo, hi] (scalars or per
    coordinate) or, when radius is given, the ball ||z - center|| <= radius."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a.reshape(-1, 1)
    n, d = a.shape
    w = np.ascontiguousarray(w, dtype=np.float64).reshape(-1)
    z = np.array(z0, dtype=np.float64).reshape(-1).copy()
    it = C.c_int64(0)
    rp = C.c_double(0.0)
    rd = C.c_double(0.0)
    if radius is None:
        lv = np.ascontiguousarray(np.broadcast_to(np.asarray(lo, np.float64), (d,)), dtype=np.float64)
        hv = np.ascontiguousarray(np.broadcast_to(np.asarray(hi, np.float64), (d,)), dtype=np.float64)
        f = _load().oracle_em_solve_wpen(n, d, _p(a, C.c_double), _p(w, C.c_double), float(mu),
                                         _p(lv, C.c_double), _p(hv, C.c_double), _p(z, C.c_double),
                                         int(max_iter), float(tol), C.byref(it), C.byref(rp), C.byref(rd))
    else:
        cen = np.zeros(d) if center is None else np.asarray(center, np.float64)
        cen = np.ascontiguousarray(np.broadcast_to(cen, (d,)), dtype=np.float64)
        f = _load().oracle_em_solve_wpen_ball(n, d, _p(a, C.c_double), _p(w, C.c_double), float(mu),
                                              _p(cen, C.c_double), float(radius), _p(z, C.c_double),
                                              int(max_iter), float(tol), C.byref(it), C.byref(rp),
                                              C.byref(rd))
    return dict(z=z, iters=int(it.value), r_pri=rp.value, r_dual=rd.value, flags=int(f))


def em_solve_fast(a, w, mu: float, lo, hi, z0, max_iter: int = 100, tol: float = 0.0,
                  eta: float = 0.999) -> dict:
    """Accelerated ADMM (fast ADMM with restart) in FP64 over the box [lo, hi];
    returns z, iters, residuals, flags and the number of restarts."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a.reshape(-1, 1)
    n, d = a.shape
    w = np.ascontiguousarray(w, dtype=np.float64).reshape(-1)
    z = np.array(z0, dtype=np.float64).reshape(-1).copy()
    assert w.size == n and z.size == d
    lv, hv = _box(lo, hi, d)
    it = C.c_int64(0)
    rs = C.c_int64(0)
    rp = C.c_double(0.0)
    rd = C.c_double(0.0)
    f = _load().oracle_em_solve_fast(n, d, _p(a, C.c_double), _p(w, C.c_double), float(mu),
                                     _p(lv, C.c_double), _p(hv, C.c_double), _p(z, C.c_double),
                                     int(max_iter), float(tol), float(eta), C.byref(it),
                                     C.byref(rp), C.byref(rd), C.byref(rs))
    return dict(z=z, iters=int(it.value), r_pri=rp.value, r_dual=rd.value, flags=int(f),
                restarts=int(rs.value))


def em_batch(batch, mu: float, max_iter: int, tol: float, init: int = INIT_MAXW, z0=None,
             max_iter_each=None, nthreads: int = 0, solver: int = SOLVER_ADMM, eps: float = 1e-6,
             box_lo=None, box_hi=None, adapt_every: int = 0, adapt_ratio: float = 10.0,
             adapt_factor: float = 2.0, eta: float = 0.999, ball_center=None,
             ball_radius=None, tie_band: float = 2e-6) -> dict:
    """Batch of instances (a ``synth.PointSetBatch`` or anything with a, w, inst,
    z_size, lo, hi).  solver: SOLVER_ADMM (adapt_every > 0: adaptive penalty),
    SOLVER_IRLS, SOLVER_FAST_ADMM (restart parameter eta) or SOLVER_WPEN (the
    weighted-mean variant, penalties mu w_k); box_lo / box_hi:
    optional float32 per-coordinate bounds indexed like z; ball_radius
    (float32, one per instance) selects the ball constraint with centres
    ball_center (float32 indexed like z, None = origin).  Returns z (float64,
    concatenated), iters, flags, residuals, the final penalties and the
    accelerated ADMM's restart counts and its near-tie decisions (ties: those
    with |c - thr| <= tie_band thr, thr = eta (1 - 2^-16) c_prev, where a run
    in a lower precision may take either branch)."""
    inst = batch.inst
    B = int(inst.shape[0])
    a = np.ascontiguousarray(batch.a, dtype=np.float32)
    w = np.ascontiguousarray(batch.w, dtype=np.float32)
    a_off = np.ascontiguousarray(inst["a_off"], dtype=np.int64)
    w_off = np.ascontiguousarray(inst["w_off"], dtype=np.int64)
    z_off = np.ascontiguousarray(inst["z_off"], dtype=np.int64)
    n = np.ascontiguousarray(inst["n"], dtype=np.int32)
    d = np.ascontiguousarray(inst["d"], dtype=np.int32)
    z = np.zeros(batch.z_size, dtype=np.float64) if z0 is None else np.array(z0, np.float64).copy()
    bl = None if box_lo is None else np.ascontiguousarray(box_lo, dtype=np.float32)
    bh = None if box_hi is None else np.ascontiguousarray(box_hi, dtype=np.float32)
    bc = None if ball_center is None else np.ascontiguousarray(ball_center, dtype=np.float32)
    br = None if ball_radius is None else np.ascontiguousarray(ball_radius, dtype=np.float32)
    iters = np.zeros(B, np.int32)
    flags = np.zeros(B, np.int32)
    rp = np.zeros(B)
    rd = np.zeros(B)
    mf = np.zeros(B)
    rs = np.zeros(B, np.int32)
    ti = np.zeros(B, np.int32)
    mie = None if max_iter_each is None else np.ascontiguousarray(max_iter_each, dtype=np.int32)
    _load().oracle_em_batch_ex(B, _p(a, C.c_float), _p(w, C.c_float), _p(a_off, C.c_int64),
                               _p(w_off, C.c_int64), _p(z_off, C.c_int64), _p(n, C.c_int32),
                               _p(d, C.c_int32), int(solver), float(mu), float(eps), float(batch.lo),
                               float(batch.hi), _p(bl, C.c_float), _p(bh, C.c_float),
                               _p(bc, C.c_float), _p(br, C.c_float), int(max_iter),
                               _p(mie, C.c_int32), float(tol), int(init), int(adapt_every),
                               float(adapt_ratio), float(adapt_factor), _p(z, C.c_double),
                               _p(iters, C.c_int32), _p(flags, C.c_int32), _p(rp, C.c_double),
                               _p(rd, C.c_double), _p(mf, C.c_double), float(eta),
                               _p(rs, C.c_int32), int(nthreads), float(tie_band), _p(ti, C.c_int32))
    return dict(z=z, iters=iters, flags=flags, r_pri=rp, r_dual=rd, mu=mf, restarts=rs, ties=ti)


def nlem(img, patch_radius: int, window_radius: int, h: float, lo: float, hi: float,
         mu: float, max_iter: int, tol: float, pix=None, max_iter_each=None,
         want_z: bool = False, want_weights: bool = False, nthreads: int = 0,
         solver: int = SOLVER_ADMM, init: int = NLEM_INIT_NOISY, eps: float = 1e-6) -> dict:
    """NLEM on the float32 image ``img`` (H x W) for the pixels ``pix`` (linear
    indices; None = all).  solver: SOLVER_ADMM (Algorithm 1, penalty mu) or
    SOLVER_IRLS (surrogate with eps); init: the noisy patch or the NLM patch.
    Returns out (float64), iters, flags, residuals and optionally the full
    patches z and the window weights."""
    img = np.ascontiguousarray(img, dtype=np.float32)
    H, W = img.shape
    d = (2 * patch_radius + 1) ** 2
    nmax = (2 * window_radius + 1) ** 2
    pixa = None if pix is None else np.ascontiguousarray(pix, dtype=np.int64)
    npix = H * W if pixa is None else int(pixa.size)
    out = np.zeros(npix)
    zf = np.zeros((npix, d)) if want_z else None
    wo = np.zeros((npix, nmax)) if want_weights else None
    iters = np.zeros(npix, np.int32)
    flags = np.zeros(npix, np.int32)
    rp = np.zeros(npix)
    rd = np.zeros(npix)
    mie = None if max_iter_each is None else np.ascontiguousarray(max_iter_each, dtype=np.int32)
    _load().oracle_nlem_ex(H, W, _p(img, C.c_float), int(patch_radius), int(window_radius),
                           float(h), float(lo), float(hi), int(solver), int(init), float(mu),
                           float(eps), int(max_iter), _p(mie, C.c_int32), float(tol), npix,
                           _p(pixa, C.c_int64), _p(out, C.c_double), _p(zf, C.c_double),
                           _p(wo, C.c_double), _p(iters, C.c_int32), _p(flags, C.c_int32),
                           _p(rp, C.c_double), _p(rd, C.c_double), int(nthreads))
    res = dict(out=out, iters=iters, flags=flags, r_pri=rp, r_dual=rd)
    if want_z:
        res["z"] = zf
    if want_weights:
        res["weights"] = wo
    return res


def nlm(img, patch_radius: int, window_radius: int, h: float, pix=None, want_z: bool = False,
        nthreads: int = 0) -> dict:
    """Non-Local Means: per pixel the weighted mean sum_j w_ij P_j / sum_j w_ij of
    the window's patches (the NLEM weights); ``out`` is its centre pixel."""
    return nlem(img, patch_radius, window_radius, h, 0.0, 1.0, 1.0, 0, 0.0, pix=pix,
                want_z=want_z, nthreads=nthreads, init=NLEM_INIT_NLM)


def irls_solve(a, w, eps: float, lo: float, hi: float, z0, max_iter: int = 100,
               tol: float = 0.0) -> dict:
    """IRLS (majorise-minimise) on the surrogate sum_k w_k (||z - a_k||^2 + eps)^(1/2)
    over the box [lo, hi] (scalars or per-coordinate arrays), in FP64; returns
    z, iters, r_dual, flags."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a.reshape(-1, 1)
    n, d = a.shape
    w = np.ascontiguousarray(w, dtype=np.float64).reshape(-1)
    z = np.array(z0, dtype=np.float64).reshape(-1).copy()
    assert w.size == n and z.size == d
    lv, hv = _box(lo, hi, d)
    it = C.c_int64(0)
    rp = C.c_double(0.0)
    rd = C.c_double(0.0)
    f = _load().oracle_irls_solve_ex(n, d, _p(a, C.c_double), _p(w, C.c_double), float(eps),
                                     _p(lv, C.c_double), _p(hv, C.c_double), _p(z, C.c_double),
                                     int(max_iter), float(tol), C.byref(it), C.byref(rp), C.byref(rd))
    return dict(z=z, iters=int(it.value), r_dual=rd.value, flags=int(f))


def em_objective(a, w, z) -> float:
    """sum_k w_k ||z - a_k|| (the objective of (EM))."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a.reshape(-1, 1)
    n, d = a.shape
    w = np.ascontiguousarray(w, dtype=np.float64).reshape(-1)
    z = np.ascontiguousarray(z, dtype=np.float64).reshape(-1)
    return float(_load().oracle_em_objective(n, d, _p(a, C.c_double), _p(w, C.c_double),
                                             _p(z, C.c_double)))


def surrogate_objective(a, w, eps: float, z) -> float:
    """sum_k w_k (||z - a_k||^2 + eps)^(1/2), equation (EM_surrogate)."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.ndim == 1:
        a = a.reshape(-1, 1)
    n, d = a.shape
    w = np.ascontiguousarray(w, dtype=np.float64).reshape(-1)
    z = np.ascontiguousarray(z, dtype=np.float64).reshape(-1)
    return float(_load().oracle_surrogate_objective(n, d, _p(a, C.c_double), _p(w, C.c_double),
                                                    float(eps), _p(z, C.c_double)))