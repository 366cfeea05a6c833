"""GPU parity of em_solve_batch (persistent shape-class kernels) and
em_solve_plain (one launch per instance) against the FP64 oracle
(Algorithm 1 per instance).

Tolerance: max |z_gpu - z_oracle| <= 1e-4 * D per coordinate, D = hi - lo.
"""

import numpy as np
import pytest

import oracle
import synth
from helpers import rel_errors, report, run_batch

pytestmark = pytest.mark.gpu


def _z_blocks(batch, z):
    out = []
    for b in range(batch.B):
        e = batch.inst[b]
        out.append(z[e["z_off"]:e["z_off"] + e["d"]])
    return out


def _check(batch, got, ref, D, name, tol=1e-4):
    emax, erms = rel_errors(got[:batch.z_size], ref[:batch.z_size], D)
    report(name, emax, erms)
    assert emax <= tol


@pytest.mark.parametrize("plain", [False, True])
def test_mixed_shapes_fixed_iterations(plain):
    """Uneven n in [1, 512] and d in {1..64} across all shape classes, 25 iterations."""
    b = synth.make_pointset_batch(11, 60 if plain else 400, n_lo=1, n_hi=512,
                                  d_choices=(1, 2, 3, 4, 5, 8, 15, 16, 17, 31, 33, 48, 49, 64))
    got, st = run_batch(b, 0.5, 25, 0.0, oracle.INIT_MAXW, plain=plain)
    ref = oracle.em_batch(b, 0.5, 25, 0.0, init=oracle.INIT_MAXW)
    _check(b, got, ref["z"], 6.0, f"batch mixed T25 plain={plain}")
    assert np.all(st["iters"] == 25)


def test_pointset_workload_tolerance_mode():
    """The point-set workload's distribution (n ~ U{8..512}, d ~ {2,3,16,49,64},
    Student-t outliers, box [-3,3]) at tol 1e-4: the oracle is rerun at the
    GPU's iteration count per instance."""
    b = synth.make_pointset_batch(505, 512)
    mu = synth.configs.POINTSET_MU
    got, st = run_batch(b, mu, synth.configs.POINTSET_MAX_ITER, synth.configs.POINTSET_TOL,
                        oracle.INIT_MAXW)
    ref = oracle.em_batch(b, mu, synth.configs.POINTSET_MAX_ITER, 0.0, init=oracle.INIT_MAXW,
                          max_iter_each=st["iters"])
    _check(b, got, ref["z"], 6.0, "pointsets tol-mode (oracle at GPU iterations)")
    print(f"[parity] pointsets: mean iters {st['iters'].mean():.1f}, "
          f"converged {np.mean(st['flags'] == 1):.3f}", flush=True)


def test_large_instances_patch_regression():
    """n = 441, d = 49: window patches of a noisy image as an explicit batch."""
    wl = synth.nlem_256()
    img = wl.images[0].noisy.astype(np.float64)
    P = np.pad(img, 3, mode="symmetric")
    rng = np.random.default_rng(3)
    pts, ws = [], []
    for _ in range(24):
        iy, ix = rng.integers(10, 246, size=2)
        win = [P[y:y + 7, x:x + 7].reshape(-1) for y in range(iy - 10, iy + 11) for x in range(ix - 10, ix + 11)]
        a = np.array(win)
        c = P[iy:iy + 7, ix:ix + 7].reshape(-1)
        pts.append(a.astype(np.float32))
        ws.append(np.exp(-np.sum((a - c) ** 2, axis=1) / 200.0 ** 2).astype(np.float32))
    b = synth.pointsets.pack_instances(pts, ws, 0.0, 255.0)
    got, st = run_batch(b, 1e-3, 30, 0.0, oracle.INIT_MAXW)
    ref = oracle.em_batch(b, 1e-3, 30, 0.0, init=oracle.INIT_MAXW)
    _check(b, got, ref["z"], 255.0, "batch n441 d49 T30")


def test_edge_instances():
    """n = 0 (EMPTY, z untouched), a negative weight and a NaN point
    (BAD_INPUT, z = NaN), n = 1, d = 1, all-zero weights, max_iter = 0 with a
    given start, and an unbounded box."""
    rng = np.random.default_rng(5)
    pts = [np.zeros((0, 3), np.float32), rng.normal(size=(5, 2)).astype(np.float32),
           np.array([[1.0, np.nan]], np.float32), rng.normal(size=(1, 4)).astype(np.float32) * 5,
           rng.normal(size=(9, 1)).astype(np.float32), rng.normal(size=(6, 3)).astype(np.float32)]
    ws = [np.zeros(0, np.float32), np.array([1, 1, -1, 1, 1], np.float32), np.ones(1, np.float32),
          np.ones(1, np.float32), rng.uniform(0.1, 2, 9).astype(np.float32), np.zeros(6, np.float32)]
    b = synth.pointsets.pack_instances(pts, ws, -3.0, 3.0)
    z0 = rng.uniform(-1, 1, b.z_size).astype(np.float32)
    got, st = run_batch(b, 0.7, 40, 0.0, oracle.INIT_GIVEN, z0=z0)
    ref = oracle.em_batch(b, 0.7, 40, 0.0, init=oracle.INIT_GIVEN, z0=z0)
    zg, zr = _z_blocks(b, got), _z_blocks(b, ref["z"])
    assert st["flags"][0] == 4 and np.array_equal(zg[0], z0[0:3].astype(np.float64))
    assert st["flags"][1] == 8 and np.all(np.isnan(zg[1]))
    assert st["flags"][2] == 8 and np.all(np.isnan(zg[2]))
    for k in (3, 4, 5):
        emax, _ = rel_errors(zg[k], zr[k], 6.0)
        assert emax <= 1e-4, (k, zg[k], zr[k])
    np.testing.assert_array_equal(st["flags"][3:], ref["flags"][3:])
    got0, st0 = run_batch(b, 0.7, 0, 1e-4, oracle.INIT_GIVEN, z0=z0)
    for k in (3, 4, 5):
        np.testing.assert_array_equal(_z_blocks(b, got0)[k], _z_blocks(b, z0.astype(np.float64))[k])
    bu = synth.pointsets.pack_instances(pts[3:], ws[3:], float("-inf"), float("inf"))
    gu, su = run_batch(bu, 0.7, 3000, 1e-5, oracle.INIT_MAXW)
    ru = oracle.em_batch(bu, 0.7, 3000, 0.0, init=oracle.INIT_MAXW, max_iter_each=su["iters"])
    for zg_, zr_, e in zip(_z_blocks(bu, gu), _z_blocks(bu, ru["z"]), bu.inst):
        emax, _ = rel_errors(zg_, zr_, 1.0)
        assert emax <= 1e-4


def test_invalid_arguments_rejected():
    import torch
    import paper_1501_03879_amd as emx
    from helpers import gpu, handle
    dev = gpu()
    b = synth.make_pointset_batch(1, 4, n_hi=20)
    a = torch.from_numpy(b.a).to(dev)
    w = torch.from_numpy(b.w).to(dev)
    inst = emx.instances_tensor(b.inst, dev)
    z = torch.zeros(b.z_size, device=dev)
    hd = handle()
    for kw in (dict(rho=0.0), dict(rho=float("nan")), dict(max_iter=-1), dict(tol=float("nan")),
               dict(lo=1.0, hi=0.0), dict(init=7)):
        args = dict(lo=-3.0, hi=3.0, rho=0.5, max_iter=5, tol=0.0)
        args.update(kw)
        with pytest.raises(emx.EmxError) as ei:
            hd.em_solve_batch(a, w, inst, z, None, **args)
        assert ei.value.status == emx.EM_ERR_INVALID_ARG
