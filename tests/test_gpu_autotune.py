"""Autotuners and plans (nlem_autotune, nlem_plan_get / nlem_plan_set,
em_batch_autotune, em_batch_plan_get / em_batch_plan_set): a tuned plan
holds values from the searched sets, the handle uses it afterwards, every
variant a plan can name keeps parity with the FP64 oracle (NLEM: 1e-4 of
the intensity range, the oracle rerun at the GPU's per-pixel iteration
counts in tolerance mode, and the GPU's count within the one-iteration lag
of the residual test; batch: 1e-4 D per coordinate), and plans survive in
the EMX_AUTOTUNE_CACHE file for a new handle; cache lines for another
architecture, for an uncompiled variant or garbled ones are ignored."""

import os

import numpy as np
import pytest

import oracle
import synth
from helpers import gpu, rel_errors, report

pytestmark = pytest.mark.gpu
D = 255.0


def _img(seed, H, W, sigma=30.0):
    rng = np.random.default_rng(seed)
    return synth.add_gaussian_noise(rng, synth.piecewise_smooth_image(rng, H, W), sigma).astype(np.float32)


def _item(img):
    import torch
    dev = gpu()
    t = torch.from_numpy(img).to(dev)
    return dict(img=t, out=torch.full(t.shape, -7.0, dtype=torch.float32, device=dev),
                stats=torch.zeros((t.numel(), 4), dtype=torch.int32, device=dev),
                patch_radius=3, window_radius=10, h=300.0)


def _new_handle(monkeypatch, cache):
    import paper_1501_03879_amd as emx
    monkeypatch.setenv("EMX_AUTOTUNE_CACHE", str(cache))
    monkeypatch.delenv("EMX_NLEM_WC", raising=False)
    return emx.Handle(0)


def test_autotune_plan_parity_and_cache(tmp_path, monkeypatch):
    import torch
    cache = tmp_path / "plans.txt"
    hd = _new_handle(monkeypatch, cache)
    default = hd.nlem_plan(3, 10)
    img = _img(3, 40, 44)
    chosen = hd.nlem_autotune(_item(img), max_iter=6, tol=0.0, repeats=2)
    hd.sync()
    assert chosen in (2, 3, 4), chosen          # compiled counts for patch radius 3
    assert hd.nlem_plan(3, 10) == chosen
    print(f"[autotune] r3 R10 chose {chosen} coordinate waves (default {default})", flush=True)

    it = _item(img)
    hd.nlem_denoise_ex([it], max_iter=6, tol=0.0)
    hd.sync()
    got = it["out"].cpu().numpy().reshape(-1).astype(np.float64)
    ref = oracle.nlem(img, 3, 10, 300.0, 0, 255, 1e-3, 6, 0.0)
    e, r = rel_errors(got, ref["out"], D)
    report("nlem after autotune T6", e, r)
    assert e <= 1e-4
    assert torch.all(it["stats"][:, 0] == 6)
    hd.close()

    lines = cache.read_text().split("\n")
    # nlem2 <arch> <pr> <m> <solver> <fp16> <waves> <chunk> <order> <arm>
    tuned = [ln.split() for ln in lines if ln.startswith("nlem2 ")]
    assert any(t[2:7] == ["3", "7", "0", "0", str(chosen)] for t in tuned), tuned
    arch = tuned[0][1]

    # a new handle loads the plan; other lines are filtered
    with open(cache, "a") as f:
        f.write(f"nlem {arch} 2 4 0 1\n")          # compiled, not the default (2)
        f.write(f"nlem {arch} 1 2 0 3\n")          # not compiled for patch radius 1: ignored
        f.write("nlem gfx000 0 1 0 4\n")            # another architecture: ignored
    h2 = _new_handle(monkeypatch, cache)
    assert h2.nlem_plan(3, 10) == chosen
    assert h2.nlem_plan_get(3, 10)["source"] == "cache"
    # the line "2 4 0 1" is patch radius 2, 4 points per lane (window radius 7)
    assert h2.nlem_plan_get(2, 7)["source"] == "cache"         # a line without queue fields
    assert h2.nlem_plan_get(2, 7, f16=True)["source"] == "cache"   # applies to both storages
    assert h2.nlem_plan_get(2, 4)["source"] == "builtin"       # 2 points per lane: no line
    assert h2.nlem_plan(2, 4) == 1
    assert h2.nlem_plan(1, 4) == 1
    assert h2.nlem_plan(0, 4) == 1
    h2.close()

    with open(cache, "a") as f:
        f.write("garbled line\n")
    h3 = _new_handle(monkeypatch, cache)       # stops reading at the bad line, keeps what it read
    assert h3.nlem_plan(2, 4) == 1
    h3.close()


def test_autotune_errors(tmp_path, monkeypatch):
    import paper_1501_03879_amd as emx
    hd = _new_handle(monkeypatch, tmp_path / "none.txt")
    img = _img(4, 16, 16)
    with pytest.raises(emx.EmxError):
        hd.nlem_autotune(_item(img), repeats=0)
    with pytest.raises(emx.EmxError):
        hd.nlem_plan(9, 10)
    assert not os.path.exists(tmp_path / "none.txt")
    hd.close()


def _parity_tol(hd, img, name, pr=3, wr=10, h=300.0, mu=1e-3, tol=1e-4, max_iter=200, max_lag=1):
    """NLEM in tolerance mode under the handle's current plan: every pixel
    against the oracle rerun at the GPU's iteration counts, and the GPU's
    count at most max_lag above the oracle's own stop (one for a plan that
    checks every iteration, the check interval otherwise).  Returns out,
    iters."""
    it = _item(img)
    it.update(patch_radius=pr, window_radius=wr, h=h)
    hd.nlem_denoise_ex([it], lo=0.0, hi=255.0, rho=mu, max_iter=max_iter, tol=tol)
    hd.sync()
    got = it["out"].cpu().numpy().reshape(-1).astype(np.float64)
    iters = it["stats"][:, 0].cpu().numpy()
    ref = oracle.nlem(img, pr, wr, h, 0, 255, mu, max_iter, 0.0, max_iter_each=iters)
    e, r = rel_errors(got, ref["out"], D)
    report(name, e, r)
    assert e <= 1e-4
    own = oracle.nlem(img, pr, wr, h, 0, 255, mu, max_iter, tol)
    lag = iters.astype(int) - own["iters"]
    # (FP32 rounding of a residual at the threshold can move a stop; cf. test_gpu_nlem)
    assert np.mean((lag >= 0) & (lag <= max_lag)) >= 0.99, np.unique(lag, return_counts=True)
    return got, iters


def test_every_nlem_plan_variant_keeps_parity(tmp_path, monkeypatch):
    """Each value a plan can name (waves, chunk, order, arm factor), set
    through nlem_plan_set on the 7x7-patch, 21x21-window shape: parity in
    tolerance mode; chunk and order change only the schedule, so their
    results are bitwise those of the built-in plan; a larger arm factor
    evaluates the primal residual on more iterations, so a pixel stops at
    the same iteration or one earlier."""
    monkeypatch.delenv("EMX_NLEM_CHUNK", raising=False)
    monkeypatch.delenv("EMX_NLEM_ORDER", raising=False)
    hd = _new_handle(monkeypatch, tmp_path / "plans.txt")
    img = _img(7, 30, 34)
    assert hd.nlem_plan_get(3, 10)["source"] == "builtin"
    default_wc = hd.nlem_plan_get(3, 10)["waves"]
    assert default_wc == 4
    # a short queue in tolerance mode runs with the most waves compiled (4)
    # when no plan is set, so the variants below with waves = 4 schedule the
    # same arithmetic as the built-in run
    base_out, base_it = _parity_tol(hd, img, "plan built-in")
    for wc in (2, 3, 4):
        hd.nlem_plan_set(3, 10, dict(waves=wc))
        _parity_tol(hd, img, f"plan waves={wc}")
    for chunk, order in ((1, 0), (8, 1), (3, 1), (2, 0)):
        hd.nlem_plan_set(3, 10, dict(waves=4, chunk=chunk, order=order))
        out, iters = _parity_tol(hd, img, f"plan chunk={chunk} order={order}")
        np.testing.assert_array_equal(out, base_out)
        np.testing.assert_array_equal(iters, base_it)
    for arm in (1.5, 2.0, 3.0):
        hd.nlem_plan_set(3, 10, dict(waves=4, arm_factor=arm))
        _, iters = _parity_tol(hd, img, f"plan arm={arm}")
        assert np.all((iters <= base_it) & (iters >= base_it - 1))
    for check in (2, 4, 8):
        hd.nlem_plan_set(3, 10, dict(waves=4, check_every=check))
        _, iters = _parity_tol(hd, img, f"plan check_every={check}", max_lag=check)
        # the same iterates, tested on fewer iterations: never earlier, at most
        # check_every - 1 later while the residuals stay within tol
        assert np.all(iters >= base_it) and np.mean(iters < base_it + check) >= 0.99
    p = hd.nlem_plan_get(3, 10)
    assert p["source"] == "set" and p["check_every"] == 8
    hd.nlem_plan_set(3, 10, None)
    assert hd.nlem_plan_get(3, 10)["source"] == "builtin"
    import paper_1501_03879_amd as emx
    for bad in (dict(waves=1), dict(waves=4, chunk=65), dict(waves=4, order=2), dict(waves=4, arm_factor=0.5),
                dict(waves=4, arm_factor=float("nan")), dict(waves=4, check_every=3)):
        with pytest.raises(emx.EmxError):
            hd.nlem_plan_set(3, 10, bad)
    hd.close()


def test_nlem_autotune_tolerance_mode_full_search(tmp_path, monkeypatch):
    """The widened search in tolerance mode: the plan it keeps holds values
    from the searched sets, names its source, is written to the cache with
    every field and gives parity; FP16 storage has a plan of its own."""
    import torch
    monkeypatch.delenv("EMX_NLEM_CHUNK", raising=False)
    monkeypatch.delenv("EMX_NLEM_ORDER", raising=False)
    cache = tmp_path / "plans.txt"
    hd = _new_handle(monkeypatch, cache)
    img = _img(8, 48, 40)
    it = _item(img)
    chosen = hd.nlem_autotune(it, max_iter=200, tol=1e-4, repeats=2)
    hd.sync()
    p = hd.nlem_plan_get(3, 10)
    print(f"[autotune] tolerance mode r3 R10: {p}", flush=True)
    assert p["waves"] == chosen and p["source"] == "tuned"
    assert p["chunk"] in (0, 1, 2, 4, 8) and p["order"] in (-1, 0, 1) and p["arm_factor"] in (1.0, 1.5, 2.0, 3.0)
    assert p["check_every"] in (1, 2, 4, 8)
    assert hd.nlem_plan_get(3, 10, f16=True)["source"] == "builtin"
    _parity_tol(hd, img, "nlem after tolerance-mode autotune", max_lag=p["check_every"])
    it16 = _item(img)
    it16["img"] = it16["img"].half()
    hd.nlem_autotune(it16, max_iter=200, tol=1e-4, repeats=1)
    assert hd.nlem_plan_get(3, 10, f16=True)["source"] == "tuned"
    hd.close()
    t = [ln.split() for ln in cache.read_text().split("\n") if ln.startswith("nlem2 ")]
    assert [x[5] for x in t] == ["0", "1"] and all(len(x) == 11 for x in t)   # the fp16 field
    h2 = _new_handle(monkeypatch, cache)
    q = h2.nlem_plan_get(3, 10)
    keys = ("waves", "chunk", "order", "arm_factor", "check_every")
    assert q["source"] == "cache" and {k: q[k] for k in keys} == {k: p[k] for k in keys}
    h2.close()


def _sliced_batch(seed, B):
    # d in (16, 64] and n <= 448: the sliced classes (plus some generic ones)
    return synth.make_pointset_batch(seed, B, n_lo=8, n_hi=448, d_choices=(17, 25, 33, 49, 64, 8))


def _batch_parity(hd, b, name, mu=0.5, tol=1e-4, max_lag=1):
    import torch
    import paper_1501_03879_amd as emx
    dev = gpu()
    a = torch.from_numpy(b.a).to(dev)
    w = torch.from_numpy(b.w).to(dev)
    inst = emx.instances_tensor(b.inst, dev)
    z = torch.zeros(b.z_size, dtype=torch.float32, device=dev)
    st = torch.zeros((b.B, 4), dtype=torch.int32, device=dev)
    hd.em_solve_batch(a, w, inst, z, st, lo=b.lo, hi=b.hi, rho=mu, max_iter=2000, tol=tol, init=emx.INIT_MAXW)
    hd.sync()
    iters, flags = emx.stats_view(st)[0].cpu().numpy(), emx.stats_view(st)[1].cpu().numpy()
    ref = oracle.em_batch(b, mu, 2000, 0.0, init=oracle.INIT_MAXW, max_iter_each=iters)
    got = z.cpu().numpy().astype(np.float64)
    e, r = rel_errors(got, ref["z"], b.hi - b.lo)
    report(name, e, r)
    assert e <= 1e-4
    assert np.all(flags == 1)
    own = oracle.em_batch(b, mu, 2000, tol, init=oracle.INIT_MAXW)
    lag = iters.astype(int) - own["iters"]
    assert np.mean((lag >= 0) & (lag <= max_lag)) >= 0.99, np.unique(lag, return_counts=True)
    return got, iters, (a, w, inst, z, st)


def test_batch_plans_autotune_variants_and_cache(tmp_path, monkeypatch):
    """em_batch_autotune on a batch over the sliced classes: the plan names
    only populated classes, parity under it; every sliced class routed to the
    generic kernels, and arm factors 2 and 3, each keep parity; the plain
    path follows the routing (bitwise equal to the batched results); the
    plan is cached and reloaded."""
    import torch
    import paper_1501_03879_amd as emx
    monkeypatch.delenv("EMX_BATCH_WIDE", raising=False)
    cache = tmp_path / "plans.txt"
    hd = _new_handle(monkeypatch, cache)
    b = _sliced_batch(41, 600)
    assert hd.em_batch_plan_get() == dict(generic_classes=0, arm_factor=1.0, check_every=1, host_counts=0,
                                          source="builtin")
    z0, it0, (a, w, inst, z, st) = _batch_parity(hd, b, "batch built-in plan")
    # the host-counts dispatch changes only which classes are launched where:
    # bitwise the built-in results
    hd.em_batch_plan_set(dict(host_counts=1))
    zh, ith, _ = _batch_parity(hd, b, "batch plan host_counts=1")
    np.testing.assert_array_equal(zh, z0)
    np.testing.assert_array_equal(ith, it0)
    hd.em_batch_plan_set(None)
    p = hd.em_batch_autotune(a, w, inst, z, st, lo=b.lo, hi=b.hi, rho=0.5, max_iter=2000, tol=1e-4, repeats=2)
    print(f"[autotune] batch plan {p}", flush=True)
    assert p["source"] == "tuned" and p["arm_factor"] in (1.0, 1.5, 2.0, 3.0) and p["check_every"] in (1, 2, 4, 8)
    populated = 0
    for e in b.inst:
        n, d = int(e["n"]), int(e["d"])
        if 16 < d <= 64 and n <= 448:
            populated |= 1 << (7 * ((d + 12) // 13 - 2) + (n + 63) // 64 - 1)
    assert p["generic_classes"] & ~populated == 0
    assert hd.em_batch_plan_get() == p
    _batch_parity(hd, b, "batch tuned plan", max_lag=p["check_every"])
    all_generic = (1 << 28) - 1
    for plan in (dict(generic_classes=all_generic), dict(arm_factor=2.0), dict(check_every=4),
                 dict(generic_classes=populated, arm_factor=3.0)):
        hd.em_batch_plan_set(plan)
        got, iters, _ = _batch_parity(hd, b, f"batch plan {plan}", max_lag=plan.get("check_every", 1))
        if plan.get("arm_factor", 1.0) > 1.0:
            assert np.all((iters <= it0) & (iters >= it0 - 1))
        if plan.get("check_every", 1) > 1:
            assert np.all(iters >= it0)
    # the plain path under the routing and arm factor of the plan in force
    # (it does not defer far outliers: max |a| > 300 D sqrt(n) compared apart)
    far = np.array([np.abs(b.points(i)).max() > 300.0 * (b.hi - b.lo) * np.sqrt(b.inst[i]["n"])
                    for i in range(b.B)])
    near = np.concatenate([np.full(int(e["d"]), not f) for e, f in zip(b.inst, far)])
    zp = torch.zeros_like(z)
    sp = torch.zeros_like(st)
    hd.em_solve_plain(a, w, inst, b.inst, zp, sp, lo=b.lo, hi=b.hi, rho=0.5, max_iter=2000, tol=1e-4,
                      init=emx.INIT_MAXW)
    hd.sync()
    np.testing.assert_array_equal(zp.cpu().numpy()[near], got.astype(np.float32)[near])
    hd.em_batch_plan_set(None)
    assert hd.em_batch_plan_get()["source"] == "builtin"
    for bad in (dict(generic_classes=1 << 28), dict(arm_factor=0.9), dict(check_every=16), dict(host_counts=2)):
        with pytest.raises(emx.EmxError):
            hd.em_batch_plan_set(bad)
    hd.close()
    lines = [ln.split() for ln in cache.read_text().split("\n") if ln.startswith("batch ")]
    assert len(lines) == 1 and int(lines[0][4], 16) == p["generic_classes"]
    h2 = _new_handle(monkeypatch, cache)
    q = h2.em_batch_plan_get()
    assert q["source"] == "cache" and q["generic_classes"] == p["generic_classes"]
    assert q["arm_factor"] == p["arm_factor"] and q["check_every"] == p["check_every"]
    h2.close()
