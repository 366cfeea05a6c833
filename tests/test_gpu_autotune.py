"""NLEM autotuner (nlem_autotune / nlem_plan): the tuned plan is one of the
compiled coordinate-wave counts, the handle uses it afterwards (parity with
the FP64 oracle at the NLEM bar, 1e-4 of the intensity range, fixed
iteration count), and the plan survives in the EMX_AUTOTUNE_CACHE file for a
new handle; cache lines for another architecture, for an uncompiled
variant or garbled ones are ignored."""

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
    assert any(ln.startswith("nlem ") and ln.split()[2:] == ["3", "7", "0", str(chosen)] for ln in lines)
    arch = next(ln.split()[1] for ln in lines if ln.startswith("nlem "))

    # a new handle loads the plan; other lines are filtered
    with open(cache, "a") as f:
        f.write(f"nlem {arch} 2 4 0 1\n")          # compiled, not the default (2)
        f.write(f"nlem {arch} 1 2 0 3\n")          # not compiled for patch radius 1: ignored
        f.write("nlem gfx000 0 1 0 4\n")            # another architecture: ignored
    h2 = _new_handle(monkeypatch, cache)
    assert h2.nlem_plan(3, 10) == chosen
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
