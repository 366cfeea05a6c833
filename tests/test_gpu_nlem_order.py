"""The longest-first queue order of the NLEM kernel (pixels by decreasing
patch standard deviation) changes only which workgroup solves a pixel and
when: outputs and per-pixel statistics must be identical, bit for bit, with
the order switched off (EMX_NLEM_ORDER=0), for one image, for several images
and shapes in one call, for the multi-image graph and for FP16 storage."""

import numpy as np
import pytest

import synth
from helpers import gpu, handle

pytestmark = pytest.mark.gpu


def _img(seed, H, W, sigma=20.0):
    rng = np.random.default_rng(seed)
    return synth.add_gaussian_noise(rng, synth.piecewise_smooth_image(rng, H, W), sigma).astype(np.float32)


def _items(specs, fp16=False):
    import torch
    dev = gpu()
    items = []
    for seed, H, W, pr, wr in specs:
        t = torch.from_numpy(_img(seed, H, W)).to(dev)
        if fp16:
            t = t.half()
        items.append(dict(img=t, out=torch.full(t.shape, -7.0, dtype=torch.float32, device=dev),
                          stats=torch.zeros((t.numel(), 4), dtype=torch.int32, device=dev),
                          patch_radius=pr, window_radius=wr, h=200.0))
    return items


def _snapshot(items):
    return [(it["out"].clone(), it["stats"].clone()) for it in items]


# the order is used in tolerance mode for queues of at least 4 rounds of the
# resident grid (768 workgroups for patch radius 3, window radius 10): the
# 128x131 and 96x200 images are ordered, the small ones keep raster order
SPECS = [(1, 128, 131, 3, 10), (2, 33, 41, 2, 7), (3, 96, 200, 3, 10), (4, 17, 90, 1, 5)]


@pytest.mark.parametrize("fp16", [False, True])
def test_order_does_not_change_results(fp16, monkeypatch):
    gpu()   # torch sets up the device before the library's handle
    hd = handle()
    runs = []
    for flag in ("0", "1"):
        monkeypatch.setenv("EMX_NLEM_ORDER", flag)
        items = _items(SPECS, fp16)
        hd.nlem_denoise_ex(items, max_iter=200, tol=1e-4)
        hd.sync()
        runs.append(_snapshot(items))
    for (o0, s0), (o1, s1) in zip(*runs):
        assert torch_equal(o0, o1) and torch_equal(s0, s1)
        assert float(o1.min()) >= 0.0   # every pixel written (the fill value is -7)
    print(f"[order] fp16={fp16}: identical outputs and stats with and without the order", flush=True)


def test_order_multi_graph(monkeypatch):
    gpu()
    hd = handle()
    runs = []
    for flag in ("0", "1", "1"):
        monkeypatch.setenv("EMX_NLEM_ORDER", flag)
        items = _items(SPECS)
        hd.nlem_denoise_multi(items, max_iter=200, tol=1e-4)
        hd.sync()
        runs.append(_snapshot(items))
    for r in runs[1:]:
        for (o0, s0), (o1, s1) in zip(runs[0], r):
            assert torch_equal(o0, o1) and torch_equal(s0, s1)
    print("[order] multi-image graph: identical with and without the order", flush=True)


def torch_equal(a, b):
    import torch
    return bool(torch.equal(a, b))


@pytest.mark.parametrize("chunk", [3, 8])
def test_queue_chunks_parity(chunk, monkeypatch):
    """Several queue positions per atomic (forced with EMX_NLEM_CHUNK): the
    same outputs and statistics as one per atomic, bit for bit, and parity
    with the oracle at a fixed iteration count (1e-4 of the range)."""
    import oracle
    from helpers import rel_errors, report
    gpu()
    hd = handle()
    img = _img(21, 45, 52)
    runs = []
    for c in ("1", str(chunk)):
        monkeypatch.setenv("EMX_NLEM_CHUNK", c)
        items = _items([(21, 45, 52, 2, 5)])
        hd.nlem_denoise_ex(items, max_iter=9, tol=0.0)
        hd.sync()
        runs.append(_snapshot(items))
    (o1, s1), = runs[0]
    (ok, sk), = runs[1]
    assert torch_equal(o1, ok) and torch_equal(s1, sk)
    ref = oracle.nlem(img, 2, 5, 200.0, 0, 255, 1e-3, 9, 0.0)
    e, r = rel_errors(ok.cpu().numpy().reshape(-1).astype(np.float64), ref["out"], 255.0)
    report(f"nlem r2 R5 T9, {chunk} queue positions per atomic", e, r)
    assert e <= 1e-4


@pytest.mark.parametrize("pr,wr,fp16", [(0, 4, False), (1, 5, True), (2, 7, False), (3, 5, True)])
def test_forced_order_every_patch_size(pr, wr, fp16):
    """A plan with the order forced on (order = 1) runs the order kernels on
    small images too, for every patch size (each size has its own unrolled
    patch-statistics kernel): outputs and statistics identical, bit for bit,
    to the same plan with the order off, and every pixel written."""
    gpu()
    hd = handle()
    base = hd.nlem_plan_get(pr, wr, f16=fp16)
    runs = []
    try:
        for order in (0, 1):
            hd.nlem_plan_set(pr, wr, dict(base, order=order), f16=fp16)
            items = _items([(30 + pr, 37, 45, pr, wr)], fp16)
            hd.nlem_denoise_ex(items, max_iter=200, tol=1e-4)
            hd.sync()
            runs.append(_snapshot(items))
    finally:
        hd.nlem_plan_set(pr, wr, None, f16=fp16)
    (o0, s0), = runs[0]
    (o1, s1), = runs[1]
    assert torch_equal(o0, o1) and torch_equal(s0, s1)
    assert float(o1.min()) >= 0.0   # every pixel written (the fill value is -7)
    print(f"[order] forced on, r={pr} R={wr} fp16={fp16}: identical to the order off", flush=True)
