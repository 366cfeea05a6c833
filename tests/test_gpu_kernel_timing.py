"""em_kernel_timing: HIP events around each NLEM solve launch.  One pair per
nlem_denoise / nlem_denoise_ex launch while enabled, none while disabled or
inside a stream capture, and the timed duration of a launch lies within the
duration of the whole call measured around it on the same stream."""

import numpy as np
import pytest

import synth
from helpers import gpu, handle

pytestmark = pytest.mark.gpu


def _image(dev, seed=71, H=96, W=80):
    import torch
    rng = np.random.default_rng(seed)
    img = synth.add_gaussian_noise(rng, synth.piecewise_smooth_image(rng, H, W), 20.0).astype(np.float32)
    t = torch.from_numpy(img).to(dev)
    return t, torch.empty_like(t), torch.zeros((t.numel(), 4), dtype=torch.int32, device=dev)


KW = dict(patch_radius=3, window_radius=10, h=200.0, lo=0.0, hi=255.0, rho=1e-3, max_iter=200, tol=1e-4)


@pytest.fixture
def hd():
    """The shared handle, with timing switched off again whatever the test did."""
    gpu()
    h = handle()
    yield h
    h.kernel_timing(False)


def test_launches_are_counted_and_bounded_by_the_call(hd):
    import torch
    dev = gpu()
    img, out, st = _image(dev)
    hd.nlem_denoise(img, out, st, **KW)              # warm-up, untimed
    hd.kernel_timing(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        hd.nlem_denoise(img, out, st, **KW)
    e1.record()
    torch.cuda.synchronize()
    total, n = hd.kernel_timing_read()
    assert n == 3
    whole = e0.elapsed_time(e1)
    assert 0.0 < total <= whole * 1.001
    print(f"[timing] 3 launches: kernels {total:.3f} ms of {whole:.3f} ms", flush=True)
    # read clears; disabled records nothing
    assert hd.kernel_timing_read() == (0.0, 0)
    hd.kernel_timing(False)
    hd.nlem_denoise(img, out, st, **KW)
    torch.cuda.synchronize()
    assert hd.kernel_timing_read()[1] == 0


def test_ex_groups_and_capture(hd):
    import torch
    dev = gpu()
    a, b = _image(dev, 72, 64, 70), _image(dev, 73, 40, 52)
    items = [dict(img=a[0], out=a[1], stats=a[2], patch_radius=3, window_radius=10, h=200.0),
             dict(img=b[0], out=b[1], stats=b[2], patch_radius=2, window_radius=5, h=200.0)]
    hd.kernel_timing(True)
    hd.nlem_denoise_ex(items, max_iter=200, tol=1e-4)  # two shape groups: two launches
    torch.cuda.synchronize()
    assert hd.kernel_timing_read()[1] == 2
    # a captured launch records no events; the eager one after it does
    img, out, st = _image(dev, 74)
    hd.nlem_denoise(img, out, st, **KW)
    torch.cuda.synchronize()
    hd.kernel_timing_read()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        hd.nlem_denoise(img, out, st, **KW)
    assert hd.kernel_timing_read()[1] == 0
    g.replay()
    torch.cuda.synchronize()
    assert hd.kernel_timing_read()[1] == 0
    hd.nlem_denoise(img, out, st, **KW)
    torch.cuda.synchronize()
    assert hd.kernel_timing_read()[1] == 1
    hd.kernel_timing(False)
    print("[timing] ex groups and capture: as documented", flush=True)
