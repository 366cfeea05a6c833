"""HIP graph capture of the C-ABI calls: em_solve_batch and nlem_denoise are
recorded into a torch.cuda.CUDAGraph (their launches go to the capture
stream; the work-queue heads are cleared by a kernel, not a memset node) and
replayed several times, with eager work and synchronisations between the
replays; every replay must reproduce the eager result bit for bit (the
per-instance arithmetic does not depend on which workgroup ran it)."""

import numpy as np
import pytest

import synth
from helpers import gpu, handle

pytestmark = pytest.mark.gpu
DIMS = (1, 2, 3, 4, 5, 8, 15, 16, 17, 31, 33, 48, 49, 64)


def test_batch_solve_graph_replays():
    import torch
    import paper_1501_03879_amd as emx
    dev = gpu()
    b = synth.make_pointset_batch(61, 300, n_lo=1, n_hi=512, d_choices=DIMS)
    a = torch.from_numpy(b.a).to(dev)
    w = torch.from_numpy(b.w).to(dev)
    it = emx.instances_tensor(b.inst, dev)
    z = torch.zeros(b.z_size, dtype=torch.float32, device=dev)
    st = torch.zeros((b.B, 4), dtype=torch.int32, device=dev)
    hd = handle()
    kw = dict(lo=b.lo, hi=b.hi, rho=0.5, max_iter=80, tol=1e-4, init=emx.INIT_MAXW)
    hd.em_solve_batch(a, w, it, z, st, **kw)   # eager: the reference, and sizes the workspace
    hd.sync()
    z_ref, st_ref = z.clone(), st.clone()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        hd.em_solve_batch(a, w, it, z, st, **kw)
    for r in range(3):
        z.fill_(float(r) - 7.0)        # eager work between replays
        st.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(z, z_ref), f"replay {r}: z differs"
        assert torch.equal(st, st_ref), f"replay {r}: stats differ"
        print(f"[graph] batch replay {r}: identical to the eager solve", flush=True)


def test_nlem_graph_replays():
    import torch
    dev = gpu()
    rng = np.random.default_rng(62)
    img = synth.add_gaussian_noise(rng, synth.piecewise_smooth_image(rng, 61, 57), 20.0).astype(np.float32)
    t = torch.from_numpy(img).to(dev)
    out = torch.zeros_like(t)
    st = torch.zeros((t.numel(), 4), dtype=torch.int32, device=dev)
    hd = handle()
    kw = dict(patch_radius=3, window_radius=10, h=200.0, lo=0.0, hi=255.0, rho=1e-3, max_iter=200, tol=1e-4)
    hd.nlem_denoise(t, out, st, **kw)
    hd.sync()
    out_ref, st_ref = out.clone(), st.clone()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        hd.nlem_denoise(t, out, st, **kw)
    for r in range(3):
        out.fill_(-1.0)
        st.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, out_ref), f"replay {r}: output differs"
        assert torch.equal(st, st_ref), f"replay {r}: stats differ"
        print(f"[graph] nlem replay {r}: identical to the eager call", flush=True)
