"""Full-size GPU runs of the remaining workloads, checked on sampled outputs
that the oracle recomputes one by one at the GPU's iteration counts.

* 512 x 512 mixed-noise image (Gaussian sigma 30 + 10% impulses), d = 49,
  n <= 441, FP32 and FP16 image storage (per-pixel error of the FP16 run
  against the FP32-image oracle, and of both against their own inputs),
  ~6,000 pixels stratified over impulses, the border band and the image;
* 16 images of uneven size and radii in one nlem_denoise_multi graph, per
  image 1,024 random pixels, 128 from the band of truncated windows and the
  four corners;
* 1,048,576 uneven point sets (drawn on the device), 10,240 sampled
  instances (2,048 per d); the same batch with IRLS and with the
  weighted-penalty ADMM from the weighted-mean start, 1,280 sampled.
"""

import numpy as np
import pytest

import oracle
import synth
from helpers import gpu, handle, rel_errors, report, run_nlem

pytestmark = pytest.mark.gpu


def _strata(img, rng, k):
    """k pixels each from: impulse pixels, border band, everything."""
    H, W = img.shape
    flat = img.reshape(-1)
    imp = np.flatnonzero((flat == 0.0) | (flat == 255.0))
    yy, xx = np.divmod(np.arange(H * W), W)
    border = np.flatnonzero(np.minimum.reduce([yy, xx, H - 1 - yy, W - 1 - xx]) < 10)
    parts = [rng.choice(imp, k, replace=False), rng.choice(border, k, replace=False),
             rng.choice(H * W, k, replace=False), [0, W - 1, H * W - W, H * W - 1]]
    return np.unique(np.concatenate(parts))


def test_512_mixed_noise_fp32_and_fp16():
    wl = synth.nlem_512_mixed()
    im = wl.images[0]
    rng = np.random.default_rng(1)
    pix = _strata(im.noisy, rng, 2048)
    got32, st32 = run_nlem(im.noisy, 3, 10, im.h, wl.mu, wl.max_iter, wl.tol)
    got16, st16 = run_nlem(im.noisy, 3, 10, im.h, wl.mu, wl.max_iter, wl.tol, fp16=True)
    ref32 = oracle.nlem(im.noisy, 3, 10, im.h, 0, 255, wl.mu, wl.max_iter, 0.0, pix=pix,
                        max_iter_each=st32["iters"][pix])
    e, r = rel_errors(got32[pix], ref32["out"], 255.0)
    report(f"512 mixed FP32 storage, {pix.size} sampled px (oracle at GPU iterations)", e, r)
    assert e <= 1e-4
    img16 = im.noisy.astype(np.float16).astype(np.float32)
    ref16 = oracle.nlem(img16, 3, 10, im.h, 0, 255, wl.mu, wl.max_iter, 0.0, pix=pix,
                        max_iter_each=st16["iters"][pix])
    e, r = rel_errors(got16[pix], ref16["out"], 255.0)
    report("512 mixed FP16 storage vs oracle on the FP16-rounded image", e, r)
    assert e <= 1e-4
    ref16_32 = oracle.nlem(im.noisy, 3, 10, im.h, 0, 255, wl.mu, wl.max_iter, 0.0, pix=pix,
                           max_iter_each=st16["iters"][pix])
    err = np.abs(got16[pix] - ref16_32["out"]) / 255.0
    report("512 mixed FP16 storage vs oracle on the FP32 image", float(err.max()),
           float(np.sqrt(np.mean(err ** 2))))
    print(f"[parity] FP16 per-pixel error: p50 {np.percentile(err, 50):.2e} p99 "
          f"{np.percentile(err, 99):.2e} max {err.max():.2e}; FP32 run mean iters "
          f"{st32['iters'].mean():.1f}, FP16 run {st16['iters'].mean():.1f}", flush=True)
    assert err.max() <= 2e-3
    assert np.mean(st32["flags"] == 1) >= 0.99


def test_multi_image_workload():
    import torch
    import paper_1501_03879_amd as emx
    dev = gpu()
    wl = synth.nlem_multi_image()
    items = []
    for im in wl.images:
        t = torch.from_numpy(im.noisy).to(dev)
        items.append(dict(img=t, out=torch.zeros_like(t), patch_radius=im.patch_radius,
                          window_radius=im.window_radius, h=im.h,
                          stats=torch.zeros((im.noisy.size, 4), dtype=torch.int32, device=dev)))
    hd = handle()
    hd.nlem_denoise_multi(items, lo=wl.lo, hi=wl.hi, rho=wl.mu, max_iter=wl.max_iter, tol=wl.tol)
    hd.sync()
    rng = np.random.default_rng(2)
    worst = 0.0
    for k, (im, it) in enumerate(zip(wl.images, items)):
        H, W = im.noisy.shape
        iters = emx.stats_view(it["stats"])[0].cpu().numpy()
        yy, xx = np.divmod(np.arange(H * W), W)
        border = np.flatnonzero(np.minimum.reduce([yy, xx, H - 1 - yy, W - 1 - xx]) < im.window_radius)
        pix = np.unique(np.concatenate([[0, W - 1, H * W - W, H * W - 1], rng.choice(H * W, 1024, replace=False),
                                        rng.choice(border, 128, replace=False)]))
        ref = oracle.nlem(im.noisy, im.patch_radius, im.window_radius, im.h, 0, 255, wl.mu,
                          wl.max_iter, 0.0, pix=pix, max_iter_each=iters[pix])
        got = it["out"].cpu().numpy().reshape(-1).astype(np.float64)
        e, r = rel_errors(got[pix], ref["out"], 255.0)
        worst = max(worst, e)
        print(f"[parity] multi image {k}: {H}x{W} r={im.patch_radius} R={im.window_radius} "
              f"{pix.size} px max_rel={e:.2e} rms_rel={r:.2e} mean iters {iters.mean():.1f}", flush=True)
    assert worst <= 1e-4


def test_pointsets_full_batch_sampled():
    import torch
    import paper_1501_03879_amd as emx
    dev = gpu()
    B = 1 << 20
    a, w, inst, zs = synth.pointsets.make_pointset_batch_device(505, B, dev)
    it = emx.instances_tensor(inst, dev)
    z = torch.zeros(zs, dtype=torch.float32, device=dev)
    stats = torch.zeros((B, 4), dtype=torch.int32, device=dev)
    mu = synth.configs.POINTSET_MU
    hd = handle()
    hd.em_solve_batch(a, w, it, z, stats, lo=-3.0, hi=3.0, rho=mu,
                      max_iter=synth.configs.POINTSET_MAX_ITER, tol=synth.configs.POINTSET_TOL,
                      init=emx.INIT_MAXW)
    hd.sync()
    iters = emx.stats_view(stats)[0].cpu().numpy()
    flags = emx.stats_view(stats)[1].cpu().numpy()
    zc = z.cpu().numpy()
    rng = np.random.default_rng(3)
    sample = np.concatenate([rng.choice(np.flatnonzero(inst["d"] == dv), 2048, replace=False)
                             for dv in (2, 3, 16, 49, 64)])
    pts, ws = [], []
    for b in sample:
        e = inst[b]
        n, d = int(e["n"]), int(e["d"])
        pts.append(a[e["a_off"]:e["a_off"] + n * d].view(n, d).cpu().numpy())
        ws.append(w[e["w_off"]:e["w_off"] + n].cpu().numpy())
    sb = synth.pointsets.pack_instances(pts, ws, -3.0, 3.0)
    ref = oracle.em_batch(sb, mu, synth.configs.POINTSET_MAX_ITER, 0.0, init=oracle.INIT_MAXW,
                          max_iter_each=iters[sample])
    got = np.concatenate([zc[inst[b]["z_off"]:inst[b]["z_off"] + inst[b]["d"]] for b in sample])
    e, r = rel_errors(got, ref["z"], 6.0)
    report(f"pointsets 2^20 instances, {sample.size} sampled (oracle at GPU iterations)", e, r)
    print(f"[parity] pointsets full batch: mean iters {iters.mean():.1f}, converged "
          f"{np.mean(flags == 1):.4f}, max iters {iters.max()}", flush=True)
    assert e <= 1e-4
    # every instance reaches the tolerance (far-outlier instances included: they
    # are solved carrying the prox displacement itself)
    assert np.all(flags == 1), np.unique(flags, return_counts=True)


@pytest.mark.parametrize("solver", [1, 4])
def test_pointsets_full_batch_irls_and_weighted_sampled(solver):
    """The same 2^20-instance workload with IRLS (eps 1e-4 in the unit-scale
    set units) and with the weighted-penalty ADMM, weighted-mean start,
    tolerance 1e-4; 1,280 sampled instances (256 per d) against the oracle
    at the GPU's iteration counts."""
    import torch
    import paper_1501_03879_amd as emx
    dev = gpu()
    B = 1 << 20
    a, w, inst, zs = synth.pointsets.make_pointset_batch_device(505, B, dev)
    it = emx.instances_tensor(inst, dev)
    z = torch.zeros(zs, dtype=torch.float32, device=dev)
    stats = torch.zeros((B, 4), dtype=torch.int32, device=dev)
    mu = synth.configs.POINTSET_MU
    hd = handle()
    hd.em_solve_batch_ex(a, w, it, z, stats, solver=solver, init=emx.INIT_WMEAN, lo=-3.0, hi=3.0, rho=mu,
                         eps=1e-4, max_iter=synth.configs.POINTSET_MAX_ITER, tol=synth.configs.POINTSET_TOL)
    hd.sync()
    iters = emx.stats_view(stats)[0].cpu().numpy()
    flags = emx.stats_view(stats)[1].cpu().numpy()
    zc = z.cpu().numpy()
    rng = np.random.default_rng(4 + solver)
    sample = np.concatenate([rng.choice(np.flatnonzero(inst["d"] == dv), 256, replace=False)
                             for dv in (2, 3, 16, 49, 64)])
    pts, ws = [], []
    for b in sample:
        e = inst[b]
        n, d = int(e["n"]), int(e["d"])
        pts.append(a[e["a_off"]:e["a_off"] + n * d].view(n, d).cpu().numpy())
        ws.append(w[e["w_off"]:e["w_off"] + n].cpu().numpy())
    sb = synth.pointsets.pack_instances(pts, ws, -3.0, 3.0)
    ref = oracle.em_batch(sb, mu, synth.configs.POINTSET_MAX_ITER, 0.0, init=oracle.INIT_WMEAN,
                          solver=solver, eps=1e-4, max_iter_each=iters[sample])
    got = np.concatenate([zc[inst[b]["z_off"]:inst[b]["z_off"] + inst[b]["d"]] for b in sample])
    e, r = rel_errors(got, ref["z"], 6.0)
    name = "irls" if solver == 1 else "weighted-penalty admm"
    report(f"pointsets 2^20 {name}, {sample.size} sampled (oracle at GPU iterations)", e, r)
    print(f"[parity] pointsets full batch {name}: mean iters {iters.mean():.1f}, converged "
          f"{np.mean(flags == 1):.4f}, max iters {iters.max()}", flush=True)
    assert e <= 1e-4


def test_interior_pixels_as_batch_instances_sampled():
    """em_solve_batch on every interior pixel of the 256x256 workload as a
    materialised n = 441, d = 49 instance (bench.py's batch_interior leg, the
    same launch): 256 sampled instances against the oracle rerun at the GPU's
    per-instance iteration counts on the same input bits (1e-4 of 255).
    Inputs: the window patches gathered on the device and their NLM weights
    exp(-||P_i - P_j||^2 / h^2) computed there in FP64, both stored as FP32."""
    import torch
    import paper_1501_03879_amd as emx
    dev = gpu()
    wl = synth.nlem_256()
    im = wl.images[0]
    H, W = im.noisy.shape
    r, R = im.patch_radius, im.window_radius
    k, n = 2 * r + 1, (2 * R + 1) ** 2
    d = k * k
    P = torch.from_numpy(np.pad(im.noisy.astype(np.float64), r, mode="symmetric")).to(dev)
    patches = P.unfold(0, k, 1).unfold(1, k, 1).reshape(H * W, d)
    ys, xs = torch.meshgrid(torch.arange(R, H - R, device=dev), torch.arange(R, W - R, device=dev),
                            indexing="ij")
    centres = (ys * W + xs).reshape(-1)
    dy, dx = torch.meshgrid(torch.arange(-R, R + 1, device=dev), torch.arange(-R, R + 1, device=dev),
                            indexing="ij")
    idx = centres[:, None] + (dy * W + dx).reshape(-1)[None, :]
    B = int(idx.shape[0])
    a64 = patches[idx]
    w = torch.exp(-((a64 - patches[centres][:, None, :]) ** 2).sum(-1) / (im.h * im.h)).float().contiguous()
    a = a64.float().contiguous()
    del a64
    inst = np.zeros(B, dtype=synth.pointsets.INSTANCE_DTYPE)
    bi = np.arange(B, dtype=np.int64)
    inst["a_off"], inst["w_off"], inst["z_off"] = bi * n * d, bi * n, bi * d
    inst["n"], inst["d"] = n, d
    it = emx.instances_tensor(inst, dev)
    z = torch.zeros(B * d, dtype=torch.float32, device=dev)
    st = torch.zeros((B, 4), dtype=torch.int32, device=dev)
    print(f"[parity] batch interior: {B} instances n={n} d={d}", flush=True)
    hd = handle()
    hd.em_solve_batch(a.reshape(-1), w.reshape(-1), it, z, st, lo=wl.lo, hi=wl.hi, rho=wl.mu,
                      max_iter=wl.max_iter, tol=wl.tol, init=emx.INIT_MAXW)
    hd.sync()
    iters = emx.stats_view(st)[0].cpu().numpy()
    flags = emx.stats_view(st)[1].cpu().numpy()
    rng = np.random.default_rng(11)
    sample = np.sort(rng.choice(B, 256, replace=False))
    sb = synth.pointsets.pack_instances([a[b].cpu().numpy() for b in sample],
                                        [w[b].cpu().numpy() for b in sample], wl.lo, wl.hi)
    ref = oracle.em_batch(sb, wl.mu, wl.max_iter, 0.0, init=oracle.INIT_MAXW, max_iter_each=iters[sample])
    got = z.reshape(B, d)[torch.from_numpy(sample).to(dev)].cpu().numpy().reshape(-1).astype(np.float64)
    e, rr = rel_errors(got, ref["z"], wl.hi - wl.lo)
    report(f"batch interior {B} instances, 256 sampled (oracle at GPU iterations; mean iters "
           f"{iters.mean():.2f}, converged {np.mean(flags == 1):.4f})", e, rr)
    assert e <= 1e-4
    assert np.mean(flags == 1) >= 0.999
