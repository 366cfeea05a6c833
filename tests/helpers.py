"""Shared helpers for the GPU parity tests (run the HIP path through the C ABI
and the FP64 oracle on the same input bits)."""

from __future__ import annotations

import numpy as np


def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    return torch.device("cuda:0")


def handle():
    import paper_1501_03879_amd as emx
    return emx.handle(0)


def run_nlem(img_np, pr, wr, h, mu, max_iter, tol, lo=0.0, hi=255.0, fp16=False):
    """NLEM on the GPU; returns (out float64 [H*W], stats dict of numpy arrays)."""
    import torch
    import paper_1501_03879_amd as emx
    dev = gpu()
    t = torch.from_numpy(np.ascontiguousarray(img_np, dtype=np.float32)).to(dev)
    if fp16:
        t = t.half()
    out = torch.full(t.shape, -7.0, dtype=torch.float32, device=dev)
    stats = torch.zeros((t.numel(), 4), dtype=torch.int32, device=dev)
    hd = handle()
    hd.nlem_denoise(t, out, stats, patch_radius=pr, window_radius=wr, h=h, lo=lo, hi=hi, rho=mu,
                    max_iter=max_iter, tol=tol)
    hd.sync()
    it, fl, rp, rd = emx.stats_view(stats)
    return (out.cpu().numpy().reshape(-1).astype(np.float64),
            dict(iters=it.cpu().numpy(), flags=fl.cpu().numpy(), r_pri=rp.cpu().numpy(),
                 r_dual=rd.cpu().numpy()))


def run_batch(batch, mu, max_iter, tol, init, z0=None, plain=False):
    """em_solve_batch (or em_solve_plain) on the GPU for a synth.PointSetBatch."""
    import torch
    import paper_1501_03879_amd as emx
    dev = gpu()
    a = torch.from_numpy(np.ascontiguousarray(batch.a, dtype=np.float32)).to(dev)
    w = torch.from_numpy(np.ascontiguousarray(batch.w, dtype=np.float32)).to(dev)
    inst = emx.instances_tensor(batch.inst, dev)
    zsz = max(batch.z_size, 1)
    if z0 is None:
        z = torch.zeros(zsz, dtype=torch.float32, device=dev)
    else:
        z = torch.from_numpy(np.ascontiguousarray(z0, dtype=np.float32)).to(dev)
    stats = torch.zeros((max(batch.B, 1), 4), dtype=torch.int32, device=dev)
    hd = handle()
    if plain:
        hd.em_solve_plain(a, w, inst, np.ascontiguousarray(batch.inst), z, stats, lo=batch.lo,
                          hi=batch.hi, rho=mu, max_iter=max_iter, tol=tol, init=init)
    else:
        hd.em_solve_batch(a, w, inst, z, stats, lo=batch.lo, hi=batch.hi, rho=mu,
                          max_iter=max_iter, tol=tol, init=init)
    hd.sync()
    it, fl, rp, rd = emx.stats_view(stats)
    return (z.cpu().numpy().astype(np.float64),
            dict(iters=it.cpu().numpy()[:batch.B], flags=fl.cpu().numpy()[:batch.B],
                 r_pri=rp.cpu().numpy()[:batch.B], r_dual=rd.cpu().numpy()[:batch.B]))


def rel_errors(got, ref, D):
    """(max |got - ref| / D, rms |got - ref| / D) over finite reference entries."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    diff = np.abs(got - ref) / D
    return float(diff.max()) if diff.size else 0.0, float(np.sqrt(np.mean(diff ** 2))) if diff.size else 0.0


def report(name, emax, erms):
    print(f"[parity] {name}: max_rel={emax:.3e} rms_rel={erms:.3e}", flush=True)


def run_nlem_ex(images, *, solver, init, max_iter, tol, mu=1e-3, eps=1e-6, lo=0.0, hi=255.0,
                fp16=False):
    """nlem_denoise_ex on the GPU for a list of (img_np, pr, wr, h); returns a
    list of (out float64 [H*W], stats dict)."""
    import torch
    import paper_1501_03879_amd as emx
    dev = gpu()
    items = []
    for img_np, pr, wr, h in images:
        t = torch.from_numpy(np.ascontiguousarray(img_np, dtype=np.float32)).to(dev)
        if fp16:
            t = t.half()
        items.append(dict(img=t, out=torch.full(t.shape, -7.0, dtype=torch.float32, device=dev),
                          stats=torch.zeros((t.numel(), 4), dtype=torch.int32, device=dev),
                          patch_radius=pr, window_radius=wr, h=h))
    hd = handle()
    hd.nlem_denoise_ex(items, solver=solver, init=init, lo=lo, hi=hi, rho=mu, eps=eps,
                       max_iter=max_iter, tol=tol)
    hd.sync()
    res = []
    for it in items:
        i, f, rp, rd = emx.stats_view(it["stats"])
        res.append((it["out"].cpu().numpy().reshape(-1).astype(np.float64),
                    dict(iters=i.cpu().numpy(), flags=f.cpu().numpy(), r_pri=rp.cpu().numpy(),
                         r_dual=rd.cpu().numpy())))
    return res


def run_nlm(img_np, pr, wr, h, fp16=False):
    """nlm_denoise on the GPU; returns out float64 [H*W]."""
    import torch
    dev = gpu()
    t = torch.from_numpy(np.ascontiguousarray(img_np, dtype=np.float32)).to(dev)
    if fp16:
        t = t.half()
    out = torch.full(t.shape, -7.0, dtype=torch.float32, device=dev)
    hd = handle()
    hd.nlm_denoise(t, out, patch_radius=pr, window_radius=wr, h=h)
    hd.sync()
    return out.cpu().numpy().reshape(-1).astype(np.float64)


def run_batch_ex(batch, *, solver, max_iter, tol, init, mu=0.5, eps=1e-6, box_lo=None,
                 box_hi=None, adapt_every=1, adapt_ratio=10.0, adapt_factor=2.0, z0=None,
                 ball_center=None, ball_radius=None, radius=None, eta=0.999):
    """em_solve_batch_ex on the GPU for a synth.PointSetBatch (box from the
    batch's lo/hi unless per-coordinate arrays are given)."""
    import torch
    import paper_1501_03879_amd as emx
    dev = gpu()
    a = torch.from_numpy(np.ascontiguousarray(batch.a, dtype=np.float32)).to(dev)
    w = torch.from_numpy(np.ascontiguousarray(batch.w, dtype=np.float32)).to(dev)
    inst = emx.instances_tensor(batch.inst, dev)
    zsz = max(batch.z_size, 1)
    z = (torch.zeros(zsz, dtype=torch.float32, device=dev) if z0 is None else
         torch.from_numpy(np.ascontiguousarray(z0, dtype=np.float32)).to(dev))
    bl = None if box_lo is None else torch.from_numpy(np.ascontiguousarray(box_lo, np.float32)).to(dev)
    bh = None if box_hi is None else torch.from_numpy(np.ascontiguousarray(box_hi, np.float32)).to(dev)
    bc = None if ball_center is None else torch.from_numpy(np.ascontiguousarray(ball_center, np.float32)).to(dev)
    br = None if ball_radius is None else torch.from_numpy(np.ascontiguousarray(ball_radius, np.float32)).to(dev)
    stats = torch.zeros((max(batch.B, 1), 4), dtype=torch.int32, device=dev)
    hd = handle()
    hd.em_solve_batch_ex(a, w, inst, z, stats, solver=solver, init=init, lo=batch.lo, hi=batch.hi,
                         box_lo=bl, box_hi=bh, rho=mu, eps=eps, max_iter=max_iter, tol=tol,
                         adapt_every=adapt_every, adapt_ratio=adapt_ratio, adapt_factor=adapt_factor,
                         ball_center=bc, ball_radius=br, radius=radius, eta=eta)
    hd.sync()
    it, fl, rp, rd = emx.stats_view(stats)
    return (z.cpu().numpy().astype(np.float64),
            dict(iters=it.cpu().numpy()[:batch.B], flags=fl.cpu().numpy()[:batch.B],
                 r_pri=rp.cpu().numpy()[:batch.B], r_dual=rd.cpu().numpy()[:batch.B]))


def run_plain_ex(batch, *, solver, max_iter, tol, init, mu=0.5, eta=0.999, box_lo=None, box_hi=None):
    """em_solve_plain_ex on the GPU for a synth.PointSetBatch."""
    import torch
    import paper_1501_03879_amd as emx
    dev = gpu()
    a = torch.from_numpy(np.ascontiguousarray(batch.a, dtype=np.float32)).to(dev)
    w = torch.from_numpy(np.ascontiguousarray(batch.w, dtype=np.float32)).to(dev)
    inst = emx.instances_tensor(batch.inst, dev)
    z = torch.zeros(max(batch.z_size, 1), dtype=torch.float32, device=dev)
    bl = None if box_lo is None else torch.from_numpy(np.ascontiguousarray(box_lo, np.float32)).to(dev)
    bh = None if box_hi is None else torch.from_numpy(np.ascontiguousarray(box_hi, np.float32)).to(dev)
    stats = torch.zeros((max(batch.B, 1), 4), dtype=torch.int32, device=dev)
    hd = handle()
    hd.em_solve_plain_ex(a, w, inst, np.ascontiguousarray(batch.inst), z, stats, solver=solver, init=init,
                         lo=batch.lo, hi=batch.hi, box_lo=bl, box_hi=bh, rho=mu, max_iter=max_iter,
                         tol=tol, eta=eta)
    hd.sync()
    it, fl, rp, rd = emx.stats_view(stats)
    return (z.cpu().numpy().astype(np.float64),
            dict(iters=it.cpu().numpy()[:batch.B], flags=fl.cpu().numpy()[:batch.B],
                 r_pri=rp.cpu().numpy()[:batch.B], r_dual=rd.cpu().numpy()[:batch.B]))
