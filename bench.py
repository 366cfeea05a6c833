"""Benchmark: Non-Local Euclidean Medians and the batched Euclidean-median
solver on one MI355X.

One step = nlem_denoise over the whole 256 x 256 synthetic image (sigma 20,
patch 7x7 so d = 49, window 21x21 so n <= 441, h = 10 sigma, box [0, 255],
mu = 1e-3, primal/dual residual 1e-4 relative to 255 or 200 iterations):
staging, weights, per-pixel EM-ADMM and the centre-pixel output all run in
the library's kernels; `value` is its rate in Mpixel/s.

Also in the line: em_solves_per_s_n441_d49, em_solve_batch over the 55,696
interior pixels' materialised windows (n = 441, d = 49 exactly), with the
plain one-instance-per-launch path on the same instances (speedup_vs_plain)
and FP64-oracle error on sampled instances; the roofline of the NLEM kernel
on the FP32 FLOP model (6 flop per point coordinate per iteration plus 3
per point coordinate for the weights); one sub-record per workload in
`configs` (64 x 64 with 50 fixed iterations, the 256 x 256 step, 512 x 512
mixed noise with FP32 and FP16 storage, 16 images in one graph, 1,048,576
point sets), each with its time, rate, model TFLOP/s and max-abs / RMS
error against the FP64 oracle at the GPU's iteration counts; and the
oracle itself timed on this host's cores (cpu_baseline), whose outputs
cover every pixel of the step's image.  Before the warm-up, the built-in
schedules are timed and the autotuners (nlem_autotune, em_batch_autotune)
pick the plans the timed steps run; `plan` and `batch_interior.plan`
record both, with the plans' source (--tune 0 keeps the built-in plans).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-batch] [--no-configs] [--plain 0|1]
                    [--tune 0|1]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "EM solves/sec & Mpixel/s at n=441,d=49, residual 1e-4 (batched FP32 vs plain)"
FP32_PEAK_TFLOPS = 157.3      # MI355X published FP32 vector peak (packed FP32)
FP32_NONPACKED_TFLOPS = 78.6  # 256 CU x 64 lanes x 2 flop (FMA) x 2.4 GHz
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip em_solve_batch over the interior pixels' materialised windows")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the other workloads' sub-records (64x64, 512x512 FP32/FP16, 16 images, "
                         "point sets)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target oracle CPU time")
    ap.add_argument("--plain", type=int, default=1,
                    help="also time the plain one-instance-per-launch path on the same n=441, d=49 "
                         "instances (speedup_vs_plain in the line; 0 skips it)")
    ap.add_argument("--study", choices=["psnr", "evolution", "objective"], default=None,
                    help="instead of the timing line, run a denoising-quality study on the GPU: "
                         "the PSNR table (NLM / NLEM-IRLS / NLEM-ADMM, 4 iterations), PSNR per "
                         "iteration, or the objective per iteration at sampled pixels")
    ap.add_argument("--realizations", type=int, default=10, help="noise realizations per study cell")
    ap.add_argument("--pointsets", action="store_true",
                    help="instead of the NLEM line, time em_solve_batch on the 1,048,576-instance "
                         "point-set workload (n ~ U{8..512}, d in {2,3,16,49,64}) and print its own line")
    ap.add_argument("--batch-interior", action="store_true",
                    help="instead of the NLEM line, time only em_solve_batch over the 55,696 interior "
                         "pixels of the 256x256 image as materialised n=441, d=49 instances (its own line)")
    ap.add_argument("--tune", type=int, default=1,
                    help="tune the NLEM and batch schedules (nlem_autotune, em_batch_autotune) during the "
                         "untimed warm-up and time the tuned plans, after timing the built-in ones; "
                         "0 keeps the built-in plans")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 512 MiB device-to-device copy (3 times): the known-size "
                         "kernel that scales the FETCH_SIZE / WRITE_SIZE counters")
    return ap.parse_args()


def copy_calibration():
    """A device copy of 512 MiB whose source was written before 2 GiB of other
    writes (so it is not resident in the 256 MB last-level cache): the
    known-size kernel that scales the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = (512 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    flush = torch.empty(4 * n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        flush.fill_(2.0)
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copy calibration: 3 copies of {src.numel() * 4} bytes", flush=True)


def profiled_traffic(waves):
    """HBM bytes per launch of the NLEM kernel from the committed rocprofv3
    counter summary, or None when the kernel sources changed since or the
    plan runs another coordinate-wave count than the profiled kernel."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "nlem_256x256_d49_counters.md")
    csrc = os.path.join(ROOT, "paper_1501_03879_amd", "csrc")
    try:
        text = open(path).read()
        src = "".join(open(os.path.join(csrc, f)).read()
                      for f in ("nlem_kernel.hpp", "em_device.hpp", "nlem_table.hpp", "emx_internal.hpp"))
    except OSError:
        return None
    h = hashlib.sha256(src.encode()).hexdigest()[:16]
    m_h = re.search(r"kernel_source_sha256_16: (\w+)", text)
    m_t = re.search(r"traffic_bytes_per_launch: (\d+)", text)
    m_k = re.search(r"nlem_solve_kernel<3, 7, (\d), 0>", text)
    if not m_h or not m_t or m_h.group(1) != h or not m_k or int(m_k.group(1)) != waves:
        return None
    return float(m_t.group(1))


def _denoise(hd, noisy, method, sigma, iters, init):
    """One GPU denoising run (patch 7x7, window 21x21, h = 10 sigma, box
    [0, 255], mu = 1e-3, eps = 1e-6, fixed iteration count)."""
    import torch

    import paper_1501_03879_amd as emx
    img = torch.from_numpy(noisy).cuda()
    out = torch.empty_like(img)
    if method == "nlm":
        hd.nlm_denoise(img, out, patch_radius=3, window_radius=10, h=10.0 * sigma)
    else:
        item = dict(img=img, out=out, patch_radius=3, window_radius=10, h=10.0 * sigma)
        hd.nlem_denoise_ex([item], solver=emx.SOLVER_ADMM if method == "admm" else emx.SOLVER_IRLS,
                           init=init, lo=0.0, hi=255.0, rho=1e-3, eps=1e-6, max_iter=iters, tol=0.0)
    hd.sync()
    return out.cpu().numpy()


def study_psnr(args):
    """Table 1 analogue: PSNR (dB, mean over noise realizations) of NLM,
    NLEM-IRLS and NLEM-ADMM (4 iterations each; starting from the noisy patch
    for sigma <= 60 and from the NLM patch above, as in Section 3)."""
    import numpy as np

    import paper_1501_03879_amd as emx
    import synth
    hd = emx.handle(0)
    rows = []
    for name, clean in synth.study_images().items():
        for sigma in synth.STUDY_SIGMAS:
            init = emx.NLEM_INIT_NOISY if sigma <= 60 else emx.NLEM_INIT_NLM
            acc = {"noisy": [], "nlm": [], "irls": [], "admm": []}
            for r in range(args.realizations):
                noisy = synth.study_noise(clean, sigma, r)
                acc["noisy"].append(synth.psnr(noisy, clean))
                for m in ("nlm", "irls", "admm"):
                    acc[m].append(synth.psnr(_denoise(hd, noisy, m, sigma, 4, init), clean))
            row = {"image": name, "sigma": sigma, "init": "noisy" if init == 0 else "nlm",
                   **{k: float(np.mean(v)) for k, v in acc.items()},
                   "admm_std": float(np.std(acc["admm"])), "realizations": args.realizations}
            rows.append(row)
            print(json.dumps(row), flush=True)
    print(json.dumps({"study": "psnr", "rows": len(rows),
                      "admm_minus_nlm_mean_db": float(np.mean([r["admm"] - r["nlm"] for r in rows])),
                      "admm_minus_irls_mean_db": float(np.mean([r["admm"] - r["irls"] for r in rows]))}),
          flush=True)


def study_evolution(args):
    """PSNR after t = 0..10 iterations of NLEM-ADMM and NLEM-IRLS started from
    the noisy patch (the PSNR-evolution figure of Section 3), sigma 10 and 40."""
    import numpy as np

    import paper_1501_03879_amd as emx
    import synth
    hd = emx.handle(0)
    for name in ("smooth-512", "shapes-512"):
        clean = synth.study_images()[name]
        for sigma in (10.0, 40.0):
            curves = {"admm": np.zeros(11), "irls": np.zeros(11)}
            K = max(1, min(args.realizations, 3))
            for r in range(K):
                noisy = synth.study_noise(clean, sigma, r)
                for m in curves:
                    for t in range(11):
                        curves[m][t] += synth.psnr(_denoise(hd, noisy, m, sigma, t, emx.NLEM_INIT_NOISY),
                                                   clean) / K
            print(json.dumps({"image": name, "sigma": sigma, "realizations": K,
                              **{m: [round(float(v), 3) for v in c] for m, c in curves.items()}}),
                  flush=True)


def _window_instances(noisy, pixels, sigma):
    """The NLEM instances (window patches, NLM weights) of the given pixels as
    an explicit point-set batch, built on the host in float64."""
    import numpy as np

    import synth
    H, W = noisy.shape
    P = np.pad(noisy.astype(np.float64), 3, mode="symmetric")
    pts, ws, z0 = [], [], []
    for iy, ix in pixels:
        a = np.array([P[y:y + 7, x:x + 7].reshape(-1) for y in range(max(iy - 10, 0), min(iy + 10, H - 1) + 1)
                      for x in range(max(ix - 10, 0), min(ix + 10, W - 1) + 1)])
        c = P[iy:iy + 7, ix:ix + 7].reshape(-1)
        pts.append(a.astype(np.float32))
        ws.append(np.exp(-np.sum((a - c) ** 2, axis=1) / (10.0 * sigma) ** 2).astype(np.float32))
        z0.append(c.astype(np.float32))
    return synth.pointsets.pack_instances(pts, ws, 0.0, 255.0), np.concatenate(z0)


def study_objective(args):
    """Objective per iteration at sampled pixels (the convergence figure of
    Section 3): (EM) along the EM-ADMM iterates (mu = 1e-3) and the surrogate
    along the IRLS iterates (eps = 1e-6), both from the noisy patch, sigma 40,
    computed by em_solve_batch_ex with max_iter = t; reported relative to the
    best value found (2000 ADMM iterations) and as the first iteration that
    is within 1e-3 of it."""
    import numpy as np
    import torch

    import paper_1501_03879_amd as emx
    import synth
    hd = emx.handle(0)
    clean = synth.study_images()["shapes-256"]
    noisy = synth.study_noise(clean, 40.0, 0)
    rng = np.random.default_rng(8)
    pixels = [tuple(int(v) for v in rng.integers(10, 246, size=2)) for _ in range(64)]
    b, z0 = _window_instances(noisy, pixels, 40.0)
    dev = torch.device("cuda:0")
    a = torch.from_numpy(b.a).to(dev)
    w = torch.from_numpy(b.w).to(dev)
    inst = emx.instances_tensor(b.inst, dev)

    def run(solver, T):
        z = torch.from_numpy(z0.copy()).to(dev)
        hd.em_solve_batch_ex(a, w, inst, z, solver=solver, init=emx.INIT_GIVEN, lo=0.0, hi=255.0,
                             rho=1e-3, eps=1e-6, max_iter=T, tol=0.0)
        hd.sync()
        return z.cpu().numpy().astype(np.float64)

    def objective(zs, eps=None):
        out = []
        for k in range(b.B):
            e = b.inst[k]
            n, d = int(e["n"]), int(e["d"])
            A = b.a[e["a_off"]:e["a_off"] + n * d].reshape(n, d).astype(np.float64)
            Wk = b.w[e["w_off"]:e["w_off"] + n].astype(np.float64)
            q = np.sum((zs[e["z_off"]:e["z_off"] + d][None, :] - A) ** 2, axis=1)
            out.append(np.sum(Wk * np.sqrt(q if eps is None else q + eps)))
        return np.array(out)

    best = objective(run(emx.SOLVER_ADMM, 2000))
    curves = {"admm": [], "irls": []}
    for t in range(11):
        curves["admm"].append(objective(run(emx.SOLVER_ADMM, t)) / best - 1.0)
        curves["irls"].append(objective(run(emx.SOLVER_IRLS, t), 1e-6) / best - 1.0)
    res = {"study": "objective", "pixels": len(pixels), "sigma": 40.0}
    for m, c in curves.items():
        c = np.array(c)                                    # [t, pixel]
        res[m + "_median_rel_gap"] = [float(f"{v:.3e}") for v in np.median(c, axis=1)]
        first = [int(np.argmax(c[:, k] <= 1e-3)) if np.any(c[:, k] <= 1e-3) else -1 for k in range(c.shape[1])]
        res[m + "_iters_to_1e-3_median"] = float(np.median([f for f in first if f >= 0])) if any(
            f >= 0 for f in first) else None
        res[m + "_reached_1e-3_within_10"] = float(np.mean([f >= 0 for f in first]))
    print(json.dumps(res), flush=True)


def window_sizes(H, W, R):
    import numpy as np
    y = np.arange(H)
    x = np.arange(W)
    ny = np.minimum(y + R, H - 1) - np.maximum(y - R, 0) + 1
    nx = np.minimum(x + R, W - 1) - np.maximum(x - R, 0) + 1
    return (ny[:, None] * nx[None, :]).reshape(-1)


def _events_ms(fn, reps):
    """Mean time of fn() over reps calls, from HIP events on the current stream
    (the library's calls run on it; their side streams join back into it)."""
    import torch
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _err(got, ref, D):
    import numpy as np
    e = np.abs(np.asarray(got, np.float64) - np.asarray(ref, np.float64)) / D
    return {"max_abs_over_range": float(e.max()) if e.size else 0.0,
            "rms_over_range": float(np.sqrt(np.mean(e ** 2))) if e.size else 0.0}


def _rate_record(ms, flops, **extra):
    tf = flops / (ms * 1e-3) / 1e12
    return {"ms": ms, "model_tflops": tf, "frac_of_157.3": tf / FP32_PEAK_TFLOPS, **extra}


def nlem_image_config(hd, dev, img_np, pr, wr, h, wl, fp16, reps, oracle_pix, rng, oracle_images=None):
    """nlem_denoise on one image: time per call, Mpixel/s, the 6-flop model
    throughput (+3 flop per point coordinate for the weights) and, on
    `oracle_pix` sampled pixels (all when it is >= the pixel count), the FP64
    oracle's error at the GPU's per-pixel iteration counts; oracle_images maps
    a label to the image the oracle is fed (default: the image itself)."""
    import numpy as np
    import torch

    import oracle
    import paper_1501_03879_amd as emx
    H, W = img_np.shape
    d = (2 * pr + 1) ** 2
    t = torch.from_numpy(img_np).to(dev)
    if fp16:
        t = t.half()
    out = torch.empty((H, W), dtype=torch.float32, device=dev)
    st = torch.zeros((H * W, 4), dtype=torch.int32, device=dev)

    def call():
        hd.nlem_denoise(t, out, st, patch_radius=pr, window_radius=wr, h=h, lo=wl.lo, hi=wl.hi, rho=wl.mu,
                        max_iter=wl.max_iter, tol=wl.tol)
    for _ in range(3):
        call()
    ms = _events_ms(call, reps)
    iters = emx.stats_view(st)[0].cpu().numpy().astype(np.int64)
    n = window_sizes(H, W, wr).astype(np.int64)
    flops = 6.0 * float(np.sum(n * d * iters)) + 3.0 * float(np.sum(n * d))
    got = out.cpu().numpy().reshape(-1)
    pix = np.arange(H * W) if oracle_pix >= H * W else np.sort(rng.choice(H * W, oracle_pix, replace=False))
    errs = {}
    for label, im in (oracle_images or {"oracle": img_np}).items():
        r = oracle.nlem(im, pr, wr, h, wl.lo, wl.hi, wl.mu, wl.max_iter, 0.0, pix=pix,
                        max_iter_each=iters[pix])
        errs[label] = {"pixels": int(pix.size), **_err(got[pix], r["out"], wl.hi - wl.lo)}
    return _rate_record(ms, flops, mpixel_per_s=H * W / (ms * 1e-3) / 1e6, mean_iters=float(iters.mean()),
                        reps=reps, oracle_error=errs)


def multi_config(hd, dev, reps, per_image, rng):
    """The 16-image workload as one cached nlem_denoise_multi graph."""
    import numpy as np
    import torch

    import oracle
    import paper_1501_03879_amd as emx
    import synth
    wl = synth.nlem_multi_image()
    items = []
    for im in wl.images:
        t = torch.from_numpy(im.noisy).to(dev)
        items.append(dict(img=t, out=torch.zeros_like(t), patch_radius=im.patch_radius,
                          window_radius=im.window_radius, h=im.h,
                          stats=torch.zeros((im.noisy.size, 4), dtype=torch.int32, device=dev)))

    def call():
        hd.nlem_denoise_multi(items, lo=wl.lo, hi=wl.hi, rho=wl.mu, max_iter=wl.max_iter, tol=wl.tol)
    for _ in range(2):
        call()
    ms = _events_ms(call, reps)
    flops, px, got_all, ref_all = 0.0, 0, [], []
    for im, it in zip(wl.images, items):
        H, W = im.noisy.shape
        d = (2 * im.patch_radius + 1) ** 2
        iters = emx.stats_view(it["stats"])[0].cpu().numpy().astype(np.int64)
        n = window_sizes(H, W, im.window_radius).astype(np.int64)
        flops += 6.0 * float(np.sum(n * d * iters)) + 3.0 * float(np.sum(n * d))
        px += H * W
        pix = np.sort(rng.choice(H * W, per_image, replace=False))
        r = oracle.nlem(im.noisy, im.patch_radius, im.window_radius, im.h, wl.lo, wl.hi, wl.mu, wl.max_iter,
                        0.0, pix=pix, max_iter_each=iters[pix])
        got_all.append(it["out"].cpu().numpy().reshape(-1)[pix])
        ref_all.append(r["out"])
    return _rate_record(ms, flops, mpixel_per_s=px / (ms * 1e-3) / 1e6, images=len(wl.images), pixels=px,
                        reps=reps, oracle_error={"pixels": int(per_image * len(wl.images)),
                                                 **_err(np.concatenate(got_all), np.concatenate(ref_all), 255.0)})


def pointsets_config(hd, dev, reps, per_d, rng):
    """em_solve_batch on the 1,048,576 point sets (drawn on the device)."""
    import numpy as np
    import torch

    import oracle
    import paper_1501_03879_amd as emx
    import synth
    B = 1 << 20
    a, w, inst, zs = synth.pointsets.make_pointset_batch_device(505, B, dev)
    it = emx.instances_tensor(inst, dev)
    z = torch.zeros(zs, dtype=torch.float32, device=dev)
    st = torch.zeros((B, 4), dtype=torch.int32, device=dev)
    mu, T, tol = synth.configs.POINTSET_MU, synth.configs.POINTSET_MAX_ITER, synth.configs.POINTSET_TOL

    def call():
        hd.em_solve_batch(a, w, it, z, st, lo=-3.0, hi=3.0, rho=mu, max_iter=T, tol=tol, init=emx.INIT_MAXW)
    call()
    ms = _events_ms(call, reps)
    iters = emx.stats_view(st)[0].cpu().numpy().astype(np.int64)
    flags = emx.stats_view(st)[1].cpu().numpy()
    nd = inst["n"].astype(np.float64) * inst["d"].astype(np.float64)
    flops = 6.0 * float(np.sum(nd * iters))
    sample = np.concatenate([rng.choice(np.flatnonzero(inst["d"] == dv), per_d, replace=False)
                             for dv in (2, 3, 16, 49, 64)])
    pts, ws = [], []
    for b in sample:
        e = inst[b]
        n, d = int(e["n"]), int(e["d"])
        pts.append(a[e["a_off"]:e["a_off"] + n * d].view(n, d).cpu().numpy())
        ws.append(w[e["w_off"]:e["w_off"] + n].cpu().numpy())
    sub = synth.pointsets.pack_instances(pts, ws, -3.0, 3.0)
    ref = oracle.em_batch(sub, mu, T, 0.0, init=oracle.INIT_MAXW, max_iter_each=iters[sample])
    zc = z.cpu().numpy()
    got = np.concatenate([zc[inst[b]["z_off"]:inst[b]["z_off"] + inst[b]["d"]] for b in sample])
    res = _rate_record(ms, flops, solves_per_s=B / (ms * 1e-3), instances=B, mean_iters=float(iters.mean()),
                       converged_fraction=float(np.mean(flags == 1)),
                       maxiter_instances=int(np.sum(flags == 2)), reps=reps,
                       oracle_error={"instances": int(sample.size), **_err(got, ref["z"], 6.0)},
                       plan=hd.em_batch_plan_get())
    del a, w, z, st, it
    torch.cuda.empty_cache()
    return res


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.pointsets:
        pointsets(args)
        return
    if args.batch_interior:
        import torch

        import paper_1501_03879_amd as emx
        import synth
        wl = synth.nlem_256()
        r = batch_interior_rate(wl.images[0], wl, torch.device("cuda:0"), emx.handle(0), None,
                                reps=max(1, min(args.steps, 20)), tune=args.tune != 0)
        print(json.dumps({"workload": "em_solve_batch, the 256x256 image's interior pixels as n=441, "
                                      "d=49 instances", **r}), flush=True)
        return
    if args.study:
        if args.gpus != 1:
            print("studies run on one GPU (--gpus 1)", file=sys.stderr)
            sys.exit(2)
        import torch
        torch.zeros(1, device="cuda:0")   # the device is set up by torch before the library
        {"psnr": study_psnr, "evolution": study_evolution, "objective": study_objective}[args.study](args)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: each pixel's solve is independent, so the "
              "image would be split by rows across GPUs with no exchange; "
              "this benchmark runs on one GPU only (use --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1501_03879_amd as emx
    import synth

    wl = synth.nlem_256()
    im = wl.images[0]
    H, W = im.noisy.shape
    pr, wr = im.patch_radius, im.window_radius
    d = (2 * pr + 1) ** 2
    dev = torch.device("cuda:0")
    img = torch.from_numpy(im.noisy).to(dev)
    out = torch.empty_like(img)
    stats = torch.zeros((H * W, 4), dtype=torch.int32, device=dev)
    hd = emx.handle(0)
    stream = torch.cuda.current_stream()

    def step():
        hd.nlem_denoise(img, out, stats, patch_radius=pr, window_radius=wr, h=im.h, lo=wl.lo,
                        hi=wl.hi, rho=wl.mu, max_iter=wl.max_iter, tol=wl.tol)

    # schedule: the built-in plan is timed, then nlem_autotune keeps the
    # fastest plan of its search (both untimed for the line); the timed steps
    # run the plan in force
    plan = {"nlem_builtin": hd.nlem_plan_get(pr, wr)}
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if args.tune:
        plan["nlem_builtin_ms_per_step"] = _events_ms(step, 20)
        t_tune = time.perf_counter()
        hd.nlem_autotune(dict(img=img, out=out, stats=stats, patch_radius=pr, window_radius=wr, h=im.h),
                         lo=wl.lo, hi=wl.hi, rho=wl.mu, max_iter=wl.max_iter, tol=wl.tol, repeats=5)
        hd.sync()
        plan["tune_s"] = time.perf_counter() - t_tune
    plan["nlem"] = hd.nlem_plan_get(pr, wr)
    plan["nlem_same_as_builtin"] = all(plan["nlem"][k] == plan["nlem_builtin"][k]
                                       for k in ("waves", "chunk", "order", "arm_factor", "check_every"))
    waves = plan["nlem"]["waves"]
    for _ in range(3 if args.tune else 0):   # (the warm-up ran before the tuning)
        step()
    torch.cuda.synchronize()
    # the library brackets each NLEM solve launch with HIP events on the same
    # stream, which times the dominant kernel alone for the roofline
    hd.kernel_timing(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1) / args.steps
    k_total_ms, k_launches = hd.kernel_timing_read()
    hd.kernel_timing(False)
    if k_launches != args.steps:
        raise RuntimeError(f"expected {args.steps} timed NLEM launches, got {k_launches}")
    kernel_ms = k_total_ms / k_launches
    hd.sync()

    it, fl, rp, rd = emx.stats_view(stats)
    iters = it.cpu().numpy().astype(np.int64)
    flags = fl.cpu().numpy()
    n = window_sizes(H, W, wr).astype(np.int64)
    elem_iters = float(np.sum(n * d * iters))
    flops = 6.0 * elem_iters + 3.0 * float(np.sum(n * d))
    tflops = flops / (kernel_ms * 1e-3) / 1e12          # the NLEM kernel alone
    tflops_step = flops / (ms * 1e-3) / 1e12            # whole step (with the queue kernels)
    solves_per_s = H * W / (ms * 1e-3)

    res = {
        "metric": METRIC,
        "value": solves_per_s / 1e6,
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"nlem {H}x{W} sigma=20 patch 7x7 (d={d}) window 21x21 (n<=441) "
                               f"h=200 box [0,255] mu={wl.mu} tol={wl.tol} max_iter={wl.max_iter}",
                   "pixels": H * W, "patch_radius": pr, "window_radius": wr},
        "mpixel_per_s": solves_per_s / 1e6,
        "nlem_solves_per_s_all_pixels": solves_per_s,
        "nlem_solves_note": "one EM solve per pixel, border pixels included (their windows are "
                            "truncated: n from 121 to 441, mean 423.2); the rate at n=441, d=49 "
                            "exactly is em_solves_per_s_n441_d49",
        "mean_iters": float(iters.mean()),
        "converged_fraction": float(np.mean(flags == 1)),
        "plan": plan,
        "elem_iters_per_s": elem_iters / (ms * 1e-3),
        "host_wall_s": wall,
        "roofline": {"bound": "alu", "achieved": tflops, "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": tflops / FP32_PEAK_TFLOPS,
                     "frac_nonpacked_fma_peak": tflops / FP32_NONPACKED_TFLOPS,
                     "flops_per_launch": flops, "traffic": profiled_traffic(waves),
                     "kernel": f"nlem_solve_kernel<{pr}, 7, {waves}, 0> ({waves} coordinate waves, "
                               f"plan {plan['nlem']['source']})", "kernel_ms": kernel_ms,
                     "achieved_per_step": tflops_step,
                     "timing": "achieved: flops per launch / the NLEM kernel's mean duration, from "
                               "HIP events the library records around each NLEM launch on the "
                               "launch stream over the timed steps (em_kernel_timing); "
                               "achieved_per_step and ms_per_step: events around whole steps "
                               "(one nlem_denoise call: the three queue-order "
                               "kernels and one NLEM kernel launch)"},
    }

    rng = np.random.default_rng(12)
    if not args.no_batch:
        bi = batch_interior_rate(im, wl, dev, hd, out, plain=args.plain != 0, oracle_instances=1024,
                                 tune=args.tune != 0)
        res["em_solves_per_s_n441_d49"] = bi["solves_per_s"]
        res["batch_interior"] = bi
        if "plain" in bi:
            res["speedup_vs_plain"] = bi["speedup_vs_plain"]
    if not args.no_configs:
        cfg = {}
        sm = synth.nlem_small()
        s_im = sm.images[0]
        cfg["small_64x64_r2_R5_T50"] = nlem_image_config(
            hd, dev, s_im.noisy, s_im.patch_radius, s_im.window_radius, s_im.h, sm, False, 20, 1 << 30, rng)
        cfg["nlem_256x256_d49"] = {"ms": ms, "model_tflops": tflops_step,
                                   "frac_of_157.3": tflops_step / FP32_PEAK_TFLOPS,
                                   "mpixel_per_s": solves_per_s / 1e6, "mean_iters": float(iters.mean()),
                                   "note": "the timed step above; oracle error over every pixel in "
                                           "cpu_baseline.oracle_error"}
        for f16 in (False, True):
            mw = synth.nlem_512_mixed(fp16_storage=f16)
            m_im = mw.images[0]
            refs = {"oracle": m_im.noisy}
            if f16:
                refs = {"oracle_fp32_image": m_im.noisy,
                        "oracle_fp16_rounded_image": m_im.noisy.astype(np.float16).astype(np.float32)}
            cfg["mixed_512x512_" + ("fp16" if f16 else "fp32")] = nlem_image_config(
                hd, dev, m_im.noisy, 3, 10, m_im.h, mw, f16, 5, 4096, rng, refs)
        cfg["multi_16_images_graph"] = multi_config(hd, dev, 3, 256, rng)
        cfg["pointsets_1m"] = pointsets_config(hd, dev, 3, 512, rng)
        res["configs"] = cfg
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(im, wl, args.cpu_seconds,
                                           out.cpu().numpy().reshape(-1).astype(np.float64), iters)
    print(json.dumps(res), flush=True)


def pointsets(args):
    """em_solve_batch on the point-set workload: 1,048,576 instances, n ~
    U{8..512}, d uniform over {2, 3, 16, 49, 64}, 20% Student-t outliers
    scaled by 50, weights Exp(1), box [-3, 3]^d, max-weight start, mu 0.5,
    tol 1e-4, at most 1000 iterations; inputs drawn on the device, resident
    in HBM before the timed region.  One JSON line with the rate, the FP32
    model throughput (6 flop per point coordinate per iteration) and the
    per-d iteration counts."""
    import numpy as np
    import torch

    import paper_1501_03879_amd as emx
    import synth
    if args.gpus != 1:
        print("the point-set line measures one GPU (--gpus 1)", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    B = 1 << 20
    a, w, inst, zs = synth.pointsets.make_pointset_batch_device(505, B, dev)
    it = emx.instances_tensor(inst, dev)
    z = torch.zeros(zs, dtype=torch.float32, device=dev)
    st = torch.zeros((B, 4), dtype=torch.int32, device=dev)
    hd = emx.handle(0)
    kw = dict(lo=-3.0, hi=3.0, rho=synth.configs.POINTSET_MU, max_iter=synth.configs.POINTSET_MAX_ITER,
              tol=synth.configs.POINTSET_TOL, init=emx.INIT_MAXW)
    for _ in range(max(1, args.warmup // 5)):
        z.zero_()
        hd.em_solve_batch(a, w, it, z, st, **kw)
    torch.cuda.synchronize()
    reps = max(1, min(args.steps, 5))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        hd.em_solve_batch(a, w, it, z, st, **kw)   # z is the max-weight start each time (init MAXW)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    iters = emx.stats_view(st)[0].cpu().numpy().astype(np.float64)
    flags = emx.stats_view(st)[1].cpu().numpy()
    nd = inst["n"].astype(np.float64) * inst["d"].astype(np.float64)
    flops = float(np.sum(nd * 6.0 * iters))
    per_d = {int(dv): {"instances": int(np.sum(inst["d"] == dv)),
                       "mean_iters": float(iters[inst["d"] == dv].mean()),
                       "elem_iter_share": float(np.sum((nd * iters)[inst["d"] == dv]) / np.sum(nd * iters))}
             for dv in (2, 3, 16, 49, 64)}
    print(json.dumps({"workload": "em_solve_batch, 1,048,576 point sets", "instances": B, "ms": ms,
                      "solves_per_s": B / (ms * 1e-3), "mean_iters": float(iters.mean()),
                      "converged_fraction": float(np.mean(flags == 1)),
                      "model_tflops": flops / (ms * 1e-3) / 1e12,
                      "frac_of_157.3": flops / (ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS,
                      "reps": reps, "per_d": per_d}), flush=True)


def batch_interior_rate(im, wl, dev, hd, out_nlem, reps=5, plain=False, oracle_instances=0, tune=False):
    """em_solve_batch on every interior pixel of the image (full 21 x 21
    windows: n = 441, d = 49) as materialised instances, the EM-solves half of
    the metric.  Input preparation (untimed): patches gathered on the device,
    NLM weights exp(-||P_i - P_j||^2 / h^2) in FP64 there, both stored as
    FP32; start = the largest weight (the centre patch).  With plain=True the
    same instances also go through em_solve_plain (one launch per instance),
    timed with HIP events; oracle_instances > 0: that many sampled instances
    are solved by the FP64 oracle at the GPU's iteration counts (every
    coordinate of z compared).  tune=True: the built-in plan is timed, then
    em_batch_autotune picks the plan the timed calls use (both reported)."""
    import numpy as np
    import torch

    import oracle
    import paper_1501_03879_amd as emx
    import synth
    from synth.pointsets import INSTANCE_DTYPE
    H, W = im.noisy.shape
    r, R = im.patch_radius, im.window_radius
    k, nwin = 2 * r + 1, (2 * R + 1) ** 2
    d = k * k
    P = torch.from_numpy(np.pad(im.noisy.astype(np.float64), r, mode="symmetric")).to(dev)
    patches = P.unfold(0, k, 1).unfold(1, k, 1).reshape(H * W, d)      # row-major patches
    ys, xs = torch.meshgrid(torch.arange(R, H - R, device=dev), torch.arange(R, W - R, device=dev),
                            indexing="ij")
    centres = (ys * W + xs).reshape(-1)
    dy, dx = torch.meshgrid(torch.arange(-R, R + 1, device=dev), torch.arange(-R, R + 1, device=dev),
                            indexing="ij")
    idx = centres[:, None] + (dy * W + dx).reshape(-1)[None, :]       # B x n, row-major window
    B = int(idx.shape[0])
    a64 = patches[idx]                                                # B x n x d
    w = torch.exp(-((a64 - patches[centres][:, None, :]) ** 2).sum(-1) / (im.h * im.h)).float()
    a = a64.float().reshape(-1)
    del a64, patches, P
    w = w.reshape(-1).contiguous()
    inst = np.zeros(B, dtype=INSTANCE_DTYPE)
    bi = np.arange(B, dtype=np.int64)
    inst["a_off"], inst["w_off"], inst["z_off"] = bi * nwin * d, bi * nwin, bi * d
    inst["n"], inst["d"] = nwin, d
    it = emx.instances_tensor(inst, dev)
    z = torch.zeros(B * d, dtype=torch.float32, device=dev)
    st = torch.zeros((B, 4), dtype=torch.int32, device=dev)
    kw = dict(lo=wl.lo, hi=wl.hi, rho=wl.mu, max_iter=wl.max_iter, tol=wl.tol, init=emx.INIT_MAXW)
    hd.em_solve_batch(a, w, it, z, st, **kw)   # warm-up (workspace, code objects)
    torch.cuda.synchronize()
    plan = {"batch_builtin": hd.em_batch_plan_get()}
    if tune:
        for _ in range(3):
            hd.em_solve_batch(a, w, it, z, st, **kw)
        plan["batch_builtin_ms"] = _events_ms(lambda: hd.em_solve_batch(a, w, it, z, st, **kw), reps)
        t_tune = time.perf_counter()
        hd.em_batch_autotune(a, w, it, z, st, lo=wl.lo, hi=wl.hi, rho=wl.mu, max_iter=wl.max_iter,
                             tol=wl.tol, init=emx.INIT_MAXW, repeats=3)
        hd.sync()
        plan["tune_s"] = time.perf_counter() - t_tune
    plan["batch"] = hd.em_batch_plan_get()
    plan["batch_same_as_builtin"] = all(plan["batch"][k] == plan["batch_builtin"][k]
                                        for k in ("generic_classes", "arm_factor", "check_every", "host_counts"))
    ms = _events_ms(lambda: hd.em_solve_batch(a, w, it, z, st, **kw), reps)
    iters, flags = emx.stats_view(st)[0].cpu().numpy(), emx.stats_view(st)[1].cpu().numpy()
    centre = z.reshape(B, d)[:, (d - 1) // 2]
    diff = (None if out_nlem is None else
            float((centre - out_nlem.reshape(-1)[centres]).abs().max()) / (wl.hi - wl.lo))
    flops = 6.0 * nwin * d * float(np.sum(iters.astype(np.float64)))
    res = {"instances": B, "n": nwin, "d": d, "solves_per_s": B / (ms * 1e-3),
           **_rate_record(ms, flops), "mean_iters": float(iters.mean()),
           "converged_fraction": float(np.mean(flags == 1)),
           "max_abs_diff_vs_nlem_over_range": diff,
           "note": "em_solve_batch over the interior pixels' materialised windows (inputs in HBM, "
                   "weights computed outside the timed region); the NLEM kernel solves the same "
                   "instances from the image tile",
           "plan": plan}
    if oracle_instances > 0:
        rng = np.random.default_rng(5)
        sample = np.sort(rng.choice(B, min(oracle_instances, B), replace=False))
        ah = a.view(B, nwin, d)[torch.from_numpy(sample).to(dev)].cpu().numpy()
        wh = w.view(B, nwin)[torch.from_numpy(sample).to(dev)].cpu().numpy()
        sub = synth.pointsets.pack_instances(list(ah), list(wh), wl.lo, wl.hi)
        ref = oracle.em_batch(sub, wl.mu, wl.max_iter, 0.0, init=oracle.INIT_MAXW,
                              max_iter_each=iters[sample])
        got = z.view(B, d)[torch.from_numpy(sample).to(dev)].cpu().numpy().reshape(-1)
        res["oracle_error"] = {"instances": int(sample.size), **_err(got, ref["z"], wl.hi - wl.lo)}
    if plain:
        zp = torch.zeros_like(z)
        stp = torch.zeros_like(st)
        pk = dict(kw)
        hd.em_solve_plain(a[:nwin * d * 64], w[:nwin * 64], emx.instances_tensor(inst[:64], dev), inst[:64],
                          zp, stp, **pk)   # warm-up
        torch.cuda.synchronize()
        pms = _events_ms(lambda: hd.em_solve_plain(a, w, it, inst, zp, stp, **pk), 1)
        same = bool(torch.equal(zp, z))
        res["plain"] = {"ms": pms, "solves_per_s": B / (pms * 1e-3), "instances": B,
                        "bitwise_equal_to_batched": same,
                        "note": "em_solve_plain on the same instances: the batched class kernel launched as "
                                "one workgroup per instance, back to back on one stream (HIP events)"}
        res["speedup_vs_plain"] = res["solves_per_s"] / res["plain"]["solves_per_s"]
        del zp, stp
    del a, w, z, st, it
    torch.cuda.empty_cache()
    return res


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(im, wl, target_s, gpu_out, gpu_iters):
    """The FP64 oracle on all host threads, run on the same image at the
    GPU's per-pixel iteration counts (reading R18: a solve stops at most one
    iteration after the oracle's own stopping rule would), over a random
    pixel order until about target_s seconds of CPU time (the whole image
    when the host is fast enough).  Its outputs double as the parity check
    of the timed GPU run: max-abs and RMS of |gpu - oracle| / (hi - lo) over
    the pixels it covered."""
    import numpy as np

    import oracle
    H, W = im.noisy.shape
    D = wl.hi - wl.lo
    rng = np.random.default_rng(0)
    order = rng.permutation(H * W)
    threads = oracle.max_threads()
    npix = 1024
    done = 0
    total_t = 0.0
    errs = []
    while True:
        pix = order[done:done + npix]
        t0 = time.perf_counter()
        r = oracle.nlem(im.noisy, im.patch_radius, im.window_radius, im.h, wl.lo, wl.hi, wl.mu,
                        wl.max_iter, 0.0, pix=pix, max_iter_each=gpu_iters[pix], nthreads=threads)
        total_t += time.perf_counter() - t0
        errs.append(np.abs(gpu_out[pix] - r["out"]) / D)
        done += len(pix)
        if total_t >= target_s or done >= H * W:
            break
        rate = done / total_t
        npix = int(min(H * W - done, max(1024, rate * (target_s - total_t))))
    e = np.concatenate(errs)
    # one thread on a fixed 256-pixel sample, for the per-core rate
    one = order[:256]
    t0 = time.perf_counter()
    oracle.nlem(im.noisy, im.patch_radius, im.window_radius, im.h, wl.lo, wl.hi, wl.mu,
                wl.max_iter, 0.0, pix=one, max_iter_each=gpu_iters[one], nthreads=1)
    t1 = time.perf_counter() - t0
    return {"value": done / total_t, "unit": "EM solves/s", "cores": threads, "cpu_model": cpu_model(),
            "kind": "oracle",
            "sample": f"{done} random pixels of the 256x256 image ({done / (H * W):.1%}), FP64, "
                      f"each run to the GPU's iteration count for that pixel, {total_t:.1f} s",
            "value_1_thread": len(one) / t1, "sample_1_thread": f"{len(one)} of the same pixels, {t1:.2f} s",
            "oracle_error": {"pixels": int(done), "max_abs_over_range": float(e.max()),
                             "rms_over_range": float(np.sqrt(np.mean(e ** 2))),
                             "what": "|nlem_denoise output of the timed run - FP64 oracle at the GPU's "
                                     "per-pixel iteration counts| / (hi - lo)"}}


if __name__ == "__main__":
    main()
