#!/usr/bin/env python3
"""Forward+backward rasterize iterations/s and Gaussian-tile pairs/s on one MI355X, batched vs plain.

One step = one pass of the whole hot path over one batch of views: EWA
projection and SH colour, depth sort, tile binning (prefix sum + pair
emission), tile sort, per-tile ranges, front-to-back blend with the entropy
term, per-view mean entropy, L1 loss and its gradient, back-to-front blend
backward with Alg. 1, per-Gaussian gradient reduction, projection backward.
Every stage runs in the HIP library (libgsr.so); inputs are resident in HBM
before the timed region.

Default workload (the metric's configuration): 3,000,000 Gaussians, SH degree
3, eight orbit cameras at the resolution scheduler's stages (2x 486x324,
3x 972x648, 3x 1944x1296), loss L1 + 0.015 L_E.  Two forms run on the same
views in the same process:

  batched  all eight views in one launch sequence, SH stored in BF16, FP32
           blending, tile shape / LDS batch / scheduling from gsr_autotune,
           eager launches at a fixed pair capacity (GSR_NO_SYNC); the same
           form replayed from HIP graphs is timed too;
  plain    eight single-view launch sequences, SH in FP32 (the unrounded
           draw), plain mode (exact pair sizing, one host sync per view).

`value` is the batched form's views/s.  Other workloads (--workload) time one
form.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+bwd rasterize iters/s and Gaussian-tile pairs/s at 1 MI355X; batched vs plain"
METRIC_RENDER = "forward-only render views/s (test-time FPS) at 1 MI355X"
METRIC_TRAIN = "synthetic training iterations/s (L1 + D-SSIM + entropy, Adam, scale reset, r_max scheduler) at 1 MI355X"
GAMMA = 0.015
HBM_PEAK_GBS = 8000.0
# MI355X published dense FP32 vector peak (256 CUs x 2.4 GHz x 256 FLOP/clock: FMA = 2, packed dual rate)
FP32_PEAK_TFLOPS = 157.3
# issue rate of unpacked FP32 VALU operations: 256 CUs x 64 lanes x 2.4 GHz (one op per lane per clock)
VALU_ISSUE_TOPS = 256 * 64 * 2.4e9 / 1e12

# Work of the blend kernels per evaluated (pixel, list position), the method's own
# count: every position a pixel visits costs the alpha test, a blended one its
# blending on top (forward), and the backward replays every position up to the
# pixel's last contributor.
OPS_EVAL_FWD = 21           # ~20 VALU + exp per visited position
OPS_BLENDED_FWD = 3         # + log + 2 per blended position (entropy term)
OPS_EVAL_BWD = 53           # ~50 VALU + exp + log + rcp per position walked back
# Post-cull model: what the kernels execute after the exact 8x8-block cull.
OPS_ALPHA_TEST = 11         # per tested position: offset, exponent, exp2, opacity scale, clamp, skip test
OPS_BLEND_FWD = 10          # per blended pair: transmittance, stop test, colour, entropy term
OPS_BLEND_BWD = 49          # per blended pair: T recovery, dC/dalpha, Alg. 1, 9 gradient terms and their sums
OPS_ENTROPY = 2             # of OPS_BLEND_FWD / OPS_BLENDED_FWD: log2 and the entropy FMA (absent when rendering)


def blend_ops_method(kind, st, render=False):
    """Operations of the method's per-evaluation model (no cull)."""
    if kind == "blend_fwd":
        return OPS_EVAL_FWD * st["evals_fwd"] + (0 if render else OPS_BLENDED_FWD) * st["blended"]
    return OPS_EVAL_BWD * st["evals_bwd"]


def blend_ops_post_cull(kind, st, render=False):
    """Operations the kernels execute on the positions that survive the block cull."""
    if kind == "blend_fwd":
        return OPS_ALPHA_TEST * st["tested_fwd"] + (OPS_BLEND_FWD - (OPS_ENTROPY if render else 0)) * st["blended"]
    return OPS_ALPHA_TEST * st["tested_bwd"] + OPS_BLEND_BWD * st["blended"]


WORKLOAD_NAMES = {
    "tiny": "2k Gaussians, 1x128x128, SH0",
    "single": "200k Gaussians, 1x1296x840, SH3",
    "sweep": "1M Gaussians, 1x1600x1060, SH3",
    "sweep_half": "1M Gaussians (scales x0.5), 1x1600x1060, SH3",
    "batched": "3M Gaussians, 8 views (2x486x324, 3x972x648, 3x1944x1296), SH3",
    "diff": "6M Gaussians, 4x1920x1080, SH3",
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="batched", choices=sorted(WORKLOAD_NAMES))
    ap.add_argument("--form", choices=["compare", "batched", "plain"], default=None,
                    help="batched workload: both forms (default), or one; other workloads: one launch sequence "
                         "for all views (batched) or one per view (plain)")
    ap.add_argument("--tile", default=None, help="tile shape WxH (default: autotuned for the batched workload, else 16x16)")
    ap.add_argument("--lds", type=int, default=None)
    ap.add_argument("--graph", action="store_true", help="one form: replay captured HIP graphs")
    ap.add_argument("--no-sync", action="store_true",
                    help="one form: eager launches at a fixed pair capacity, no host synchronisation per step")
    ap.add_argument("--persistent", action="store_true", help="persistent blend kernels pulling tiles from per-XCD queues")
    ap.add_argument("--autotune", action="store_true", help="one form: pick tile shape and LDS batch with gsr_autotune first")
    ap.add_argument("--no-autotune", action="store_true", help="compare form: 16x16 tiles, LDS batch 128")
    ap.add_argument("--forward-only", action="store_true",
                    help="test-time rendering (gsr_render): colour only, no entropy, no backward; value = views/s")
    ap.add_argument("--per-view", action="store_true", help="same as --form plain")
    ap.add_argument("--sh", choices=["auto", "f32", "bf16"], default="auto", help="SH storage (auto: the workload's)")
    ap.add_argument("--bf16", action="store_true", help="same as --sh bf16")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true", help="do not bracket stages with HIP events")
    ap.add_argument("--breakdown-steps", type=int, default=20,
                    help="untimed steps after the timed region with every stage bracketed by events")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (3 launches), to scale HBM counters")
    ap.add_argument("--aux", action="store_true",
                    help="time the training-step and scheduler entry points (scale reset, opacity regulariser, "
                         "Adam, D-SSIM, base loss, r_max selection) at the training workload's sizes")
    ap.add_argument("--train", action="store_true",
                    help="time a synthetic training run (loss of Eq. 6 + 12, Adam, scale reset, resolution scheduler)")
    ap.add_argument("--train-iters", type=int, default=30000,
                    help="iterations of the training run (the paper's 30K by default); its 150-epoch schedule "
                         "is laid out over this many")
    ap.add_argument("--train-gaussians", type=int, default=3_300_000)
    ap.add_argument("--train-res", default="1296x840")
    ap.add_argument("--train-regulariser", choices=["entropy", "opacity", "none"], default="entropy",
                    help="entropy constraint (Eq. 12), the opacity regulariser it is compared with, or neither")
    a = ap.parse_args()
    if a.per_view:
        a.form = "plain"
    if a.form is None:
        a.form = "compare" if a.workload == "batched" and not a.forward_only else "batched"
    return a


def stage_bytes(stage, n, V, sh_bytes, pairs, n_tiles, npix):
    """Algorithmic HBM bytes of one launch of each stage: the data the stage must
    read and write once (per (view, Gaussian) `vn`, per pair, per tile, per pixel)."""
    vn = n * V
    return {
        "project": n * (44 + sh_bytes) + vn * 64,          # params + SH once; record 48 + key 4 + rect 8 + tt 4
        "depth_sort": vn * 4 * 20,                          # 4 passes: key+value in/out, key histogram
        "scan": vn * 36,                                    # order, tt and rect gathered, depth-ordered copies, offsets
        "duplicate": vn * 20 + pairs * 8,                   # order/tt/offset/rect; tile id, owner
        # 2 passes: keys read twice (histogram, ranking), key + value written; the first pass's
        # values are the items' indices, the last pass writes no keys (it records the tile ranges)
        "tile_sort": pairs * 16 * 2,
        "ranges": n_tiles * 16,                             # empty tiles' bounds; the tile order reads them twice
        # blend stages: every pair of every list; the forward stops reading a tile's list
        # once all its pixels have stopped, so this bounds what it reads from above
        "blend_fwd": pairs * 56 + npix * 24,                # pair value + owner + record; rgb, H, T, n_contrib
        "entropy_mean": 0,
        "blend_bwd": pairs * 96 + npix * 24,                # pair value + owner + record + row + stamp; per-pixel state
        # params + SH in, grads out; per view the row stamp and the 2D-gradient row (read only
        # where the stamp is this frame's: every row counted, an upper bound)
        "project_bwd": n * (88 + 2 * sh_bytes) + vn * 40,
        "grad_reduce": pairs * 8,                           # stamps + owners in (rows and 2D grads only where blended)
    }[stage]


def source_hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def percentiles(xs):
    a = np.asarray(xs, np.float64)
    return {"median_ms": round(float(np.median(a)), 4), "p10_ms": round(float(np.percentile(a, 10)), 4),
            "p90_ms": round(float(np.percentile(a, 90)), 4)}


def _pixel_sample(cam, frac, seed, v):
    """The seeded pixel sample of view v: sorted packed indices (shared by every oracle timing)."""
    M = cam.width * cam.height
    rng = np.random.default_rng(seed + v)
    return np.sort(rng.choice(M, max(1, int(round(frac * M))), replace=False))


def _oracle_view(orc, scene, cam, target, tile, forward_only, sel):
    """One view through the oracle: projection and binning (and the projection backward)
    in full, the blend (and entropy and blend backward) on the packed pixels `sel`.
    Returns (seconds of the per-view part, seconds of the per-pixel part, oracle image)."""
    tw, th = tile
    W, H = cam.width, cam.height
    M = W * H
    pix = np.zeros(M, np.uint8)
    pix[sel] = 1
    pix = pix.reshape(H, W)
    t0 = time.perf_counter()
    pr = orc.project(scene, cam)
    vals, ranges = orc.bin_lists(pr["mean2d"], pr["radius"], pr["depth32"], W, H, tw, th)
    t1 = time.perf_counter()
    img = orc.render(W, H, tw, th, pr["mean2d"], pr["conic"], pr["opacity"], pr["rgb"], ranges, vals, pix)
    t2 = t3 = t4 = time.perf_counter()
    if not forward_only:
        gC = np.sign(img["rgb"] - target) / (3.0 * M)
        gH = np.full((H, W), GAMMA / M)
        t2 = time.perf_counter()
        g2 = orc.backward_render(W, H, tw, th, pr["mean2d"], pr["conic"], pr["opacity"], pr["rgb"], ranges, vals,
                                 gC, gH, pix)
        t3 = time.perf_counter()
        orc.backward_project(scene, cam, g2)
        t4 = time.perf_counter()
    return (t1 - t0) + (t4 - t3), (t2 - t1) + (t3 - t2), img


def _per_iteration(cams, per_view):
    """Seconds per iteration over all views: each unsampled view is charged the time of
    the sampled view of its resolution."""
    total = 0.0
    for v, cam in enumerate(cams):
        if v in per_view:
            total += per_view[v]
        else:
            same = [u for u in per_view if (cams[u].width, cams[u].height) == (cam.width, cam.height)]
            if not same:
                raise ValueError(f"no sampled view of resolution {cam.width}x{cam.height}")
            total += per_view[same[0]]
    return total


def cpu_baseline(scene, cams, tile, targets, forward_only=False, views=None, frac=0.5, seed=77):
    """The FP64 oracle (single-threaded) on a bounded sample of the same workload.

    For each sampled view: projection and binning (and the projection backward)
    in full; blend + entropy + blend backward (the blend alone for test-time
    rendering) on a seeded fraction `frac` of the view's pixels.  Per-pixel work
    is extrapolated to the whole view, and each unsampled view is charged the
    time of the sampled view of its resolution.  Returns the record and the
    oracle's images of the sampled pixels (for the image-error check)."""
    from oracle import oracle as orc
    views = list(range(len(cams))) if views is None else list(views)
    per_view = {}
    measured = 0.0
    sampled_px = {}
    for v in views:
        cam = cams[v]
        M = cam.width * cam.height
        sel = _pixel_sample(cam, frac, seed, v)
        fixed, pixel, img = _oracle_view(orc, scene, cam, targets[v], tile, forward_only, sel)
        per_view[v] = fixed + pixel * M / len(sel)
        measured += fixed + pixel
        sampled_px[v] = (sel, img["rgb"].reshape(-1, 3)[sel], img["flags"].reshape(-1)[sel])
    total = _per_iteration(cams, per_view)
    n_sel = sum(len(s[0]) for s in sampled_px.values())
    res = [f"{cams[v].width}x{cams[v].height}" for v in views]
    rec = {"value": len(cams) / total, "unit": "views/s" if forward_only else "iters/s", "cores": 1,
           "kind": "oracle",
           "sample": (f"FP64 oracle, 1 thread, on views {views} ({', '.join(res)}) of the {len(cams)}: projection, "
                      f"binning{'' if forward_only else ' and projection backward'} in full, "
                      f"{'blend' if forward_only else 'blend, entropy and blend backward'} on a seeded "
                      f"{frac:.0%} of each sampled view's pixels ({n_sel} pixels); extrapolated per pixel and, for "
                      f"the unsampled views, per resolution; {measured:.1f} s measured, {total:.1f} s per "
                      f"{len(cams)}-view iteration")}
    return rec, sampled_px


def _stripe_worker(job):
    """One of P oracle processes: the workload drawn again from its seed, and on each
    sampled view every P-th pixel of the seeded sample (a disjoint stripe)."""
    name, sh_f32, tile, forward_only, views, frac, seed, i, P = job
    from oracle import oracle as orc
    from paper_2603_09277_amd import scenes
    scene, cams, _ = scenes.workload(name, sh_f32=sh_f32)
    out = {}
    for v in views:
        cam = cams[v]
        target = scenes.target_image(1000 + v, cam.height, cam.width)
        sel = _pixel_sample(cam, frac, seed, v)
        fixed, pixel, _ = _oracle_view(orc, scene, cam, target, tile, forward_only, sel[i::P])
        out[v] = (fixed, pixel, len(sel))
    return out


def cpu_baseline_processes(name, sh_f32, cams, tile, forward_only=False, views=None, frac=0.01, seed=77, procs=None):
    """The same oracle sample as P independent processes (P = the host's CPUs available
    to this process, at most 16), each taking a disjoint stripe of every sampled view's
    pixels and repeating the view's projection and binning.  A view's time is the
    slowest stripe, its pixel part extrapolated to a 1/P share of the view."""
    import multiprocessing as mp
    views = list(range(len(cams))) if views is None else list(views)
    P = procs or max(1, min(16, len(os.sched_getaffinity(0))))
    jobs = [(name, sh_f32, tile, forward_only, views, frac, seed, i, P) for i in range(P)]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(P) as pool:
        res = pool.map(_stripe_worker, jobs)
    wall = time.perf_counter() - t0
    per_view = {}
    for v in views:
        M = cams[v].width * cams[v].height
        per_view[v] = max(r[v][0] + r[v][1] * M / r[v][2] for r in res)
    total = _per_iteration(cams, per_view)
    res_s = [f"{cams[v].width}x{cams[v].height}" for v in views]
    return {"value": len(cams) / total, "unit": "views/s" if forward_only else "iters/s", "cores": P,
            "kind": "oracle",
            "sample": (f"FP64 oracle in {P} processes, one thread each, on views {views} ({', '.join(res_s)}): each "
                       f"process projects and bins the view in full and takes every {P}-th pixel of the same seeded "
                       f"{frac:.0%} sample; a view costs its slowest process with that process's pixel time "
                       f"extrapolated to 1/{P} of the view; {total:.1f} s per {len(cams)}-view iteration; "
                       f"{wall:.1f} s wall including each process drawing the scene")}


def run_train(args, torch, dev):
    """A training run with the paper's schedule on a synthetic scene (the held-out scene renders the targets).

    Untimed: the targets at every scale the scheduler visits, and `warmup` iterations after which the
    parameters and the optimiser are put back to their initial state.  Timed: the whole run."""
    from paper_2603_09277_amd.train import TrainConfig, Trainer
    W, H = (int(x) for x in args.train_res.split("x"))
    cfg = TrainConfig(n_gaussians=args.train_gaussians, width=W, height=H, iterations=args.train_iters,
                      tile=tuple(int(x) for x in (args.tile or "16x16").split("x")), lds=args.lds or 128,
                      regulariser=args.train_regulariser)
    tr = Trainer(cfg, dev)
    tr.prepare()
    p0 = tr.psnr()
    for it in range(min(args.warmup, cfg.iterations)):
        tr.step(it)
    tr.restart()
    res = tr.run(log_every=5000)
    p1 = tr.psnr()
    ls = tr.list_stats()
    ips = res["iters_per_s"]
    result = {
        "metric": METRIC_TRAIN, "value": round(ips, 3), "unit": "iters/s", "n_gpus": 1, "steps": cfg.iterations,
        "warmup": args.warmup, "ms_per_step": round(1e3 / ips, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"synthetic training, {cfg.n_gaussians} Gaussians, {cfg.n_views} views {W}x{H}, "
                               f"{cfg.iterations} iterations as 150 epochs",
                   "n_gaussians": cfg.n_gaussians, "views": cfg.n_views, "resolution": [W, H],
                   "iterations": cfg.iterations, "epoch_views": tr.epoch_views, "reset_every_epochs": cfg.reset_every,
                   "zeta": cfg.zeta, "gamma": cfg.gamma, "lambda": cfg.lam, "r_max": tr.r_max,
                   "regulariser": cfg.regulariser + (f" ({cfg.opacity_weight})" if cfg.regulariser == "opacity" else ""),
                   "tile": list(cfg.tile), "lds_batch": cfg.lds},
        "train_seconds": round(res["seconds"], 3),
        "seconds_per_30k_iters": round(30000.0 / ips, 2),
        "psnr_before": round(p0, 3), "psnr_after": round(p1, 3),
        "final_mean_list_len": round(ls["mean_list_len"], 2), "final_mean_entropy": round(ls["mean_entropy"], 4),
        "paper_context": "Tab. 1: 99.58 s for 30K iterations of the whole training, 3.3M Gaussians, Mip-NeRF 360, "
                         "one RTX 5090 D (not the same workload)",
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(result), flush=True)


METRIC_AUX = "auxiliary entry points: per-call time and HBM rate at 1 MI355X"


def run_aux(args, torch, dev):
    """Per-call time of the element-wise and image entry points around the rasterizer, at the
    training workload's sizes, with their algorithmic HBM bytes (read and written once)."""
    from paper_2603_09277_amd import gsr, scenes
    n = args.train_gaussians
    W, H = (int(x) for x in args.train_res.split("x"))
    scene = scenes.gmm_scene(9, n)
    t = {k: torch.from_numpy(np.ascontiguousarray(getattr(scene, k))).to(dev) for k in
         ("means", "scales", "quats", "opacities", "sh")}
    R = gsr.Rasterizer(max_views=1)
    cam = scenes.orbit_cameras(np.random.default_rng(10), [(W, H)])[0]
    opts = gsr.RasterOptions(tile=(16, 16), lds_batch=args.lds or 128, sh_degree=3)
    g = torch.Generator(device="cpu").manual_seed(11)
    sc = t["scales"].clone()
    lsc = torch.log(sc).contiguous()
    grad_o = torch.zeros(n, device=dev)
    loss1 = torch.zeros(1, device=dev)
    P = W * H
    img = torch.rand((P, 3), generator=g).to(dev)
    tgt = torch.rand((P, 3), generator=g).to(dev)
    grad_img = torch.zeros_like(img)
    lv = torch.zeros(1, device=dev)
    lv2 = torch.zeros(1, device=dev)
    # Adam over the 59 floats of every Gaussian, kinds as in training
    attrs = [(3, 0), (3, 1), (4, 0), (1, 2), (48, 0)]     # means, log-scales, quats, opacity logits, SH
    ad = []
    for width, kind in attrs:
        raw = torch.randn((n * width,), generator=g).to(dev)
        ad.append((raw, torch.zeros_like(raw), torch.zeros_like(raw), torch.empty_like(raw) if kind else None,
                   (torch.randn((n * width,), generator=g) * 1e-3).to(dev), kind))
    state = {"step": 0}

    def adam_all():
        state["step"] += 1
        for raw, m, v, act, gr, kind in ad:
            R.adam(raw, m, v, act, gr, kind, 1e-3, state["step"])

    ops = {
        "scale_reset": (lambda: R.scale_reset(sc, 1.0, lsc), n * 3 * 16),
        "opacity_loss": (lambda: R.opacity_loss(t["opacities"], 3.0, grad_o, loss1), n * 12),
        "adam": (adam_all, n * (59 * 28 + 4 * 4)),
        "dssim": (lambda: R.dssim([cam], img, tgt, 0.2, grad_img, lv), P * 3 * 16),
        "select_rmax": (lambda: R.select_rmax(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], cam, opts),
                        None),
    }
    res = {}
    for name, (fn, nbytes) in ops.items():
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        r = {"ms": round(ms, 4)}
        if nbytes:
            gbs = nbytes / (ms * 1e-3) / 1e9
            r.update({"algorithmic_bytes": nbytes, "GB_s": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 3)})
        res[name] = r
    R.close()
    print(json.dumps({"metric": METRIC_AUX, "unit": "ms per call", "n_gpus": 1, "data": "synthetic",
                      "config": {"workload": f"{n} Gaussians (Adam over 59 floats each), one {W}x{H} image",
                                 "gaussians": n, "resolution": [W, H]},
                      "ops": res}), flush=True)


KEYS = ("means", "scales", "quats", "opacities", "sh")


def upload(torch, dev, scene, bf16):
    t = {k: torch.from_numpy(np.ascontiguousarray(getattr(scene, k))).to(dev) for k in KEYS}
    if bf16:
        t["sh"] = t["sh"].to(torch.bfloat16).contiguous()
    return t


class Form:
    """One form of the step on a set of views: its own rasterizer context and options, and
    its launch groups (one per view in the plain form, one for all views in the batched form)."""

    def __init__(self, torch, gsr, t, cams, opts, per_view, target, forward_only=False):
        self.torch, self.gsr, self.t, self.cams, self.opts = torch, gsr, t, cams, opts
        self.forward_only = forward_only
        self.R = gsr.Rasterizer(max_views=len(cams))
        dev = t["means"].device
        off = [0]
        for c in cams:
            off.append(off[-1] + c.width * c.height)
        groups = [[v] for v in range(len(cams))] if per_view else [list(range(len(cams)))]
        self.work = []
        for gv in groups:
            p0, p1 = off[gv[0]], off[gv[-1] + 1]
            self.work.append(dict(views=gv, cams=[cams[v] for v in gv], target=target[p0:p1], out=None, rgb=None,
                                  grad_rgb=torch.empty((p1 - p0, 3), device=dev),
                                  loss=torch.empty(len(gv), device=dev),
                                  g_le=torch.full((len(gv),), GAMMA, device=dev)))
        self.grads = {k: torch.empty_like(v) for k, v in t.items()}

    def step(self):
        t, R, opts = self.t, self.R, self.opts
        for w in self.work:
            if self.forward_only:
                w["rgb"] = R.render_image(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], w["cams"],
                                          opts, rgb=w["rgb"])
                continue
            out = R.forward(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], w["cams"], opts, out=w["out"])
            w["out"] = out
            R.l1_loss(w["cams"], out["rgb"], w["target"], w["grad_rgb"], w["loss"])
            R.backward(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], w["cams"], opts, out,
                       w["grad_rgb"], None, w["g_le"], self.grads)

    def run(self, steps, warmup, timing=True, breakdown_steps=0):
        """Warm-up, then exactly `steps` timed steps bracketed by synchronisations.  Inside
        the timed region only the blend stages (the candidates for the dominant kernel)
        are bracketed by HIP events on the launch stream, plus one event pair per step;
        the full per-stage breakdown comes from extra steps afterwards."""
        torch, R = self.torch, self.R
        for _ in range(warmup):
            self.step()
        torch.cuda.synchronize()
        hot = ["blend_fwd"] if self.forward_only else ["blend_fwd", "blend_bwd"]
        if timing:
            R.stage_times(reset=True)
            R.set_timing(True, hot)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            ev[i][0].record()
            self.step()
            ev[i][1].record()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        res = {"sec": (t1 - t0) / steps, "step_ms": [a.elapsed_time(b) for a, b in ev], "hot": {}, "stages": {}}
        if timing:
            R.set_timing(False)
            res["hot"] = {k: v for k, v in R.stage_times(reset=True).items() if k in hot and v[1] > 0}
            if breakdown_steps:
                R.set_timing(True)
                for _ in range(breakdown_steps):
                    self.step()
                R.set_timing(False)
                res["stages"] = R.stage_times(reset=True)
        return res

    def stats(self):
        """Statistics summed over the launch groups (each forwarded once more, untimed)."""
        tile = self.opts.tile
        if len(self.work) == 1 and not self.forward_only:
            return self.R.stats(len(self.cams))
        t = self.t
        st = dict(pairs=0, evals_fwd=0, evals_bwd=0, blended=0, tested_fwd=0, tested_bwd=0, mean_len=0.0, p99_len=0,
                  overflow=False)
        n_t = 0
        for w in self.work:
            self.R.forward(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], w["cams"], self.opts)
            sv = self.R.stats(len(w["cams"]))
            nt = sum(((c.width + tile[0] - 1) // tile[0]) * ((c.height + tile[1] - 1) // tile[1]) for c in w["cams"])
            for k in ("pairs", "evals_fwd", "evals_bwd", "blended", "tested_fwd", "tested_bwd"):
                st[k] += sv[k]
            st["mean_len"] += sv["mean_len"] * nt
            n_t += nt
            st["p99_len"] = max(st["p99_len"], sv["p99_len"])   # the largest per-launch p99
            st["overflow"] = st["overflow"] or sv["overflow"]
        st["mean_len"] /= max(n_t, 1)
        return st

    def images(self):
        """Packed rgb [P, 3] of the latest step (host)."""
        key = "rgb" if self.forward_only else "out"
        parts = [(w["rgb"] if self.forward_only else w["out"]["rgb"]).cpu().numpy() for w in self.work if w[key] is not None]
        return np.concatenate(parts)

    def close(self):
        self.R.close()


def stage_report(res, st, n, V, sh_bytes, n_tiles, npix, launches, render=False):
    """Per-stage average launch time, algorithmic HBM rate and, for the blend stages,
    both operation models.  Stage times are per launch sequence."""
    stl = {k: st[k] / launches for k in ("pairs", "evals_fwd", "evals_bwd", "blended", "tested_fwd", "tested_bwd")}
    rep = {}
    for name, (ms, cnt) in list(res["stages"].items()) + list(res["hot"].items()):   # the timed region's last
        if cnt == 0:
            continue
        avg_s = ms / cnt / 1e3
        b = stage_bytes(name, n, V / launches, sh_bytes, stl["pairs"], n_tiles / launches, npix / launches)
        r = {"avg_ms": round(ms / cnt, 4), "hbm_GBs": round(b / avg_s / 1e9, 1) if b else None,
             "timed_region": name in res["hot"]}
        if name in ("blend_fwd", "blend_bwd"):
            r["method_TFLOPs"] = round(blend_ops_method(name, stl, render) / avg_s / 1e12, 3)
            r["post_cull_Tops"] = round(blend_ops_post_cull(name, stl, render) / avg_s / 1e12, 3)
            r["evals_G_per_s"] = round(stl["evals_fwd" if name == "blend_fwd" else "evals_bwd"] / avg_s / 1e9, 2)
        rep[name] = r
    return rep, stl


def roofline_of(res, rep, stl, traffic_key, render=False):
    """Roofline record of the dominant kernel of the timed region (the slower blend stage)."""
    if not res["hot"]:
        return None
    dom = max(res["hot"], key=lambda k: rep[k]["avg_ms"])
    avg_s = rep[dom]["avg_ms"] / 1e3
    traffic = None
    tf = os.path.join(ROOT, "profiles", f"{dom}_{traffic_key}_traffic.json")
    if os.path.exists(tf):
        with open(tf) as f:
            rec = json.load(f)
        src = os.path.join(ROOT, "paper_2603_09277_amd", "csrc", rec.get("source", ""))
        if os.path.exists(src) and source_hash(src) == rec.get("source_sha256_16"):
            traffic = rec.get("bytes_per_launch")
    ops = blend_ops_method(dom, stl, render)
    ach = ops / avg_s / 1e12
    pc = blend_ops_post_cull(dom, stl, render) / avg_s / 1e12
    return {"bound": "alu", "kernel": dom, "achieved": round(ach, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(ach / FP32_PEAK_TFLOPS, 4), "traffic": traffic,
            "work": (f"{OPS_EVAL_BWD} ops x evals_bwd" if dom == "blend_bwd" else
                     f"{OPS_EVAL_FWD} ops x evals_fwd" + ("" if render else f" + {OPS_BLENDED_FWD} x blended")),
            "ops_per_launch": int(ops), "avg_launch_ms": rep[dom]["avg_ms"],
            "post_cull": {"achieved": round(pc, 3), "peak": round(VALU_ISSUE_TOPS, 2), "unit": "T VALU op/s",
                          "frac": round(pc / VALU_ISSUE_TOPS, 4)},
            # measured HBM bytes (the traffic record) over this launch time, against 8 TB/s
            "traffic_GBs": round(traffic / avg_s / 1e9, 1) if traffic else None,
            "traffic_frac": round(traffic / avg_s / 1e9 / HBM_PEAK_GBS, 4) if traffic else None}


def image_errors(sampled, cams, imgs):
    """max |GPU - oracle| over the oracle's sampled, unflagged pixels, per form."""
    off = [0]
    for c in cams:
        off.append(off[-1] + c.width * c.height)
    out = {}
    for name, img in imgs.items():
        err = 0.0
        for v, (sel, ref, flags) in sampled.items():
            g = img[off[v]:off[v + 1]][sel]
            ok = flags == 0
            if ok.any():
                err = max(err, float(np.abs(g[ok] - ref[ok]).max()))
        out[name] = float(f"{err:.3g}")
    return out


def run_compare(args, torch, dev, gsr, scenes):
    """The metric's configuration: batched BF16-SH vs plain per-view FP32 on the same eight views."""
    scene, cams, meta = scenes.workload("batched", sh_f32=True)        # the FP32 draw; the batched form rounds it
    n, V = scene.n, len(cams)
    npix = sum(c.width * c.height for c in cams)
    t32 = upload(torch, dev, scene, False)
    t16 = dict(t32)
    t16["sh"] = torch.from_numpy(scenes.bf16_round(scene.sh)).to(dev).to(torch.bfloat16).contiguous()
    targets = [scenes.target_image(1000 + v, c.height, c.width) for v, c in enumerate(cams)]
    target = torch.from_numpy(np.concatenate([x.reshape(-1, 3) for x in targets])).to(dev).contiguous()

    tile = tuple(int(x) for x in args.tile.split("x")) if args.tile else (16, 16)
    ob = gsr.RasterOptions(tile=tile, lds_batch=args.lds or 128, sh_degree=3, sh_bf16=True,
                           flags=gsr.GSR_DEFAULT_FLAGS | (gsr.GSR_PERSISTENT if args.persistent else 0))
    tuned = False
    if not args.no_autotune and not args.tile:
        Rt = gsr.Rasterizer(max_views=V)
        cache = os.path.join(tempfile.gettempdir(), "gsr_autotune_cache.txt")
        ob = Rt.autotune(t16["means"], t16["scales"], t16["quats"], t16["opacities"], t16["sh"], cams, ob, cache)
        Rt.close()
        tuned = True
    ob_nosync = gsr.RasterOptions(tile=ob.tile, lds_batch=ob.lds_batch, sh_degree=3, sh_bf16=True,
                                  flags=ob.flags | gsr.GSR_NO_SYNC)
    ob_graph = gsr.RasterOptions(tile=ob.tile, lds_batch=ob.lds_batch, sh_degree=3, sh_bf16=True,
                                 flags=ob.flags | gsr.GSR_GRAPH)
    op = gsr.RasterOptions(tile=ob.tile, lds_batch=ob.lds_batch, sh_degree=3, sh_bf16=False,
                           flags=gsr.GSR_DEFAULT_FLAGS)

    fb = Form(torch, gsr, t16, cams, ob_nosync, False, target)
    rb = fb.run(args.steps, args.warmup, timing=not args.no_timing, breakdown_steps=args.breakdown_steps)
    st_b = fb.stats()
    img_b = fb.images()
    fb.close()
    fg = Form(torch, gsr, t16, cams, ob_graph, False, target)
    rg = fg.run(args.steps, args.warmup, timing=False)
    st_g = fg.stats()
    fg.close()
    fp = Form(torch, gsr, t32, cams, op, True, target)
    rp = fp.run(args.steps, args.warmup, timing=not args.no_timing, breakdown_steps=0)
    img_p = fp.images()
    st_p = fp.stats()
    fp.close()

    sh_b = 16 * 3 * 2
    n_tiles = sum(((c.width + ob.tile[0] - 1) // ob.tile[0]) * ((c.height + ob.tile[1] - 1) // ob.tile[1]) for c in cams)
    rep_b, stl_b = stage_report(rb, st_b, n, V, sh_b, n_tiles, npix, 1)
    rep_p, stl_p = stage_report(rp, st_p, n, V, 16 * 3 * 4, n_tiles, npix, V)
    roof = roofline_of(rb, rep_b, stl_b, "batched")
    vb, vg, vp = V / rb["sec"], V / rg["sec"], V / rp["sec"]

    def form_rec(r, st, views_s, mode, sh):
        d = {"views_per_s": round(views_s, 3), "ms_per_step": round(r["sec"] * 1e3, 4), "mode": mode,
             "sh_storage": sh, "pairs_per_s": round(st["pairs"] / r["sec"], 1), "overflow": bool(st["overflow"])}
        d.update(percentiles(r["step_ms"]))
        return d

    pers = "+persistent" if ob.flags & gsr.GSR_PERSISTENT else ""
    result = {
        "metric": METRIC, "value": round(vb, 3), "unit": "iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(rb["sec"] * 1e3, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOAD_NAMES["batched"] + "; batched BF16-SH vs plain per-view FP32",
                   "gaussians": n, "views": V, "resolutions": [f"{c.width}x{c.height}" for c in cams],
                   "tile": f"{ob.tile[0]}x{ob.tile[1]}", "lds_batch": ob.lds_batch, "autotuned": tuned,
                   "loss": "L1 + 0.015 L_E", "iteration": "one view through every stage, forward and backward"},
        "batched": form_rec(rb, st_b, vb, "one launch sequence, eager, fixed pair capacity (no host sync)" + pers,
                            "bf16"),
        "batched_graph": form_rec(rg, st_g, vg, "one launch sequence replayed from HIP graphs" + pers, "bf16"),
        "plain": form_rec(rp, st_p, vp, "one launch sequence per view, exact pair sizing", "f32"),
        "speedup_batched_vs_plain": round(vb / vp, 3),
        "speedup_batched_graph_vs_plain": round(vg / vp, 3),
        "pairs_per_s": round(st_b["pairs"] / rb["sec"], 1), "pairs": st_b["pairs"],
        "mean_list_len": round(st_b["mean_len"], 2), "p99_list_len": st_b["p99_len"],
        "evals_fwd": st_b["evals_fwd"], "evals_bwd": st_b["evals_bwd"], "blended": st_b["blended"],
        "tested_fwd": st_b["tested_fwd"], "tested_bwd": st_b["tested_bwd"],
        "stages": rep_b, "plain_stages": {k: v for k, v in rep_p.items() if v["timed_region"]},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        # one view of each resolution (views 0, 2, 5), at the forms' tile shape
        cb, sampled = cpu_baseline(scene, cams, ob.tile, targets, views=[0, 2, 5], frac=0.01)
        cb["processes"] = cpu_baseline_processes("batched", True, cams, ob.tile, views=[0, 2, 5], frac=0.01)
        result["cpu_baseline"] = cb
        result["image_err_vs_oracle"] = dict(
            image_errors(sampled, cams, {"batched_bf16_sh": img_b, "plain_f32_sh": img_p}),
            note="max |GPU - oracle| over the baseline's sampled pixels (flagged FP32/FP64 decision pixels "
                 "excluded); the oracle projects the FP32 SH draw, so the batched figure includes its BF16 rounding")
    print(json.dumps(result), flush=True)


def run_one(args, torch, dev, gsr, scenes):
    """One form of any workload."""
    tile = tuple(int(x) for x in args.tile.split("x")) if args.tile else (16, 16)
    scene, cams, meta = scenes.workload(args.workload)
    bf16 = args.bf16 or args.sh == "bf16" or (args.sh == "auto" and meta["sh_dtype"] == "bf16")
    n, V = scene.n, len(cams)
    npix = sum(c.width * c.height for c in cams)
    t = upload(torch, dev, scene, bf16)
    flags = (gsr.GSR_DEFAULT_FLAGS | (gsr.GSR_GRAPH if args.graph else 0) | (gsr.GSR_PERSISTENT if args.persistent else 0)
             | (gsr.GSR_NO_SYNC if args.no_sync else 0))
    opts = gsr.RasterOptions(tile=tile, lds_batch=args.lds or 128, sh_degree=scene.sh_degree, sh_bf16=bf16, flags=flags)
    targets_np = [scenes.target_image(1000 + v, c.height, c.width) for v, c in enumerate(cams)]
    target = torch.from_numpy(np.concatenate([x.reshape(-1, 3) for x in targets_np])).to(dev).contiguous()
    if args.autotune:
        Rt = gsr.Rasterizer(max_views=V)
        cache = os.path.join(tempfile.gettempdir(), "gsr_autotune_cache.txt")
        opts = Rt.autotune(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], cams, opts, cache)
        Rt.close()
        tile = opts.tile
    per_view = args.form == "plain"
    f = Form(torch, gsr, t, cams, opts, per_view, target, args.forward_only)
    timing = not args.no_timing and not args.graph
    r = f.run(args.steps, args.warmup, timing=timing, breakdown_steps=args.breakdown_steps)
    st = f.stats()
    f.close()
    sec = r["sec"]
    K = (scene.sh_degree + 1) ** 2
    sh_bytes = K * 3 * (2 if bf16 else 4)
    n_tiles = sum(((c.width + tile[0] - 1) // tile[0]) * ((c.height + tile[1] - 1) // tile[1]) for c in cams)
    launches = V if per_view else 1
    rep, stl = stage_report(r, st, n, V, sh_bytes, n_tiles, npix, launches, args.forward_only)
    roof = roofline_of(r, rep, stl, args.workload, args.forward_only)
    mode = (("forward-only " if args.forward_only else "") + ("per-view" if per_view else ("batched" if V > 1 else "single-view"))
            + ("+graph" if args.graph else "") + ("+no-sync" if args.no_sync and not args.graph else "")
            + ("+persistent" if opts.flags & gsr.GSR_PERSISTENT else "") + ("+autotuned" if args.autotune else ""))
    result = {
        "metric": METRIC_RENDER if args.forward_only else METRIC, "value": round(V / sec, 3),
        "unit": "views/s" if args.forward_only else "iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOAD_NAMES[args.workload], "gaussians": n, "views": V, "tile": f"{tile[0]}x{tile[1]}",
                   "lds_batch": opts.lds_batch, "sh_storage": "bf16" if bf16 else "f32", "mode": mode,
                   "loss": None if args.forward_only else "L1 + 0.015 L_E"},
        "pairs_per_s": round(st["pairs"] / sec, 1), "pairs": st["pairs"], "mean_list_len": round(st["mean_len"], 2),
        "p99_list_len": st["p99_len"], "evals_fwd": st["evals_fwd"], "evals_bwd": st["evals_bwd"],
        "blended": st["blended"], "tested_fwd": st["tested_fwd"], "tested_bwd": st["tested_bwd"],
        "overflow": st["overflow"], "stages": rep, "roofline": roof,
    }
    result.update(percentiles(r["step_ms"]))
    if not args.no_cpu_baseline:
        views = sorted({min(v for v, c2 in enumerate(cams) if (c2.width, c2.height) == (c.width, c.height))
                        for c in cams})
        frac = 0.5 if args.workload in ("tiny", "single") else 0.01
        result["cpu_baseline"], _ = cpu_baseline(scene, cams, tile, targets_np, args.forward_only, views=views,
                                                 frac=frac)
        result["cpu_baseline"]["processes"] = cpu_baseline_processes(args.workload, False, cams, tile,
                                                                     args.forward_only, views=views, frac=frac)
    print(json.dumps(result), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported by this build "
              "(the multi-GPU sharding over views is described in the design notes, not implemented)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2603_09277_amd import gsr, scenes

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes, "launches": 3}))
        return
    if args.train:
        run_train(args, torch, dev)
        return
    if args.aux:
        run_aux(args, torch, dev)
        return
    if args.form == "compare":
        run_compare(args, torch, dev, gsr, scenes)
    else:
        run_one(args, torch, dev, gsr, scenes)


if __name__ == "__main__":
    main()
