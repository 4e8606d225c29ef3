#!/usr/bin/env python3
"""Error of every output of the HIP path against the FP64 oracle, per workload.

Run on a GPU machine from the repository root:  python tests/error_report.py [names]
Prints one JSON line per workload.  Test infrastructure: it calls the oracle.

For each workload the GPU renders all views in one launch; on a seeded sample of
pixels per view (every pixel for the tiny scene) it reports, over the pixels
whose skip/stop decisions are not within the oracle's decision band:

  stagewise   the oracle blending the GPU's float32 records (isolates the blend)
  end_to_end  the oracle's own FP64 projection of the parameters (for BF16 SH
              the oracle uses the FP32 draw, so the BF16 storage error shows)

and the relative L2 error of every parameter gradient of the loss
L1 + 0.015 * mean entropy restricted to the sampled pixels, against the oracle
backward (blend on the GPU's records, FP64 projection backward).
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

from oracle import oracle as orc                      # noqa: E402
from paper_2603_09277_amd import gsr, scenes          # noqa: E402
from gpu_helpers import DEV, KEYS, gpu_records, oracle_stagewise, rel_norm, to_dev   # noqa: E402

GAMMA = 0.015
SAMPLES = 2000


def report(name, tile=(16, 16), lds=64, flags=gsr.GSR_DEFAULT_FLAGS):
    scene, cams, meta = scenes.workload(name)
    bf16 = meta["sh_dtype"] == "bf16"
    scene_f32 = None
    if bf16:                                    # the FP32 draw the BF16 storage rounds
        scene_f32 = scenes.workload(name, sh_f32=True)[0]
    R = gsr.Rasterizer(max_views=len(cams))
    t = to_dev(scene, bf16=bf16)
    opts = gsr.RasterOptions(tile=tile, lds_batch=lds, sh_degree=scene.sh_degree, sh_bf16=bf16, flags=flags)
    out = R.forward(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], cams, opts)
    torch.cuda.synchronize()
    recs = gpu_records(R, scene.n, len(cams))
    off = gsr.pixel_offsets(cams)
    rng = np.random.default_rng(77)
    rgb = out["rgb"].cpu().numpy()
    H = out["entropy"].cpu().numpy()
    T = out["t_final"].cpu().numpy()
    g_rgb = np.zeros_like(rgb, dtype=np.float64)
    g_H = np.zeros(len(H))
    err = dict(stagewise=dict(rgb=0.0, H=0.0, T=0.0), end_to_end=dict(rgb=0.0, H=0.0, T=0.0))
    nflag = nchk = 0
    sel_all, imgs = [], []
    for v, cam in enumerate(cams):
        M = cam.width * cam.height
        s = np.arange(M) if M <= SAMPLES * 10 else np.sort(rng.choice(M, SAMPLES, replace=False))
        pix = np.zeros(M, np.uint8)
        pix[s] = 1
        pix = pix.reshape(cam.height, cam.width)
        o0 = off[v]
        st = oracle_stagewise(recs[v], cam, tile, pix)
        e2e = orc.forward_view(scene_f32 if bf16 else scene, cam, tile, pix=pix)
        for key, img in (("stagewise", st), ("end_to_end", e2e)):
            ok = img["flags"].reshape(-1)[s] == 0
            if key == "stagewise":
                nflag += int((~ok).sum())
                nchk += int(ok.sum())
            err[key]["rgb"] = max(err[key]["rgb"], float(np.abs(rgb[o0 + s] - img["rgb"].reshape(-1, 3)[s])[ok].max()))
            err[key]["H"] = max(err[key]["H"], float(np.abs(H[o0 + s] - img["H"].reshape(-1)[s])[ok].max()))
            err[key]["T"] = max(err[key]["T"], float(np.abs(T[o0 + s] - img["T"].reshape(-1)[s])[ok].max()))
        sel_all.append(o0 + s)
        imgs.append((s, pix, st))
    sel = np.concatenate(sel_all)
    tgt = np.concatenate([scenes.target_image(900 + v, c.height, c.width).reshape(-1, 3) for v, c in enumerate(cams)])
    g_rgb[sel] = np.sign(rgb[sel] - tgt[sel]) / (3 * len(sel))
    g_H[sel] = GAMMA / len(sel)
    g = R.backward(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], cams, opts, out,
                   torch.from_numpy(g_rgb.astype(np.float32)).to(DEV), torch.from_numpy(g_H.astype(np.float32)).to(DEV),
                   None)
    torch.cuda.synchronize()
    g = {k: v.float().cpu().numpy().astype(np.float64) for k, v in g.items()}
    acc = None
    for v, (cam, (s, pix, st)) in enumerate(zip(cams, imgs)):
        M = cam.width * cam.height
        o0 = off[v]
        pg = recs[v]
        g2 = orc.backward_render(cam.width, cam.height, tile[0], tile[1], pg["mean2d"], pg["conic"], pg["opacity"],
                                 pg["rgb"], st["ranges"], st["values"], g_rgb[o0:o0 + M].reshape(cam.height, cam.width, 3),
                                 g_H[o0:o0 + M].reshape(cam.height, cam.width), pix)
        acc = orc.backward_project(scene, cam, g2, orc.DEFAULT_FLAGS, acc)
    R.close()
    grads = {k: rel_norm(g[k], acc[k]) for k in KEYS}
    return dict(workload=name, views=len(cams), gaussians=scene.n, tile=f"{tile[0]}x{tile[1]}", sh=meta["sh_dtype"],
                pixels_checked=nchk, pixels_flagged=nflag, image_max_abs=err,
                grad_rel_l2=grads, loss="L1 + 0.015 mean H over the sampled pixels")


CONFIGS = {
    "tiny": dict(),
    "single": dict(),
    "sweep": dict(),
    "sweep_half": dict(),
    "batched": dict(lds=256, flags=gsr.GSR_DEFAULT_FLAGS | gsr.GSR_PERSISTENT),
    "diff": dict(lds=128, flags=gsr.GSR_DEFAULT_FLAGS | gsr.GSR_PERSISTENT),
}

if __name__ == "__main__":
    names = sys.argv[1:] or list(CONFIGS)
    for nm in names:
        print(json.dumps(report(nm, **CONFIGS[nm])), flush=True)
