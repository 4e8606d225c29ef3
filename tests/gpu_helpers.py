"""Shared helpers of the GPU parity tests: run the HIP path through the C-ABI
binding and the FP64 oracle on the same seeded inputs, and compare."""
from __future__ import annotations

import numpy as np
import torch

from oracle import oracle as orc
from paper_2603_09277_amd import gsr, scenes

DEV = torch.device("cuda:0")
KEYS = ("means", "scales", "quats", "opacities", "sh")


def to_dev(scene: scenes.Scene, bf16: bool = False):
    out = {}
    for k in KEYS:
        a = torch.from_numpy(np.ascontiguousarray(getattr(scene, k))).to(DEV)
        if k == "sh" and bf16:
            a = a.to(torch.bfloat16)
        out[k] = a.contiguous()
    return out


def gpu_forward(R: gsr.Rasterizer, t: dict, cams, opts: gsr.RasterOptions):
    out = R.forward(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], cams, opts)
    torch.cuda.synchronize()
    return out


def gpu_backward(R, t, cams, opts, saved, grad_rgb, grad_H=None, grad_LE=None):
    g = R.backward(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], cams, opts, saved,
                   grad_rgb, grad_H, grad_LE)
    torch.cuda.synchronize()
    return {k: v.float().cpu().numpy().astype(np.float64) for k, v in g.items()}


def gpu_records(R: gsr.Rasterizer, n: int, n_views: int):
    """The GPU's float32 projection per view, in the oracle's dict layout."""
    rec = R.inspect(gsr.BUF_RECORDS).reshape(n_views, n, 12)
    rad = R.inspect(gsr.BUF_RADIUS).reshape(n_views, n)
    dep = R.inspect(gsr.BUF_DEPTH).reshape(n_views, n)
    views = []
    for v in range(n_views):
        r = rec[v]
        views.append(dict(mean2d=r[:, 0:2].astype(np.float64), conic=r[:, 2:5].astype(np.float64),
                          opacity=r[:, 5].astype(np.float64), rgb=r[:, 6:9].astype(np.float64),
                          radius=rad[v].copy(), depth32=dep[v].astype(np.float32),
                          mean2d_f32=r[:, 0:2].copy()))
    return views


def split_pixels(arr: np.ndarray, cams, v: int):
    off = gsr.pixel_offsets(cams)
    c = cams[v]
    return arr[off[v]:off[v + 1]].reshape((c.height, c.width) + arr.shape[1:])


def rel_norm(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def oracle_stagewise(pr_gpu: dict, cam, tile, pix=None):
    """Oracle binning + blend on the GPU's own float32 records (reading R1)."""
    W, H = cam.width, cam.height
    vals, ranges = orc.bin_lists(pr_gpu["mean2d"], pr_gpu["radius"], pr_gpu["depth32"], W, H, tile[0], tile[1])
    img = orc.render(W, H, tile[0], tile[1], pr_gpu["mean2d"], pr_gpu["conic"], pr_gpu["opacity"], pr_gpu["rgb"],
                     ranges, vals, pix)
    img["values"], img["ranges"] = vals, ranges
    return img
