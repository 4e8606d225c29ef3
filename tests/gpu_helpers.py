"""Shared helpers of the GPU parity tests: run the HIP path through the C-ABI
binding and the FP64 oracle on the same seeded inputs, and compare."""
from __future__ import annotations

import numpy as np
import torch

from oracle import oracle as orc
from paper_2603_09277_amd import gsr, scenes

DEV = torch.device("cuda:0")
LOG2E = 1.4426950408889634
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
    # the library stores the conic pre-scaled to log2 units
    unscale = np.array([-2.0 / LOG2E, -1.0 / LOG2E, -2.0 / LOG2E])
    for v in range(n_views):
        r = rec[v]
        views.append(dict(mean2d=r[:, 0:2].astype(np.float64), conic=r[:, 2:5].astype(np.float64) * unscale,
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


def oracle_grads(scene, cams, targets, gamma, tile, gpu_rgb=None, ambiguous=1e-5, flags=orc.DEFAULT_FLAGS):
    """FP64 oracle gradient of L = sum_v [L1_v + gamma L_E,v].

    L1 has a kink at C = target.  Where |C_oracle - target| <= `ambiguous`
    (below the FP32 image tolerance) either sign is a correct reading, so the
    oracle takes the GPU's sign there (`gpu_rgb`, packed [P, 3]); everywhere
    else the two sign patterns must agree, which is asserted."""
    acc = None
    L = 0.0
    off = 0
    for cam, tgt in zip(cams, targets):
        f = orc.forward_view(scene, cam, tile, flags)
        M = cam.width * cam.height
        diff = f["rgb"] - tgt.astype(np.float64)
        sign = np.sign(diff)
        if gpu_rgb is not None:
            g_img = np.asarray(gpu_rgb[off:off + M], np.float64).reshape(cam.height, cam.width, 3)
            gs = np.sign(g_img - tgt.astype(np.float64))
            amb = np.abs(diff) <= ambiguous
            assert np.all((sign == gs) | amb), "L1 sign disagreement outside the ambiguity band"
            sign = np.where(amb, gs, sign)
        L += float(np.abs(diff).mean()) + gamma * f["L_E"]
        pr = f["proj"]
        g2 = orc.backward_render(cam.width, cam.height, tile[0], tile[1], pr["mean2d"], pr["conic"],
                                 pr["opacity"], pr["rgb"], f["ranges"], f["values"], sign / diff.size,
                                 np.full((cam.height, cam.width), gamma / M))
        acc = orc.backward_project(scene, cam, g2, flags, acc)
        off += M
    return L, acc


GRAD_TOL = 1e-3       # relative gradient tolerance
GRAD_FLOOR = 1e-5     # element-wise floor, as a fraction of the tensor's largest |g*|


def check_grad(g, ref, name="", tol=GRAD_TOL, floor=GRAD_FLOOR, mask=None):
    """The gradient tolerance for FP32 gradients, per tensor and per element:
    ||g - g*||_2 <= tol ||g*||_2 and |g - g*| <= tol |g*| + floor max|g*| for every
    element (of the rows selected by `mask`, a boolean over the first axis, when given;
    the L2 check always covers the whole tensor)."""
    g = np.asarray(g, np.float64)
    ref = np.asarray(ref, np.float64)
    assert g.shape == ref.shape, (name, g.shape, ref.shape)
    rn = rel_norm(g, ref)
    assert rn <= tol, (name, "relative L2 error", rn)
    if ref.size == 0:
        return rn
    scale = float(np.abs(ref).max())
    gs, rs = (g, ref) if mask is None else (g[mask], ref[mask])
    err = np.abs(gs - rs)
    bound = tol * np.abs(rs) + floor * scale
    bad = np.flatnonzero((err > bound).reshape(-1))
    if bad.size:
        worst = bad[np.argsort(-(err.reshape(-1)[bad] / np.maximum(bound.reshape(-1)[bad], 1e-300)))[:5]]
        raise AssertionError((name, f"{bad.size} of {err.size} elements beyond tol |g*| + floor max|g*|",
                              [(int(i), float(gs.reshape(-1)[i]), float(rs.reshape(-1)[i])) for i in worst]))
    return rn


def check_grad2d(g2g, g2o, tol=GRAD_TOL, floor=GRAD_FLOOR):
    """The blend backward's per-Gaussian 2D gradients (BUF_GRAD2D rows) against the
    oracle's, component group by component group."""
    check_grad(g2g[:, 0:2], g2o["mean2d"], "mean2d", tol, floor)
    check_grad(g2g[:, 2:5], g2o["conic"], "conic", tol, floor)
    check_grad(g2g[:, 5], g2o["opacity"], "opacity", tol, floor)
    check_grad(g2g[:, 6:9], g2o["rgb"], "rgb", tol, floor)
