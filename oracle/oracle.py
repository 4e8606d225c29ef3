"""Python front end of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of bench.py.  The product path never imports it.

All arithmetic of the method lives in oracle.c; this module marshals arrays,
loops over views, and evaluates the test loss L = sum_v [L1_v + gamma L_E,v]
(Eq. 6 with lambda = 0, Eq. 11-12).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

DILATE, JAC_CLAMP, COLOR_CLAMP = 1, 2, 4
DEFAULT_FLAGS = DILATE | JAC_CLAMP | COLOR_CLAMP
NEAR_SKIP, NEAR_STOP, NEAR_CLAMP = 1, 2, 4

_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (strict IEEE double, no FMA contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-Wall", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        i64, i32, u32, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_uint, ctypes.c_double
        L.orc_sh_basis.argtypes = [i32, dbl, dbl, dbl, P, P]
        L.orc_project.argtypes = [i64, P, P, P, P, P, i32, P, u32, P, P, P, P, P, P, P]
        L.orc_count_pairs.argtypes = [i64, P, P, i32, i32, i32, i32, P, P]
        L.orc_count_pairs.restype = i64
        L.orc_bin.argtypes = [i64, P, P, P, i32, i32, i32, i32, i64, P, P]
        L.orc_render.argtypes = [i32, i32, i32, i32, i64, P, P, P, P, P, P, P, P, P, P, P, P, P, P, P]
        L.orc_render_bruteforce.argtypes = [i32, i32, i32, i32, i64, P, P, P, P, P, P, P, P, P, P, P]
        L.orc_backward_render.argtypes = [i32, i32, i32, i32, i64, P, P, P, P, P, P, P, P, P, P, P, P, P]
        L.orc_backward_project.argtypes = [i64, P, P, P, P, i32, P, u32, P, P, P, P, P, P, P]
        for f in ("orc_dH_dalpha_chain", "orc_dH_dalpha_alg1", "orc_dH_dalpha_cancelled"):
            getattr(L, f).argtypes = [i32, P, P]
        L.orc_entropy_of_alphas.argtypes = [i32, P]
        L.orc_entropy_of_alphas.restype = dbl
        L.orc_opacity_loss.argtypes = [i64, P, dbl, P]
        L.orc_opacity_loss.restype = dbl
        L.orc_scale_reset.argtypes = [i64, P, dbl]
        L.orc_ssim.argtypes = [i32, i32, P, P, P]
        L.orc_ssim.restype = dbl
        L.orc_adam_step.argtypes = [i64, P, P, P, P, P, i32, dbl, dbl, dbl, dbl, i64]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, np.float32)


def _f64(a):
    return np.ascontiguousarray(a, np.float64)


# --------------------------------------------------------------------------- #
# Building blocks
# --------------------------------------------------------------------------- #

def sh_basis(deg: int, d: Sequence[float]):
    K = (deg + 1) ** 2
    Y = np.zeros(K)
    dY = np.zeros((K, 3))
    lib().orc_sh_basis(deg, float(d[0]), float(d[1]), float(d[2]), _p(Y), _p(dY))
    return Y, dY


def project(scene, cam, flags: int = DEFAULT_FLAGS) -> Dict[str, np.ndarray]:
    n = scene.n
    out = dict(mean2d=np.zeros((n, 2)), conic=np.zeros((n, 3)), cov2d=np.zeros((n, 3)),
               depth=np.zeros(n), radius=np.zeros(n, np.int32), rgb=np.zeros((n, 3)),
               mask=np.zeros(n, np.uint8))
    keep = [_f32(scene.means), _f32(scene.scales), _f32(scene.quats), _f32(scene.opacities), _f32(scene.sh)]
    camv = _f64(cam.as_array())
    lib().orc_project(n, *[_p(a) for a in keep], scene.sh_degree, _p(camv), flags,
                      _p(out["mean2d"]), _p(out["conic"]), _p(out["cov2d"]), _p(out["depth"]),
                      _p(out["radius"]), _p(out["rgb"]), _p(out["mask"]))
    out["opacity"] = scene.opacities.astype(np.float64)
    out["depth32"] = out["depth"].astype(np.float32)
    return out


def opacity_loss(opacities, weight):
    """(L_O, dL_O/dsigma) of the opacity regulariser, FP64."""
    op = _f32(opacities)
    g = np.zeros(len(op))
    L = lib().orc_opacity_loss(len(op), _p(op), float(weight), _p(g))
    return float(L), g


def scale_reset(scales, zeta):
    """s <- zeta * s (Eq. 7) with zeta a float32 value (as every parameter at the
    library's boundary), float32 result."""
    s = np.array(scales, np.float32, copy=True, order="C")
    lib().orc_scale_reset(len(s), _p(s), float(np.float32(zeta)))
    return s


def ssim(x, y, grad: bool = True):
    """(SSIM, dSSIM/dx) of two [H, W, 3] images (FP64, 11x11 Gaussian window)."""
    x = _f64(x)
    y = _f64(y)
    H, W = x.shape[:2]
    g = np.zeros_like(x) if grad else None
    s = lib().orc_ssim(W, H, _p(x), _p(y), None if g is None else _p(g))
    return float(s), g


def adam_step(raw, m, v, grad_act, kind, lr, t, b1=0.9, b2=0.999, eps=1e-15):
    """One Adam step on float64 copies: returns (raw, m, v, activated)."""
    raw, m, v = (np.array(a, np.float64, copy=True) for a in (raw, m, v))
    act = np.zeros_like(raw)
    ga = _f64(grad_act)
    lib().orc_adam_step(raw.size, _p(raw), _p(m), _p(v), _p(act), _p(ga), int(kind), float(lr), float(b1), float(b2),
                        float(eps), int(t))
    return raw, m, v, act


def scaled_camera(cam, r):
    """The camera at downsampling factor r: width and height divided by r and rounded
    down (at least 1), intrinsics divided by r, pose unchanged."""
    from paper_2603_09277_amd.scenes import Camera
    r = max(1, int(r))
    f32 = lambda x: float(np.float32(np.float32(x) / np.float32(r)))
    return Camera(max(1, cam.width // r), max(1, cam.height // r), f32(cam.fx), f32(cam.fy), f32(cam.cx),
                  f32(cam.cy), np.asarray(cam.R, np.float32), np.asarray(cam.t, np.float32), cam.near)


def select_rmax(scene, cam, tile=(16, 16), r_cap=4, max_mean_len=150.0, flags: int = DEFAULT_FLAGS):
    """Resolution-scheduler r_max: the largest r <= r_cap whose scaled camera keeps the mean
    per-tile list length (pairs / tiles) <= max_mean_len, else 1; also the pair counts."""
    tw, th = tile
    best, counts = 1, []
    for r in range(1, r_cap + 1):
        k = scaled_camera(cam, r)
        pr = project(scene, k, flags)
        total, _, _ = count_pairs(pr["mean2d"], pr["radius"], k.width, k.height, tw, th)
        tiles = ((k.width + tw - 1) // tw) * ((k.height + th - 1) // th)
        counts.append(total)
        if total / tiles <= max_mean_len:
            best = r
    return best, counts


def count_pairs(mean2d, radius, W, H, tw, th):
    n = len(radius)
    tt = np.zeros(n, np.int32)
    rects = np.zeros((n, 4), np.int32)
    m2 = _f64(mean2d)
    r = np.ascontiguousarray(radius, np.int32)
    total = lib().orc_count_pairs(n, _p(m2), _p(r), W, H, tw, th, _p(tt), _p(rects))
    return int(total), tt, rects


def bin_lists(mean2d, radius, depth32, W, H, tw, th):
    """Sorted per-tile lists: (values[P] int32, ranges[n_tiles, 2] int32)."""
    total, _, _ = count_pairs(mean2d, radius, W, H, tw, th)
    gx, gy = (W + tw - 1) // tw, (H + th - 1) // th
    values = np.zeros(max(total, 1), np.int32)
    ranges = np.zeros((gx * gy, 2), np.int32)
    m2 = _f64(mean2d)
    r = np.ascontiguousarray(radius, np.int32)
    d = _f32(depth32)
    rc = lib().orc_bin(len(r), _p(m2), _p(r), _p(d), W, H, tw, th, max(total, 1), _p(values), _p(ranges))
    if rc != 0:
        raise RuntimeError(f"orc_bin failed ({rc})")
    return values[:total], ranges


def render(W, H, tw, th, mean2d, conic, opac, rgb, ranges, values, pix=None):
    n = len(opac)
    m2, cn, op, cl = _f64(mean2d), _f64(conic), _f64(opac), _f64(rgb)
    rg, vl = np.ascontiguousarray(ranges, np.int32), np.ascontiguousarray(values, np.int32)
    if vl.size == 0:
        vl = np.zeros(1, np.int32)
    out = dict(rgb=np.zeros((H, W, 3)), H=np.zeros((H, W)), T=np.zeros((H, W)),
               ncontrib=np.zeros((H, W), np.int32), flags=np.zeros((H, W), np.uint8))
    pm = None if pix is None else np.ascontiguousarray(pix, np.uint8)
    ev = ctypes.c_int64(0)
    nb = ctypes.c_int64(0)
    sig = ctypes.c_uint64(0)
    lib().orc_render(W, H, tw, th, n, _p(m2), _p(cn), _p(op), _p(cl), _p(rg), _p(vl),
                     None if pm is None else _p(pm), _p(out["rgb"]), _p(out["H"]), _p(out["T"]),
                     _p(out["ncontrib"]), _p(out["flags"]), ctypes.byref(ev), ctypes.byref(nb), ctypes.byref(sig))
    out["n_eval"] = int(ev.value)
    out["n_blend"] = int(nb.value)
    out["sig"] = int(sig.value)
    return out


def render_bruteforce(W, H, tw, th, mean2d, conic, opac, rgb, radius, depth32):
    n = len(opac)
    args = [_f64(mean2d), _f64(conic), _f64(opac), _f64(rgb), np.ascontiguousarray(radius, np.int32), _f32(depth32)]
    out = dict(rgb=np.zeros((H, W, 3)), H=np.zeros((H, W)), T=np.zeros((H, W)),
               ncontrib=np.zeros((H, W), np.int32), flags=np.zeros((H, W), np.uint8))
    lib().orc_render_bruteforce(W, H, tw, th, n, *[_p(a) for a in args], _p(out["rgb"]), _p(out["H"]),
                                _p(out["T"]), _p(out["ncontrib"]), _p(out["flags"]))
    return out


def backward_render(W, H, tw, th, mean2d, conic, opac, rgb, ranges, values, grad_rgb, grad_H, pix=None):
    n = len(opac)
    g = dict(mean2d=np.zeros((n, 2)), conic=np.zeros((n, 3)), opacity=np.zeros(n), rgb=np.zeros((n, 3)))
    m2, cn, op, cl = _f64(mean2d), _f64(conic), _f64(opac), _f64(rgb)
    rg, vl = np.ascontiguousarray(ranges, np.int32), np.ascontiguousarray(values, np.int32)
    if vl.size == 0:
        vl = np.zeros(1, np.int32)
    gr = _f64(grad_rgb)
    gh = None if grad_H is None else _f64(grad_H)
    pm = None if pix is None else np.ascontiguousarray(pix, np.uint8)
    rc = lib().orc_backward_render(W, H, tw, th, n, _p(m2), _p(cn), _p(op), _p(cl), _p(rg), _p(vl),
                                   None if pm is None else _p(pm), _p(gr), None if gh is None else _p(gh),
                                   _p(g["mean2d"]), _p(g["conic"]), _p(g["opacity"]), _p(g["rgb"]))
    if rc != 0:
        raise RuntimeError("orc_backward_render failed")
    return g


def backward_project(scene, cam, g2d, flags: int = DEFAULT_FLAGS, acc=None):
    n = scene.n
    K = (scene.sh_degree + 1) ** 2
    if acc is None:
        acc = dict(means=np.zeros((n, 3)), scales=np.zeros((n, 3)), quats=np.zeros((n, 4)),
                   opacities=np.zeros(n), sh=np.zeros((n, K, 3)))
    keep = [_f32(scene.means), _f32(scene.scales), _f32(scene.quats), _f32(scene.sh)]
    camv = _f64(cam.as_array())
    gm, gc, gr = _f64(g2d["mean2d"]), _f64(g2d["conic"]), _f64(g2d["rgb"])
    lib().orc_backward_project(n, *[_p(a) for a in keep], scene.sh_degree, _p(camv), flags,
                               _p(gm), _p(gc), _p(gr), _p(acc["means"]), _p(acc["scales"]),
                               _p(acc["quats"]), _p(acc["sh"]))
    acc["opacities"] += g2d["opacity"]
    return acc


def dH_dalpha(alphas, method: str = "alg1"):
    a = _f64(alphas)
    out = np.zeros(len(a))
    getattr(lib(), f"orc_dH_dalpha_{method}")(len(a), _p(a), _p(out))
    return out


def entropy_of_alphas(alphas) -> float:
    a = _f64(alphas)
    return float(lib().orc_entropy_of_alphas(len(a), _p(a)))


# --------------------------------------------------------------------------- #
# Whole forward / loss / backward, one view at a time
# --------------------------------------------------------------------------- #

def forward_view(scene, cam, tile=(16, 16), flags: int = DEFAULT_FLAGS, pix=None, proj=None):
    """Project, bin and render one view entirely in FP64 (or on a supplied
    projection ``proj``, e.g. the GPU's float32 records)."""
    tw, th = tile
    pr = project(scene, cam, flags) if proj is None else proj
    values, ranges = bin_lists(pr["mean2d"], pr["radius"], pr["depth32"], cam.width, cam.height, tw, th)
    img = render(cam.width, cam.height, tw, th, pr["mean2d"], pr["conic"], pr["opacity"], pr["rgb"],
                 ranges, values, pix)
    img["values"], img["ranges"], img["proj"] = values, ranges, pr
    M = cam.width * cam.height
    img["L_E"] = float(img["H"].sum() / M) if pix is None else float("nan")
    return img


def l1_grad(img, target):
    """dL1/dC for L1 = mean over 3M of |C - target|; sign(0) = 0 (Eq. 6)."""
    diff = img - target.astype(np.float64)
    return np.sign(diff) / diff.size


def loss_and_grads(scene, cams, targets, gamma: float = 0.015, tile=(16, 16), flags: int = DEFAULT_FLAGS):
    """L = sum_v [L1_v + gamma * L_E,v] and dL/d(parameters) in FP64."""
    L = 0.0
    acc = None
    views = []
    for cam, tgt in zip(cams, targets):
        f = forward_view(scene, cam, tile, flags)
        M = cam.width * cam.height
        L += float(np.abs(f["rgb"] - tgt.astype(np.float64)).mean()) + gamma * f["L_E"]
        g_rgb = l1_grad(f["rgb"], tgt)
        g_H = np.full((cam.height, cam.width), gamma / M)
        pr = f["proj"]
        g2 = backward_render(cam.width, cam.height, tile[0], tile[1], pr["mean2d"], pr["conic"], pr["opacity"],
                             pr["rgb"], f["ranges"], f["values"], g_rgb, g_H)
        acc = backward_project(scene, cam, g2, flags, acc)
        views.append(f)
    return L, acc, views


def signature(scene, cams, tile=(16, 16), flags: int = DEFAULT_FLAGS):
    """Hash of every discrete decision of the forward (lists, skips, stops,
    clamps, tile rects, colour and Jacobian clamps)."""
    h = []
    for cam in cams:
        f = forward_view(scene, cam, tile, flags)
        pr = f["proj"]
        h.append((f["sig"], hash(pr["mask"].tobytes()), hash(pr["radius"].tobytes()),
                  hash(f["values"].tobytes()), hash(f["ranges"].tobytes())))
    return tuple(h)
