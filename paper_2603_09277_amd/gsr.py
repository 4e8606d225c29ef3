"""Python binding of libgsr.so (include/gsr.h): argument marshalling only.

Every step of the rasterizer runs in the HIP library; PyTorch supplies device
memory and the current stream.  If the library has not been built, importing
works but every call raises: there is no CPU or PyTorch fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import List, Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsr.so")

GSR_DILATE, GSR_JACOBIAN_CLAMP, GSR_COLOR_CLAMP, GSR_GRAPH, GSR_PERSISTENT, GSR_NO_SYNC = 1, 2, 4, 8, 16, 32
GSR_DEBUG_INVARIANTS = 64
GSR_DEFAULT_FLAGS = GSR_DILATE | GSR_JACOBIAN_CLAMP | GSR_COLOR_CLAMP

BUF_RECORDS, BUF_RADIUS, BUF_DEPTH, BUF_TILES_TOUCHED, BUF_PAIR_VALUES, BUF_PAIR_TILES, BUF_RANGES, BUF_GRAD2D = range(8)

STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported", 3: "pair capacity exceeded", 4: "HIP runtime error",
          5: "stale frame", 6: "out of device memory"}


class GsrError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("near_z", ctypes.c_float)]


class Opts(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("lds_batch", ctypes.c_int32),
                ("sh_degree", ctypes.c_int32), ("sh_dtype", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class Gaussians(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("means", ctypes.c_void_p), ("scales", ctypes.c_void_p),
                ("quats", ctypes.c_void_p), ("opacities", ctypes.c_void_p), ("sh", ctypes.c_void_p)]


class FwdOut(ctypes.Structure):
    _fields_ = [("rgb", ctypes.c_void_p), ("entropy", ctypes.c_void_p), ("t_final", ctypes.c_void_p),
                ("n_contrib", ctypes.c_void_p), ("entropy_mean", ctypes.c_void_p), ("frame_id", ctypes.c_int64)]


class FrameStats(ctypes.Structure):
    _fields_ = [("pairs", ctypes.c_int64), ("mean_len", ctypes.c_double), ("p99_len", ctypes.c_int32),
                ("overflow", ctypes.c_int32), ("evals_fwd", ctypes.c_int64), ("evals_bwd", ctypes.c_int64),
                ("blended", ctypes.c_int64), ("tested_fwd", ctypes.c_int64), ("tested_bwd", ctypes.c_int64),
                ("invariant_max_err", ctypes.c_double), ("invariant_violations", ctypes.c_int64)]


STAGES = ["project", "depth_sort", "scan", "duplicate", "tile_sort", "ranges", "blend_fwd", "entropy_mean",
          "blend_bwd", "project_bwd", "grad_reduce"]


class Grads(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("scales", ctypes.c_void_p), ("quats", ctypes.c_void_p),
                ("opacities", ctypes.c_void_p), ("sh", ctypes.c_void_p)]


EXPORTED = ["gsr_status_string", "gsr_last_error", "gsr_create", "gsr_destroy", "gsr_pixel_offsets",
            "gsr_forward", "gsr_render", "gsr_backward", "gsr_stats", "gsr_autotune", "gsr_inspect", "gsr_set_timing",
            "gsr_opacity_loss", "gsr_scale_reset", "gsr_pair_counts", "gsr_scaled_camera", "gsr_select_rmax",
            "gsr_dssim", "gsr_adam", "gsr_base_loss",
            "gsr_stage_times", "gsr_l1_loss", "gsr_l1_loss_noalloc", "gsr_backward_opacity_reg"]

_lib = None


def lib():
    """Load libgsr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(python -m paper_2603_09277_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
        L.gsr_status_string.argtypes = [ctypes.c_int]
        L.gsr_status_string.restype = ctypes.c_char_p
        L.gsr_last_error.argtypes = [P]
        L.gsr_last_error.restype = ctypes.c_char_p
        L.gsr_create.argtypes = [ctypes.POINTER(P), i32, i64]
        L.gsr_destroy.argtypes = [P]
        L.gsr_pixel_offsets.argtypes = [P, i32, P]
        L.gsr_forward.argtypes = [P, P, ctypes.POINTER(Gaussians), P, i32, ctypes.POINTER(Opts),
                                  ctypes.POINTER(FwdOut)]
        L.gsr_render.argtypes = [P, P, ctypes.POINTER(Gaussians), P, i32, ctypes.POINTER(Opts), P]
        L.gsr_backward.argtypes = [P, P, ctypes.POINTER(Gaussians), P, i32, ctypes.POINTER(Opts),
                                   ctypes.POINTER(FwdOut), P, P, P, ctypes.POINTER(Grads)]
        L.gsr_stats.argtypes = [P, P, P, ctypes.POINTER(FrameStats)]
        L.gsr_backward_opacity_reg.argtypes = [P, P, ctypes.POINTER(Gaussians), P, i32, ctypes.POINTER(Opts),
                                               ctypes.POINTER(FwdOut), P, P, P, ctypes.c_float, P,
                                               ctypes.POINTER(Grads)]
        L.gsr_set_timing.argtypes = [P, i32]
        L.gsr_l1_loss.argtypes = [P, P, P, i32, P, P, P, P]
        L.gsr_l1_loss_noalloc.argtypes = [P, P, P, i32, P, P, P, P]
        L.gsr_stage_times.argtypes = [P, P, P, i32]
        L.gsr_autotune.argtypes = [P, P, ctypes.POINTER(Gaussians), P, i32, ctypes.POINTER(Opts), ctypes.c_char_p]
        L.gsr_inspect.argtypes = [P, P, ctypes.c_int, P, i64, ctypes.POINTER(i64)]
        L.gsr_opacity_loss.argtypes = [P, P, P, i64, ctypes.c_float, P, P]
        L.gsr_scale_reset.argtypes = [P, P, P, P, i64, ctypes.c_float]
        L.gsr_dssim.argtypes = [P, P, P, i32, P, P, ctypes.c_float, P, P]
        L.gsr_base_loss.argtypes = [P, P, P, i32, P, P, ctypes.c_float, P, P, P]
        fl = ctypes.c_float
        L.gsr_adam.argtypes = [P, P, P, P, P, P, P, i64, i32, fl, fl, fl, fl, i64]
        L.gsr_pair_counts.argtypes = [P, P, ctypes.POINTER(Gaussians), P, i32, ctypes.POINTER(Opts), P]
        L.gsr_scaled_camera.argtypes = [ctypes.POINTER(Camera), i32]
        L.gsr_scaled_camera.restype = Camera
        L.gsr_select_rmax.argtypes = [P, P, ctypes.POINTER(Gaussians), ctypes.POINTER(Camera), ctypes.POINTER(Opts),
                                      i32, ctypes.c_double, ctypes.POINTER(i32), P]
        for f in EXPORTED:
            if f not in ("gsr_status_string", "gsr_last_error", "gsr_scaled_camera"):
                getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


@dataclasses.dataclass
class RasterOptions:
    tile: tuple = (16, 16)
    lds_batch: int = 64
    sh_degree: int = 3
    sh_bf16: bool = False
    flags: int = GSR_DEFAULT_FLAGS

    def c(self) -> Opts:
        return Opts(self.tile[0], self.tile[1], self.lds_batch, self.sh_degree, 1 if self.sh_bf16 else 0, self.flags)


def make_cameras(cams: Sequence) -> ctypes.Array:
    """Camera objects with width/height/fx/fy/cx/cy/R/t/near (e.g. scenes.Camera) -> C array."""
    arr = (Camera * len(cams))()
    for i, c in enumerate(cams):
        R = np.asarray(c.R, np.float32).reshape(9)
        t = np.asarray(c.t, np.float32).reshape(3)
        arr[i] = Camera(int(c.width), int(c.height), float(c.fx), float(c.fy), float(c.cx), float(c.cy),
                        (ctypes.c_float * 9)(*R.tolist()), (ctypes.c_float * 3)(*t.tolist()),
                        float(getattr(c, "near", getattr(c, "near_z", 0.2))))
    return arr


def scaled_camera(cam, r: int):
    """The camera at downsampling factor r (gsr_scaled_camera), as a scenes.Camera."""
    from . import scenes
    k = lib().gsr_scaled_camera(ctypes.byref(make_cameras([cam])[0]), int(r))
    return scenes.Camera(k.width, k.height, k.fx, k.fy, k.cx, k.cy, np.asarray(cam.R, np.float32),
                         np.asarray(cam.t, np.float32), float(getattr(cam, "near", 0.2)))


def pixel_offsets(cams: Sequence) -> List[int]:
    arr = make_cameras(cams)
    off = (ctypes.c_int64 * (len(cams) + 1))()
    _check(None, lib().gsr_pixel_offsets(arr, len(cams), off))
    return list(off)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check(ctx, status: int):
    if status != 0:
        msg = lib().gsr_last_error(ctx).decode() if ctx else ""
        raise GsrError(status, msg)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _gaussians(means, scales, quats, opacities, sh, opts: RasterOptions) -> Gaussians:
    n = means.shape[0]
    for name, t, shape in (("means", means, (n, 3)), ("scales", scales, (n, 3)), ("quats", quats, (n, 4)),
                           ("opacities", opacities, (n,))):
        if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shape:
            raise ValueError(f"{name} must be a contiguous float32 CUDA tensor of shape {shape}")
    K = (opts.sh_degree + 1) ** 2
    want = torch.bfloat16 if opts.sh_bf16 else torch.float32
    if sh.dtype != want or not sh.is_cuda or not sh.is_contiguous() or tuple(sh.shape) != (n, K, 3):
        raise ValueError(f"sh must be a contiguous {want} CUDA tensor of shape {(n, K, 3)}")
    return Gaussians(n, means.data_ptr(), scales.data_ptr(), quats.data_ptr(), opacities.data_ptr(), sh.data_ptr())


class Rasterizer:
    """Owns one gsr context (device scratch, graphs) on the current device."""

    def __init__(self, max_views: int = 16, pair_capacity: int = 0):
        self._ctx = ctypes.c_void_p()
        _check(None, lib().gsr_create(ctypes.byref(self._ctx), max_views, pair_capacity))
        self.last_frame = None

    def close(self):
        if self._ctx:
            lib().gsr_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- raw calls -------------------------------------------------------
    def forward(self, means, scales, quats, opacities, sh, cams, opts: RasterOptions, out: Optional[dict] = None):
        """Render; `out` (a dict returned by an earlier call with the same sizes) is reused
        when given, which keeps output pointers stable for graph replays."""
        g = _gaussians(means, scales, quats, opacities, sh, opts)
        carr = make_cameras(cams)
        npix = sum(int(c.width) * int(c.height) for c in cams)
        dev = means.device
        if out is None or out["rgb"].shape[0] != npix or out["entropy_mean"].shape[0] != len(cams):
            out = dict(rgb=torch.empty((npix, 3), device=dev, dtype=torch.float32),
                       entropy=torch.empty(npix, device=dev, dtype=torch.float32),
                       t_final=torch.empty(npix, device=dev, dtype=torch.float32),
                       n_contrib=torch.empty(npix, device=dev, dtype=torch.int32),
                       entropy_mean=torch.empty(len(cams), device=dev, dtype=torch.float32))
        else:
            out = dict(out)
        fo = FwdOut(out["rgb"].data_ptr(), out["entropy"].data_ptr(), out["t_final"].data_ptr(),
                    out["n_contrib"].data_ptr(), out["entropy_mean"].data_ptr(), 0)
        o = opts.c()
        _check(self._ctx, lib().gsr_forward(self._ctx, _stream(), ctypes.byref(g), carr, len(cams), ctypes.byref(o),
                                            ctypes.byref(fo)))
        out["frame_id"] = fo.frame_id
        self.last_frame = fo.frame_id
        return out

    def render_image(self, means, scales, quats, opacities, sh, cams, opts: RasterOptions,
                     rgb: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Test-time render (colour only, no entropy, no saved state) into rgb [P, 3]."""
        g = _gaussians(means, scales, quats, opacities, sh, opts)
        carr = make_cameras(cams)
        npix = sum(int(c.width) * int(c.height) for c in cams)
        if rgb is None or rgb.shape != (npix, 3):
            rgb = torch.empty((npix, 3), device=means.device, dtype=torch.float32)
        elif rgb.dtype != torch.float32 or not rgb.is_contiguous():
            raise ValueError("rgb must be a contiguous float32 tensor of shape [P, 3]")
        o = opts.c()
        _check(self._ctx, lib().gsr_render(self._ctx, _stream(), ctypes.byref(g), carr, len(cams), ctypes.byref(o),
                                           ctypes.c_void_p(rgb.data_ptr())))
        self.last_frame = None
        return rgb

    def opacity_loss(self, opacities: torch.Tensor, weight: float, grad: Optional[torch.Tensor] = None,
                     loss: Optional[torch.Tensor] = None) -> torch.Tensor:
        """L_O = weight / n * sum exp(-(sigma - 0.5)^2 / 0.05) into `loss` (a 1-element tensor);
        its gradient is added to `grad` when given."""
        if opacities.dtype != torch.float32 or not opacities.is_contiguous() or opacities.dim() != 1:
            raise ValueError("opacities must be a contiguous float32 vector")
        if loss is None:
            loss = torch.empty(1, device=opacities.device, dtype=torch.float32)
        _check(self._ctx, lib().gsr_opacity_loss(self._ctx, _stream(), _ptr(opacities), opacities.shape[0],
                                                 float(weight), _ptr(grad), _ptr(loss)))
        return loss

    def dssim(self, cams, rgb, target, weight: float, grad_rgb: Optional[torch.Tensor] = None,
              loss: Optional[torch.Tensor] = None) -> torch.Tensor:
        """loss[v] = weight (1 - SSIM) per view; grad_rgb (when given) += its gradient."""
        for name, t in (("rgb", rgb), ("target", target)):
            if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
        if loss is None:
            loss = torch.empty(len(cams), device=rgb.device, dtype=torch.float32)
        carr = make_cameras(cams)
        _check(self._ctx, lib().gsr_dssim(self._ctx, _stream(), carr, len(cams), _ptr(rgb), _ptr(target),
                                          float(weight), _ptr(grad_rgb), _ptr(loss)))
        return loss

    def base_loss(self, cams, rgb, target, lam: float, grad_rgb: torch.Tensor, loss_l1: Optional[torch.Tensor] = None,
                  loss_dssim: Optional[torch.Tensor] = None):
        """(1 - lam) L1 + lam D-SSIM per view (Eq. 6) for the latest forward; grad_rgb is overwritten."""
        for name, t in (("rgb", rgb), ("target", target), ("grad_rgb", grad_rgb)):
            if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
        carr = make_cameras(cams)
        _check(self._ctx, lib().gsr_base_loss(self._ctx, _stream(), carr, len(cams), _ptr(rgb), _ptr(target), float(lam),
                                              _ptr(grad_rgb), _ptr(loss_l1), _ptr(loss_dssim)))

    def adam(self, raw, m, v, act, grad_act, kind: int, lr: float, step: int, beta1: float = 0.9,
             beta2: float = 0.999, eps: float = 1e-15) -> None:
        """One Adam step on raw parameters in place; act (may be None) receives f(raw)."""
        n = raw.numel()
        for name, t in (("raw", raw), ("m", m), ("v", v), ("grad", grad_act)) + ((("act", act),) if act is not None else ()):
            if t.dtype != torch.float32 or not t.is_contiguous() or t.numel() != n:
                raise ValueError(f"{name} must be a contiguous float32 tensor of {n} elements")
        _check(self._ctx, lib().gsr_adam(self._ctx, _stream(), _ptr(raw), _ptr(m), _ptr(v), _ptr(act), _ptr(grad_act),
                                         n, int(kind), float(lr), float(beta1), float(beta2), float(eps), int(step)))

    def scale_reset(self, scales: torch.Tensor, zeta: float, log_scales: Optional[torch.Tensor] = None) -> None:
        """s <- zeta * s in place (Eq. 7); log_scales (when given) += log(zeta)."""
        for t in (scales,) + ((log_scales,) if log_scales is not None else ()):
            if t.dtype != torch.float32 or not t.is_contiguous() or t.dim() != 2 or t.shape[1] != 3:
                raise ValueError("scales must be contiguous float32 [n, 3] tensors")
        _check(self._ctx, lib().gsr_scale_reset(self._ctx, _stream(), _ptr(scales), _ptr(log_scales),
                                                scales.shape[0], float(zeta)))

    def pair_counts(self, means, scales, quats, opacities, sh, cams, opts: RasterOptions) -> List[int]:
        g = _gaussians(means, scales, quats, opacities, sh, opts)
        carr = make_cameras(cams)
        out = (ctypes.c_int64 * len(cams))()
        o = opts.c()
        _check(self._ctx, lib().gsr_pair_counts(self._ctx, _stream(), ctypes.byref(g), carr, len(cams),
                                                ctypes.byref(o), out))
        return list(out)

    def select_rmax(self, means, scales, quats, opacities, sh, cam, opts: RasterOptions, r_cap: int = 4,
                    max_mean_len: float = 150.0):
        """(r_max, [mean per-tile list length at r = 1 .. r_cap])."""
        g = _gaussians(means, scales, quats, opacities, sh, opts)
        carr = make_cameras([cam])
        r = ctypes.c_int32(0)
        ml = (ctypes.c_double * r_cap)()
        o = opts.c()
        _check(self._ctx, lib().gsr_select_rmax(self._ctx, _stream(), ctypes.byref(g), carr, ctypes.byref(o),
                                                int(r_cap), float(max_mean_len), ctypes.byref(r), ml))
        return int(r.value), list(ml)

    def backward(self, means, scales, quats, opacities, sh, cams, opts: RasterOptions, saved: dict,
                 grad_rgb, grad_entropy=None, grad_entropy_mean=None, grads: Optional[dict] = None,
                 opacity_weight: float = 0.0, opacity_loss: Optional[torch.Tensor] = None):
        """gsr_backward; with opacity_weight or opacity_loss, gsr_backward_opacity_reg (the opacity
        regulariser fused into the projection backward, its loss into the 1-element opacity_loss)."""
        g = _gaussians(means, scales, quats, opacities, sh, opts)
        carr = make_cameras(cams)
        if grads is None:
            grads = dict(means=torch.empty_like(means), scales=torch.empty_like(scales),
                         quats=torch.empty_like(quats), opacities=torch.empty_like(opacities),
                         sh=torch.empty_like(sh))
        fo = FwdOut(saved["rgb"].data_ptr(), saved["entropy"].data_ptr(), saved["t_final"].data_ptr(),
                    saved["n_contrib"].data_ptr(), saved["entropy_mean"].data_ptr(), saved["frame_id"])
        gr = Grads(grads["means"].data_ptr(), grads["scales"].data_ptr(), grads["quats"].data_ptr(),
                   grads["opacities"].data_ptr(), grads["sh"].data_ptr())
        for name, t in (("grad_rgb", grad_rgb), ("grad_entropy", grad_entropy), ("grad_entropy_mean", grad_entropy_mean)):
            if t is not None and (t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
        o = opts.c()
        if opacity_weight == 0.0 and opacity_loss is None:
            _check(self._ctx, lib().gsr_backward(self._ctx, _stream(), ctypes.byref(g), carr, len(cams),
                                                 ctypes.byref(o), ctypes.byref(fo), _ptr(grad_rgb), _ptr(grad_entropy),
                                                 _ptr(grad_entropy_mean), ctypes.byref(gr)))
        else:
            if opacity_loss is not None and (opacity_loss.dtype != torch.float32 or not opacity_loss.is_cuda):
                raise ValueError("opacity_loss must be a float32 CUDA tensor")
            _check(self._ctx, lib().gsr_backward_opacity_reg(self._ctx, _stream(), ctypes.byref(g), carr, len(cams),
                                                             ctypes.byref(o), ctypes.byref(fo), _ptr(grad_rgb),
                                                             _ptr(grad_entropy), _ptr(grad_entropy_mean),
                                                             float(opacity_weight), _ptr(opacity_loss),
                                                             ctypes.byref(gr)))
        return grads

    def stats(self, n_views: int):
        ppv = (ctypes.c_int64 * n_views)()
        fs = FrameStats()
        _check(self._ctx, lib().gsr_stats(self._ctx, _stream(), ppv, ctypes.byref(fs)))
        return dict(pairs_per_view=list(ppv), pairs=fs.pairs, mean_len=fs.mean_len, p99_len=fs.p99_len,
                    overflow=bool(fs.overflow), evals_fwd=fs.evals_fwd, evals_bwd=fs.evals_bwd,
                    blended=fs.blended, tested_fwd=fs.tested_fwd, tested_bwd=fs.tested_bwd,
                    invariant_max_err=fs.invariant_max_err, invariant_violations=fs.invariant_violations)

    def l1_loss(self, cams, rgb, target, grad_rgb=None, loss=None):
        """L1 per view and its gradient, on the GPU, for the latest forward's cameras."""
        for name, t in (("rgb", rgb), ("target", target)):
            if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
        if grad_rgb is None:
            grad_rgb = torch.empty_like(rgb)
        if loss is None:
            loss = torch.empty(len(cams), device=rgb.device, dtype=torch.float32)
        carr = make_cameras(cams)
        _check(self._ctx, lib().gsr_l1_loss(self._ctx, _stream(), carr, len(cams), _ptr(rgb), _ptr(target),
                                            _ptr(grad_rgb), _ptr(loss)))
        return grad_rgb, loss

    def l1_loss_noalloc(self, cams, rgb, target, grad_rgb: torch.Tensor, loss: torch.Tensor):
        """gsr_l1_loss_noalloc: the L1 term into caller-provided grad_rgb [P, 3] and loss [V],
        with the library allocating nothing (its partial sums live in a static device array)."""
        for name, t in (("rgb", rgb), ("target", target), ("grad_rgb", grad_rgb), ("loss", loss)):
            if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
        carr = make_cameras(cams)
        _check(self._ctx, lib().gsr_l1_loss_noalloc(self._ctx, _stream(), carr, len(cams), _ptr(rgb), _ptr(target),
                                                    _ptr(grad_rgb), _ptr(loss)))
        return grad_rgb, loss

    def set_timing(self, enable: bool, stages: Optional[Sequence[str]] = None):
        """Time every stage (or only `stages`, names from STAGES) with HIP events; False stops."""
        mask = 0
        if enable:
            mask = (1 << len(STAGES)) - 1 if stages is None else sum(1 << STAGES.index(s) for s in stages)
        _check(self._ctx, lib().gsr_set_timing(self._ctx, mask))

    def stage_times(self, reset: bool = True):
        """{stage: (total_ms, launches)} accumulated since the last reset (synchronises)."""
        ms = (ctypes.c_double * len(STAGES))()
        n = (ctypes.c_int64 * len(STAGES))()
        _check(self._ctx, lib().gsr_stage_times(self._ctx, ms, n, 1 if reset else 0))
        return {name: (ms[i], n[i]) for i, name in enumerate(STAGES)}

    def inspect(self, which: int) -> np.ndarray:
        nbytes = ctypes.c_int64()
        _check(self._ctx, lib().gsr_inspect(self._ctx, _stream(), which, None, 0, ctypes.byref(nbytes)))
        dtype = {BUF_RECORDS: np.float32, BUF_RADIUS: np.int32, BUF_DEPTH: np.float32, BUF_TILES_TOUCHED: np.int32,
                 BUF_PAIR_VALUES: np.uint32, BUF_PAIR_TILES: np.uint32, BUF_RANGES: np.uint32,
                 BUF_GRAD2D: np.float32}[which]
        out = np.empty(nbytes.value // 4, dtype)
        _check(self._ctx, lib().gsr_inspect(self._ctx, _stream(), which, out.ctypes.data_as(ctypes.c_void_p),
                                            nbytes.value, ctypes.byref(nbytes)))
        return out

    def autotune(self, means, scales, quats, opacities, sh, cams, opts: RasterOptions,
                 cache_path: Optional[str] = None) -> RasterOptions:
        g = _gaussians(means, scales, quats, opacities, sh, opts)
        carr = make_cameras(cams)
        o = opts.c()
        _check(self._ctx, lib().gsr_autotune(self._ctx, _stream(), ctypes.byref(g), carr, len(cams), ctypes.byref(o),
                                             cache_path.encode() if cache_path else None))
        return dataclasses.replace(opts, tile=(o.tile_w, o.tile_h), lds_batch=o.lds_batch, flags=o.flags)


class RasterizeEntropy(torch.autograd.Function):
    """(means, scales, quats, opacities, sh) -> (rgb [P, 3], entropy [P], entropy_mean [V]).

    The backward maps autograd's incoming gradients to dL/dC, dL/dH_j and
    dL/dL_E,v and calls the HIP backward (Alg. 1 fused into the blend
    backward).  Only per-pixel state (final transmittance, contributor count)
    is saved between the two."""

    @staticmethod
    def forward(ctx, means, scales, quats, opacities, sh, rasterizer: Rasterizer, cams, opts: RasterOptions):
        out = rasterizer.forward(means, scales, quats, opacities, sh, cams, opts)
        ctx.rasterizer, ctx.cams, ctx.opts = rasterizer, cams, opts
        ctx.frame_id = out["frame_id"]
        ctx.save_for_backward(means, scales, quats, opacities, sh, out["rgb"], out["entropy"], out["t_final"],
                              out["n_contrib"], out["entropy_mean"])
        ctx.mark_non_differentiable(out["n_contrib"])
        return out["rgb"], out["entropy"], out["entropy_mean"]

    @staticmethod
    def backward(ctx, g_rgb, g_entropy, g_entropy_mean):
        means, scales, quats, opacities, sh, rgb, ent, tf, nc, em = ctx.saved_tensors
        saved = dict(rgb=rgb, entropy=ent, t_final=tf, n_contrib=nc, entropy_mean=em, frame_id=ctx.frame_id)
        if g_rgb is None:
            g_rgb = torch.zeros_like(rgb)
        grads = ctx.rasterizer.backward(means, scales, quats, opacities, sh, ctx.cams, ctx.opts, saved,
                                        g_rgb.contiguous().float(),
                                        None if g_entropy is None else g_entropy.contiguous().float(),
                                        None if g_entropy_mean is None else g_entropy_mean.contiguous().float())
        return grads["means"], grads["scales"], grads["quats"], grads["opacities"], grads["sh"], None, None, None


def render(means, scales, quats, opacities, sh, cams, opts: RasterOptions, rasterizer: Rasterizer):
    """Differentiable render of several views: returns (rgb [P,3], entropy [P], entropy_mean [V])."""
    return RasterizeEntropy.apply(means, scales, quats, opacities, sh, rasterizer, cams, opts)
