"""A synthetic training run around the rasterizer: the paper's loss and
schedule on targets rendered from a held-out synthetic scene.

Every step of an iteration runs in the HIP library: projection, binning,
sort, blending with the entropy term (gsr_forward), the L1 + D-SSIM base
loss (gsr_base_loss), the backward with Alg. 1 (gsr_backward) and one
Adam step per attribute (gsr_adam); between epochs the scale reset
(gsr_scale_reset) and the resolution scheduler's r_max (gsr_select_rmax).
This module only orders those calls and keeps the optimiser state.

Loss (Sec. 3, Eq. 6 and 12):  L = (1 - lambda) L1 + lambda L_D-SSIM + gamma L_E,
with the entropy term on every other epoch of each scale-reset period and the
scale reset s <- zeta s every `reset_every` epochs (Sec. 4.2, Eq. 7; Sec. 5.2,
Implementation Details).  The resolution scheduler trains coarse to fine:
the downsampling factor falls linearly from r_max to 1 over the first
`coarse_frac` of the iterations, r_max being the largest r <= 4 that keeps the
mean per-tile list length under `max_list_len` (Sec. 5.2).  No densification:
the Gaussian count is fixed, as in the paper's fixed-budget comparisons.

The held-out "teacher" scene is drawn with the bench generator; the student
starts from the teacher's centres jittered, larger scales, low opacities and
grey colours, so that the run has something to learn.  Targets are the
teacher's renders at the same cameras (and scale factors).
"""
from __future__ import annotations

import dataclasses
import math
import sys
import time
from typing import Dict, List, Optional

import numpy as np
import torch

from . import gsr, scenes


@dataclasses.dataclass
class TrainConfig:
    n_gaussians: int = 200_000
    n_views: int = 32
    width: int = 648
    height: int = 432
    iterations: int = 600
    epochs: int = 150              # the schedule is laid out in epochs (Sec. 5.2: 150 epochs)
    epoch_views: int = 0           # images per epoch, sampled with replacement; 0: iterations // epochs
    lam: float = 0.2               # D-SSIM weight, Eq. 6
    gamma: float = 0.015           # entropy weight, Eq. 12
    regulariser: str = "entropy"   # "entropy" (Eq. 12), "opacity" (the Sec. 5.4 comparator) or "none"
    opacity_weight: float = 3.0    # weight of the opacity regulariser in the Sec. 5.4 comparison
    zeta: float = 0.2              # scale-reset factor, Eq. 7
    reset_every: int = 20          # epochs between scale resets (Sec. 5.2)
    r_cap: int = 4
    max_list_len: float = 150.0
    coarse_frac: float = 0.3
    sh_degree: int = 3
    tile: tuple = (16, 16)
    lds: int = 128
    seed: int = 7
    lr_means: float = 1.6e-4 * 5.0
    lr_scales: float = 5e-3
    lr_quats: float = 1e-3
    lr_opacity: float = 2.5e-2
    lr_sh: float = 2.5e-3


class Trainer:
    def __init__(self, cfg: TrainConfig, device: torch.device = torch.device("cuda:0")):
        self.cfg = cfg
        self.dev = device
        self.R = gsr.Rasterizer(max_views=1)
        rng = np.random.default_rng(cfg.seed)
        teacher = scenes.gmm_scene(cfg.seed + 1, cfg.n_gaussians)
        if cfg.sh_degree < 3:
            teacher.sh = np.ascontiguousarray(teacher.sh[:, :(cfg.sh_degree + 1) ** 2])
            teacher.sh_degree = cfg.sh_degree
        self.cams = scenes.orbit_cameras(np.random.default_rng(cfg.seed + 2), [(cfg.width, cfg.height)] * cfg.n_views)
        self.test_cams = scenes.orbit_cameras(np.random.default_rng(cfg.seed + 3), [(cfg.width, cfg.height)] * 4)
        self.opts = gsr.RasterOptions(tile=tuple(cfg.tile), lds_batch=cfg.lds, sh_degree=cfg.sh_degree)
        td = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
        self.teacher = {k: td(getattr(teacher, k)) for k in ("means", "scales", "quats", "opacities", "sh")}
        # student: jittered centres, larger scales, low opacity, grey colour
        n = cfg.n_gaussians
        means = teacher.means + rng.normal(0, 0.05, teacher.means.shape).astype(np.float32)
        log_s = np.log(teacher.scales) + np.float32(math.log(1.5))
        quats = rng.normal(0, 1, (n, 4)).astype(np.float32)
        op_logit = np.full(n, math.log(0.1 / 0.9), np.float32)
        sh = np.zeros_like(teacher.sh)
        self.raw = {"means": td(means.astype(np.float32)), "scales": td(log_s.astype(np.float32)),
                    "quats": td(quats), "opacities": td(op_logit), "sh": td(sh)}
        self.act = {"means": self.raw["means"], "quats": self.raw["quats"], "sh": self.raw["sh"],
                    "scales": torch.exp(self.raw["scales"]).contiguous(),
                    "opacities": torch.sigmoid(self.raw["opacities"]).contiguous()}
        self.kind = {"means": 0, "scales": 1, "quats": 0, "opacities": 2, "sh": 0}
        self.lr = {"means": cfg.lr_means, "scales": cfg.lr_scales, "quats": cfg.lr_quats,
                   "opacities": cfg.lr_opacity, "sh": cfg.lr_sh}
        self.m = {k: torch.zeros_like(v) for k, v in self.raw.items()}
        self.v = {k: torch.zeros_like(v) for k, v in self.raw.items()}
        self.grads = {k: torch.empty_like(v) for k, v in self.raw.items()}
        self.step_no = 0
        self.targets: Dict[tuple, torch.Tensor] = {}
        self.r_max = self._select_rmax()
        self.epoch_views = cfg.epoch_views or max(1, cfg.iterations // cfg.epochs)
        self.order = np.random.default_rng(cfg.seed + 4).integers(0, cfg.n_views, cfg.iterations)
        self._g_le = torch.full((1,), cfg.gamma, device=device)
        self._g_le0 = torch.zeros(1, device=device)
        self._g_rgb: Optional[torch.Tensor] = None
        self._g_rgb_eval: Optional[torch.Tensor] = None
        self._loss = torch.zeros(2, device=device)        # (1 - lam) L1, lam D-SSIM of the latest step
        self._loss_o = torch.zeros(1, device=device)      # opacity regulariser of the latest step
        if cfg.regulariser not in ("entropy", "opacity", "none"):
            raise ValueError(f"unknown regulariser {cfg.regulariser!r}")
        self._init = {k: (self.raw[k].clone(), self.act[k].clone()) for k in self.raw}

    def restart(self) -> None:
        """Back to the initial parameters and a fresh optimiser (after warm-up iterations)."""
        for k, (raw, act) in self._init.items():
            self.raw[k].copy_(raw)
            if self.act[k] is not self.raw[k]:
                self.act[k].copy_(act)
            self.m[k].zero_()
            self.v[k].zero_()
        self.step_no = 0

    def prepare(self) -> None:
        """Render every target the schedule will ask for (all views at every scale it visits)."""
        for r in sorted({self.r_at(it) for it in range(self.cfg.iterations)}):
            for v in range(self.cfg.n_views):
                self.target(v, r)
        for v in range(len(self.test_cams)):
            self.target(v, 1, self.test_cams)

    # --------------------------------------------------------------------- #
    def _select_rmax(self) -> int:
        t = self.teacher
        r, _ = self.R.select_rmax(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], self.cams[0],
                                  self.opts, self.cfg.r_cap, self.cfg.max_list_len)
        return r

    def r_at(self, it: int) -> int:
        coarse = max(1, int(self.cfg.coarse_frac * self.cfg.iterations))
        if it >= coarse or self.r_max == 1:
            return 1
        return max(1, int(math.ceil(self.r_max * (1.0 - it / coarse))))

    def target(self, view: int, r: int, cams=None) -> torch.Tensor:
        cams = self.cams if cams is None else cams
        key = (id(cams), view, r)
        if key not in self.targets:
            cam = gsr.scaled_camera(cams[view], r)
            t = self.teacher
            self.targets[key] = self.R.render_image(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"],
                                                    [cam], self.opts).clone()
        return self.targets[key]

    def epoch(self, it: int) -> int:
        return it // self.epoch_views

    # --------------------------------------------------------------------- #
    def step(self, it: int) -> None:
        cfg = self.cfg
        view = int(self.order[it])
        r = self.r_at(it)
        cam = gsr.scaled_camera(self.cams[view], r)
        tgt = self.target(view, r)
        a = self.act
        out = self.R.forward(a["means"], a["scales"], a["quats"], a["opacities"], a["sh"], [cam], self.opts)
        rgb = out["rgb"]
        if self._g_rgb is None or self._g_rgb.shape != rgb.shape:
            self._g_rgb = torch.empty_like(rgb)
        g_rgb = self._g_rgb
        self.R.base_loss([cam], rgb, tgt, cfg.lam, g_rgb, self._loss[0:1], self._loss[1:2])
        ep = self.epoch(it)
        reg_on = (ep % cfg.reset_every) % 2 == 1              # every other epoch of a reset period
        entropy_on = reg_on and cfg.regulariser == "entropy"
        opacity_on = reg_on and cfg.regulariser == "opacity"   # dL_O/dsigma fused into the projection backward
        g = self.R.backward(a["means"], a["scales"], a["quats"], a["opacities"], a["sh"], [cam], self.opts, out,
                            g_rgb, None, self._g_le if entropy_on else self._g_le0, self.grads,
                            opacity_weight=cfg.opacity_weight if opacity_on else 0.0,
                            opacity_loss=self._loss_o if opacity_on else None)
        self.step_no += 1
        for k in self.raw:
            act = None if self.kind[k] == 0 else self.act[k]
            self.R.adam(self.raw[k], self.m[k], self.v[k], act, g[k], self.kind[k], self.lr[k], self.step_no)
        # scale reset at the start of every reset period (not the first)
        if (it + 1) % self.epoch_views == 0:
            nxt = self.epoch(it + 1)
            if nxt % cfg.reset_every == 0:
                self.R.scale_reset(self.act["scales"], cfg.zeta, self.raw["scales"])

    def train_loss(self) -> float:
        """Mean base loss (Eq. 6) over the training views at full resolution."""
        a = self.act
        if self._g_rgb_eval is None:
            self._g_rgb_eval = torch.empty(self.cfg.width * self.cfg.height, 3, device=self.dev)
        tot = 0.0
        for v, cam in enumerate(self.cams):
            out = self.R.forward(a["means"], a["scales"], a["quats"], a["opacities"], a["sh"], [cam], self.opts)
            self.R.base_loss([cam], out["rgb"], self.target(v, 1), self.cfg.lam, self._g_rgb_eval,
                             self._loss[0:1], self._loss[1:2])
            tot += float(self._loss.sum())
        return tot / len(self.cams)

    def list_stats(self, cams=None) -> dict:
        """Mean per-tile list length and mean per-pixel entropy (nats) of the current scene over `cams`."""
        cams = self.test_cams if cams is None else cams
        a = self.act
        mean_len, ent = 0.0, 0.0
        for cam in cams:
            out = self.R.forward(a["means"], a["scales"], a["quats"], a["opacities"], a["sh"], [cam], self.opts)
            mean_len += self.R.stats(1)["mean_len"]
            ent += float(out["entropy_mean"][0])
        return {"mean_list_len": mean_len / len(cams), "mean_entropy": ent / len(cams)}

    def psnr(self, cams=None) -> float:
        cams = self.test_cams if cams is None else cams
        a = self.act
        tot = 0.0
        for v, cam in enumerate(cams):
            img = self.R.render_image(a["means"], a["scales"], a["quats"], a["opacities"], a["sh"], [cam], self.opts)
            mse = float(((img - self.target(v, 1, cams)) ** 2).mean())
            tot += -10.0 * math.log10(max(mse, 1e-12))
        return tot / len(cams)

    def run(self, iterations: Optional[int] = None, log_every: int = 0) -> dict:
        n = self.cfg.iterations if iterations is None else iterations
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for it in range(n):
            self.step(it)
            if log_every and (it + 1) % log_every == 0:
                print(f"iteration {it + 1}/{n}  {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        return {"iterations": n, "seconds": sec, "iters_per_s": n / sec}
