"""Parity of the training-step entry points with the FP64 oracle: D-SSIM and
the base loss of Eq. 6, the Adam step on raw parameters, and a short
synthetic training run (loss falls, held-out PSNR rises, bit-identical reruns).

Tolerances.  D-SSIM is accumulated in FP32: the window statistics are sums of
121 products of values in [0, 1] (relative rounding ~121 * 6e-8 of each), the
variances subtract squares of similar size, and the loss is a mean over
3 * W * H terms -- 2e-5 absolute on the loss and 1e-4 relative (L2) on the
gradient cover that with room.  Adam runs element-wise in FP32: the moments
agree to ~1e-6 relative and the update to ~1e-6 of lr per step.
"""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2603_09277_amd import gsr, scenes

from gpu_helpers import DEV, rel_norm, to_dev

pytestmark = pytest.mark.gpu

SSIM_LOSS_TOL = 2e-5
F32 = lambda x: float(np.float32(x))
SSIM_GRAD_TOL = 1e-4


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = gsr.Rasterizer(max_views=8)
    yield r
    r.close()


def _cam(W, H):
    return scenes.Camera(W, H, float(W), float(W), W / 2.0, H / 2.0, np.eye(3, dtype=np.float32),
                         np.zeros(3, np.float32), 0.2)


def _image_pair(rng, W, H, smooth=True):
    """A render-like image (smooth blobs plus noise, in [0, 1]) and a perturbed copy."""
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    x = np.zeros((H, W, 3))
    if smooth:
        for _ in range(6):
            cx, cy, s = rng.uniform(0, W), rng.uniform(0, H), rng.uniform(2, 0.3 * max(W, H) + 2)
            x += rng.uniform(0, 0.6, 3) * np.exp(-((xx - cx) ** 2 + (yy - cy) ** 2) / (2 * s * s))[..., None]
    x = np.clip(x + rng.normal(0, 0.05, x.shape), 0, 1)
    y = np.clip(x + rng.normal(0, 0.1, x.shape), 0, 1)
    return x.astype(np.float32), y.astype(np.float32)


@pytest.mark.parametrize("sizes", [[(64, 48)], [(37, 23), (1, 1), (200, 5)], [(130, 97), (16, 16)], [(11, 11)]])
def test_dssim_parity(R, sizes):
    rng = np.random.default_rng(len(sizes) * 1000 + sizes[0][0])
    xs, ys = zip(*[_image_pair(rng, W, H) for W, H in sizes])
    cams = [_cam(W, H) for W, H in sizes]
    x = torch.from_numpy(np.concatenate([a.reshape(-1, 3) for a in xs])).to(DEV)
    y = torch.from_numpy(np.concatenate([a.reshape(-1, 3) for a in ys])).to(DEV)
    base = torch.from_numpy(rng.normal(0, 1e-3, x.shape).astype(np.float32)).to(DEV)
    grad = base.clone()
    w = 0.2
    loss = R.dssim(cams, x, y, w, grad)
    torch.cuda.synchronize()
    loss = loss.cpu().numpy()
    g = (grad - base).cpu().numpy()
    off = 0
    for v, (W, H) in enumerate(sizes):
        s, gs = orc.ssim(xs[v], ys[v])
        assert abs(loss[v] - w * (1.0 - s)) <= SSIM_LOSS_TOL, (v, W, H, loss[v], w * (1 - s))
        gv = g[off:off + W * H].reshape(H, W, 3)
        assert rel_norm(gv, -w * gs) <= SSIM_GRAD_TOL, (v, W, H, rel_norm(gv, -w * gs))
        off += W * H


def test_dssim_identical_images(R):
    rng = np.random.default_rng(3)
    x, _ = _image_pair(rng, 40, 30)
    xt = torch.from_numpy(x.reshape(-1, 3)).to(DEV)
    grad = torch.zeros_like(xt)
    loss = R.dssim([_cam(40, 30)], xt, xt.clone(), 1.0, grad)
    torch.cuda.synchronize()
    assert abs(float(loss[0])) <= 1e-6
    assert float(grad.abs().max()) <= 1e-6


def test_base_loss_parity(R):
    scene, cams, _ = scenes.workload("tiny")
    t = to_dev(scene)
    opts = gsr.RasterOptions(tile=(16, 16), sh_degree=0)
    out = R.forward(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], cams, opts)
    rgb = out["rgb"]
    rng = np.random.default_rng(11)
    tgt_np = rng.uniform(0, 1, tuple(rgb.shape)).astype(np.float32)
    tgt = torch.from_numpy(tgt_np).to(DEV)
    lam = 0.2
    grad = torch.full_like(rgb, 7.0)            # overwritten
    l1 = torch.empty(len(cams), device=DEV)
    ds = torch.empty(len(cams), device=DEV)
    R.base_loss(cams, rgb, tgt, lam, grad, l1, ds)
    torch.cuda.synchronize()
    x = rgb.cpu().numpy().astype(np.float64)
    W, H = cams[0].width, cams[0].height
    s, gs = orc.ssim(x.reshape(H, W, 3), tgt_np.reshape(H, W, 3))
    d = x - tgt_np
    assert abs(float(l1[0]) - (1 - lam) * np.abs(d).mean()) <= 1e-6
    assert abs(float(ds[0]) - lam * (1 - s)) <= SSIM_LOSS_TOL
    want = (1 - lam) * np.sign(d) / d.size - lam * gs.reshape(-1, 3)
    assert rel_norm(grad.cpu().numpy(), want) <= SSIM_GRAD_TOL
    # lambda = 0 is plain L1 (the D-SSIM outputs are left alone)
    ds.fill_(-1.0)
    R.base_loss(cams, rgb, tgt, 0.0, grad, l1, ds)
    torch.cuda.synchronize()
    assert float(ds[0]) == -1.0
    assert rel_norm(grad.cpu().numpy(), np.sign(d) / d.size) <= 1e-6


def test_base_loss_rejects(R):
    scene, cams, _ = scenes.workload("tiny")
    t = to_dev(scene)
    opts = gsr.RasterOptions(tile=(16, 16), sh_degree=0)
    out = R.forward(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], cams, opts)
    g = torch.empty_like(out["rgb"])
    with pytest.raises(gsr.GsrError):
        R.base_loss(cams, out["rgb"], out["rgb"], 1.5, g)
    with pytest.raises(gsr.GsrError):
        R.base_loss(cams + cams, out["rgb"], out["rgb"], 0.2, g)


@pytest.mark.parametrize("offset", [0, 1])      # 1: views one float past a 16-byte boundary (the scalar path)
@pytest.mark.parametrize("kind", [0, 1, 2])
def test_adam_parity(R, kind, offset):
    rng = np.random.default_rng(20 + kind + 10 * offset)
    n = 100_003                                   # several blocks and a ragged tail
    buf = lambda: torch.zeros(n + offset, device=DEV)[offset:]
    raw_d = buf()
    raw_d.copy_(torch.from_numpy(rng.normal(0, 1.5, n).astype(np.float32)))
    m_d, v_d = buf(), buf()
    act_d = buf() if kind else None
    lr = 1e-2
    for step in range(1, 8):
        g = rng.normal(0, 1, n).astype(np.float32) * np.float32(10.0 ** rng.uniform(-6, 0))
        g[::97] = 0.0                             # exact zeros: the update is 0 / (0 + eps) = 0
        # the oracle steps from the library's own float32 state, so every step is compared on its own
        before = [t.cpu().numpy() for t in (raw_d, m_d, v_d)]
        # hyper-parameters cross the boundary as float32 (1 - 0.999f differs from 1e-3 by 1.3e-5 relative)
        r64, m64, v64, a64 = orc.adam_step(*before, g, kind, F32(lr), step, b1=F32(0.9), b2=F32(0.999), eps=F32(1e-15))
        g_d = buf()
        g_d.copy_(torch.from_numpy(g))
        R.adam(raw_d, m_d, v_d, act_d, g_d, kind, lr, step)
        torch.cuda.synchronize()
        got_raw, got_m, got_v = raw_d.cpu().numpy(), m_d.cpu().numpy(), v_d.cpu().numpy()
        # m = b1 m + (1 - b1) g may cancel: bound its rounding by the size of its two terms
        g_eff = (m64 - 0.9 * before[1]) / 0.1
        m_scale = 0.9 * np.abs(before[1]) + 0.1 * np.abs(g_eff)
        assert np.all(np.abs(got_m - m64) <= 1e-6 * m_scale), step
        assert np.all(np.abs(got_v - v64) <= 1e-6 * np.abs(v64)), step
        assert np.all(np.abs(got_raw - r64) <= 1e-6 * np.abs(before[0]) + 1e-5 * lr), step
        if kind:
            got_a = act_d.cpu().numpy()
            assert np.all(np.abs(got_a - a64) <= 4e-6 * np.abs(a64) + 1e-7), step


def test_adam_rejects(R):
    x = torch.zeros(4, device=DEV)
    with pytest.raises(gsr.GsrError):
        R.adam(x, x.clone(), x.clone(), None, x.clone(), 3, 1e-3, 1)
    with pytest.raises(gsr.GsrError):
        R.adam(x, x.clone(), x.clone(), None, x.clone(), 0, 1e-3, 0)


# --------------------------------------------------------------------------- #
# a short synthetic training run
# --------------------------------------------------------------------------- #

def _small_cfg():
    from paper_2603_09277_amd.train import TrainConfig
    return TrainConfig(n_gaussians=20_000, n_views=8, width=160, height=120, iterations=120, epoch_views=8,
                       reset_every=4, seed=5)


def test_training_run_learns_and_is_deterministic():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_09277_amd.train import Trainer
    finals = []
    for rep in range(2):
        tr = Trainer(_small_cfg())
        p0, l0 = tr.psnr(), tr.train_loss()
        tr.run()
        p1, l1 = tr.psnr(), tr.train_loss()
        print(f"run {rep}: r_max {tr.r_max} held-out psnr {p0:.2f} -> {p1:.2f}, training loss {l0:.4f} -> {l1:.4f}",
              flush=True)
        assert math.isfinite(l1) and math.isfinite(p1)
        assert p1 > p0 + 0.5
        assert l1 < l0
        finals.append({k: v.cpu().numpy().copy() for k, v in tr.raw.items()})
        tr.R.close()
    for k in finals[0]:
        assert np.array_equal(finals[0][k], finals[1][k]), k


def test_training_with_opacity_regulariser_adds_its_gradient():
    """The comparator of the Sec. 5.4 ablation: on an epoch where the regulariser is on, the
    opacity gradient of the step is the image and entropy-free gradient plus dL_O/dsigma
    (weight 3.0, mean over Gaussians) at the step's opacities."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import dataclasses
    from paper_2603_09277_amd.train import Trainer
    cfg = _small_cfg()
    tr_o = Trainer(dataclasses.replace(cfg, regulariser="opacity"))
    tr_n = Trainer(dataclasses.replace(cfg, regulariser="none"))
    for it in range(cfg.epoch_views):                # epoch 0: no regulariser, identical runs
        tr_o.step(it)
        tr_n.step(it)
    torch.cuda.synchronize()
    for k in tr_o.raw:
        assert torch.equal(tr_o.raw[k], tr_n.raw[k]), k
    op = tr_o.act["opacities"].cpu().numpy().copy()
    it = cfg.epoch_views                             # first iteration of epoch 1: the regulariser is on
    tr_o.step(it)
    tr_n.step(it)
    torch.cuda.synchronize()
    g_o = tr_o.grads["opacities"].cpu().numpy().astype(np.float64)
    g_n = tr_n.grads["opacities"].cpu().numpy().astype(np.float64)
    L_want, g_want = orc.opacity_loss(op, 3.0)
    assert abs(float(tr_o._loss_o[0]) - L_want) <= 1e-6 * L_want
    # (a + b) - a recovers b up to one rounding of the sum; b itself is FP32 (exp and 4 products)
    err = np.abs((g_o - g_n) - g_want)
    assert np.all(err <= 2.0 ** -22 * (np.abs(g_n) + np.abs(g_want)) + 1e-6 * np.abs(g_want)), err.max()
    tr_o.R.close()
    tr_n.R.close()


@pytest.mark.parametrize("reg", ["opacity", "none"])
def test_training_run_with_other_regularisers(reg):
    """The comparator runs of the Sec. 5.4 ablation: the opacity regulariser in place of the
    entropy term (its gradient is added to the opacity gradient), or no regulariser."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import dataclasses
    from paper_2603_09277_amd.train import Trainer
    tr = Trainer(dataclasses.replace(_small_cfg(), regulariser=reg, iterations=64))
    lo0 = float(tr.R.opacity_loss(tr.act["opacities"], 3.0)[0])
    p0 = tr.psnr()
    tr.run()
    p1 = tr.psnr()
    lo1 = float(tr.R.opacity_loss(tr.act["opacities"], 3.0)[0])
    ls = tr.list_stats()
    print(f"{reg}: psnr {p0:.2f} -> {p1:.2f}, L_O {lo0:.4f} -> {lo1:.4f}, mean list {ls['mean_list_len']:.1f}, "
          f"entropy {ls['mean_entropy']:.3f}", flush=True)
    assert math.isfinite(p1) and ls["mean_list_len"] > 0 and math.isfinite(ls["mean_entropy"])
    if reg == "none":
        assert p1 > p0 + 0.5
    tr.R.close()
