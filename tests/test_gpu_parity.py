"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (FP32 blending against an FP64 oracle):
  * tile counts, sorted per-tile lists and ranges: bit-exact, with the oracle
    binning the GPU's own float32 projection (a Gaussian's rect and depth key
    are integer decisions taken from float32 values);
  * image, entropy, final transmittance: 1e-5 absolute on every pixel whose
    alpha-skip / transmittance-stop decisions are not within 1e-4 (relative)
    of their thresholds -- the oracle flags those pixels, where FP32 and FP64
    may legitimately decide differently; flagged pixels are counted and bounded;
  * FP32 gradients: relative L2 error per tensor <= 1e-3 and, per element,
    |g - g*| <= 1e-3 |g*| + 1e-5 max|g*| (check_grad).
"""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as orc
from paper_2603_09277_amd import gsr, scenes

from gpu_helpers import (DEV, GRAD_TOL, KEYS, check_grad, check_grad2d, gpu_backward, gpu_forward, gpu_records,
                         oracle_grads, oracle_stagewise, rel_norm, split_pixels, to_dev)

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-5
GAMMA = 0.015


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = gsr.Rasterizer(max_views=16)
    yield r
    r.close()


@pytest.fixture(scope="module")
def tiny():
    scene, cams, _ = scenes.workload("tiny")
    return scene, cams


def l1_grad_torch(rgb, target_np):
    tgt = torch.from_numpy(target_np.reshape(-1, 3)).to(DEV)
    return (torch.sign(rgb - tgt) / rgb.numel()).contiguous()


# --------------------------------------------------------------------------- #
# (a) projection
# --------------------------------------------------------------------------- #

def test_projection_parity_tiny(R, tiny):
    scene, cams = tiny
    t = to_dev(scene)
    opts = gsr.RasterOptions(tile=(16, 16), sh_degree=0)
    gpu_forward(R, t, cams, opts)
    pg = gpu_records(R, scene.n, 1)[0]
    po = orc.project(scene, cams[0])
    assert np.array_equal(pg["radius"] > 0, po["radius"] > 0)
    v = po["radius"] > 0
    assert np.all(np.abs(pg["mean2d"] - po["mean2d"])[v] <= 1e-6 * np.abs(po["mean2d"][v]) + 1e-5)
    scale = np.maximum(np.abs(po["conic"][:, 0]), np.abs(po["conic"][:, 2]))[:, None]
    assert np.all((np.abs(pg["conic"] - po["conic"]) / scale)[v] <= 1e-4)
    assert np.all(np.abs(pg["rgb"] - po["rgb"])[v] <= 1e-6)
    assert np.all(np.abs(pg["depth32"].astype(np.float64) - po["depth"])[v] <= 1e-6 * po["depth"][v])
    a, b, c = po["cov2d"][:, 0], po["cov2d"][:, 1], po["cov2d"][:, 2]
    mid = 0.5 * (a + c)
    r_exact = 3 * np.sqrt(mid + np.sqrt(np.maximum(mid * mid - (a * c - b * b), 0)))
    near_int = np.abs(r_exact - np.round(r_exact)) < 1e-3
    assert np.array_equal(pg["radius"][v & ~near_int], po["radius"][v & ~near_int])


def test_projection_parity_sh3_rotated_camera(R):
    scene = scenes.gmm_scene(21, 4000)
    cams = scenes.orbit_cameras(np.random.default_rng(22), [(320, 200)])
    t = to_dev(scene)
    opts = gsr.RasterOptions(tile=(16, 16), sh_degree=3)
    gpu_forward(R, t, cams, opts)
    pg = gpu_records(R, scene.n, 1)[0]
    po = orc.project(scene, cams[0])
    assert np.array_equal(pg["radius"] > 0, po["radius"] > 0)
    v = po["radius"] > 0
    assert v.sum() > 1000
    assert np.all(np.abs(pg["rgb"] - po["rgb"])[v] <= 2e-6)
    assert np.all(np.abs(pg["mean2d"] - po["mean2d"])[v] <= 1e-6 * np.abs(po["mean2d"][v]) + 1e-5)


# --------------------------------------------------------------------------- #
# (b)-(d) binning, sort, ranges: bit-exact on the GPU's float32 projection
# --------------------------------------------------------------------------- #

@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8)])
def test_binning_sort_ranges_bit_exact(R, tiny, tile):
    scene, cams = tiny
    t = to_dev(scene)
    opts = gsr.RasterOptions(tile=tile, sh_degree=0)
    gpu_forward(R, t, cams, opts)
    pg = gpu_records(R, scene.n, 1)[0]
    cam = cams[0]
    total, tt, _ = orc.count_pairs(pg["mean2d"], pg["radius"], cam.width, cam.height, *tile)
    assert np.array_equal(R.inspect(gsr.BUF_TILES_TOUCHED), tt)
    vals, ranges = orc.bin_lists(pg["mean2d"], pg["radius"], pg["depth32"], cam.width, cam.height, *tile)
    gv = R.inspect(gsr.BUF_PAIR_VALUES)
    gr = R.inspect(gsr.BUF_RANGES).reshape(-1, 2)
    assert len(gv) == total
    assert np.array_equal(gv.astype(np.int64), vals.astype(np.int64))
    assert np.array_equal(gr.astype(np.int64), ranges.astype(np.int64))


def test_binning_bit_exact_mid_size_sort(R):
    """A tile sort of 2.8e5-3.3e5 pairs: 129-256 radix blocks, the pass size whose spine
    takes one count a thread (smaller passes have no spine, larger ones 8 or 32)."""
    scene, cams = scenes.tiny_scene(41, 8000)
    scene.scales = (scene.scales * np.float32(7.0)).astype(np.float32)
    t = to_dev(scene)
    gpu_forward(R, t, cams, gsr.RasterOptions(tile=(16, 16), sh_degree=0))
    pg = gpu_records(R, scene.n, 1)[0]
    cam = cams[0]
    vals, ranges = orc.bin_lists(pg["mean2d"], pg["radius"], pg["depth32"], cam.width, cam.height, 16, 16)
    assert 128 * 2048 < len(vals) <= 256 * 2048, len(vals)
    assert np.array_equal(R.inspect(gsr.BUF_PAIR_VALUES).astype(np.int64), vals.astype(np.int64))
    assert np.array_equal(R.inspect(gsr.BUF_RANGES).reshape(-1, 2).astype(np.int64), ranges.astype(np.int64))


def test_binning_bit_exact_single_view_full(R):
    """The 200k-Gaussian 1296x840 workload: every one of ~1e6 pairs in order."""
    scene, cams, _ = scenes.workload("single")
    t = to_dev(scene)
    opts = gsr.RasterOptions(tile=(16, 16), sh_degree=3)
    gpu_forward(R, t, cams, opts)
    pg = gpu_records(R, scene.n, 1)[0]
    cam = cams[0]
    vals, ranges = orc.bin_lists(pg["mean2d"], pg["radius"], pg["depth32"], cam.width, cam.height, 16, 16)
    assert len(vals) > 100_000
    assert np.array_equal(R.inspect(gsr.BUF_PAIR_VALUES).astype(np.int64), vals.astype(np.int64))
    assert np.array_equal(R.inspect(gsr.BUF_RANGES).reshape(-1, 2).astype(np.int64), ranges.astype(np.int64))


# --------------------------------------------------------------------------- #
# (e)-(f) blend and entropy
# --------------------------------------------------------------------------- #

def _cmp_image(out, img_o, cam, v=0, cams=None, tol=IMG_TOL, max_flag_frac=0.01):
    cams = cams or [cam]
    rgb = split_pixels(out["rgb"].cpu().numpy(), cams, v)
    H = split_pixels(out["entropy"].cpu().numpy(), cams, v)
    T = split_pixels(out["t_final"].cpu().numpy(), cams, v)
    nc = split_pixels(out["n_contrib"].cpu().numpy(), cams, v)
    ok = img_o["flags"] == 0
    assert ok.mean() >= 1 - max_flag_frac
    e_rgb = np.abs(rgb - img_o["rgb"])[ok].max(initial=0.0)
    e_H = np.abs(H - img_o["H"])[ok].max(initial=0.0)
    e_T = np.abs(T - img_o["T"])[ok].max(initial=0.0)
    assert e_rgb <= tol, e_rgb
    assert e_H <= tol, e_H
    assert e_T <= tol, e_T
    assert np.array_equal(nc[ok], img_o["ncontrib"][ok])
    return e_rgb, e_H, e_T


@pytest.mark.parametrize("tile,lds", [((16, 16), 64), ((8, 8), 32), ((32, 8), 128), ((16, 16), 256)])
def test_blend_stagewise_tiny(R, tiny, tile, lds):
    scene, cams = tiny
    t = to_dev(scene)
    opts = gsr.RasterOptions(tile=tile, lds_batch=lds, sh_degree=0)
    out = gpu_forward(R, t, cams, opts)
    pg = gpu_records(R, scene.n, 1)[0]
    img_o = oracle_stagewise(pg, cams[0], tile)
    _cmp_image(out, img_o, cams[0])
    le = float(out["entropy_mean"].cpu()[0])
    assert abs(le - img_o["H"].mean()) <= 1e-6


def test_end_to_end_tiny_vs_fp64_oracle(R, tiny):
    """Oracle with its own FP64 projection: lists identical, image within 1e-5."""
    scene, cams = tiny
    t = to_dev(scene)
    opts = gsr.RasterOptions(tile=(16, 16), sh_degree=0)
    out = gpu_forward(R, t, cams, opts)
    f = orc.forward_view(scene, cams[0], (16, 16))
    assert np.array_equal(R.inspect(gsr.BUF_PAIR_VALUES).astype(np.int64), f["values"].astype(np.int64))
    _cmp_image(out, f, cams[0])
    assert abs(float(out["entropy_mean"].cpu()[0]) - f["L_E"]) <= 1e-6


def test_weights_sum_to_one_on_gpu(R, tiny):
    """Eq. 9 on the GPU: with every colour 1, rgb + T_final = 1."""
    scene, cams = tiny
    s = scene.copy()
    s.sh[:] = np.float32(0.5 * 2.0 * math.sqrt(math.pi))      # Y00 * k + 0.5 = 1
    t = to_dev(s)
    out = gpu_forward(R, t, cams, gsr.RasterOptions(tile=(16, 16), sh_degree=0))
    rgb = out["rgb"].cpu().numpy().astype(np.float64)
    T = out["t_final"].cpu().numpy().astype(np.float64)
    assert np.abs(rgb + T[:, None] - 1.0).max() < 3e-6
    assert T.min() >= 1e-4
    H = out["entropy"].cpu().numpy()
    nc = out["n_contrib"].cpu().numpy()
    assert np.all(H >= -1e-6) and np.all(H <= np.log(nc + 1.0) + 1e-5)


def test_determinism(R, tiny):
    scene, cams = tiny
    t = to_dev(scene)
    opts = gsr.RasterOptions(tile=(16, 16), sh_degree=0)
    a = gpu_forward(R, t, cams, opts)
    va = R.inspect(gsr.BUF_PAIR_VALUES)
    b = gpu_forward(R, t, cams, opts)
    vb = R.inspect(gsr.BUF_PAIR_VALUES)
    for k in ("rgb", "entropy", "t_final", "n_contrib", "entropy_mean"):
        assert torch.equal(a[k], b[k]), k
    assert np.array_equal(va, vb)


# --------------------------------------------------------------------------- #
# (g) backward
# --------------------------------------------------------------------------- #

def _tiny_backward(R, scene, cams, tile=(16, 16), lds=64):
    t = to_dev(scene)
    opts = gsr.RasterOptions(tile=tile, lds_batch=lds, sh_degree=scene.sh_degree)
    out = gpu_forward(R, t, cams, opts)
    target = scenes.target_image(101, cams[0].height, cams[0].width)
    g_rgb = l1_grad_torch(out["rgb"], target)
    g_le = torch.full((1,), GAMMA, device=DEV)
    grads = gpu_backward(R, t, cams, opts, out, g_rgb, None, g_le)
    return t, opts, out, target, g_rgb, grads


def test_blend_backward_stagewise(R, tiny):
    scene, cams = tiny
    cam = cams[0]
    t, opts, out, target, g_rgb, grads = _tiny_backward(R, scene, cams)
    pg = gpu_records(R, scene.n, 1)[0]
    vals, ranges = orc.bin_lists(pg["mean2d"], pg["radius"], pg["depth32"], cam.width, cam.height, 16, 16)
    M = cam.width * cam.height
    g2o = orc.backward_render(cam.width, cam.height, 16, 16, pg["mean2d"], pg["conic"], pg["opacity"], pg["rgb"],
                              ranges, vals, g_rgb.cpu().numpy().reshape(cam.height, cam.width, 3).astype(np.float64),
                              np.full((cam.height, cam.width), GAMMA / M))
    g2g = R.inspect(gsr.BUF_GRAD2D).reshape(scene.n, 9).astype(np.float64)
    check_grad2d(g2g, g2o)


@pytest.mark.parametrize("tile,lds", [((16, 16), 128), ((32, 8), 64), ((16, 16), 256)])
def test_long_lists_shared_batches_vs_oracle(R, tile, lds):
    """Mean list length above 512: the forward stages each batch once per tile for its four
    8x8 blocks (the short-list tests cover the per-block staging).  Image, entropy and
    transmittance stage-wise, and the blend backward, against the oracle."""
    scene, cams = scenes.tiny_scene(41, 8000)
    scene.scales = (scene.scales * np.float32(4.0)).astype(np.float32)
    cam = cams[0]
    t = to_dev(scene)
    opts = gsr.RasterOptions(tile=tile, lds_batch=lds, sh_degree=0)
    out = gpu_forward(R, t, cams, opts)
    st = R.stats(1)
    assert st["mean_len"] >= 512, st["mean_len"]
    pg = gpu_records(R, scene.n, 1)[0]
    img_o = oracle_stagewise(pg, cam, tile)
    _cmp_image(out, img_o, cam)
    g_rgb = l1_grad_torch(out["rgb"], scenes.target_image(43, cam.height, cam.width))
    M = cam.width * cam.height
    gpu_backward(R, t, cams, opts, out, g_rgb, None, torch.full((1,), GAMMA, device=DEV))
    vals, ranges = orc.bin_lists(pg["mean2d"], pg["radius"], pg["depth32"], cam.width, cam.height, tile[0], tile[1])
    g2o = orc.backward_render(cam.width, cam.height, tile[0], tile[1], pg["mean2d"], pg["conic"], pg["opacity"],
                              pg["rgb"], ranges, vals,
                              g_rgb.cpu().numpy().reshape(cam.height, cam.width, 3).astype(np.float64),
                              np.full((cam.height, cam.width), GAMMA / M))
    g2g = R.inspect(gsr.BUF_GRAD2D).reshape(scene.n, 9).astype(np.float64)
    check_grad2d(g2g, g2o)
    # the persistent scheduling of the same kernels: bit-identical outputs and gradients
    ref = {k: out[k].clone() for k in ("rgb", "entropy", "t_final", "n_contrib", "entropy_mean")}
    gref = gpu_backward(R, t, cams, opts, gpu_forward(R, t, cams, opts), g_rgb, None,
                        torch.full((1,), GAMMA, device=DEV))
    popts = gsr.RasterOptions(tile=tile, lds_batch=lds, sh_degree=0, flags=gsr.GSR_DEFAULT_FLAGS | gsr.GSR_PERSISTENT)
    pout = gpu_forward(R, t, cams, popts)
    for k in ref:
        assert torch.equal(pout[k], ref[k]), k
    pg_ = gpu_backward(R, t, cams, popts, pout, g_rgb, None, torch.full((1,), GAMMA, device=DEV))
    for k in KEYS:
        assert np.array_equal(pg_[k], gref[k]), k


def test_projection_backward_stagewise(R, tiny):
    scene, cams = tiny
    t, opts, out, target, g_rgb, grads = _tiny_backward(R, scene, cams)
    g2g = R.inspect(gsr.BUF_GRAD2D).reshape(scene.n, 9).astype(np.float64)
    g2d = dict(mean2d=g2g[:, 0:2], conic=g2g[:, 2:5], opacity=g2g[:, 5], rgb=g2g[:, 6:9])
    acc = orc.backward_project(scene, cams[0], g2d)
    for k in KEYS:
        check_grad(grads[k], acc[k], k)


def test_gradients_end_to_end_tiny(R, tiny):
    scene, cams = tiny
    t, opts, out, target, g_rgb, grads = _tiny_backward(R, scene, cams)
    L, g_o = oracle_grads(scene, cams, [target], GAMMA, (16, 16), out["rgb"].cpu().numpy())
    for k in KEYS:
        check_grad(grads[k], g_o[k], k)


def test_gradients_sh3_scene(R):
    """SH degree 3 and a rotated camera: exercises the colour -> direction chain."""
    scene = scenes.gmm_scene(31, 3000)
    scene.scales *= np.float32(4.0)
    cams = scenes.orbit_cameras(np.random.default_rng(32), [(160, 120)])
    t = to_dev(scene)
    opts = gsr.RasterOptions(tile=(16, 16), sh_degree=3)
    out = gpu_forward(R, t, cams, opts)
    target = scenes.target_image(33, 120, 160)
    g_rgb = l1_grad_torch(out["rgb"], target)
    g_le = torch.full((1,), 0.3, device=DEV)
    grads = gpu_backward(R, t, cams, opts, out, g_rgb, None, g_le)
    L, g_o = oracle_grads(scene, cams, [target], 0.3, (16, 16), out["rgb"].cpu().numpy())
    for k in KEYS:
        check_grad(grads[k], g_o[k], k)


# --------------------------------------------------------------------------- #
# batching, precision, graphs, autograd
# --------------------------------------------------------------------------- #

def _tiny_cams():
    from scipy.spatial.transform import Rotation
    out = []
    for (w, h, f, ang, tx) in [(128, 128, 128.0, 0.0, 0.0), (96, 64, 90.0, 0.08, 0.2), (50, 37, 40.0, -0.1, -0.1)]:
        Rm = Rotation.from_euler("y", ang).as_matrix().astype(np.float32)
        out.append(scenes.Camera(w, h, f, f, w / 2.0, h / 2.0, Rm, np.array([tx, 0.0, 0.1], np.float32), 0.2))
    return out


def test_batched_equals_plain(R, tiny):
    scene, _ = tiny
    cams = _tiny_cams()
    t = to_dev(scene)
    opts = gsr.RasterOptions(tile=(16, 16), sh_degree=0)
    ob = gpu_forward(R, t, cams, opts)
    g_rgb_b = torch.full_like(ob["rgb"], 1e-4)
    g_le_b = torch.full((3,), GAMMA, device=DEV)
    gb = gpu_backward(R, t, cams, opts, ob, g_rgb_b, None, g_le_b)
    off = gsr.pixel_offsets(cams)
    gsum = {k: np.zeros_like(v) for k, v in gb.items()}
    for v, cam in enumerate(cams):
        os_ = gpu_forward(R, t, [cam], opts)
        for k in ("rgb", "entropy", "t_final", "n_contrib"):
            assert torch.equal(ob[k][off[v]:off[v + 1]], os_[k]), (v, k)
        assert torch.equal(ob["entropy_mean"][v:v + 1], os_["entropy_mean"])
        gv = gpu_backward(R, t, [cam], opts, os_, torch.full_like(os_["rgb"], 1e-4), None,
                          torch.full((1,), GAMMA, device=DEV))
        for k in gsum:
            gsum[k] += gv[k]
    for k in gsum:
        assert rel_norm(gb[k], gsum[k]) < 1e-5, k


def test_many_views_one_launch_equals_per_view(tiny):
    """More views than the projection kernels stage in LDS at once (16): 20 views in one
    launch give bit-identical images and the summed per-view gradients."""
    from scipy.spatial.transform import Rotation
    scene, _ = tiny
    cams = []
    for k in range(20):
        w, h = (64, 48) if k % 2 else (48, 40)
        Rm = Rotation.from_euler("y", -0.2 + 0.02 * k).as_matrix().astype(np.float32)
        cams.append(scenes.Camera(w, h, 60.0, 60.0, w / 2.0, h / 2.0, Rm,
                                  np.array([0.01 * k - 0.1, 0.0, 0.1], np.float32), 0.2))
    G = gsr.Rasterizer(max_views=len(cams))
    t = to_dev(scene)
    opts = gsr.RasterOptions(tile=(16, 16), sh_degree=0)
    ob = gpu_forward(G, t, cams, opts)
    gb = gpu_backward(G, t, cams, opts, ob, torch.full_like(ob["rgb"], 1e-4), None,
                      torch.full((len(cams),), GAMMA, device=DEV))
    off = gsr.pixel_offsets(cams)
    gsum = {k: np.zeros_like(v) for k, v in gb.items()}
    for v, cam in enumerate(cams):
        os_ = gpu_forward(G, t, [cam], opts)
        for k in ("rgb", "entropy", "t_final", "n_contrib"):
            assert torch.equal(ob[k][off[v]:off[v + 1]], os_[k]), (v, k)
        gv = gpu_backward(G, t, [cam], opts, os_, torch.full_like(os_["rgb"], 1e-4), None,
                          torch.full((1,), GAMMA, device=DEV))
        for k in gsum:
            gsum[k] += gv[k]
    for k in gsum:
        assert rel_norm(gb[k], gsum[k]) < 1e-5, k


def test_batched_views_vs_oracle(R, tiny):
    scene, _ = tiny
    cams = _tiny_cams()
    t = to_dev(scene)
    opts = gsr.RasterOptions(tile=(8, 8), sh_degree=0)
    out = gpu_forward(R, t, cams, opts)
    recs = gpu_records(R, scene.n, len(cams))
    for v, cam in enumerate(cams):
        img_o = oracle_stagewise(recs[v], cam, (8, 8))
        _cmp_image(out, img_o, cam, v, cams)


def test_bf16_sh_storage(R):
    scene = scenes.gmm_scene(41, 20000)
    scene.sh = scenes.bf16_round(scene.sh)
    scene.scales *= np.float32(2.0)
    cams = scenes.orbit_cameras(np.random.default_rng(42), [(256, 192)])
    t = to_dev(scene, bf16=True)
    opts = gsr.RasterOptions(tile=(16, 16), sh_degree=3, sh_bf16=True)
    out = gpu_forward(R, t, cams, opts)
    pg = gpu_records(R, scene.n, 1)[0]
    img_o = oracle_stagewise(pg, cams[0], (16, 16))
    _cmp_image(out, img_o, cams[0])
    f = orc.forward_view(scene, cams[0], (16, 16))          # oracle on the bf16-rounded SH
    ok = f["flags"] == 0
    rgb = out["rgb"].cpu().numpy().reshape(192, 256, 3)
    assert np.abs(rgb - f["rgb"])[ok].max() <= 1e-4
    target = scenes.target_image(43, 192, 256)
    g_rgb = l1_grad_torch(out["rgb"], target)
    grads = gpu_backward(R, t, cams, opts, out, g_rgb, None, torch.full((1,), GAMMA, device=DEV))
    L, g_o = oracle_grads(scene, cams, [target], GAMMA, (16, 16), out["rgb"].cpu().numpy())
    for k in ("means", "scales", "quats", "opacities"):
        check_grad(grads[k], g_o[k], k)
    # SH gradients are stored in bfloat16: within 1 bf16 ulp of bf16(g*) where g* is well away from zero
    gs, go = grads["sh"], g_o["sh"]
    ref = scenes.bf16_round(go.astype(np.float32)).astype(np.float64)
    big = np.abs(go) > 1e-3 * np.abs(go).max()
    ulp = np.abs(ref) * 2.0 ** -7
    assert np.all(np.abs(gs - ref)[big] <= ulp[big] * 1.01 + 1e-12)
    assert rel_norm(gs, go) < 5e-3


def test_graph_mode_replays_match_plain(R, tiny):
    scene, cams = tiny
    t = to_dev(scene)
    plain = gsr.RasterOptions(tile=(16, 16), sh_degree=0)
    ref = gpu_forward(R, t, cams, plain)
    g_rgb = torch.full_like(ref["rgb"], 2e-5)
    g_le = torch.full((1,), GAMMA, device=DEV)
    gref = gpu_backward(R, t, cams, plain, ref, g_rgb, None, g_le)
    G = gsr.Rasterizer(max_views=2)
    graph = gsr.RasterOptions(tile=(16, 16), sh_degree=0, flags=gsr.GSR_DEFAULT_FLAGS | gsr.GSR_GRAPH)
    outs = dict(rgb=torch.empty_like(ref["rgb"]), entropy=torch.empty_like(ref["entropy"]))
    for rep in range(4):
        o = G.forward(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], cams, graph)
        gg = G.backward(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], cams, graph, o, g_rgb, None, g_le)
        torch.cuda.synchronize()
        _ = (torch.randn(1000, device=DEV) * 2).sum().item()    # unrelated eager work between replays
        for k in ("rgb", "entropy", "t_final", "n_contrib", "entropy_mean"):
            assert torch.equal(o[k], ref[k]), (rep, k)
        for k in KEYS:
            assert rel_norm(gg[k].cpu().numpy(), gref[k]) < 1e-5, (rep, k)
        st = G.stats(1)
        assert not st["overflow"]
    G.close()


def test_no_sync_mode_matches_plain_and_grows(R, tiny):
    """GSR_NO_SYNC: eager launches at a fixed pair capacity give the plain mode's outputs
    bit for bit and its gradients, with stage timing; a frame past the capacity is flagged
    as an overflow and the next frame runs at a grown capacity."""
    scene, cams = tiny
    t = to_dev(scene)
    plain = gsr.RasterOptions(tile=(16, 16), sh_degree=0)
    ref = gpu_forward(R, t, cams, plain)
    p_small = R.stats(1)["pairs"]
    g_rgb = torch.full_like(ref["rgb"], 2e-5)
    g_le = torch.full((1,), GAMMA, device=DEV)
    gref = gpu_backward(R, t, cams, plain, ref, g_rgb, None, g_le)
    big = dict(t)
    big["scales"] = (t["scales"] * 6.0).contiguous()
    ref_big = gpu_forward(R, big, cams, plain)
    p_big = R.stats(1)["pairs"]
    assert p_big > 1.5 * p_small + 4096
    gref_big = gpu_backward(R, big, cams, plain, ref_big, g_rgb, None, g_le)
    G = gsr.Rasterizer(max_views=1)
    G.set_timing(True)
    ns = gsr.RasterOptions(tile=(16, 16), sh_degree=0, flags=gsr.GSR_DEFAULT_FLAGS | gsr.GSR_NO_SYNC)
    for rep in range(3):                          # the first frame sizes the capacity, the others do not wait
        o = G.forward(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], cams, ns)
        gg = G.backward(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], cams, ns, o, g_rgb, None, g_le)
        torch.cuda.synchronize()
        for k in ("rgb", "entropy", "t_final", "n_contrib", "entropy_mean"):
            assert torch.equal(o[k], ref[k]), (rep, k)
        for k in KEYS:
            assert rel_norm(gg[k].cpu().numpy(), gref[k]) < 1e-6, (rep, k)
        assert not G.stats(1)["overflow"]
    times = G.stage_times()
    assert times["blend_fwd"][1] == 3 and times["blend_bwd"][1] == 3 and times["blend_bwd"][0] > 0
    # six times the scales: more pairs than the capacity the small frames set
    o = G.forward(big["means"], big["scales"], big["quats"], big["opacities"], big["sh"], cams, ns)
    assert G.stats(1)["overflow"]
    for rep in range(2):
        o = G.forward(big["means"], big["scales"], big["quats"], big["opacities"], big["sh"], cams, ns)
        gg = G.backward(big["means"], big["scales"], big["quats"], big["opacities"], big["sh"], cams, ns, o, g_rgb,
                        None, g_le)
        torch.cuda.synchronize()
        st = G.stats(1)
        assert not st["overflow"] and st["pairs"] == p_big, rep
        for k in ("rgb", "entropy", "t_final", "n_contrib", "entropy_mean"):
            assert torch.equal(o[k], ref_big[k]), (rep, k)
        for k in KEYS:
            assert rel_norm(gg[k].cpu().numpy(), gref_big[k]) < 1e-6, (rep, k)
    G.close()


def test_autograd_function_matches_raw(R, tiny):
    scene, cams = tiny
    t = {k: v.clone().requires_grad_(True) for k, v in to_dev(scene).items()}
    opts = gsr.RasterOptions(tile=(16, 16), sh_degree=0)
    rgb, ent, em = gsr.render(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], cams, opts, R)
    target = scenes.target_image(101, 128, 128)
    loss = (rgb - torch.from_numpy(target.reshape(-1, 3)).to(DEV)).abs().mean() + GAMMA * em.sum()
    loss.backward()
    L, g_o = oracle_grads(scene, cams, [target], GAMMA, (16, 16), rgb.detach().cpu().numpy())
    assert abs(float(loss.detach()) - L) < 1e-5
    for k in KEYS:
        check_grad(t[k].grad.cpu().numpy(), g_o[k], k)


def test_autograd_vs_central_fd_of_fp64_oracle(R, tiny):
    """GPU autograd gradient against central finite differences (eps 1e-4) of the
    FP64 oracle loss, on 64 seeded Gaussians; probes that cross a discrete
    decision (list, skip, stop, clamp, L1 sign) are redrawn."""
    scene, cams = tiny
    t = {k: v.clone().requires_grad_(True) for k, v in to_dev(scene).items()}
    opts = gsr.RasterOptions(tile=(16, 16), sh_degree=0)
    target = scenes.target_image(101, 128, 128)
    gamma = 0.5
    rgb, ent, em = gsr.render(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], cams, opts, R)
    loss = (rgb - torch.from_numpy(target.reshape(-1, 3)).to(DEV)).abs().mean() + gamma * em.sum()
    loss.backward()
    grads = {k: t[k].grad.cpu().numpy().astype(np.float64) for k in KEYS}
    rng = np.random.default_rng(505)
    cam = cams[0]

    def loss_sig(sc):
        f = orc.forward_view(sc, cam, (16, 16))
        L = float(np.abs(f["rgb"] - target).mean()) + gamma * f["L_E"]
        return L, (f["sig"], f["values"].tobytes(), f["proj"]["mask"].tobytes(),
                   np.sign(f["rgb"] - target).astype(np.int8).tobytes())

    sc = scene.copy()
    checked = redrawn = 0
    for g in rng.choice(scene.n, 64, replace=False):
        for name in ("means", "scales", "opacities"):
            flat = getattr(sc, name).reshape(sc.n, -1)
            j = int(rng.integers(flat.shape[1]))
            x0 = flat[g, j]
            eps = 1e-4 * (abs(float(x0)) if name == "scales" else max(1.0, abs(float(x0))))
            xp, xm = np.float32(x0 + eps), np.float32(x0 - eps)
            flat[g, j] = xp
            Lp, sp = loss_sig(sc)
            flat[g, j] = xm
            Lm, sm = loss_sig(sc)
            flat[g, j] = x0
            if sp != sm:
                redrawn += 1
                continue
            fd = (Lp - Lm) / (float(xp) - float(xm))
            an = grads[name].reshape(sc.n, -1)[g, j]
            scale = np.abs(grads[name]).max()
            assert abs(an - fd) <= 2e-3 * abs(fd) + 2e-4 * scale + 1e-9, (name, g, j, an, fd)
            checked += 1
    assert checked >= 100, (checked, redrawn)


# --------------------------------------------------------------------------- #
# the single-view workload at full size, sampled
# --------------------------------------------------------------------------- #

@pytest.mark.parametrize("bench_cfg", [(16, 16, 64)])
def test_single_view_full_size_sampled(R, bench_cfg):
    """200k Gaussians, 1296x840, SH3, in the bench's launch configuration: image,
    entropy, T on 2,000 seeded pixels; gradients of a loss restricted to those
    pixels against the oracle's gradient of the same loss."""
    tw, th, lds = bench_cfg
    scene, cams, _ = scenes.workload("single")
    cam = cams[0]
    t = to_dev(scene)
    opts = gsr.RasterOptions(tile=(tw, th), lds_batch=lds, sh_degree=3)
    out = gpu_forward(R, t, cams, opts)
    pg = gpu_records(R, scene.n, 1)[0]
    rng = np.random.default_rng(55)
    M = cam.width * cam.height
    sel = rng.choice(M, 2000, replace=False)
    pix = np.zeros(M, np.uint8)
    pix[sel] = 1
    img_o = oracle_stagewise(pg, cam, (tw, th), pix.reshape(cam.height, cam.width))
    ok = (img_o["flags"].reshape(-1) == 0) & (pix == 1)
    rgb = out["rgb"].cpu().numpy()
    assert np.abs(rgb - img_o["rgb"].reshape(-1, 3))[ok].max() <= IMG_TOL
    assert np.abs(out["entropy"].cpu().numpy() - img_o["H"].reshape(-1))[ok].max() <= IMG_TOL
    assert np.abs(out["t_final"].cpu().numpy() - img_o["T"].reshape(-1))[ok].max() <= IMG_TOL
    assert np.array_equal(out["n_contrib"].cpu().numpy()[ok], img_o["ncontrib"].reshape(-1)[ok])
    # masked loss: L1 on the sampled pixels + gamma * mean entropy over them
    target = scenes.target_image(202, cam.height, cam.width).reshape(-1, 3)
    g_rgb = np.zeros((M, 3))
    g_rgb[sel] = np.sign(rgb[sel] - target[sel]) / (3 * len(sel))
    g_H = np.zeros(M)
    g_H[sel] = GAMMA / len(sel)
    grads = gpu_backward(R, t, cams, opts, out, torch.from_numpy(g_rgb.astype(np.float32)).to(DEV),
                         torch.from_numpy(g_H.astype(np.float32)).to(DEV), None)
    g2o = orc.backward_render(cam.width, cam.height, tw, th, pg["mean2d"], pg["conic"], pg["opacity"], pg["rgb"],
                              img_o["ranges"], img_o["values"], g_rgb.reshape(cam.height, cam.width, 3),
                              g_H.reshape(cam.height, cam.width), pix.reshape(cam.height, cam.width))
    g2g = R.inspect(gsr.BUF_GRAD2D).reshape(scene.n, 9).astype(np.float64)
    check_grad2d(g2g, g2o)
    acc = orc.backward_project(scene, cam, g2o)
    for k in KEYS:
        check_grad(grads[k], acc[k], k)


# --------------------------------------------------------------------------- #
# statistics, edge cases, errors
# --------------------------------------------------------------------------- #

def test_stats_match_lists(R, tiny):
    scene, cams = tiny
    t = to_dev(scene)
    opts = gsr.RasterOptions(tile=(8, 8), sh_degree=0)
    out = gpu_forward(R, t, cams, opts)
    assert R.stats(1)["tested_bwd"] == 0                    # counted by the backward, which has not run
    g = torch.ones_like(out["rgb"]) / out["rgb"].numel()
    gpu_backward(R, t, cams, opts, out, g, torch.full_like(out["entropy"], 1e-3))
    st = R.stats(1)
    rg = R.inspect(gsr.BUF_RANGES).reshape(-1, 2).astype(np.int64)
    lens = np.sort(rg[:, 1] - rg[:, 0])
    assert st["pairs_per_view"][0] == lens.sum()
    assert abs(st["mean_len"] - lens.mean()) < 1e-9
    assert st["p99_len"] == lens[int(math.ceil(0.99 * len(lens))) - 1]
    assert not st["overflow"]
    # work counts against the oracle walking the same lists with the GPU's float32
    # records: alpha evaluations and blended (pixel, Gaussian) pairs; a pixel whose
    # skip/stop decision lies within the oracle's decision band may differ by its list
    c = cams[0]
    ref = oracle_stagewise(gpu_records(R, scene.n, 1)[0], c, (8, 8))
    gx = (c.width + 7) // 8
    tile_of = (np.arange(c.height)[:, None] // 8) * gx + np.arange(c.width)[None, :] // 8
    rr = np.asarray(ref["ranges"]).reshape(-1, 2)
    slack = int((rr[tile_of, 1] - rr[tile_of, 0])[ref["flags"] != 0].sum())
    assert abs(st["blended"] - ref["n_blend"]) <= slack
    assert abs(st["evals_fwd"] - ref["n_eval"]) <= slack
    assert 0 < st["blended"] <= st["evals_bwd"] <= st["evals_fwd"]
    # alpha tests the kernels make: positions that survive the block cull, a subset of the
    # visited ones; every blended entry is tested, and the backward tests no further than the
    # last contributor
    assert st["blended"] <= st["tested_bwd"] <= st["tested_fwd"] <= st["evals_fwd"]
    assert st["tested_bwd"] <= st["evals_bwd"]


def _single_gaussian_scene(means, scales, opac, n_extra=0):
    n = len(means)
    q = np.tile(np.array([[1, 0, 0, 0]], np.float32), (n, 1))
    sh = np.full((n, 1, 3), 0.8, np.float32)
    return scenes.Scene(np.asarray(means, np.float32), np.asarray(scales, np.float32), q,
                        np.asarray(opac, np.float32), sh, 0)


def _e2e(R, scene, cams, tile=(16, 16)):
    t = to_dev(scene)
    opts = gsr.RasterOptions(tile=tile, sh_degree=scene.sh_degree)
    out = gpu_forward(R, t, cams, opts)
    for v, cam in enumerate(cams):
        f = orc.forward_view(scene, cam, tile)
        _cmp_image(out, f, cam, v, cams)
    return t, opts, out


def test_edge_empty_scene(R):
    sc = _single_gaussian_scene(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0))
    cams = [scenes.Camera(64, 48, 50.0, 50.0, 32.0, 24.0, np.eye(3, dtype=np.float32), np.zeros(3, np.float32))]
    t, opts, out = _e2e(R, sc, cams)
    assert float(out["rgb"].abs().max()) == 0.0 and float(out["t_final"].min()) == 1.0
    assert float(out["entropy_mean"][0]) == 0.0
    assert not np.any(R.inspect(gsr.BUF_RANGES))                      # every tile [0, 0)
    g = gpu_backward(R, t, cams, opts, out, torch.ones_like(out["rgb"]), None, torch.ones(1, device=DEV))
    assert all(v.size == 0 for v in g.values())


def test_edge_all_culled_and_nan(R):
    cams = [scenes.Camera(64, 48, 50.0, 50.0, 32.0, 24.0, np.eye(3, dtype=np.float32), np.zeros(3, np.float32))]
    sc = _single_gaussian_scene([[0, 0, -3.0], [0, 0, 0.1], [np.nan, 0, 4.0], [0.1, 0.0, 4.0]],
                                [[0.1] * 3, [0.1] * 3, [0.1] * 3, [0.2] * 3], [0.9, 0.9, 0.9, 0.8])
    t, opts, out = _e2e(R, sc, cams)
    rad = R.inspect(gsr.BUF_RADIUS)
    assert list(rad[:3]) == [0, 0, 0] and rad[3] > 0
    # the one visible Gaussian's tiles hold one pair each, in tile order; the others are [0, 0)
    tt = int(R.inspect(gsr.BUF_TILES_TOUCHED)[3])
    rg = R.inspect(gsr.BUF_RANGES).reshape(-1, 2).astype(np.int64)
    hit = rg[:, 1] > rg[:, 0]
    assert hit.sum() == tt and np.all(rg[~hit] == 0)
    assert np.array_equal(rg[hit, 0], np.arange(tt)) and np.array_equal(rg[hit, 1], np.arange(1, tt + 1))
    assert list(R.inspect(gsr.BUF_PAIR_VALUES)) == [3] * tt
    assert np.array_equal(R.inspect(gsr.BUF_PAIR_TILES), np.nonzero(hit)[0])
    g = gpu_backward(R, t, cams, opts, out, torch.full_like(out["rgb"], 1e-3), None, torch.ones(1, device=DEV))
    assert np.all(g["means"][:3] == 0) and np.any(g["means"][3] != 0)


def test_edge_giant_gaussian_and_clamp(R):
    """One Gaussian covering every tile, alpha at the 0.99 clamp in its centre."""
    cams = [scenes.Camera(160, 96, 80.0, 80.0, 80.0, 48.0, np.eye(3, dtype=np.float32), np.zeros(3, np.float32))]
    sc = _single_gaussian_scene([[0.1, -0.05, 3.0], [0.2, 0.1, 5.0]], [[2.0, 1.5, 1.0], [0.05, 0.08, 0.03]],
                                [0.999, 0.7])
    sc.quats[:] = np.array([[0.9, 0.2, -0.3, 0.1], [0.5, -0.4, 0.6, 0.2]], np.float32)   # no symmetry
    t, opts, out = _e2e(R, sc, cams)
    assert R.inspect(gsr.BUF_TILES_TOUCHED)[0] == 10 * 6
    g = gpu_backward(R, t, cams, opts, out, torch.full_like(out["rgb"], 1e-3), None, torch.ones(1, device=DEV))
    target = np.zeros((96, 160, 3))
    # compare with the oracle for the same upstream gradients
    f = orc.forward_view(sc, cams[0], (16, 16))
    pr = f["proj"]
    g2 = orc.backward_render(160, 96, 16, 16, pr["mean2d"], pr["conic"], pr["opacity"], pr["rgb"], f["ranges"],
                             f["values"], np.full((96, 160, 3), 1e-3), np.full((96, 160), 1.0 / (160 * 96)))
    acc = orc.backward_project(sc, cams[0], g2)
    for k in KEYS:
        check_grad(g[k], acc[k], k)
    del target


@pytest.mark.parametrize("wh", [(100, 75), (37, 23), (1, 1), (17, 200)])
def test_edge_ragged_sizes(R, tiny, wh):
    scene, _ = tiny
    w, h = wh
    f = 128.0 * max(w, h) / 128.0
    cams = [scenes.Camera(w, h, f, f, w / 2.0, h / 2.0, np.eye(3, dtype=np.float32), np.zeros(3, np.float32))]
    for tile in [(16, 16), (32, 8)]:
        _e2e(R, scene, cams, tile)


def test_edge_equal_depths_keep_index_order(R):
    n = 6
    sc = _single_gaussian_scene(np.tile([[0.0, 0.0, 4.0]], (n, 1)), np.full((n, 3), 0.05), np.full(n, 0.3))
    cams = [scenes.Camera(32, 32, 40.0, 40.0, 16.0, 16.0, np.eye(3, dtype=np.float32), np.zeros(3, np.float32))]
    _e2e(R, sc, cams)
    vals = R.inspect(gsr.BUF_PAIR_VALUES)
    rg = R.inspect(gsr.BUF_RANGES).reshape(-1, 2)
    for t_ in range(len(rg)):
        assert list(vals[rg[t_, 0]:rg[t_, 1]]) == list(range(n))


def test_invalid_arguments_rejected(R, tiny):
    scene, cams = tiny
    t = to_dev(scene)
    bad = [gsr.RasterOptions(tile=(16, 8), sh_degree=0), gsr.RasterOptions(tile=(16, 16), sh_degree=4),
           gsr.RasterOptions(tile=(16, 16), lds_batch=48, sh_degree=0)]
    for o in bad:
        K = (o.sh_degree + 1) ** 2
        sh = torch.zeros((scene.n, K, 3), device=DEV)
        with pytest.raises(gsr.GsrError) as e:
            R.forward(t["means"], t["scales"], t["quats"], t["opacities"], sh, cams, o)
        assert e.value.status == 2
    bad_cam = [scenes.Camera(0, 10, 1.0, 1.0, 0.0, 0.0, np.eye(3, dtype=np.float32), np.zeros(3, np.float32))]
    with pytest.raises(gsr.GsrError) as e:
        R.forward(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], bad_cam,
                  gsr.RasterOptions(sh_degree=0))
    assert e.value.status == 1
    opts = gsr.RasterOptions(tile=(16, 16), sh_degree=0)
    a = gpu_forward(R, t, cams, opts)
    gpu_forward(R, t, cams, opts)
    with pytest.raises(gsr.GsrError) as e:
        R.backward(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], cams, opts, a,
                   torch.zeros_like(a["rgb"]))
    assert e.value.status == 5


def test_fixed_capacity_overflow_is_reported(tiny):
    """A replayed forward whose pairs outgrow the capacity its graph was captured with
    (same pointers and sizes, every scale 8x larger in place) is flagged by gsr_stats, its
    backward is refused, and the next forward captures again at the new count."""
    scene, cams = tiny
    t = to_dev(scene)
    G = gsr.Rasterizer(max_views=1, pair_capacity=64)
    graph = gsr.RasterOptions(tile=(16, 16), sh_degree=0, flags=gsr.GSR_DEFAULT_FLAGS | gsr.GSR_GRAPH)
    args = (t["means"], t["scales"], t["quats"], t["opacities"], t["sh"])
    try:
        out = G.forward(*args, cams, graph)          # a capture sizes the capacity itself
        out = G.forward(*args, cams, graph, out=out)  # a replay
        assert not G.stats(1)["overflow"]
        t["scales"].mul_(8.0)
        out = G.forward(*args, cams, graph, out=out)
        assert G.stats(1)["overflow"]
        with pytest.raises(gsr.GsrError) as ei:
            G.backward(*args, cams, graph, out, torch.zeros_like(out["rgb"]))
        assert ei.value.status == 3
        out = G.forward(*args, cams, graph, out=out)
        assert not G.stats(1)["overflow"]
        G.backward(*args, cams, graph, out, torch.zeros_like(out["rgb"]))
        torch.cuda.synchronize()
    finally:
        G.close()


def test_autotune_picks_a_valid_shape(R, tiny, tmp_path):
    scene, cams = tiny
    t = to_dev(scene)
    opts = gsr.RasterOptions(tile=(16, 16), sh_degree=0)
    cache = str(tmp_path / "tune.txt")
    best = R.autotune(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], cams, opts, cache)
    assert best.tile in [(8, 8), (16, 16), (32, 8)] and best.lds_batch in (32, 64, 128, 256)
    # only the scheduling bit of the flags may change
    assert best.flags & ~gsr.GSR_PERSISTENT == opts.flags & ~gsr.GSR_PERSISTENT
    again = R.autotune(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], cams, opts, cache)
    assert again == best
    # the tuned options render
    gpu_forward(R, t, cams, best)


@pytest.mark.parametrize("tile,lds,persist", [((16, 16), 64, False), ((8, 8), 32, False), ((32, 8), 128, True)])
def test_render_only_matches_forward(R, tiny, tile, lds, persist):
    """gsr_render: the forward's colour bit for bit, the same work counts; it replaces the
    frame (a backward of the earlier forward is stale); graph mode is refused."""
    scene, cams = tiny
    t = to_dev(scene)
    flags = gsr.GSR_DEFAULT_FLAGS | (gsr.GSR_PERSISTENT if persist else 0)
    opts = gsr.RasterOptions(tile=tile, lds_batch=lds, sh_degree=0, flags=flags)
    out = gpu_forward(R, t, cams, opts)
    st_f = R.stats(1)
    rgb = R.render_image(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], cams, opts)
    torch.cuda.synchronize()
    assert torch.equal(rgb, out["rgb"])
    st_r = R.stats(1)
    for k in ("pairs", "evals_fwd", "evals_bwd", "blended"):
        assert st_r[k] == st_f[k], k
    g_rgb = l1_grad_torch(out["rgb"], scenes.target_image(101, 128, 128))
    with pytest.raises(gsr.GsrError) as ei:
        R.backward(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], cams, opts, out, g_rgb, None, None)
    assert ei.value.status == 5                                  # GSR_ERR_STALE_FRAME
    with pytest.raises(gsr.GsrError) as ei:
        R.render_image(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], cams,
                       gsr.RasterOptions(tile=tile, lds_batch=lds, sh_degree=0, flags=flags | gsr.GSR_GRAPH))
    assert ei.value.status == 2                                  # GSR_ERR_UNSUPPORTED


def test_render_only_single_view_full_size(R):
    scene, cams, _ = scenes.workload("single")
    t = to_dev(scene)
    opts = gsr.RasterOptions(tile=(16, 16), lds_batch=128, sh_degree=3)
    out = gpu_forward(R, t, cams, opts)
    rgb = R.render_image(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], cams, opts)
    torch.cuda.synchronize()
    assert torch.equal(rgb, out["rgb"])


def test_l1_loss_entry_point(R):
    """gsr_l1_loss on packed views of uneven size: gradient sign/(3 M_v) exactly, loss per view."""
    scene, _, _ = scenes.workload("tiny")
    cams = _tiny_cams()
    t = to_dev(scene)
    out = gpu_forward(R, t, cams, gsr.RasterOptions(tile=(16, 16), sh_degree=0))
    tg = np.concatenate([scenes.target_image(7 + v, c.height, c.width).reshape(-1, 3) for v, c in enumerate(cams)])
    tg[5] = out["rgb"][5].cpu().numpy()               # one exact tie: sign(0) = 0
    target = torch.from_numpy(tg).to(DEV)
    grad, loss = R.l1_loss(cams, out["rgb"], target)
    torch.cuda.synchronize()
    rgb = out["rgb"].cpu().numpy()
    off = gsr.pixel_offsets(cams)
    for v, c in enumerate(cams):
        M = c.width * c.height
        d = rgb[off[v]:off[v + 1]] - tg[off[v]:off[v + 1]]
        exp_g = (np.sign(d) * np.float32(1.0 / (3.0 * M))).astype(np.float32)
        assert np.array_equal(grad.cpu().numpy()[off[v]:off[v + 1]], exp_g)
        assert abs(float(loss[v]) - np.abs(d.astype(np.float64)).mean()) <= 1e-6 * np.abs(d).mean()
    assert float(grad[5].abs().sum()) == 0.0


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8)])
def test_gradients_bit_reproducible(R, tile):
    """The backward uses no float atomics: two runs give bit-identical gradients."""
    scene = scenes.gmm_scene(61, 8000)
    scene.scales *= np.float32(2.0)
    cams = scenes.orbit_cameras(np.random.default_rng(62), [(200, 150), (120, 90)])
    t = to_dev(scene)
    opts = gsr.RasterOptions(tile=tile, sh_degree=3)
    res = []
    for _ in range(2):
        out = gpu_forward(R, t, cams, opts)
        g_rgb = torch.full_like(out["rgb"], 1e-4)
        g = R.backward(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], cams, opts, out, g_rgb, None,
                       torch.full((2,), GAMMA, device=DEV))
        torch.cuda.synchronize()
        res.append({k: v.clone() for k, v in g.items()})
    for k in KEYS:
        assert torch.equal(res[0][k], res[1][k]), k


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8)])
def test_persistent_mode_matches_plain_bit_exactly(R, tile):
    """Persistent blend kernels (tiles pulled from per-XCD device queues, with stealing) give
    bit-identical outputs and gradients, on uneven views."""
    scene = scenes.gmm_scene(71, 10000)
    scene.scales *= np.float32(1.5)
    cams = scenes.orbit_cameras(np.random.default_rng(72), [(243, 162), (486, 324), (97, 65)])
    t = to_dev(scene)
    res = []
    for flags in (gsr.GSR_DEFAULT_FLAGS, gsr.GSR_DEFAULT_FLAGS | gsr.GSR_PERSISTENT):
        opts = gsr.RasterOptions(tile=tile, sh_degree=3, flags=flags)
        out = gpu_forward(R, t, cams, opts)
        g = R.backward(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], cams, opts, out,
                       torch.full_like(out["rgb"], 1e-4), None, torch.full((3,), GAMMA, device=DEV))
        torch.cuda.synchronize()
        res.append(({k: out[k].clone() for k in ("rgb", "entropy", "t_final", "n_contrib", "entropy_mean")},
                    {k: v.clone() for k, v in g.items()}, R.stats(3)))
    for k in res[0][0]:
        assert torch.equal(res[0][0][k], res[1][0][k]), k
    for k in KEYS:
        assert torch.equal(res[0][1][k], res[1][1][k]), k
    assert res[0][2]["evals_fwd"] == res[1][2]["evals_fwd"]


def test_persistent_graph_batched_vs_oracle(R):
    """The batched form (several uneven views, BF16 SH, persistent kernels, graph replay)
    against the oracle on every view."""
    scene = scenes.gmm_scene(81, 6000)
    scene.sh = scenes.bf16_round(scene.sh)
    cams = scenes.orbit_cameras(np.random.default_rng(82), [(122, 81), (122, 81), (243, 162), (486, 324)])
    t = to_dev(scene, bf16=True)
    G = gsr.Rasterizer(max_views=4)
    opts = gsr.RasterOptions(tile=(16, 16), sh_degree=3, sh_bf16=True,
                             flags=gsr.GSR_DEFAULT_FLAGS | gsr.GSR_GRAPH | gsr.GSR_PERSISTENT)
    out = None
    for _ in range(3):
        out = G.forward(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], cams, opts, out=out)
        torch.cuda.synchronize()
    recs = gpu_records(G, scene.n, len(cams))
    for v, cam in enumerate(cams):
        img_o = oracle_stagewise(recs[v], cam, (16, 16))
        _cmp_image(out, img_o, cam, v, cams)
    assert not G.stats(len(cams))["overflow"]
    G.close()


# --------------------------------------------------------------------------- #
# next rows: opacity regulariser, scale reset, r_max policy
# --------------------------------------------------------------------------- #

def test_opacity_loss_vs_oracle(R):
    rng = np.random.default_rng(31)
    op = rng.uniform(0.0, 1.0, 100_003).astype(np.float32)
    w = 3.0
    L_o, g_o = orc.opacity_loss(op, w)
    t = torch.from_numpy(op).to(DEV)
    base = rng.normal(0, 1e-3, op.shape).astype(np.float32)
    grad = torch.from_numpy(base).to(DEV)
    loss = R.opacity_loss(t, w, grad)
    loss2 = R.opacity_loss(t, w)                     # no gradient
    torch.cuda.synchronize()
    assert abs(float(loss.cpu()[0]) - L_o) <= 1e-6 * abs(L_o)
    assert float(loss2.cpu()[0]) == float(loss.cpu()[0])   # fixed-order sum
    got = grad.cpu().numpy().astype(np.float64) - base.astype(np.float64)
    assert rel_norm(got, g_o) < 1e-5


@pytest.mark.parametrize("graph", [False, True])
def test_opacity_regulariser_fused_into_projection_backward(R, tiny, graph):
    """gsr_backward_opacity_reg: the opacity gradient equals gsr_backward's followed by
    gsr_opacity_loss bit for bit, the other gradients equal gsr_backward's, and L_O matches
    the separate pass and the oracle."""
    scene, cams = tiny
    t = to_dev(scene)
    flags = gsr.GSR_DEFAULT_FLAGS | (gsr.GSR_GRAPH if graph else 0)
    opts = gsr.RasterOptions(tile=(16, 16), sh_degree=0, flags=flags)
    out = R.forward(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], cams, opts)
    g_rgb = l1_grad_torch(out["rgb"], scenes.target_image(101, 128, 128))
    g_le = torch.full((1,), GAMMA, device=DEV)
    ref = R.backward(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], cams, opts, out, g_rgb, None, g_le)
    ref = {k: v.clone() for k, v in ref.items()}
    loss_sep = R.opacity_loss(t["opacities"], 3.0, ref["opacities"])
    loss_f = torch.zeros(1, device=DEV)
    fused = {k: torch.empty_like(v) for k, v in t.items()}
    for _ in range(2 if graph else 1):                 # capture, then a replay
        R.backward(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], cams, opts, out, g_rgb, None, g_le,
                   fused, opacity_weight=3.0, opacity_loss=loss_f)
        torch.cuda.synchronize()
        for k in KEYS:
            assert torch.equal(fused[k], ref[k]), k
        L_want, _ = orc.opacity_loss(scene.opacities, 3.0)
        assert abs(float(loss_f[0]) - float(loss_sep[0])) <= 1e-6 * float(loss_sep[0])
        assert abs(float(loss_f[0]) - L_want) <= 1e-6 * L_want


@pytest.mark.parametrize("name,tile", [("tiny", (16, 16)), ("single", (16, 16)), ("single", (8, 8)),
                                       ("sweep_half", (32, 8))])
def test_debug_invariants_weights_sum_to_one(R, name, tile):
    """GSR_DEBUG_INVARIANTS: every pixel's blending weights plus T_final sum to one (Eq. 9)
    within the FP32 bound of its walk; the images are those of an unchecked forward."""
    scene, cams, _ = scenes.workload(name)
    t = to_dev(scene)
    opts = gsr.RasterOptions(tile=tile, lds_batch=128, sh_degree=scene.sh_degree)
    chk = gsr.RasterOptions(tile=tile, lds_batch=128, sh_degree=scene.sh_degree,
                            flags=gsr.GSR_DEFAULT_FLAGS | gsr.GSR_DEBUG_INVARIANTS)
    ref = gpu_forward(R, t, cams, opts)
    ref = {k: ref[k].clone() for k in ("rgb", "entropy", "t_final", "n_contrib")}
    assert R.stats(1)["invariant_violations"] == -1            # not checked
    out = gpu_forward(R, t, cams, chk)
    st = R.stats(1)
    nmax = int(out["n_contrib"].max())
    assert st["invariant_violations"] == 0, st
    assert 0.0 <= st["invariant_max_err"] <= 4 * 2.0 ** -24 * (nmax + 1), (st["invariant_max_err"], nmax)
    for k in ref:
        assert torch.equal(out[k], ref[k]), k


def test_scale_reset_bit_exact(R):
    scene = scenes.gmm_scene(32, 50_000)
    s = torch.from_numpy(scene.scales.copy()).to(DEV)
    R.scale_reset(s, 0.2)
    torch.cuda.synchronize()
    assert np.array_equal(s.cpu().numpy(), orc.scale_reset(scene.scales, 0.2))


def test_pair_counts_and_rmax_vs_oracle(R):
    """Per-view pair counts equal the oracle's count on the GPU's records bit for bit,
    and r_max follows the rule on them (and on the oracle's own FP64 projection)."""
    scene = scenes.gmm_scene(11, 30_000)
    t = to_dev(scene)
    cam = scenes.orbit_cameras(np.random.default_rng(12), [(1296, 840)])[0]
    opts = gsr.RasterOptions(tile=(16, 16), sh_degree=3)
    counts = []
    for r in range(1, 5):
        k = gsr.scaled_camera(cam, r)
        ko = orc.scaled_camera(cam, r)
        assert (k.width, k.height, k.fx, k.fy, k.cx, k.cy) == (ko.width, ko.height, ko.fx, ko.fy, ko.cx, ko.cy)
        (p,) = R.pair_counts(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], [k], opts)
        pg = gpu_records(R, scene.n, 1)[0]
        total, _, _ = orc.count_pairs(pg["mean2d"], pg["radius"], k.width, k.height, 16, 16)
        assert p == total
        counts.append(p)
    thr = float(np.median([c / (((1296 // r + 15) // 16) * ((840 // r + 15) // 16))
                           for r, c in zip(range(1, 5), counts)]))
    r_gpu, means = R.select_rmax(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], cam, opts, 4, thr)
    exp = [c / (((1296 // r + 15) // 16) * ((840 // r + 15) // 16)) for r, c in zip(range(1, 5), counts)]
    assert np.allclose(means, exp, rtol=0, atol=0)
    ok = [r for r, m in zip(range(1, 5), exp) if m <= thr]
    assert r_gpu == (max(ok) if ok else 1)
    r_o, counts_o = orc.select_rmax(scene, cam, (16, 16), 4, thr)
    assert r_o == r_gpu
    assert all(abs(a - b) <= 2e-4 * b for a, b in zip(counts, counts_o))
