"""The allocation-free L1 entry point (gsr_l1_loss_noalloc) against gsr_l1_loss.

Both run the same kernels on the same images; the variant keeps its per-block
partial sums in the library's static device array instead of context memory,
so gradients and per-view losses must be bit-identical.  Two calls in a row,
the second on fewer and smaller views (the array keeps the first call's
contents), and a third after a call of the allocating entry point.
"""
import numpy as np
import pytest
import torch

from paper_2603_09277_amd import gsr, scenes

from gpu_helpers import DEV, to_dev

pytestmark = pytest.mark.gpu


def _case(R, t, cams, sh_degree, seed):
    opts = gsr.RasterOptions(tile=(16, 16), lds_batch=64, sh_degree=sh_degree)
    out = R.forward(t["means"], t["scales"], t["quats"], t["opacities"], t["sh"], cams, opts)
    rng = np.random.default_rng(seed)
    P = out["rgb"].shape[0]
    target = torch.from_numpy(rng.uniform(0, 1, (P, 3)).astype(np.float32)).to(DEV)
    # a few targets equal to the image: sign(0) = 0 must come out of both
    target[::97] = out["rgb"][::97]
    g_ref, l_ref = R.l1_loss(cams, out["rgb"], target)
    g_na = torch.full_like(g_ref, float("nan"))
    l_na = torch.full_like(l_ref, float("nan"))
    R.l1_loss_noalloc(cams, out["rgb"], target, g_na, l_na)
    torch.cuda.synchronize()
    assert torch.equal(g_na, g_ref)
    assert torch.equal(l_na, l_ref)
    assert torch.isfinite(l_ref).all() and (l_ref > 0).all()
    return l_ref


def test_noalloc_l1_matches_allocating_entry_point():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    R = gsr.Rasterizer(max_views=8)
    try:
        scene = scenes.gmm_scene(201, 40000)
        t = to_dev(scene)
        big = scenes.orbit_cameras(np.random.default_rng(202), [(972, 648), (486, 324), (640, 480)])
        small = scenes.orbit_cameras(np.random.default_rng(203), [(123, 77)])
        _case(R, t, big, 3, 204)                    # first call
        _case(R, t, small, 3, 205)                  # second call, smaller: the array holds the first call's sums
        _case(R, t, big[:2], 3, 206)                # again after the allocating entry point ran
    finally:
        R.close()
