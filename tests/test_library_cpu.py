"""Host-side checks of the C-ABI library and the input generator (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest
import torch

from paper_2603_09277_amd import gsr, scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    with open(os.path.join(ROOT, "include", "gsr.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gsr_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 12
    lib = ctypes.CDLL(gsr.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(names) == sorted(gsr.EXPORTED)


def test_host_only_entry_points():
    lib = gsr.lib()
    assert lib.gsr_status_string(0) == b"ok"
    assert lib.gsr_status_string(3) == b"pair capacity exceeded"
    _, cams, _ = scenes.workload("tiny")
    cams2 = cams + [scenes.Camera(7, 5, 1.0, 1.0, 0.0, 0.0, np.eye(3, dtype=np.float32), np.zeros(3, np.float32))]
    assert gsr.pixel_offsets(cams2) == [0, 128 * 128, 128 * 128 + 35]
    assert lib.gsr_pixel_offsets(None, 1, None) == 1
    assert lib.gsr_destroy(None) == 1
    assert lib.gsr_last_error(None) == b"null context"


@pytest.mark.skipif(torch.cuda.is_available(), reason="checks behaviour without a GPU")
def test_create_without_gpu_reports_hip_error():
    ctx = ctypes.c_void_p()
    assert gsr.lib().gsr_create(ctypes.byref(ctx), 4, 0) == 4
    assert not ctx.value


def test_invalid_create_arguments():
    ctx = ctypes.c_void_p()
    assert gsr.lib().gsr_create(ctypes.byref(ctx), 0, 0) == 1
    assert gsr.lib().gsr_create(ctypes.byref(ctx), 65, 0) == 1
    assert gsr.lib().gsr_create(ctypes.byref(ctx), 4, -1) == 1


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(gsr, "_lib", None)
    monkeypatch.setattr(gsr, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="missing"):
        gsr.lib()


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(100_000) * np.exp(rng.uniform(-20, 20, 100_000))).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(scenes.bf16_round(x), ref)


def test_generators_are_seeded():
    a, ca, _ = scenes.workload("tiny")
    b, cb, _ = scenes.workload("tiny")
    for k in ("means", "scales", "quats", "opacities", "sh"):
        assert np.array_equal(getattr(a, k), getattr(b, k))
    g1 = scenes.gmm_scene(3, 1000)
    g2 = scenes.gmm_scene(3, 1000)
    assert np.array_equal(g1.sh, g2.sh)
    cams = scenes.orbit_cameras(np.random.default_rng(1), [(100, 80)])
    R = cams[0].R.astype(np.float64)
    assert np.allclose(R @ R.T, np.eye(3), atol=1e-6)
    # the camera looks at the origin: the world origin projects to the principal point
    t = cams[0].t.astype(np.float64)
    assert abs(t[0]) < 1e-5 and abs(t[1]) < 1e-5 and t[2] > 0


def test_oracle_baseline_in_processes_matches_its_record():
    """bench.py's P-process oracle timing: every process takes a disjoint stripe of the
    same seeded pixel sample, and the record states the process count it used."""
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    scene, cams, _ = scenes.workload("tiny")
    sel = bench._pixel_sample(cams[0], 0.5, 77, 0)
    stripes = [sel[i::3] for i in range(3)]
    assert sum(len(x) for x in stripes) == len(sel)
    assert len(np.unique(np.concatenate(stripes))) == len(sel)
    rec = bench.cpu_baseline_processes("tiny", False, cams, (16, 16), views=[0], frac=0.5, procs=2)
    assert rec["cores"] == 2 and rec["kind"] == "oracle" and rec["unit"] == "iters/s"
    assert rec["value"] > 0 and "2 processes" in rec["sample"]
