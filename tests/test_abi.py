"""The C ABI library loads and exports every symbol include/*.h declares;
host-only entry points and argument checks work without a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("gsr.h", "gsr_scorer.h")]


def _lib():
    from paper_2403_11367_amd import build, gsr  # noqa: F401
    return gsr


@pytest.fixture(scope="module")
def gsr():
    try:
        from paper_2403_11367_amd import gsr as g
    except ImportError:
        from paper_2403_11367_amd import build
        build.build()
        from paper_2403_11367_amd import gsr as g
    return g


def _declared():
    import glob
    assert sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))) == sorted(HEADERS)
    src = "".join(open(h).read() for h in HEADERS)
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gsr_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ["gsr_create", "gsr_submap_load", "gsr_render", "gsr_ncc", "gsr_topk", "gsr_crop",
                 "gsr_scorer_create", "gsr_scorer_forward", "gsr_scorer_backward", "gsr_scorer_train_step"]:
        assert must in names


def test_every_declared_symbol_is_exported(gsr):
    names = _declared()
    assert sorted(gsr.EXPORTS) == names
    for n in names:
        assert hasattr(gsr.LIB, n), n


def test_exported_dynamic_symbols_match(gsr):
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", gsr.LIB_PATH], capture_output=True, text=True).stdout
    exported = sorted(set(re.findall(r" T (gsr_\w+)", out)))
    assert exported == _declared()


def test_status_strings(gsr):
    assert gsr.LIB.gsr_status_string(0) == b"ok"
    assert gsr.LIB.gsr_status_string(-5) == b"pair buffer overflow"


def test_default_cfg_values(gsr):
    c = gsr.default_cfg()
    assert (c.tile_w, c.tile_h) == (16, 16)
    assert c.eps_dilate == np.float32(0.3) and c.z_near == np.float32(0.2) and c.jac_clamp == np.float32(1.3)
    assert c.cutoff_d2 == 9.0 and c.alpha_max == np.float32(0.99) and c.t_min == np.float32(1e-4)
    assert c.alpha_min == np.float32(1.0 / 255.0) and c.pair_capacity == 0 and c.pose_groups == 0


def test_create_without_gpu_reports_enodev(gsr):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    assert gsr.LIB.gsr_create(C.byref(h), 0, None) == -4
    assert gsr.LIB.gsr_create(None, 0, None) == -1


def test_null_context_is_einval(gsr):
    assert gsr.LIB.gsr_sync(None) == -1
    assert gsr.LIB.gsr_render(None, None, None, None, 1, None, None, None, None) == -1
    assert gsr.LIB.gsr_ncc(None, None, None, 1, 1, 1, None) == -1
    assert gsr.LIB.gsr_default_cfg(None) == -1


def test_native_crop_matches_oracle_on_config1(gsr):
    import workloads as W
    from oracle import crop as ocrop
    sc = W.config1()
    for voxel in (sc.crop_voxel, 0.0, 0.25):
        got = gsr.crop(sc.gaussians.means, sc.crop_cell, sc.prior_center[:2], sc.crop_radius, voxel)
        ref = ocrop.crop_indices(sc.gaussians.means, sc.crop_cell, sc.prior_center[:2], sc.crop_radius, voxel)
        assert np.array_equal(got, ref)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_native_crop_matches_oracle_random(gsr, seed):
    from oracle import crop as ocrop
    rng = np.random.default_rng(seed)
    means = rng.uniform([-100, -80, 0], [100, 80, 3], size=(30000, 3)).astype(np.float32)
    cx, cy = rng.uniform(-50, 50, 2)
    r = float(rng.uniform(5, 70))
    cell = float(rng.choice([1.0, 2.5, 10.0]))
    for voxel in (0.0, 1.0, 3.0):
        got = gsr.crop(means, cell, (cx, cy), r, voxel)
        ref = ocrop.crop_indices(means, cell, (cx, cy), r, voxel)
        assert np.array_equal(got, ref)


def test_native_crop_edge_cases(gsr):
    empty = np.zeros((0, 3), np.float32)
    assert gsr.crop(empty, 10.0, (0, 0), 50.0).size == 0
    m = np.array([[1, 1, 0], [np.nan, 0, 0], [500, 500, 0], [2, 2, np.nan], [3, 1, 0]], np.float32)
    from oracle import crop as ocrop
    assert gsr.crop(m, 10.0, (0, 0), 20.0).tolist() == ocrop.crop_indices(m, 10.0, (0, 0), 20.0).tolist()
    assert sorted(gsr.crop(m, 10.0, (0, 0), 20.0).tolist()) == [0, 3, 4]
    with pytest.raises(gsr.GsrError):
        gsr.crop(m, 0.0, (0, 0), 20.0)
    # capacity too small is an error that still reports the count
    cnt = C.c_int64(0)
    out = np.empty(1, np.int64)
    m2 = np.zeros((5, 3), np.float32)
    assert gsr.LIB.gsr_crop(m2.ctypes.data, 5, 10.0, 0.0, 0.0, 50.0, 1.0, out.ctypes.data, 1, C.byref(cnt)) == -1
    assert cnt.value == 5
