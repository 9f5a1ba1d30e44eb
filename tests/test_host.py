"""Host-side logic that runs without a GPU: the camera struct of the C ABI, argument handling of
the Python layer, the autotuner's choice and cache, the scene generators' determinism, and the
benchmark's refusal of more than one GPU."""
import ctypes
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import gsinputs
import oracle
from paper_2604_02120_amd import _lib, api, autotune

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_camera_struct_layout_matches_header():
    # struct gsb_camera: float R[9], t[3], fx, fy, cx, cy; int32 width, height; float near
    C = _lib.GsbCamera
    assert ctypes.sizeof(C) == 76
    offs = {name: getattr(C, name).offset for name, _ in C._fields_}
    assert offs == {"R": 0, "t": 36, "fx": 48, "fy": 52, "cx": 56, "cy": 60, "width": 64,
                    "height": 68, "near": 72}
    cam = gsinputs.look_at((1.0, 2.0, -3.0), (0.0, 0.0, 5.0), (0.0, 1.0, 0.0), 700.0, 710.0, 320, 240)
    c = api.camera_struct(cam.R, cam.t, cam.fx, cam.fy, cam.cx, cam.cy, cam.width, cam.height, 0.3)
    np.testing.assert_array_equal(np.array(c.R[:]), np.ravel(cam.R).astype(np.float32))
    np.testing.assert_array_equal(np.array(c.t[:]), np.asarray(cam.t, np.float32))
    assert (c.fx, c.fy, c.width, c.height) == (700.0, 710.0, 320, 240)
    assert abs(c.near - 0.3) < 1e-7
    with pytest.raises(ValueError):
        api.camera_struct(((1, 0), (0, 1)), (0, 0, 0), 1, 1, 0, 0, 8, 8)


def test_oracle_camera_is_the_fp32_camera():
    cam = gsinputs.look_at((0.3, -0.7, -2.0), (0.1, 0.2, 4.0), (0.0, 1.0, 0.0), 901.3, 899.7, 640, 480)
    arr = oracle.camera_array(cam)
    f32 = np.asarray([*np.ravel(cam.R), *cam.t, cam.fx, cam.fy, cam.cx, cam.cy], np.float32)
    np.testing.assert_array_equal(arr[:16], f32.astype(np.float64))
    assert arr[16:18].tolist() == [640, 480]


def test_bin_mode_arguments():
    assert api._bin_mode("rect", None, None) == (_lib.GSB_BIN_RECT, 0, 0)
    with pytest.raises(ValueError):
        api._bin_mode("visible", None, None)
    with pytest.raises(KeyError):
        api._bin_mode("tight", None, None)


def test_scene_generators_are_deterministic():
    a = gsinputs.make_scene3d(n=500, seed=3, width=64, height=48)
    b = gsinputs.make_scene3d(n=500, seed=3, width=64, height=48)
    c = gsinputs.make_scene3d(n=500, seed=4, width=64, height=48)
    for k in ("means3d", "scales", "quats", "opacity", "sh"):
        np.testing.assert_array_equal(a[k], b[k])
        assert a[k].dtype == np.float32
        assert not np.array_equal(a[k], c[k])
    assert a["sh"].shape == (500, 16, 3) and a["quats"].shape == (500, 4)
    np.testing.assert_allclose(np.linalg.norm(a["quats"], axis=1), 1.0, atol=1e-6)
    s1 = gsinputs.make_scene("C1")
    s2 = gsinputs.make_scene("C1")
    for k in ("means2d", "conics", "opacity", "colors", "depths", "radii"):
        np.testing.assert_array_equal(s1[k], s2[k])


class FakeViews:
    """Stands in for api.BatchedViews: records the plans it is given."""

    def __init__(self):
        self.views = [{"width": 854, "height": 480, "n": 300_000},
                      {"width": 1920, "height": 1080, "n": 300_000}]
        self.prec = "fp16"
        self.plans = []
        self.binned = 0

    def _make_plan(self, tuning):
        self.plans.append(dict(tuning))

    def bin(self):
        self.binned += 1


def test_autotune_picks_fastest_and_caches(tmp_path, monkeypatch):
    monkeypatch.setenv("GSBLEND_TUNING_CACHE", str(tmp_path / "sub" / "tuning.json"))
    monkeypatch.setattr(autotune, "workload_key",
                        lambda bv: json.dumps({"arch": "gfx950", "prec": bv.prec}))
    calls = []

    def fake_measure(bv, cand, reps=5, warmup=2):
        calls.append(dict(cand))
        return 10.0 - 0.001 * cand["batch_bwd"] + (0.5 if cand["launch"] == 0 else 0.0)

    monkeypatch.setattr(autotune, "measure", fake_measure)
    bv = FakeViews()
    best = autotune.tune(bv)
    assert len(calls) == len(autotune.CANDIDATES)
    assert best["launch"] == 1 and best["batch_bwd"] == 256
    assert bv.plans[-1] == {k: best[k] for k in autotune.KEYS}
    assert [t["ms"] for t in best["trials"]] == sorted(t["ms"] for t in best["trials"])
    # the second call reads the cache: no measurement, no binning, same plan
    calls.clear()
    bv2 = FakeViews()
    again = autotune.tune(bv2)
    assert calls == [] and bv2.binned == 0
    assert {k: again[k] for k in autotune.KEYS} == {k: best[k] for k in autotune.KEYS}
    # a damaged cache file is ignored, not fatal
    (tmp_path / "sub" / "tuning.json").write_text("{not json")
    assert autotune._load() == {}


def test_autotune_candidates_are_valid_shapes():
    seen = set()
    for c in autotune.CANDIDATES:
        assert c["batch_fwd"] in (64, 128, 256) and c["batch_bwd"] in (64, 128, 256)
        assert c["launch"] in (0, 1) and c["blocks_per_cu"] >= 0
        assert c["bwd_reduce"] in (0, 1) and set(c) == set(autotune.KEYS)
        # the matrix-core reduction's LDS tiles are tried only where 4-5 blocks fit per CU
        assert c["bwd_reduce"] == 0 or (c["launch"] == 1 and c["batch_bwd"] in (64, 128))
        key = tuple(sorted(c.items()))
        assert key not in seen
        seen.add(key)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
