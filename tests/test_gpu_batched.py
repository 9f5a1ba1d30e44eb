"""Batched multi-view blending (one persistent launch per direction), hipGraph capture and the
autotuner, checked against the single-view calls and the FP64 oracle."""
import numpy as np
import pytest
import torch

import gsinputs
import oracle
from gpu_util import GEMM_GRAD, check_gemm, normwise, say
from paper_2604_02120_amd import api, autotune

pytestmark = pytest.mark.gpu
GRADS = ("dL_dmeans2d", "dL_dconics", "dL_dopacity", "dL_dcolors")


def upload_views(scenes, dev):
    out = []
    for s in scenes:
        d = {"width": s["width"], "height": s["height"]}
        for k in ("means2d", "conics", "opacity", "colors", "depths", "radii"):
            d[k] = torch.from_numpy(np.ascontiguousarray(s[k])).to(dev)
        out.append(d)
    return out


def fill_dloss(bv, seed0=500):
    for i, v in enumerate(bv.views):
        g = gsinputs.make_dloss(v["width"], v["height"], seed0 + i)
        v["dL_dimage"].copy_(torch.from_numpy(g))


def single_view(v, prec, bg):
    img, T, last = api.blend_forward(v["means2d"], v["conics"], v["opacity"], v["colors"],
                                     v["ranges"], v["point_list"][: v["pairs"]], v["width"],
                                     v["height"], bg, prec)
    grads = api.blend_backward(v["means2d"], v["conics"], v["opacity"], v["colors"], v["ranges"],
                               v["point_list"][: v["pairs"]], v["width"], v["height"], T, last,
                               v["dL_dimage"], bg, prec)
    return img, T, last, grads


@pytest.fixture(scope="module")
def small_views(gpu):
    scenes = gsinputs.make_views(scale=0.25)          # 16 views, ~213..480 px wide, ~19k G each
    return scenes, upload_views(scenes, gpu)


@pytest.mark.parametrize("prec", ["fp16", "fp32", "bf16"])
def test_batched_equals_single_view(gpu, small_views, prec):
    scenes, views = small_views
    bg = (0.1, 0.2, 0.3)
    bv = api.BatchedViews(views, prec=prec, bg=bg)
    fill_dloss(bv)
    say(f"[batched] {len(views)} views {prec}")
    bv.step()
    torch.cuda.synchronize()
    for i, v in enumerate(bv.views):
        img, T, last, grads = single_view(v, prec, bg)
        torch.cuda.synchronize()
        assert torch.equal(img, v["image"]) and torch.equal(T, v["final_T"]), i
        assert torch.equal(last, v["last_contrib"]), i
        for g, k in zip(grads, GRADS):      # same sums, atomics in another order
            e = normwise(v[k].cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64))
            assert e <= 1e-5, (i, k, e)
    bv.close()


@pytest.mark.parametrize("prec", ["fp16", "fp32", "bf16"])
def test_batched_every_shape_same_results(gpu, small_views, prec):
    """Every launch shape (LDS batch 64 / 128 / 256 each way, grid or persistent launch): the same
    images and, up to the order of the gradient atomics, the same gradients as the default plan.
    The backward's flush splits each batch's slots among the wavefronts differently per batch
    size, so every size is checked."""
    _, views = small_views
    bv = api.BatchedViews(views, prec=prec)
    fill_dloss(bv)
    bv.step()
    torch.cuda.synchronize()
    ref = [v["image"].clone() for v in bv.views]
    ref_g = [[v[k].clone() for k in GRADS] for v in bv.views]
    for cand in autotune.CANDIDATES:
        say(f"[batched-shape] {prec} {cand}")
        bv._make_plan(cand)
        for v in bv.views:
            for k in GRADS:
                v[k].fill_(123.0)          # the backward must overwrite every gradient
        bv.forward()
        bv.backward()
        torch.cuda.synchronize()
        # the matrix-core reduction rounds dL/dpower to FP16 hi + lo (2^-20 relative) and forms
        # the geometric sums from moments about the tile centre: not the same rounding
        bound = 1e-5 if cand["bwd_reduce"] == 0 else 1e-4
        worst = 0.0
        for i, v in enumerate(bv.views):
            assert torch.equal(v["image"], ref[i]), (cand, i)
            for k, r in zip(GRADS, ref_g[i]):
                e = normwise(v[k].cpu().numpy().astype(np.float64),
                             r.cpu().numpy().astype(np.float64))
                worst = max(worst, e)
                assert e <= bound, (cand, i, k, e)
        say(f"  worst gradient difference from the default shape: {worst:.3e}")
    bv.close()


def test_batched_vs_oracle(gpu, small_views):
    scenes, views = small_views
    bv = api.BatchedViews(views, prec="fp16")
    fill_dloss(bv)
    bv.step()
    torch.cuda.synchronize()
    for i in (0, 5, 11):
        s, v = scenes[i], bv.views[i]
        W, H = s["width"], s["height"]
        pl, rg = oracle.bin_tiles(s["means2d"], s["radii"], s["depths"], W, H)
        ref = oracle.forward(W, H, rg, pl, s["means2d"], s["conics"], s["opacity"], s["colors"])
        check_gemm(ref, v["image"].cpu().numpy().astype(np.float64),
                   v["final_T"].cpu().numpy().astype(np.float64), v["last_contrib"].cpu().numpy(),
                   "fp16", f"view {i} {W}x{H}")
        g = v["dL_dimage"].cpu().numpy()
        gref = oracle.backward(W, H, rg, pl, s["means2d"], s["conics"], s["opacity"], s["colors"], g)
        errs = {k: normwise(v[k].cpu().numpy().astype(np.float64), gref[k[3:]]) for k in GRADS}
        say(f"  view {i} {W}x{H}: grads {errs}")
        assert max(errs.values()) <= GEMM_GRAD
    bv.close()


def test_hipgraph_capture_and_replay(gpu, small_views):
    """bin + forward + backward of all views captured once and replayed; every replay (with eager
    work and synchronisation in between) must reproduce the eager results."""
    _, views = small_views
    bv = api.BatchedViews(views, prec="fp16")
    fill_dloss(bv)
    bv.step()
    torch.cuda.synchronize()
    ref_img = [v["image"].clone() for v in bv.views]
    ref_last = [v["last_contrib"].clone() for v in bv.views]
    ref_g = [[v[k].clone() for k in GRADS] for v in bv.views]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        bv.step()
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        bv.step()
    torch.cuda.synchronize()
    for rep in range(3):
        for v in bv.views:                  # eager work between replays: clobber the outputs
            v["image"].fill_(-1.0)
            v["last_contrib"].fill_(-7)
            for k in GRADS:
                v[k].fill_(123.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        say(f"[graph] replay {rep}")
        for i, v in enumerate(bv.views):
            assert torch.equal(v["image"], ref_img[i]), (rep, i)
            assert torch.equal(v["last_contrib"], ref_last[i]), (rep, i)
            for k, r in zip(GRADS, ref_g[i]):
                e = normwise(v[k].cpu().numpy().astype(np.float64), r.cpu().numpy().astype(np.float64))
                assert e <= 1e-5, (rep, i, k, e)
    del graph
    bv.close()


def test_autotune_picks_a_candidate(gpu, small_views, tmp_path, monkeypatch):
    monkeypatch.setenv("GSBLEND_TUNING_CACHE", str(tmp_path / "tuning.json"))
    _, views = small_views
    bv = api.BatchedViews(views, prec="fp16")
    best = autotune.tune(bv, reps=2)
    say(f"[autotune] {best}")
    keys = autotune.KEYS
    assert {k: best[k] for k in keys} in autotune.CANDIDATES
    assert len(best["trials"]) == len(autotune.CANDIDATES)
    again = autotune.tune(bv)            # from the cache
    assert {k: again[k] for k in keys} == {k: best[k] for k in keys}
    bv.close()


def test_c4_full_size(gpu):
    """The full multi-view workload (16 views, 300k Gaussians each, 854x480..1920x1080): every view
    bit-identical to the single-view forward; the smallest and the largest view against the
    oracle, forward (image, last contributor) and backward (all four gradients)."""
    scenes = gsinputs.make_views()
    views = upload_views(scenes, gpu)
    bv = api.BatchedViews(views, prec="fp16")
    fill_dloss(bv)
    say(f"[c4] {[(v['width'], v['height']) for v in bv.views]}")
    bv.step()
    torch.cuda.synchronize()
    for i, v in enumerate(bv.views):
        img, T, last = api.blend_forward(v["means2d"], v["conics"], v["opacity"], v["colors"],
                                         v["ranges"], v["point_list"][: v["pairs"]], v["width"],
                                         v["height"], (0.0, 0.0, 0.0), "fp16")
        torch.cuda.synchronize()
        assert torch.equal(img, v["image"]), i
    areas = [s["width"] * s["height"] for s in scenes]
    for i in (int(np.argmin(areas)), int(np.argmax(areas))):
        s, v = scenes[i], bv.views[i]
        W, H = s["width"], s["height"]
        pl, rg = oracle.bin_tiles(s["means2d"], s["radii"], s["depths"], W, H)
        assert np.array_equal(v["ranges"].cpu().numpy().astype(np.uint32), rg)
        ref = oracle.forward(W, H, rg, pl, s["means2d"], s["conics"], s["opacity"], s["colors"])
        check_gemm(ref, v["image"].cpu().numpy().astype(np.float64),
                   v["final_T"].cpu().numpy().astype(np.float64), v["last_contrib"].cpu().numpy(),
                   "fp16", f"C4 view {i} {W}x{H}")
        gref = oracle.backward(W, H, rg, pl, s["means2d"], s["conics"], s["opacity"], s["colors"],
                               v["dL_dimage"].cpu().numpy())
        errs = {k: normwise(v[k].cpu().numpy().astype(np.float64), gref[k[3:]]) for k in GRADS}
        say(f"  view {i} {W}x{H} batched backward: {errs}")
        assert max(errs.values()) <= GEMM_GRAD, errs
    bv.close()
