"""GPU parity: libgsblend (through its C ABI) against the FP64 CPU oracle on seeded scenes.

Binning must be bit-exact; the plain FP32 blend within 1e-5 of the oracle on every pixel whose
decisions are not marginal; the FP16/BF16 GEMM blends at >= 50 dB PSNR; gradients within the
normwise bounds in gpu_util.
"""
import json
import os

import numpy as np
import pytest
import torch

import gsinputs
import oracle
from gpu_util import (GEMM_GRAD, PLAIN_GRAD, check_gemm, check_plain, plain_grad_bound,
                      gpu_forward, normwise, say, upload, upload_bins)
from paper_2604_02120_amd import _lib, api
from paper_2604_02120_amd.autograd import blend

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
PRECS = ["fp32", "fp16", "bf16"]


def ragged_scene(seed=41, n=1500, W=70, H=37):
    s = gsinputs.make_scene("C1", seed=seed, n=n, width=W, height=H)
    s["means2d"][:20] -= np.float32(25.0)       # off-screen to the top-left
    s["means2d"][20:30] += np.float32([W + 4, H + 4])
    s["radii"][30:40] = 0                       # not rendered
    s["opacity"][40:60] = 0.001                 # below the skip threshold everywhere
    return s


def scenes():
    return {
        "C1": gsinputs.make_scene("C1"),
        "ragged": ragged_scene(),
        "ties": gsinputs.make_scene("C1", seed=42, n=3000, width=96, height=80, depth_levels=4),
        "lognormal": gsinputs.make_scene("C2", seed=43, n=12000, width=200, height=120),
        # large footprints: ~150 tiles per Gaussian, so a block's output segment exceeds what
        # the fill kernel stages in LDS and most rectangles are emitted wavefront-cooperatively
        "bigrects": gsinputs.make_scene(
            gsinputs.SceneConfig("bigrects", 1024, 1024, 3000, "loguniform", 8.0, 64.0,
                                 "uniform", 44)),
        # means bunched around a few centres: tile lists up to ~8700 long (68 batches of 128),
        # most pixels saturate and stop early
        "clustered": gsinputs.make_scene(
            gsinputs.SceneConfig("clustered", 512, 384, 60000, "lognormal", 2.0, 0.0,
                                 "uniform", 47, clustered=True)),
    }


SCENES = scenes()


# ----------------------------------------------------------------------------- binning
@pytest.mark.parametrize("name", list(SCENES))
def test_bin_bitexact(gpu, name):
    s = SCENES[name]
    say(f"[bin] {name} {s['width']}x{s['height']} n={len(s['radii'])}")
    pl_ref, rg_ref = oracle.bin_tiles(s["means2d"], s["radii"], s["depths"], s["width"], s["height"])
    sd = upload(s, gpu)
    pl, rg = api.bin_tiles(sd["means2d"], sd["radii"], sd["depths"], s["width"], s["height"])
    np.testing.assert_array_equal(rg.cpu().numpy().astype(np.uint32), rg_ref)
    np.testing.assert_array_equal(pl.cpu().numpy().astype(np.uint32), pl_ref)


def test_bin_capacity_overflow_flag(gpu):
    s = SCENES["C1"]
    sd = upload(s, gpu)
    W, H = s["width"], s["height"]
    n = len(s["radii"])
    ws = api.BinWorkspace(n, 1000, W, H, device=gpu)
    npairs = api.bin_count(sd["means2d"], sd["radii"], W, H, ws)
    pl = torch.full((1000,), -1, dtype=torch.int32, device=gpu)
    rg = torch.empty((16, 2), dtype=torch.int32, device=gpu)
    st = api.bin_fill(sd["means2d"], sd["radii"], sd["depths"], W, H, ws, pl, rg)
    torch.cuda.synchronize()
    assert int(npairs.item()) > 1000
    assert int(st.item()) == 2        # GSB_ERR_CAPACITY
    ok = api.BinWorkspace(n, int(npairs.item()), W, H, device=gpu)
    ok.buf[: ws.nbytes].copy_(ws.buf[: ws.nbytes])
    pl2 = torch.empty(int(npairs.item()), dtype=torch.int32, device=gpu)
    st2 = api.bin_fill(sd["means2d"], sd["radii"], sd["depths"], W, H, ok, pl2, rg)
    torch.cuda.synchronize()
    assert int(st2.item()) == 0


# ----------------------------------------------------------------------------- forward
@pytest.mark.parametrize("name", list(SCENES))
@pytest.mark.parametrize("prec", PRECS)
def test_forward_parity(gpu, name, prec):
    s = SCENES[name]
    bg = (0.05, 0.1, 0.2)
    say(f"[fwd] {name} {prec} {s['width']}x{s['height']} n={len(s['radii'])}")
    ref = oracle.render(s, bg)
    sd = upload(s, gpu)
    pl, rg = upload_bins(ref["point_list"], ref["ranges"], gpu)
    img, T, last = gpu_forward(sd, pl, rg, prec, bg)
    if prec == "fp32":
        check_plain(ref, img, T, last, name)
    else:
        check_gemm(ref, img, T, last, prec, name)


@pytest.mark.parametrize("prec", PRECS)
def test_forward_deterministic(gpu, prec):
    s = SCENES["lognormal"]
    sd = upload(s, gpu)
    pl, rg = api.bin_tiles(sd["means2d"], sd["radii"], sd["depths"], s["width"], s["height"])
    a = gpu_forward(sd, pl, rg, prec)
    b = gpu_forward(sd, pl, rg, prec)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("prec", PRECS)
def test_forward_five_stack_golden(gpu, prec):
    g = json.load(open(os.path.join(GOLDEN, "five_stack.json")))
    s = gsinputs.stack_scene(g["n"], g["opacity"], at=tuple(g["pixel"]))
    sd = upload(s, gpu)
    pl, rg = api.bin_tiles(sd["means2d"], sd["radii"], sd["depths"], 16, 16)
    img, T, last = gpu_forward(sd, pl, rg, prec)
    px, py = g["pixel"]
    assert last[py, px] == g["last_contrib"]
    np.testing.assert_allclose(img[:, py, px], g["image"], atol=2e-6)
    assert abs(T[py, px] - g["final_T"]) < 1e-7


@pytest.mark.parametrize("prec", PRECS)
def test_forward_empty_and_degenerate(gpu, prec):
    bg = (0.25, 0.5, 0.75)
    # no Gaussians at all, odd-sized image
    empty = gsinputs.make_scene("C1", seed=9, n=5, width=33, height=17)
    empty["radii"][:] = 0
    sd = upload(empty, gpu)
    pl, rg = api.bin_tiles(sd["means2d"], sd["radii"], sd["depths"], 33, 17)
    assert pl.numel() == 0
    img, T, last = gpu_forward(sd, pl, rg, prec, bg)
    for c in range(3):
        assert np.all(img[c] == np.float32(bg[c]))
    assert np.all(T == 1.0) and np.all(last == 0)
    # a 1x1 image with a single Gaussian on the pixel
    one = gsinputs.stack_scene(1, 0.5, width=1, height=1, at=(0.0, 0.0))
    sd = upload(one, gpu)
    pl, rg = api.bin_tiles(sd["means2d"], sd["radii"], sd["depths"], 1, 1)
    img, T, last = gpu_forward(sd, pl, rg, prec)
    assert last[0, 0] == 1 and abs(T[0, 0] - 0.5) < 1e-6
    np.testing.assert_allclose(img[:, 0, 0], [0.5, 0.25, 0.125], atol=1e-6)


def test_forward_c2_full_size(gpu):
    """The benchmark's forward workload (1920x1080, 1M Gaussians), GPU binning, all three
    precisions against the full-frame oracle."""
    s = gsinputs.make_scene("C2")
    say("[fwd-full] C2 1920x1080 n=1e6: oracle")
    ref = oracle.render(s)
    sd = upload(s, gpu)
    pl, rg = api.bin_tiles(sd["means2d"], sd["radii"], sd["depths"], 1920, 1080)
    np.testing.assert_array_equal(rg.cpu().numpy().astype(np.uint32), ref["ranges"])
    np.testing.assert_array_equal(pl.cpu().numpy().astype(np.uint32), ref["point_list"])
    say("[fwd-full] C2 visible-tile binning")
    pl1_ref, rg1_ref = oracle.bin_tiles(s["means2d"], s["radii"], s["depths"], 1920, 1080,
                                        s["conics"], s["opacity"], oracle.BIN_VISIBLE)
    pl1, rg1 = api.bin_tiles(sd["means2d"], sd["radii"], sd["depths"], 1920, 1080,
                             conics=sd["conics"], opacity=sd["opacity"], mode="visible")
    np.testing.assert_array_equal(rg1.cpu().numpy().astype(np.uint32), rg1_ref)
    np.testing.assert_array_equal(pl1.cpu().numpy().astype(np.uint32), pl1_ref)
    say(f"  pairs {len(ref['point_list'])} -> {len(pl1_ref)}")
    for prec in PRECS:
        say(f"[fwd-full] C2 {prec}")
        img, T, last = gpu_forward(sd, pl, rg, prec)
        if prec == "fp32":
            check_plain(ref, img, T, last, "C2")
        else:
            check_gemm(ref, img, T, last, prec, "C2")


# ----------------------------------------------------------------------------- backward
_REF_CACHE = {}


def backward_case(s, gpu, prec, seed=77, bg=(0.1, 0.3, 0.2)):
    W, H = s["width"], s["height"]
    g = gsinputs.make_dloss(W, H, seed)
    key = (id(s), seed, bg)
    if key not in _REF_CACHE:
        pl_ref, rg_ref = oracle.bin_tiles(s["means2d"], s["radii"], s["depths"], W, H)
        ref = oracle.backward(W, H, rg_ref, pl_ref, s["means2d"], s["conics"], s["opacity"],
                              s["colors"], g, bg)
        _REF_CACHE.clear()
        _REF_CACHE[key] = (pl_ref, rg_ref, ref)
    pl_ref, rg_ref, ref = _REF_CACHE[key]
    sd = upload(s, gpu)
    pl, rg = upload_bins(pl_ref, rg_ref, gpu)
    img, T, last = api.blend_forward(sd["means2d"], sd["conics"], sd["opacity"], sd["colors"], rg,
                                     pl, W, H, bg, prec)
    gd = torch.from_numpy(g).to(gpu)
    out = api.blend_backward(sd["means2d"], sd["conics"], sd["opacity"], sd["colors"], rg, pl, W,
                             H, T, last, gd, bg, prec)
    torch.cuda.synchronize()
    names = ["dmeans2d", "dconics", "dopacity", "dcolors"]
    return {k: v.cpu().numpy().astype(np.float64) for k, v in zip(names, out)}, ref


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", ["C1", "ragged", "lognormal", "clustered"])
def test_backward_parity(gpu, prec, name):
    s = SCENES[name]
    say(f"[bwd] {name} {prec}")
    got, ref = backward_case(s, gpu, prec)
    bound = plain_grad_bound(name) if prec == "fp32" else GEMM_GRAD
    for k in ref:
        e = normwise(got[k], ref[k])
        say(f"  {k}: normwise rel err {e:.3e}")
        assert e <= bound, (k, e)


@pytest.mark.parametrize("prec", PRECS)
def test_backward_sparse_and_zero_upstream_gradient(gpu, prec):
    """The block flushes a Gaussian's per-batch sums only if one of them is nonzero. An upstream
    gradient on three pixels leaves almost every reached Gaussian with sums of exactly zero: the
    gradients must still match the oracle's (normwise) and be exactly zero for every Gaussian
    listed in none of the three pixels' tiles; a zero upstream gradient must give exactly zero
    gradients, also when the output buffers hold an earlier call's values."""
    s = SCENES["lognormal"]
    W, H = s["width"], s["height"]
    bg = (0.1, 0.3, 0.2)
    say(f"[bwd sparse] lognormal {prec}")
    pl_ref, rg_ref = oracle.bin_tiles(s["means2d"], s["radii"], s["depths"], W, H)
    g = np.zeros((3, H, W), np.float32)
    # Gaussians listed in none of the three pixels' tiles cannot reach them on any path
    untouched = np.ones(s["opacity"].shape[0], bool)
    gx = (W + 15) // 16
    for (y, x, c, v) in [(3, 5, 0, 1.0), (H // 2, W // 2, 1, -2.0), (H - 1, W - 1, 2, 0.5)]:
        g[c, y, x] = v
        t = (y // 16) * gx + x // 16
        untouched[pl_ref[int(rg_ref[t][0]):int(rg_ref[t][1])]] = False
    ref = oracle.backward(W, H, rg_ref, pl_ref, s["means2d"], s["conics"], s["opacity"],
                          s["colors"], g, bg)
    sd = upload(s, gpu)
    pl, rg = upload_bins(pl_ref, rg_ref, gpu)
    img, T, last = api.blend_forward(sd["means2d"], sd["conics"], sd["opacity"], sd["colors"], rg,
                                     pl, W, H, bg, prec)
    out = api.blend_backward(sd["means2d"], sd["conics"], sd["opacity"], sd["colors"], rg, pl, W,
                             H, T, last, torch.from_numpy(g).to(gpu), bg, prec)
    torch.cuda.synchronize()
    bound = plain_grad_bound("lognormal") if prec == "fp32" else GEMM_GRAD
    names = ["dmeans2d", "dconics", "dopacity", "dcolors"]
    for k, v in zip(names, out):
        got = v.cpu().numpy().astype(np.float64)
        e = normwise(got, ref[k])
        say(f"  {k}: normwise rel err {e:.3e}")
        assert e <= bound, (k, e)
    assert untouched.sum() > 0.5 * len(untouched)
    for k, v in zip(names, out):
        got = v.cpu().numpy().reshape(len(untouched), -1)
        assert np.all(got[untouched] == 0.0), k
    zero = torch.zeros((3, H, W), dtype=torch.float32, device=gpu)
    out2 = api.blend_backward(sd["means2d"], sd["conics"], sd["opacity"], sd["colors"], rg, pl, W,
                              H, T, last, zero, bg, prec, out=out)
    torch.cuda.synchronize()
    for k, v in zip(names, out2):
        assert torch.count_nonzero(v).item() == 0, k


@pytest.mark.parametrize("prec", PRECS)
def test_alpha_clamp(gpu, prec):
    """The 0.99 clamp of alpha (Eq. (alpha)): the kernels apply it to the exponent's argument,
    min(2^x, 0.99) = 2^min(x, log2f(0.99f)), which is exact only because the exp2 instruction
    returns exactly 0.99f there. An opaque Gaussian centred on a pixel must leave exactly
    1 - 0.99f at it; then a scene of opacities 0.97 to 1 (the clamp active around most centres)
    against the oracle, image and gradients."""
    s1 = gsinputs.stack_scene(1, 1.0, at=(8.0, 8.0))
    sd1 = upload(s1, gpu)
    pl1, rg1 = api.bin_tiles(sd1["means2d"], sd1["radii"], sd1["depths"], 16, 16)
    _, T1, last1 = gpu_forward(sd1, pl1, rg1, prec)
    assert last1[8, 8] == 1
    assert T1[8, 8] == float(np.float32(1.0) - np.float32(0.99)), T1[8, 8]
    s = dict(SCENES["C1"])
    rng = np.random.default_rng(99)
    s["opacity"] = rng.uniform(0.97, 1.0, len(s["opacity"])).astype(np.float32)
    W, H = s["width"], s["height"]
    say(f"[clamp] C1 with opacities in [0.97, 1] {prec}")
    pl_ref, rg_ref = oracle.bin_tiles(s["means2d"], s["radii"], s["depths"], W, H)
    ref = oracle.forward(W, H, rg_ref, pl_ref, s["means2d"], s["conics"], s["opacity"], s["colors"])
    sd = upload(s, gpu)
    pl, rg = upload_bins(pl_ref, rg_ref, gpu)
    img, T, last = gpu_forward(sd, pl, rg, prec)
    if prec == "fp32":
        check_plain(ref, img, T, last, "clamp")
    else:
        check_gemm(ref, img, T, last, prec, "clamp")
    got, gref = backward_case(s, gpu, prec)
    bound = PLAIN_GRAD if prec == "fp32" else GEMM_GRAD
    for k in gref:
        e = normwise(got[k], gref[k])
        say(f"  {k}: normwise rel err {e:.3e}")
        assert e <= bound, (k, e)


@pytest.mark.parametrize("prec", PRECS)
def test_autograd_matches_oracle_on_fd_subscene(gpu, prec):
    """The 32x32, 200-Gaussian subscene whose oracle gradient is pinned to finite differences."""
    s = gsinputs.fd_subscene(33)
    W, H = s["width"], s["height"]
    s32 = {k: (v.astype(np.float32) if isinstance(v, np.ndarray) and v.dtype == np.float64 else v)
           for k, v in s.items()}
    bg = (0.2, 0.4, 0.1)
    g = gsinputs.make_dloss(W, H, 34)
    pl_ref, rg_ref = oracle.bin_tiles(s32["means2d"], s32["radii"], s32["depths"], W, H)
    ref = oracle.backward(W, H, rg_ref, pl_ref, s32["means2d"], s32["conics"], s32["opacity"],
                          s32["colors"], g, bg)
    sd = upload(s32, gpu)
    pl, rg = upload_bins(pl_ref, rg_ref, gpu)
    leaves = [sd[k].clone().requires_grad_(True) for k in ("means2d", "conics", "opacity", "colors")]
    img, T, last = blend(*leaves, rg, pl, W, H, bg, prec)
    (img * torch.from_numpy(g).to(gpu)).sum().backward()
    bound = PLAIN_GRAD if prec == "fp32" else GEMM_GRAD
    for leaf, k in zip(leaves, ["dmeans2d", "dconics", "dopacity", "dcolors"]):
        e = normwise(leaf.grad.cpu().numpy().astype(np.float64), ref[k])
        say(f"  {prec} {k}: {e:.3e}")
        assert e <= bound, (k, e)


def test_backward_c3_full_size(gpu):
    """The benchmark-shaped differentiable workload at full size (1280x720, 500k Gaussians)."""
    s = gsinputs.make_scene("C3")
    for prec in PRECS:
        say(f"[bwd-full] C3 {prec}")
        got, ref = backward_case(s, gpu, prec, seed=1003, bg=(0.0, 0.0, 0.0))
        bound = PLAIN_GRAD if prec == "fp32" else GEMM_GRAD
        for k in ref:
            e = normwise(got[k], ref[k])
            say(f"  {k}: {e:.3e}")
            assert e <= bound, (k, e)


# ----------------------------------------------------------------------------- 4K, sampled tiles
def c5_sample_tiles(gx, gy, k=40, seed=5):
    rng = np.random.default_rng(seed)
    corners = [0, gx - 1, (gy - 1) * gx, gx * gy - 1]
    return sorted(set(corners) | set(rng.choice(gx * gy, size=k, replace=False).tolist()))


def test_c5_4k_full_frame(gpu):
    """The largest workload (3840x2160, 3M Gaussians, 54.7M pairs) whole, as the benchmark runs
    it: GPU binning bit-exact against the oracle's, the forward from packed records in every
    precision against the full-frame oracle image, and the backward's gradients against the
    oracle's gradient of the whole frame."""
    s = gsinputs.make_scene("C5")
    W, H = s["width"], s["height"]
    say("[c5-full] 3840x2160 n=3e6: oracle binning")
    pl_ref, rg_ref = oracle.bin_tiles(s["means2d"], s["radii"], s["depths"], W, H)
    sd = upload(s, gpu)
    pl, rg = api.bin_tiles(sd["means2d"], sd["radii"], sd["depths"], W, H)
    np.testing.assert_array_equal(rg.cpu().numpy().astype(np.uint32), rg_ref)
    np.testing.assert_array_equal(pl.cpu().numpy().astype(np.uint32), pl_ref)
    say(f"[c5-full] {len(pl_ref)} pairs bit-exact; oracle forward + backward")
    ref = oracle.forward(W, H, rg_ref, pl_ref, s["means2d"], s["conics"], s["opacity"], s["colors"])
    g = gsinputs.make_dloss(W, H, 1005)
    gref = oracle.backward(W, H, rg_ref, pl_ref, s["means2d"], s["conics"], s["opacity"],
                           s["colors"], g)
    rec = api.pack_gaussians(sd["means2d"], sd["conics"], sd["opacity"], sd["colors"])
    gd = torch.from_numpy(g).to(gpu)
    for prec in PRECS:
        img, T, last = api.blend_forward_packed(rec, rg, pl, W, H, (0.0, 0.0, 0.0), prec)
        grads = api.blend_backward_packed(rec, rg, pl, W, H, T, last, gd, (0.0, 0.0, 0.0), prec)
        torch.cuda.synchronize()
        img = img.cpu().numpy().astype(np.float64)
        T, last = T.cpu().numpy().astype(np.float64), last.cpu().numpy()
        if prec == "fp32":
            check_plain(ref, img, T, last, "C5 full frame")
        else:
            check_gemm(ref, img, T, last, prec, "C5 full frame")
        bound = plain_grad_bound("C5") if prec == "fp32" else GEMM_GRAD
        for k, v in zip(("dmeans2d", "dconics", "dopacity", "dcolors"), grads):
            e = normwise(v.cpu().numpy().astype(np.float64), gref[k])
            say(f"  C5 full frame bwd {prec} {k}: {e:.3e}")
            assert e <= bound, (prec, k, e)


def test_c5_4k_sampled_tiles(gpu):
    """The largest workload (3840x2160, 3M Gaussians) at full size in the benchmark's launch
    configuration: GPU binning of the whole frame, checked bit-exactly against the oracle's lists of
    a sample of tiles (each built on its own from every Gaussian); the whole-frame forward of every
    precision checked on those tiles' pixels; the backward run on the sampled tiles' lists only
    (every other tile empty) against the oracle's gradients of that same restricted frame."""
    s = gsinputs.make_scene("C5")
    W, H = s["width"], s["height"]
    gx, gy = oracle.grid(W, H)
    tiles = c5_sample_tiles(gx, gy)
    say(f"[c5] 3840x2160 n=3e6, {len(tiles)} sampled tiles: oracle")
    pl_ref, rg_ref = oracle.sampled_bins(s["means2d"], s["radii"], s["depths"], W, H, tiles)
    sd = upload(s, gpu)
    pl, rg = api.bin_tiles(sd["means2d"], sd["radii"], sd["depths"], W, H)
    pl, rg = pl.cpu().numpy().astype(np.uint32), rg.cpu().numpy().astype(np.uint32)
    for t in tiles:
        a, b = rg[t]
        np.testing.assert_array_equal(pl[a:b], pl_ref[rg_ref[t, 0]:rg_ref[t, 1]], err_msg=str(t))
    mask = np.zeros((H, W), bool)
    for t in tiles:
        tx, ty = t % gx, t // gx
        mask[16 * ty:16 * ty + 16, 16 * tx:16 * tx + 16] = True
    ref = oracle.forward(W, H, rg_ref, pl_ref, s["means2d"], s["conics"], s["opacity"], s["colors"])
    pl_t = torch.from_numpy(pl.astype(np.int32)).to(gpu)
    rg_t = torch.from_numpy(rg.astype(np.int32)).to(gpu)
    for prec in PRECS:
        img, T, last = gpu_forward(sd, pl_t, rg_t, prec)
        if prec == "fp32":
            check_plain(ref, img, T, last, "C5 sampled tiles", mask=mask)
        else:
            check_gemm(ref, img, T, last, prec, "C5 sampled tiles", mask=mask)
    g = gsinputs.make_dloss(W, H, 1005)
    gref = oracle.backward(W, H, rg_ref, pl_ref, s["means2d"], s["conics"], s["opacity"],
                           s["colors"], g)
    pl_s, rg_s = upload_bins(pl_ref, rg_ref, gpu)
    gd = torch.from_numpy(g).to(gpu)
    for prec in PRECS:
        img, T, last = api.blend_forward(sd["means2d"], sd["conics"], sd["opacity"], sd["colors"],
                                         rg_s, pl_s, W, H, (0.0, 0.0, 0.0), prec)
        out = api.blend_backward(sd["means2d"], sd["conics"], sd["opacity"], sd["colors"], rg_s,
                                 pl_s, W, H, T, last, gd, (0.0, 0.0, 0.0), prec)
        torch.cuda.synchronize()
        bound = PLAIN_GRAD if prec == "fp32" else GEMM_GRAD
        for k, v in zip(["dmeans2d", "dconics", "dopacity", "dcolors"], out):
            e = normwise(v.cpu().numpy().astype(np.float64), gref[k])
            say(f"  bwd {prec} {k}: {e:.3e}")
            assert e <= bound, (prec, k, e)


# ----------------------------------------------------------------------------- binning mode 1
def needle_scene(seed=61, n=400, W=120, H=72):
    """Strongly anisotropic Gaussians at all angles, opacities down to 1/255."""
    rng = np.random.default_rng(seed)
    s = gsinputs.make_scene("C1", seed=seed, n=n, width=W, height=H)
    th = rng.uniform(0, np.pi, n)
    s1, s2 = rng.uniform(0.5, 1.0, n), rng.uniform(4.0, 32.0, n)
    s["conics"] = gsinputs.conic_from_axes(th, s1, s2).astype(np.float32)
    s["radii"] = np.ceil(3.0 * np.maximum(s1, s2)).astype(np.int32)
    s["opacity"] = rng.uniform(1.0 / 255.0, 0.99, n).astype(np.float32)
    return s


VIS = dict(SCENES, needles=needle_scene())


def gpu_bins(sd, mode):
    pl, rg = api.bin_tiles(sd["means2d"], sd["radii"], sd["depths"], sd["width"], sd["height"],
                           conics=sd["conics"], opacity=sd["opacity"], mode=mode)
    torch.cuda.synchronize()
    return pl, rg


@pytest.mark.parametrize("name", list(VIS))
def test_bin_visible_bitexact(gpu, name):
    """Binning mode 1 (tiles where alpha can reach 1/255) equals the oracle's bit for bit."""
    s = VIS[name]
    W, H = s["width"], s["height"]
    say(f"[bin-visible] {name} {W}x{H} n={len(s['radii'])}")
    pl_ref, rg_ref = oracle.bin_tiles(s["means2d"], s["radii"], s["depths"], W, H, s["conics"],
                                      s["opacity"], oracle.BIN_VISIBLE)
    sd = upload(s, gpu)
    pl, rg = gpu_bins(sd, "visible")
    np.testing.assert_array_equal(rg.cpu().numpy().astype(np.uint32), rg_ref)
    np.testing.assert_array_equal(pl.cpu().numpy().astype(np.uint32), pl_ref)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", ["lognormal", "needles"])
def test_visible_binning_same_blend(gpu, prec, name):
    """Forward and backward over mode-1 lists reproduce those over the 3-sigma lists: image and
    final T bit for bit, the same last Gaussian per pixel, gradients up to atomic order."""
    s = VIS[name]
    W, H = s["width"], s["height"]
    sd = upload(s, gpu)
    bg = (0.1, 0.3, 0.2)
    g = torch.from_numpy(gsinputs.make_dloss(W, H, 77)).to(gpu)
    out = {}
    for mode in ("rect", "visible"):
        pl, rg = gpu_bins(sd, mode)
        img, T, last = api.blend_forward(sd["means2d"], sd["conics"], sd["opacity"], sd["colors"],
                                         rg, pl, W, H, bg, prec)
        grads = api.blend_backward(sd["means2d"], sd["conics"], sd["opacity"], sd["colors"], rg,
                                   pl, W, H, T, last, g, bg, prec)
        torch.cuda.synchronize()
        gx, _ = oracle.grid(W, H)
        lastc = last.cpu().numpy()
        rgn = rg.cpu().numpy().astype(np.int64)
        pln = pl.cpu().numpy().astype(np.int64)
        tile = (np.arange(H)[:, None] // 16) * gx + np.arange(W)[None, :] // 16
        who = np.where(lastc > 0, pln[np.clip(rgn[tile, 0] + lastc - 1, 0, max(len(pln) - 1, 0))], -1)
        out[mode] = (img.cpu().numpy(), T.cpu().numpy(), who,
                     [x.cpu().numpy().astype(np.float64) for x in grads], len(pln))
    a, b = out["rect"], out["visible"]
    say(f"  {name} {prec}: pairs {a[4]} -> {b[4]}")
    assert b[4] < a[4]
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    for ga, gb in zip(a[3], b[3]):
        assert normwise(gb, ga) <= 1e-5


def test_three_tile_sort_passes(gpu):
    """More than 65536 tiles (4112 x 4112 pixels: 257 x 257 tiles, 17-bit tile ids) take the
    tile sort through three passes, an odd count above one, which routes the sorted values
    through the other buffer. Both binning modes bit for bit over the whole frame, then the plain
    forward on every pixel."""
    cfg = gsinputs.SceneConfig("tiles66k", 4112, 4112, 30000, "loguniform", 0.5, 8.0, "uniform", 46)
    s = gsinputs.make_scene(cfg)
    W, H = s["width"], s["height"]
    gx, gy = oracle.grid(W, H)
    assert gx * gy > 65536
    say(f"[bin] {W}x{H} ({gx * gy} tiles) n={len(s['radii'])}")
    sd = upload(s, gpu)
    for mode, omode in (("rect", oracle.BIN_RECT), ("visible", oracle.BIN_VISIBLE)):
        pl_ref, rg_ref = oracle.bin_tiles(s["means2d"], s["radii"], s["depths"], W, H,
                                          s["conics"], s["opacity"], omode)
        pl, rg = gpu_bins(sd, mode)
        np.testing.assert_array_equal(rg.cpu().numpy().astype(np.uint32), rg_ref)
        np.testing.assert_array_equal(pl.cpu().numpy().astype(np.uint32), pl_ref)
        if mode == "rect":
            ref = oracle.forward(W, H, rg_ref, pl_ref, s["means2d"], s["conics"], s["opacity"],
                                 s["colors"])
            img, T, last = gpu_forward(sd, pl, rg, "fp32")
            check_plain(ref, img, T, last, "66k tiles")


def test_largest_16bit_tile_grid(gpu):
    """65536 tiles (4096 x 4096 pixels) is the largest grid whose tile ids the binning sorts as
    16-bit keys; tile 65535 (the bottom-right corner, all 16 bits set) must land in place. Extra
    Gaussians around that corner and along the last row and column, then both binning modes bit for
    bit over the whole frame."""
    cfg = gsinputs.SceneConfig("tiles65536", 4096, 4096, 20000, "loguniform", 0.5, 8.0, "uniform", 48)
    s = gsinputs.make_scene(cfg)
    W, H = s["width"], s["height"]
    gx, gy = oracle.grid(W, H)
    assert gx * gy == 65536
    rng = np.random.default_rng(480)
    k = 2000                       # centres within 40 px of the right or bottom edge
    edge = rng.uniform(W - 40.0, W + 8.0, k).astype(np.float32)
    along = rng.uniform(0.0, W, k).astype(np.float32)
    s["means2d"][:k, 0] = np.where(np.arange(k) % 2 == 0, edge, along)
    s["means2d"][:k, 1] = np.where(np.arange(k) % 2 == 0, along, edge)
    s["means2d"][k:k + 50] = np.float32(W - 3.0)
    say(f"[bin] {W}x{H} ({gx * gy} tiles) n={len(s['radii'])}")
    sd = upload(s, gpu)
    for mode, omode in (("rect", oracle.BIN_RECT), ("visible", oracle.BIN_VISIBLE)):
        pl_ref, rg_ref = oracle.bin_tiles(s["means2d"], s["radii"], s["depths"], W, H,
                                          s["conics"], s["opacity"], omode)
        assert rg_ref[65535, 1] > rg_ref[65535, 0]      # the last tile has pairs
        pl, rg = gpu_bins(sd, mode)
        np.testing.assert_array_equal(rg.cpu().numpy().astype(np.uint32), rg_ref)
        np.testing.assert_array_equal(pl.cpu().numpy().astype(np.uint32), pl_ref)


# ----------------------------------------------------------------------------- backward reduction
def plan_grads(sd, prec, g, bg, bwd_reduce, batch_bwd=128):
    """Gradients from a one-view plan (one block per tile) with the given backward reduction."""
    bv = api.BatchedViews([sd], prec=prec, bg=bg,
                          tuning={"launch": 1, "batch_bwd": batch_bwd, "bwd_reduce": bwd_reduce})
    bv.views[0]["dL_dimage"].copy_(torch.from_numpy(g))
    bv.step()
    torch.cuda.synchronize()
    v = bv.views[0]
    out = {k: v["dL_" + k].cpu().numpy().astype(np.float64)
           for k in ("dmeans2d", "dconics", "dopacity", "dcolors")}
    bv.close()
    return out


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", ["C1", "lognormal", "bigrects", "clustered"])
@pytest.mark.parametrize("batch_bwd", [64, 128])
def test_backward_mfma_reduction(gpu, prec, name, batch_bwd):
    """The backward with its five geometric sums formed on the matrix cores (dL/dM_g as the
    product of dL/dpower with the pixel basis) against the FP64 oracle, at the bounds of the
    vector-ALU reduction, and against that reduction itself."""
    s = SCENES[name]
    W, H = s["width"], s["height"]
    bg = (0.1, 0.3, 0.2)
    g = gsinputs.make_dloss(W, H, 77)
    pl_ref, rg_ref = oracle.bin_tiles(s["means2d"], s["radii"], s["depths"], W, H)
    ref = oracle.backward(W, H, rg_ref, pl_ref, s["means2d"], s["conics"], s["opacity"],
                          s["colors"], g, bg)
    sd = upload(s, gpu)
    mm = plan_grads(sd, prec, g, bg, 1, batch_bwd)
    valu = plan_grads(sd, prec, g, bg, 0, batch_bwd)
    bound = plain_grad_bound(name) if prec == "fp32" else GEMM_GRAD
    for k in ref:
        e = normwise(mm[k], ref[k])
        d = normwise(mm[k], valu[k])
        say(f"  mfma reduction {name} {prec} b={batch_bwd} {k}: vs oracle {e:.3e}, "
            f"vs vector reduction {d:.3e}")
        assert e <= bound, (k, e)


# ----------------------------------------------------------------------------- packed records
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", ["C1", "ragged", "lognormal", "clustered"])
def test_packed_records_same_results(gpu, prec, name):
    """The blends that read gsb_pack_gaussians' 48-byte records give the image, final T and last
    contributor of the four-array blends bit for bit, and their gradients up to the order of the
    FP32 atomic sums; the records hold the attributes unchanged."""
    s = SCENES[name]
    W, H = s["width"], s["height"]
    bg = (0.1, 0.3, 0.2)
    sd = upload(s, gpu)
    pl, rg = api.bin_tiles(sd["means2d"], sd["radii"], sd["depths"], W, H)
    rec = api.pack_gaussians(sd["means2d"], sd["conics"], sd["opacity"], sd["colors"])
    r = rec.cpu().numpy()
    assert np.array_equal(r[:, 0:2], s["means2d"]) and np.array_equal(r[:, 2:4], s["conics"][:, :2])
    assert np.array_equal(r[:, 4], s["conics"][:, 2]) and np.array_equal(r[:, 5], s["opacity"])
    assert np.array_equal(r[:, 6:9], s["colors"]) and not r[:, 9:].any()
    g = torch.from_numpy(gsinputs.make_dloss(W, H, 77)).to(gpu)
    a = api.blend_forward(sd["means2d"], sd["conics"], sd["opacity"], sd["colors"], rg, pl, W, H,
                          bg, prec)
    b = api.blend_forward_packed(rec, rg, pl, W, H, bg, prec)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    ga = api.blend_backward(sd["means2d"], sd["conics"], sd["opacity"], sd["colors"], rg, pl, W, H,
                            a[1], a[2], g, bg, prec)
    gb = api.blend_backward_packed(rec, rg, pl, W, H, b[1], b[2], g, bg, prec)
    torch.cuda.synchronize()
    for x, y in zip(ga, gb):
        e = normwise(y.cpu().numpy().astype(np.float64), x.cpu().numpy().astype(np.float64))
        assert e <= 1e-5, e


# ----------------------------------------------------------------------------- deterministic backward
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", ["C1", "ragged", "lognormal", "bigrects", "clustered"])
def test_deterministic_backward(gpu, prec, name):
    """The deterministic backward: identical bit for bit on repeated runs (the atomic backward is
    not), the oracle's gradients at the bounds of the atomic backward, and within 1e-5 (normwise)
    of the atomic backward's gradients."""
    s = SCENES[name]
    W, H = s["width"], s["height"]
    bg = (0.1, 0.3, 0.2)
    g = gsinputs.make_dloss(W, H, 77)
    pl_ref, rg_ref = oracle.bin_tiles(s["means2d"], s["radii"], s["depths"], W, H)
    ref = oracle.backward(W, H, rg_ref, pl_ref, s["means2d"], s["conics"], s["opacity"],
                          s["colors"], g, bg)
    sd = upload(s, gpu)
    pl, rg = upload_bins(pl_ref, rg_ref, gpu)
    rec = api.pack_gaussians(sd["means2d"], sd["conics"], sd["opacity"], sd["colors"])
    img, T, last = api.blend_forward_packed(rec, rg, pl, W, H, bg, prec)
    gd = torch.from_numpy(g).to(gpu)
    ws = api.DetWorkspace(rec.shape[0], pl.numel(), device=gpu)
    runs = []
    for _ in range(3):
        out = api.blend_backward_deterministic(rec, rg, pl, W, H, T, last, gd, bg, prec, ws=ws)
        torch.cuda.synchronize()
        runs.append([x.clone() for x in out])
        ws.buf.fill_(0x7f)           # what a call leaves in the workspace must not matter
    for r in runs[1:]:
        for x, y in zip(runs[0], r):
            assert torch.equal(x, y)
    atomic = api.blend_backward_packed(rec, rg, pl, W, H, T, last, gd, bg, prec)
    torch.cuda.synchronize()
    bound = plain_grad_bound(name) if prec == "fp32" else GEMM_GRAD
    for k, x, y in zip(("dmeans2d", "dconics", "dopacity", "dcolors"), runs[0], atomic):
        e = normwise(x.cpu().numpy().astype(np.float64), ref[k])
        d = normwise(x.cpu().numpy().astype(np.float64), y.cpu().numpy().astype(np.float64))
        say(f"  deterministic {name} {prec} {k}: vs oracle {e:.3e}, vs atomic {d:.3e}")
        assert e <= bound, (k, e)
        assert d <= 1e-5, (k, d)


# ----------------------------------------------------------------------------- reach culling
def reach_scene(seed=71, n=3000, W=160, H=96):
    """Footprints at the edges of the plain form's reach test: axes from 0.05 to 60 px, needles
    at all angles, half the opacities just above 1/255 (alpha reaches 1/255 only near the
    centre), a third of the centres on tile and quadrant borders, some off-screen."""
    rng = np.random.default_rng(seed)
    s = gsinputs.make_scene("C1", seed=seed, n=n, width=W, height=H)
    k = n // 4
    th = rng.uniform(0, np.pi, n)
    s1 = np.concatenate([rng.uniform(0.05, 0.6, k), rng.uniform(0.3, 1.0, k),
                         rng.uniform(8.0, 60.0, k), rng.uniform(0.5, 8.0, n - 3 * k)])
    s2 = np.concatenate([rng.uniform(0.05, 0.6, k), rng.uniform(6.0, 40.0, k),
                         rng.uniform(8.0, 60.0, k), rng.uniform(0.5, 8.0, n - 3 * k)])
    s["conics"] = gsinputs.conic_from_axes(th, s1, s2).astype(np.float32)
    s["radii"] = np.ceil(3.0 * np.maximum(s1, s2)).astype(np.int32)
    op = rng.uniform(0.05, 0.99, n)
    op[::2] = rng.uniform(1.0 / 255.0, 3.0 / 255.0, len(op[::2]))
    s["opacity"] = op.astype(np.float32)
    m = s["means2d"]
    idx = rng.choice(n, n // 3, replace=False)
    m[idx] = (np.round(m[idx] / 8.0) * 8.0 +
              rng.choice([-0.5, 0.0, 0.5, 7.5], size=(len(idx), 2))).astype(np.float32)
    m[:40] -= np.float32(30.0)
    return s


@pytest.mark.parametrize("name", ["reach", "needles", "bigrects", "clustered", "ragged"])
def test_reach_culling_changes_nothing(gpu, name):
    """The plain form's reach culling (default) against the full scan (GSB_FULL_SCAN): image,
    final T and last contributor identical bit for bit, the deterministic backward's gradients
    identical bit for bit; the culled result also within the plain bounds of the oracle. The
    flag is a no-op for the GEMM forms."""
    s = reach_scene() if name == "reach" else VIS[name]
    W, H = s["width"], s["height"]
    bg = (0.1, 0.3, 0.2)
    ref = oracle.render(s, bg)
    sd = upload(s, gpu)
    pl, rg = upload_bins(ref["point_list"], ref["ranges"], gpu)
    rec = api.pack_gaussians(sd["means2d"], sd["conics"], sd["opacity"], sd["colors"])
    gd = torch.from_numpy(gsinputs.make_dloss(W, H, 79)).to(gpu)
    ws = api.DetWorkspace(rec.shape[0], pl.numel(), device=gpu)
    for base in ("fp32", "bf16"):
        outs = {}
        for prec in (base, api.prec_code(base) | _lib.GSB_FULL_SCAN):
            f = api.blend_forward_packed(rec, rg, pl, W, H, bg, prec)
            b = api.blend_backward_deterministic(rec, rg, pl, W, H, f[1], f[2], gd, bg, prec, ws=ws)
            a = api.blend_forward(sd["means2d"], sd["conics"], sd["opacity"], sd["colors"], rg, pl,
                                  W, H, bg, prec)
            torch.cuda.synchronize()
            outs[prec] = ([x.cpu().numpy() for x in f], [x.cpu().numpy() for x in b],
                          [x.cpu().numpy() for x in a])
        (f0, b0, a0), (f1, b1, a1) = outs.values()
        for x, y in zip(f0 + b0 + a0, f1 + b1 + a1):
            np.testing.assert_array_equal(x, y)
        for x, y in zip(f0, a0):       # records and arrays: the same blend
            np.testing.assert_array_equal(x, y)
        if base == "fp32":
            check_plain(ref, *f0, name)
    say(f"  reach {name}: pairs {pl.numel()}, identical with and without culling")
