"""GPU parity of the preprocessing step (gsb_project) against the FP64 oracle, and the whole
pipeline project -> bin -> blend.

Tolerances (FP32 kernel, unit roundoff u = 2^-24):
  * integers (radius, culling) are compared exactly wherever the oracle's decision is further
    from its threshold than the FP32 error allows: depth further than 1e-5 (relative) from the
    near plane, det / (a c) above 64 u kappa (the det's relative error bound, kappa below), the
    mean further than 1e-3 px + 1e-6 |mean| from the edge of the screen-rectangle test, and
    3 sqrt(lmax) further than 1e-5 (relative) from an integer (its FP32 error is a few u:
    lmax is a well-conditioned eigenvalue, with |(a - c) / 2| <= sqrt(disc));
  * means2d within 1e-6 relative + 2e-4 px, depth within 1e-6 relative;
  * conics: the entries of Sigma2 carry absolute errors ~ u (a + c), which its determinant and
    inverse amplify by kappa = (a + c)^2 / det; each conic entry must be within
    CONIC_C * u * kappa * max|conic| (CONIC_C = 64, measured errors stay below 1/8 of it);
  * colours (sums of <= 16 products of magnitude ~1) within 2e-5.
"""
import numpy as np
import pytest
import torch

import gsinputs
import oracle
from gpu_util import say
from paper_2604_02120_amd import api

pytestmark = pytest.mark.gpu
U32 = 2.0 ** -24
CONIC_C = 64.0


def cam_look(W, H, f=None, eye=(0.4, -0.3, -1.0), target=(0.0, 0.1, 10.0)):
    f = f or 0.52 * W
    return gsinputs.look_at(eye, target, (0.0, 1.0, 0.0), f, f, W, H)


def scene(n, W, H, seed, cam=None):
    return gsinputs.make_scene3d(n=n, seed=seed, width=W, height=H, camera=cam or cam_look(W, H))


def edge_scene(W=200, H=150):
    """Hand-made cases: behind the camera, at and around the near plane, off screen, beyond the
    Jacobian clamp, degenerate and huge scales, unnormalised quaternions."""
    cam = gsinputs.Camera(((1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0)), (0.0, 0.0, 0.0),
                          150.0, 160.0, 99.5, 74.5, W, H, 0.25)
    pts, sc, q = [], [], []

    def add(p, s=(0.02, 0.02, 0.02), quat=(1.0, 0.0, 0.0, 0.0)):
        pts.append(p), sc.append(s), q.append(quat)

    add((0.0, 0.0, -2.0))                        # behind
    add((0.0, 0.0, 0.25))                        # on the near plane
    add((0.0, 0.0, 0.2501))                      # just in front
    add((0.0, 0.0, 0.2499))                      # just behind it
    for x in (-3.0, -1.5, 1.5, 3.0):             # beyond the clamp (|x/z| up to 3 vs 0.87)
        add((x, 0.1, 1.0), s=(0.5, 0.5, 0.5))
        add((x, 0.1, 1.0), s=(0.002, 0.002, 0.002))   # same place, too small to reach the image
    add((0.1, 0.1, 3.0), s=(0.0, 0.05, 0.05))    # flat
    add((0.1, -0.1, 3.0), s=(0.0, 0.0, 0.0))     # a point: only the low-pass remains
    add((0.2, 0.0, 2.0), s=(0.3, 0.001, 0.001), quat=(0.9, 0.1, 0.3, 0.2))   # needle
    add((0.0, 0.2, 5.0), s=(1e-3, 2e-3, 3e-3), quat=(10.0, -4.0, 2.0, 1.0))  # unnormalised
    add((0.0, 0.0, 1000.0), s=(1.0, 1.0, 1.0))   # far
    add((0.0, 0.0, 0.5), s=(2.0, 2.0, 2.0))      # huge
    n = len(pts)
    rng = np.random.default_rng(9)
    return {"camera": cam, "means3d": np.asarray(pts, np.float32),
            "scales": np.asarray(sc, np.float32), "quats": np.asarray(q, np.float32),
            "opacity": np.full(n, 0.5, np.float32),
            "sh": rng.normal(0, 0.5, (n, 16, 3)).astype(np.float32)}


def gpu_project(s, dev, K=None, deg=None, guard=0):
    """Runs gsb_project on the scene's arrays (sh cut to K coefficients); outputs are views of
    buffers `guard` rows longer, filled with a sentinel, which must stay untouched."""
    K = K or s["sh"].shape[1]
    t = {k: torch.from_numpy(np.ascontiguousarray(s[k], np.float32)).to(dev)
         for k in ("means3d", "scales", "quats")}
    sh = torch.from_numpy(np.ascontiguousarray(s["sh"][:, :K], np.float32)).to(dev)
    n = s["means3d"].shape[0]
    bufs = (torch.full((n + guard, 2), -7.0, device=dev), torch.full((n + guard, 3), -7.0, device=dev),
            torch.full((n + guard,), -7.0, device=dev),
            torch.full((n + guard,), -7, dtype=torch.int32, device=dev),
            torch.full((n + guard, 3), -7.0, device=dev))
    out = tuple(b[:n] for b in bufs)
    api.project(t["means3d"], t["scales"], t["quats"], sh, s["camera"], sh_degree=deg, out=out)
    torch.cuda.synchronize()
    for b in bufs:
        assert bool((b[n:] == -7).all()), "write past n"
    return tuple(o.cpu().numpy() for o in out)


def check(ref, got, label, max_unsafe=1e-3):
    m2, con, dep, rad, col = got
    rr, mg, rc = ref["rad_real"], ref["margin"], ref["conics"]
    kappa = (rc[:, 0] + rc[:, 2]) ** 2 / np.maximum(rc[:, 0] * rc[:, 2] - rc[:, 1] ** 2, 1e-300)
    near_int = np.abs(rr - np.round(rr)) <= 1e-5 * np.maximum(rr, 1.0)
    safe = ((mg[:, 0] > 1e-5) & (mg[:, 1] > 64 * U32 * kappa) &
            (mg[:, 2] > 1e-3 + 1e-6 * np.abs(ref["means2d"]).max(axis=1)) & ~near_int)
    vis_ref, vis = ref["radii"] > 0, rad > 0
    mism_vis = int((vis_ref != vis)[safe].sum())
    mism_rad = int((rad != ref["radii"])[safe].sum())
    both = vis & vis_ref
    for name, arr in (("means2d", m2), ("conics", con), ("depths", dep), ("colors", col)):
        assert not arr[~vis].any(), f"{label}: culled {name} not zero"
    err_m = (np.abs(m2 - ref["means2d"]) / (1e-6 * np.abs(ref["means2d"]) + 2e-4))[both].max(initial=0)
    err_d = (np.abs(dep - ref["depths"]) / (1e-6 * np.abs(ref["depths"])))[both].max(initial=0)
    tol_c = CONIC_C * U32 * kappa[:, None] * np.abs(rc).max(axis=1, keepdims=True)
    err_c = (np.abs(con - rc) / tol_c)[both].max(initial=0)
    err_col = np.abs(col - ref["colors"])[both].max(initial=0)
    say(f"  {label}: n={len(rad)} visible={int(vis.sum())} unsafe={int((~safe).sum())} "
        f"vis/rad mismatches {mism_vis}/{mism_rad} | means {err_m:.3f} depth {err_d:.3f} "
        f"conic {err_c:.4f} (of tol) colour {err_col:.2e}")
    assert mism_vis == 0 and mism_rad == 0
    assert err_m <= 1 and err_d <= 1 and err_c <= 1 and err_col <= 2e-5
    assert (~safe).sum() <= max(2, max_unsafe * len(rad))
    return err_c


def test_project_parity_look_at_scene(gpu):
    s = scene(50_000, 640, 480, seed=21)
    say("[project] 50k, 640x480, look-at camera, degree 3")
    got = gpu_project(s, gpu, guard=64)
    check(oracle.project(s), got, "deg3")
    assert (got[3] == 0).mean() < 0.05


@pytest.mark.parametrize("K,deg", [(16, 3), (16, 0), (16, 1), (16, 2), (9, 2), (4, 1), (1, 0),
                                   (5, 1), (10, 2), (12, 2), (15, 2)])
def test_project_coefficient_layouts(gpu, K, deg):
    s = scene(4097, 320, 200, seed=22)
    say(f"[project] K={K} deg={deg} n=4097")
    s2 = dict(s, sh=np.ascontiguousarray(s["sh"][:, :K]))
    got = gpu_project(s, gpu, K=K, deg=deg, guard=70)
    check(oracle.project(s2, sh_degree=deg), got, f"K{K}d{deg}")


@pytest.mark.parametrize("n", [1, 63, 64, 65, 255, 256, 257, 1000])
def test_project_ragged_sizes(gpu, n):
    s = scene(n, 128, 96, seed=23 + n)
    say(f"[project] ragged n={n}")
    check(oracle.project(s), gpu_project(s, gpu, guard=65), f"n{n}")


def test_project_empty(gpu):
    s = scene(0, 64, 64, seed=1)
    z = {k: torch.empty((0,) + s[k].shape[1:], dtype=torch.float32, device=gpu)
         for k in ("means3d", "scales", "quats", "sh")}
    out = api.project(z["means3d"], z["scales"], z["quats"], z["sh"], s["camera"])
    torch.cuda.synchronize()
    assert all(o.numel() == 0 for o in out)


def test_project_edge_cases(gpu):
    s = edge_scene()
    say("[project] edge cases")
    ref = oracle.project(s)
    got = gpu_project(s, gpu, guard=3)
    check(ref, got, "edge", max_unsafe=0.34)
    rad = got[3]
    assert list(rad[:4] > 0) == [False, False, True, False]       # the near plane is exclusive
    # x/z = -3 and 3 reach no tile even with a 299 px radius; -1.5 and 1.5 do; small ones never
    assert list(rad[4:12:2] > 0) == [False, True, True, False]
    assert not (rad[5:12:2] > 0).any()
    assert (rad[12:] > 0).all()


def test_project_full_size_1080p(gpu):
    # the preprocessing workload of the 1080p, 1M-Gaussian frame, every Gaussian compared
    s = gsinputs.make_scene3d(n=1_000_000, seed=7)
    say("[project] 1M Gaussians, 1920x1080")
    check(oracle.project(s), gpu_project(s, gpu), "1080p")


def test_pipeline_project_bin_blend(gpu):
    """3D scene -> (project, bin, blend) on the GPU against the same chain in the oracle."""
    W, H = 320, 240
    s = scene(30_000, W, H, seed=24)
    say("[pipeline] 30k Gaussians 320x240")
    ref = oracle.project(s)
    pl_r, rg_r = oracle.bin_tiles(ref["means2d"], ref["radii"], ref["depths"], W, H)
    img_r = oracle.forward(W, H, rg_r, pl_r, ref["means2d"], ref["conics"], s["opacity"],
                           ref["colors"])["image"]
    t = {k: torch.from_numpy(np.ascontiguousarray(s[k], np.float32)).to(gpu)
         for k in ("means3d", "scales", "quats", "sh", "opacity")}
    m2, con, dep, rad, col = api.project(t["means3d"], t["scales"], t["quats"], t["sh"], s["camera"])
    pl, rg = api.bin_tiles(m2, rad, dep, W, H)
    img, _, _ = api.blend_forward(m2, con, t["opacity"], col, rg, pl, W, H, prec="fp32")
    torch.cuda.synchronize()
    img = img.cpu().numpy().astype(np.float64)
    d = np.abs(img - img_r)
    psnr = 10 * np.log10(1.0 / max(float(np.mean(d ** 2)), 1e-300))
    say(f"  pipeline fp32: psnr {psnr:.1f} dB, max|d| {d.max():.2e}, "
        f"pixels > 1e-4: {(d.max(axis=0) > 1e-4).mean():.2e}")
    assert psnr >= 60.0
    assert (d.max(axis=0) > 1e-4).mean() < 1e-3
    # the GEMM blend on the same GPU projection
    img16, _, _ = api.blend_forward(m2, con, t["opacity"], col, rg, pl, W, H, prec="fp16")
    torch.cuda.synchronize()
    d16 = img16.cpu().numpy().astype(np.float64) - img_r
    assert 10 * np.log10(1.0 / float(np.mean(d16 ** 2))) >= 50.0
