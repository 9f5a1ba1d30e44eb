"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each expected value comes from a closed form,
an exact-arithmetic fixture (tests/golden/), an invariant, or an independent pure-Python brute
force written here from the definitions (Eq. (alpha), Eq. (power), Eq. (volume-render), the
per-pixel loop of Alg. 1, and the duplication/sort of §2.1(b)-(c)).
"""
import json
import math
import os

import numpy as np
import pytest

import gsinputs
import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TAU = float(np.float32(1.0) / np.float32(255.0))
T_STOP = float(np.float32(1e-4))
A_MAX = float(np.float32(0.99))


# ----------------------------------------------------------------------------- brute force
def bf_covered(x, y, r, W, H):
    """Tiles (tx, ty) a Gaussian covers, by scanning every tile: tile tx is covered when its left
    edge 16 tx is <= x + r - 1 and its right edge 16 (tx + 1) is > x - r (same for y)."""
    gx, gy = (W + 15) // 16, (H + 15) // 16
    if r <= 0:
        return []
    out = []
    for ty in range(gy):
        for tx in range(gx):
            if 16 * tx <= x + r - 1 and 16 * (tx + 1) > x - r and \
               16 * ty <= y + r - 1 and 16 * (ty + 1) > y - r:
                out.append((tx, ty))
    return out


def bf_render(scene, bg=(0.0, 0.0, 0.0)):
    """Per-pixel brute force over all Gaussians: candidates are the Gaussians whose covered tiles
    include the pixel's tile, ordered by (depth, index); then Alg. 1's loop with math.exp and the
    exponent written as the quadratic form d^T Sigma^-1 d."""
    W, H = scene["width"], scene["height"]
    m = scene["means2d"].astype(float)
    con = scene["conics"].astype(float)
    op = scene["opacity"].astype(float)
    col = scene["colors"].astype(float)
    dep = scene["depths"].astype(float)
    n = len(op)
    cov = [set(bf_covered(m[i, 0], m[i, 1], int(scene["radii"][i]), W, H)) for i in range(n)]
    image = np.zeros((3, H, W))
    final_T = np.ones((H, W))
    last = np.zeros((H, W), np.int64)
    for py in range(H):
        for px in range(W):
            tile = (px // 16, py // 16)
            cands = sorted((dep[i], i) for i in range(n) if tile in cov[i])
            T, acc, lst = 1.0, [0.0, 0.0, 0.0], 0
            for pos, (_, i) in enumerate(cands):
                d = np.array([m[i, 0] - px, m[i, 1] - py])
                S = np.array([[con[i, 0], con[i, 1]], [con[i, 1], con[i, 2]]])
                power = -0.5 * float(d @ S @ d)
                alpha = min(A_MAX, op[i] * math.exp(min(power, 0.0)))
                if alpha < TAU:
                    continue
                Tn = T * (1.0 - alpha)
                if Tn < T_STOP:
                    break
                for c in range(3):
                    acc[c] += alpha * T * col[i, c]
                T, lst = Tn, pos + 1
            # last_contrib counts positions in the tile's full list; the candidate list of the
            # pixel is that list, so the position carries over.
            for c in range(3):
                image[c, py, px] = acc[c] + T * bg[c]
            final_T[py, px], last[py, px] = T, lst
    return image, final_T, last


def small_scene(seed, n=80, W=40, H=24, depth_levels=None):
    s = gsinputs.make_scene("C1", seed=seed, n=n, width=W, height=H, depth_levels=depth_levels)
    # push a few Gaussians off-screen and switch a few off, to exercise clamping and r = 0
    s["means2d"][:5] -= np.float32(30.0)
    s["means2d"][5:8] += np.float32([W + 5, H + 3])
    s["radii"][8:11] = 0
    return s


# ----------------------------------------------------------------------------- binning
@pytest.mark.parametrize("seed", [11, 12, 13])
def test_bin_matches_bruteforce_rects_and_order(seed):
    s = small_scene(seed, depth_levels=3 if seed == 13 else None)   # seed 13: many depth ties
    W, H = s["width"], s["height"]
    pl, rg = oracle.bin_tiles(s["means2d"], s["radii"], s["depths"], W, H)
    gx, gy = oracle.grid(W, H)
    per_tile = {t: [] for t in range(gx * gy)}
    m = s["means2d"].astype(float)
    for i in range(len(s["radii"])):
        for tx, ty in bf_covered(m[i, 0], m[i, 1], int(s["radii"][i]), W, H):
            per_tile[ty * gx + tx].append((float(s["depths"][i]), i))
    assert len(pl) == sum(len(v) for v in per_tile.values())
    for t in range(gx * gy):
        want = [i for _, i in sorted(per_tile[t])]
        a, b = int(rg[t, 0]), int(rg[t, 1])
        if not want:
            assert (a, b) == (0, 0)
        assert pl[a:b].tolist() == want


def test_bin_rect_edges():
    # x - r and x + r + 15 exactly on tile boundaries: tx range is [floor((x-r)/16), floor((x+r+15)/16))
    means = np.array([[16.0, 16.0], [15.999, 0.5], [47.0, 8.0]], np.float32)
    radii = np.array([16, 1, 1], np.int32)
    depths = np.array([1.0, 2.0, 3.0], np.float32)
    pl, rg = oracle.bin_tiles(means, radii, depths, 64, 32)
    tiles = {t: pl[a:b].tolist() for t, (a, b) in enumerate(rg)}
    # G0: x in [0, 47/16) -> tx 0,1 ; y same -> ty 0,1
    # G1: x-1 = 14.999 -> tx0 0 ; x+16 = 31.999 -> tx1 1 ; y: -0.5 -> 0 ; 16.5 -> 1
    # G2: 46/16 -> 2 ; 63/16 -> 3 ; y: 7/16 -> 0 ; 24/16 -> 1
    assert tiles[0] == [0, 1] and tiles[1] == [0] and tiles[4] == [0] and tiles[5] == [0]
    assert tiles[2] == [2] and tiles[3] == [] and tiles[6] == []


# ----------------------------------------------------------------------------- forward
@pytest.mark.parametrize("seed", [21, 22])
def test_forward_matches_bruteforce(seed):
    s = small_scene(seed)
    bg = (0.1, 0.2, 0.3)
    got = oracle.render(s, bg)
    image, final_T, last = bf_render(s, bg)
    np.testing.assert_allclose(got["image"], image, rtol=0, atol=1e-12)
    np.testing.assert_allclose(got["final_T"], final_T, rtol=0, atol=1e-12)
    np.testing.assert_array_equal(got["last_contrib"], last)


def test_single_gaussian_analytic_falloff():
    # rotated, anisotropic, B != 0; radius deliberately smaller than 3 sigma so the tile rect clips
    theta, s1, s2 = 0.7, 5.0, 2.0
    con = gsinputs.conic_from_axes(np.array([theta]), np.array([s1]), np.array([s2]))[0]
    x0, y0, o = 20.3, 13.6, 0.9
    scene = {"width": 48, "height": 32, "means2d": np.array([[x0, y0]], np.float32),
             "conics": con[None].astype(np.float32), "opacity": np.array([o], np.float32),
             "colors": np.array([[0.25, 0.5, 1.0]], np.float32),
             "depths": np.array([5.0], np.float32), "radii": np.array([3], np.int32)}
    got = oracle.render(scene)
    A, B, C = (float(v) for v in scene["conics"][0])
    xf, yf = (float(v) for v in scene["means2d"][0])
    of = float(scene["opacity"][0])
    # covered tiles: tx in [floor(17.3/16), floor(38.3/16)) = [1, 2), ty in [floor(10.6/16), floor(31.6/16)) = [0, 1)
    for py in range(32):
        for px in range(48):
            inside = (px // 16 == 1) and (py // 16 == 0)
            d = np.array([xf - px, yf - py])
            alpha = of * math.exp(-0.5 * float(d @ np.array([[A, B], [B, C]]) @ d))
            if inside and alpha >= TAU:
                want = [alpha * c for c in (0.25, 0.5, 1.0)]
                assert got["last_contrib"][py, px] == 1
                assert got["final_T"][py, px] == pytest.approx(1 - alpha, abs=1e-14)
            else:
                want = [0.0, 0.0, 0.0]
                assert got["last_contrib"][py, px] == 0 and got["final_T"][py, px] == 1.0
            np.testing.assert_allclose(got["image"][:, py, px], want, atol=1e-14)
    # the clip is visible: just outside the covered tile alpha is still above the skip threshold
    d = np.array([xf - 15, yf - 13])
    assert of * math.exp(-0.5 * float(d @ np.array([[A, B], [B, C]]) @ d)) > TAU
    assert got["last_contrib"][13, 15] == 0


def test_mean_on_pixel_gives_alpha_equal_opacity():
    s = gsinputs.stack_scene(1, 0.37, at=(5.0, 9.0))
    got = oracle.render(s)
    o = float(np.float32(0.37))
    assert got["final_T"][9, 5] == 1.0 - o
    np.testing.assert_array_equal(got["image"][:, 9, 5], [o * 1.0, o * 0.5, o * 0.25])


def test_zero_opacity_is_background():
    s = gsinputs.make_scene("C1", seed=5, n=300)
    s["opacity"][:] = 0.0
    bg = (0.3, 0.6, 0.9)
    got = oracle.render(s, bg)
    for c in range(3):
        assert np.all(got["image"][c] == bg[c])
    assert np.all(got["final_T"] == 1.0) and np.all(got["last_contrib"] == 0)


def test_telescoping_unit_colour():
    s = gsinputs.make_scene("C1", seed=6, n=600)
    s["colors"][:] = 1.0
    got = oracle.render(s, (0.0, 0.0, 0.0))
    for c in range(3):   # sum_i alpha_i T_i = 1 - T_final
        np.testing.assert_allclose(got["image"][c], 1.0 - got["final_T"], atol=1e-13)
    got1 = oracle.render(s, (1.0, 1.0, 1.0))
    np.testing.assert_allclose(got1["image"], 1.0, atol=1e-13)


def test_two_stack_golden():
    g = json.load(open(os.path.join(GOLDEN, "two_stack.json")))
    px, py = g["pixel"]
    base = {"width": 16, "height": 16, "means2d": np.array([[px, py]] * 2, np.float32),
            "conics": np.array([[0.1, 0.02, 0.2]] * 2, np.float32),
            "opacity": np.array(g["opacity"], np.float32),
            "colors": np.array(g["colors"], np.float32), "radii": np.array([9, 9], np.int32)}
    for key, depths in (("front_first", [1.0, 2.0]), ("swapped", [2.0, 1.0])):
        s = dict(base, depths=np.array(depths, np.float32))
        got = oracle.render(s, g["bg"])
        np.testing.assert_allclose(got["image"][:, py, px], g[key]["image"], atol=1e-15)
        assert got["final_T"][py, px] == pytest.approx(g[key]["final_T"], abs=1e-15)
        assert got["last_contrib"][py, px] == g[key]["last_contrib"]


def test_five_stack_stops_golden():
    g = json.load(open(os.path.join(GOLDEN, "five_stack.json")))
    s = gsinputs.stack_scene(g["n"], g["opacity"], at=tuple(g["pixel"]))
    got = oracle.render(s)
    px, py = g["pixel"]
    assert got["last_contrib"][py, px] == g["last_contrib"] == 5
    assert got["final_T"][py, px] == pytest.approx(g["final_T"], rel=1e-14)
    np.testing.assert_allclose(got["image"][:, py, px], g["image"], rtol=1e-14)
    assert got["n_eval"][py, px] == 6
    # truncated lists reproduce every intermediate T (Eq. (volume-render) prefix products)
    pl, rg = oracle.bin_tiles(s["means2d"], s["radii"], s["depths"], 16, 16)
    for k, Tk in enumerate(g["T_after_each"], start=1):
        r2 = rg.copy()
        r2[0, 1] = r2[0, 0] + k
        f = oracle.forward(16, 16, r2, pl, s["means2d"], s["conics"], s["opacity"], s["colors"])
        assert f["final_T"][py, px] == pytest.approx(Tk, rel=1e-14)


def test_cull_threshold_is_strict():
    # alpha == 1/255 exactly (mean on the pixel, o = fp32(1/255)) is kept; one ulp below is skipped
    o = np.float32(1.0) / np.float32(255.0)
    keep = oracle.render(gsinputs.stack_scene(1, float(o)))
    assert keep["last_contrib"][8, 8] == 1
    below = np.nextafter(o, np.float32(0))
    skip = oracle.render(gsinputs.stack_scene(1, float(below)))
    assert skip["last_contrib"][8, 8] == 0 and skip["final_T"][8, 8] == 1.0


def test_alpha_clamp():
    s = gsinputs.stack_scene(1, 1.0)
    got = oracle.render(s)
    assert got["final_T"][8, 8] == pytest.approx(1.0 - A_MAX, abs=1e-15)
    # where the clamp is active alpha does not depend on opacity or the exponent
    g = np.zeros((3, 16, 16)); g[:, 8, 8] = 1.0
    b = oracle.backward(16, 16, got["ranges"], got["point_list"], s["means2d"], s["conics"],
                        s["opacity"], s["colors"], g)
    assert b["dopacity"][0] == 0.0 and np.all(b["dconics"] == 0.0)
    np.testing.assert_allclose(b["dcolors"][0], A_MAX, rtol=1e-15)


@pytest.mark.parametrize("cfg", ["C1"])
def test_invariants(cfg):
    s = gsinputs.make_scene(cfg)
    got = oracle.render(s)
    T = got["final_T"]
    assert T.min() >= T_STOP and T.max() <= 1.0
    assert got["image"].min() >= 0.0 and got["image"].max() <= 1.0 + 1e-12
    lens = (got["ranges"][:, 1] - got["ranges"][:, 0]).astype(np.int64)
    gx, _ = oracle.grid(s["width"], s["height"])
    tile = (np.arange(64)[:, None] // 16) * gx + (np.arange(64)[None, :] // 16)
    assert np.all(got["last_contrib"] <= lens[tile])
    assert np.all(got["last_contrib"] <= got["n_eval"])
    # transmittance never increases as the list grows
    prev = np.ones_like(T)
    for k in (50, 150, 300, 10_000):
        r2 = got["ranges"].copy()
        r2[:, 1] = np.minimum(r2[:, 1], r2[:, 0] + k)
        f = oracle.forward(64, 64, r2, got["point_list"], s["means2d"], s["conics"], s["opacity"],
                           s["colors"])
        assert np.all(f["final_T"] <= prev)
        prev = f["final_T"]
    np.testing.assert_array_equal(prev, T)


def test_permutation_invariance():
    s = gsinputs.make_scene("C1", seed=7, n=800)
    perm = np.random.default_rng(0).permutation(800)
    sp = dict(s)
    for k in ("means2d", "conics", "opacity", "colors", "depths", "radii"):
        sp[k] = s[k][perm]
    a, b = oracle.render(s), oracle.render(sp)
    np.testing.assert_array_equal(a["image"], b["image"])
    np.testing.assert_array_equal(a["last_contrib"], b["last_contrib"])


def test_empty_scene_and_empty_tiles():
    s = gsinputs.make_scene("C1", seed=8, n=3, width=70, height=37)
    s["radii"][:] = 0
    got = oracle.render(s, (0.5, 0.25, 0.125))
    assert len(got["point_list"]) == 0 and np.all(got["ranges"] == 0)
    assert np.all(got["final_T"] == 1.0)
    np.testing.assert_array_equal(got["image"][2], 0.125)


# ----------------------------------------------------------------------------- Eq. (power rewritten)
def test_gemm_identity_fp64():
    """power = v_g . v_p with the reference pixel at the tile centre (x_c = x0 + 7.5) and
    x_bar = x_c - x_p (Eq. 4 and Eq. (power rewritten)); checked against the quadratic form."""
    rng = np.random.default_rng(3)
    for _ in range(200):
        A, C = rng.uniform(1e-3, 4, 2)
        B = rng.uniform(-1, 1) * math.sqrt(A * C) * 0.99
        xg, yg = rng.uniform(-80, 100, 2)
        x0, y0 = 16 * rng.integers(0, 5, 2)
        xc, yc = x0 + 7.5, y0 + 7.5
        xh, yh = xg - xc, yg - yc
        vg = np.array([-A / 2, -C / 2, -B, -A * xh - B * yh, -C * yh - B * xh,
                       -A * xh * xh / 2 - C * yh * yh / 2 - B * xh * yh])
        for px in range(x0, x0 + 16, 5):
            for py in range(y0, y0 + 16, 3):
                xb, yb = xc - px, yc - py
                vp = np.array([xb * xb, yb * yb, xb * yb, xb, yb, 1.0])
                d = np.array([xg - px, yg - py])
                direct = -0.5 * float(d @ np.array([[A, B], [B, C]]) @ d)
                assert abs(float(vg @ vp) - direct) <= 1e-12 * float(np.abs(vg * vp).sum())


# ----------------------------------------------------------------------------- backward
def _loss(scene, rg, pl, g, bg):
    f = oracle.forward(scene["width"], scene["height"], rg, pl, scene["means2d"], scene["conics"],
                       scene["opacity"], scene["colors"], bg)
    return float((f["image"] * g).sum())


def test_backward_closed_form_two_stack():
    # 1x1 image, pixel (0, 0); Gaussian 0 on the pixel, Gaussian 1 offset by (dx, dy)
    o = np.array([0.6, 0.5]); c = np.array([[0.9, 0.1, 0.2], [0.2, 0.7, 0.4]])
    A, B, C = 0.3, 0.1, 0.2
    dx, dy = 0.8, -0.6
    s = {"width": 1, "height": 1, "means2d": np.array([[0.0, 0.0], [dx, dy]]),
         "conics": np.array([[A, B, C], [A, B, C]]), "opacity": o, "colors": c,
         "depths": np.array([1.0, 2.0]), "radii": np.array([3, 3], np.int32)}
    bg = np.array([0.25, 0.5, 0.75]); g = np.array([0.3, -1.2, 0.7])
    pl, rg = oracle.bin_tiles(s["means2d"], s["radii"], s["depths"], 1, 1)
    got = oracle.backward(1, 1, rg, pl, s["means2d"], s["conics"], o, c, g.reshape(3, 1, 1), bg)
    P1 = -0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy
    G1 = math.exp(P1)
    a0, a1 = o[0], o[1] * G1
    # C = a0 c0 + (1 - a0) a1 c1 + (1 - a0)(1 - a1) bg
    dC_da0 = c[0] - a1 * c[1] - (1 - a1) * bg
    dC_da1 = (1 - a0) * (c[1] - bg)
    dL_da1 = float(g @ dC_da1)
    np.testing.assert_allclose(got["dopacity"], [float(g @ dC_da0), G1 * dL_da1], rtol=1e-13)
    np.testing.assert_allclose(got["dcolors"], [a0 * g, (1 - a0) * a1 * g], rtol=1e-13)
    dP = o[1] * G1 * dL_da1
    np.testing.assert_allclose(got["dconics"][1], [-0.5 * dx * dx * dP, -dx * dy * dP, -0.5 * dy * dy * dP], rtol=1e-12)
    np.testing.assert_allclose(got["dmeans2d"][1], [-(A * dx + B * dy) * dP, -(B * dx + C * dy) * dP], rtol=1e-12)
    np.testing.assert_allclose(got["dmeans2d"][0], 0.0, atol=1e-15)
    np.testing.assert_allclose(got["dconics"][0], 0.0, atol=1e-15)


def test_backward_matches_finite_differences():
    s = gsinputs.fd_subscene(33)
    W, H = s["width"], s["height"]
    bg = np.array([0.2, 0.4, 0.1])
    g = gsinputs.make_dloss(W, H, 34).astype(np.float64)
    pl, rg = oracle.bin_tiles(s["means2d"], s["radii"], s["depths"], W, H)
    an = oracle.backward(W, H, rg, pl, s["means2d"], s["conics"], s["opacity"], s["colors"], g, bg)
    rng = np.random.default_rng(35)
    ids = rng.choice(len(s["opacity"]), 60, replace=False)
    groups = {"dmeans2d": ("means2d", 2), "dconics": ("conics", 3), "dopacity": ("opacity", 1),
              "dcolors": ("colors", 3)}
    for gname, (key, width) in groups.items():
        fd_vals, an_vals = [], []
        for i in ids:
            for j in range(width):
                est = []
                for h_rel in (1e-6, 5e-7):
                    base = s[key].copy()
                    flat = base.reshape(len(s["opacity"]), -1)
                    h = h_rel * max(1.0, abs(flat[i, j]))
                    vals = []
                    for sign in (1, -1):
                        pert = base.copy().reshape(len(s["opacity"]), -1)
                        pert[i, j] += sign * h
                        s2 = dict(s)
                        s2[key] = pert.reshape(base.shape)
                        vals.append(_loss(s2, rg, pl, g, bg))
                    est.append((vals[0] - vals[1]) / (2 * h))
                # a decision (skip / stop) flipping inside [-h, h] makes the two estimates disagree
                if abs(est[0] - est[1]) > 1e-5 * (1.0 + abs(est[0])):
                    continue
                fd_vals.append(est[1])
                an_vals.append(an[gname].reshape(len(s["opacity"]), -1)[i, j])
        fd_vals, an_vals = np.array(fd_vals), np.array(an_vals)
        assert len(fd_vals) >= 0.9 * len(ids) * width, gname
        err = np.linalg.norm(fd_vals - an_vals) / max(np.linalg.norm(an_vals), 1e-30)
        assert err <= 1e-6, (gname, err)


def test_power_clamp_for_indefinite_conic():
    """Reading of an unstated case: a positive exponent (only reachable by rounding, or by a
    conic that is not positive definite) is clamped to 0, so alpha = min(0.99, o) there, and the
    clamped exponent passes no gradient."""
    s = gsinputs.stack_scene(1, 0.5, at=(8.0, 8.0))
    s["conics"][:] = np.float32([[-0.02, 0.0, 0.01]])     # power > 0 along x, < 0 along y
    got = oracle.render(s)
    assert got["final_T"][8, 12] == pytest.approx(0.5, abs=1e-15)     # dx = -4: power = +0.16
    c32 = float(np.float32(0.01))
    assert got["final_T"][12, 8] == pytest.approx(1 - 0.5 * math.exp(-0.5 * c32 * 16), abs=1e-15)
    pl, rg = oracle.bin_tiles(s["means2d"], s["radii"], s["depths"], 16, 16)
    g = np.zeros((3, 16, 16)); g[0, 8, 12] = 1.0
    b = oracle.backward(16, 16, rg, pl, s["means2d"], s["conics"], s["opacity"], s["colors"], g)
    assert np.all(b["dconics"] == 0.0) and np.all(b["dmeans2d"] == 0.0)
    assert b["dopacity"][0] == pytest.approx(1.0, abs=1e-15)


def test_work_counters():
    """n_contrib counts blended Gaussians: the five-stack blends 5 of 6 at its centre pixel, and
    every pixel blends at most last_contrib Gaussians, which is at most n_eval."""
    g = json.load(open(os.path.join(GOLDEN, "five_stack.json")))
    got = oracle.render(gsinputs.stack_scene(g["n"], g["opacity"], at=tuple(g["pixel"])))
    px, py = g["pixel"]
    assert got["n_contrib"][py, px] == 5 and got["n_eval"][py, px] == 6
    s = gsinputs.make_scene("C1")
    f = oracle.render(s)
    assert np.all(f["n_contrib"] <= f["last_contrib"]) and np.all(f["last_contrib"] <= f["n_eval"])
    # with the skip threshold never met nothing is blended
    s["opacity"][:] = 0.003
    f0 = oracle.render(s)
    assert f0["n_contrib"].sum() == 0
    c = oracle.work_counts(f, f["ranges"])
    assert c["K"] == int(f["n_contrib"].sum()) and c["Eb"] == int(f["last_contrib"].sum())


def tile_stacks_scene():
    """A 40x20 image (3 x 2 tiles; the right tile column is 8 px wide, the bottom row 4 px high)
    where tile t = ty * 3 + tx holds its own stack of k_t = (7, 1, 3, 2, 5, 4) nearly flat
    Gaussians (conic 1e-8 I, so alpha = 0.8 (1 - O(1e-6)) on every pixel of the tile; radius 1 at
    (16 tx + 4, 16 ty + 2) covers that tile alone), plus, in front of tile 4's stack, one sharp
    Gaussian (conic 100 I, o = 0.99) on pixel (20, 18) that reaches alpha >= 1/255 there only."""
    k = (7, 1, 3, 2, 5, 4)
    means, depth = [], []
    for t, kt in enumerate(k):
        tx, ty = t % 3, t // 3
        for j in range(kt):
            means.append((16 * tx + 4.0, 16 * ty + 2.0))
            depth.append(10.0 * (t + 1) + j)
    n = len(means)
    s = {"width": 40, "height": 20,
         "means2d": np.array(means + [(20.0, 18.0)], np.float32),
         "conics": np.array([[1e-8, 0.0, 1e-8]] * n + [[100.0, 0.0, 100.0]], np.float32),
         "opacity": np.array([0.8] * n + [0.99], np.float32),
         "colors": np.full((n + 1, 3), 0.5, np.float32),
         "depths": np.array(depth + [1.0], np.float32),
         "radii": np.ones(n + 1, np.int32)}
    return s


def test_work_counts_hand_fixture():
    """E, Eb, K, F and P of a scene whose per-pixel stop positions follow by hand (the F of
    work_counts is the per-tile maximum of the stop position, summed over tiles; a reshape or
    transpose of its tile grouping changes it). Transmittance 0.2^j after j blends of alpha 0.8:
    a stack of k blends min(k, 5) (the 6th would take T to 6.4e-5 < 1e-4), so a pixel evaluates
    min(k, 6) entries and its last contributor is position min(k, 5). On pixel (20, 18) the sharp
    Gaussian blends first (T = 0.01), then 0.002 and 0.0004, and the third stack member would take
    T to 8e-5: 4 evaluations, 3 blends, last contributor 3; tile 4's other 63 pixels skip it
    (alpha ~ 0.99 e^-50 one pixel away) and blend all 5: 6 evaluations, last contributor 6."""
    s = tile_stacks_scene()
    f = oracle.render(s)
    c = oracle.work_counts(f, f["ranges"])
    px = (256, 256, 128, 64, 64, 32)            # pixels of tiles 0..5 inside the 40x20 image
    n_eval = (6, 1, 3, 2, 6, 4)                  # per pixel; tile 4's exception is pixel (20, 18)
    blends = (5, 1, 3, 2, 5, 4)
    last = (5, 1, 3, 2, 6, 4)
    E = sum(p * e for p, e in zip(px, n_eval)) - 6 + 4
    K = sum(p * b for p, b in zip(px, blends)) - 5 + 3
    Eb = sum(p * l for p, l in zip(px, last)) - 6 + 3
    assert (E, K, Eb) == (2814, 2494, 2557)
    assert f["n_eval"][18, 20] == 4 and f["last_contrib"][18, 20] == 3
    assert c == {"E": E, "Eb": Eb, "K": K, "F": 6 + 1 + 3 + 2 + 6 + 4, "P": 7 + 1 + 3 + 2 + 6 + 4}
    # F against a pixel loop over each tile's own pixels, on a scene with uneven stops
    s2 = gsinputs.make_scene("C1", seed=12, n=600, width=70, height=37)
    f2 = oracle.render(s2)
    gx, gy = oracle.grid(70, 37)
    F = 0
    for t in range(gx * gy):
        tx, ty = t % gx, t // gx
        F += max(int(f2["n_eval"][py, px_]) for py in range(16 * ty, min(16 * ty + 16, 37))
                 for px_ in range(16 * tx, min(16 * tx + 16, 70)))
    assert oracle.work_counts(f2, f2["ranges"])["F"] == F


def test_bin_tile_matches_bruteforce():
    s = small_scene(14, depth_levels=3)
    W, H = s["width"], s["height"]
    gx, gy = oracle.grid(W, H)
    m = s["means2d"].astype(float)
    for t in range(gx * gy):
        want = sorted((float(s["depths"][i]), i) for i in range(len(s["radii"]))
                      if (t % gx, t // gx) in bf_covered(m[i, 0], m[i, 1], int(s["radii"][i]), W, H))
        got = oracle.bin_tile(s["means2d"], s["radii"], s["depths"], W, H, t)
        assert got.tolist() == [i for _, i in want]
    pl, rg = oracle.sampled_bins(s["means2d"], s["radii"], s["depths"], W, H, [0, 3, 5])
    assert np.count_nonzero(rg[:, 1] - rg[:, 0]) <= 3


# ----------------------------------------------------------------------------- binning mode 1
def bf_tile_max_alpha(scene, i, tx, ty):
    """Largest alpha = min(0.99, o exp(min(P, 0))) of Gaussian i over the pixels of tile (tx, ty)
    that lie inside the image, by direct evaluation of the quadratic form at every pixel."""
    W, H = scene["width"], scene["height"]
    px = np.arange(16 * tx, min(16 * tx + 16, W), dtype=float)
    py = np.arange(16 * ty, min(16 * ty + 16, H), dtype=float)
    X, Y = np.meshgrid(px, py)
    m = scene["means2d"][i].astype(float)
    a, b, c = scene["conics"][i].astype(float)
    dx, dy = m[0] - X, m[1] - Y
    P = -0.5 * (a * dx * dx + 2.0 * b * dx * dy + c * dy * dy)
    return float(np.max(np.minimum(A_MAX, float(scene["opacity"][i]) * np.exp(np.minimum(P, 0.0)))))


def needle_scene(seed=61, n=60, W=56, H=40):
    """Strongly anisotropic Gaussians (axis ratio up to 64) at all angles, opacities down to
    just above 1/255: the case where the 3-sigma square overstates the footprint most."""
    rng = np.random.default_rng(seed)
    s = gsinputs.make_scene("C1", seed=seed, n=n, width=W, height=H)
    th = rng.uniform(0, np.pi, n)
    s1 = rng.uniform(0.5, 1.0, n)
    s2 = rng.uniform(4.0, 32.0, n)
    s["conics"] = gsinputs.conic_from_axes(th, s1, s2).astype(np.float32)
    s["radii"] = np.ceil(3.0 * np.maximum(s1, s2)).astype(np.int32)
    s["opacity"] = rng.uniform(1.0 / 255.0, 0.99, n).astype(np.float32)
    return s


VIS_SCENES = {"C1": lambda: gsinputs.make_scene("C1"), "small": lambda: small_scene(21),
              "needles": needle_scene}


@pytest.mark.parametrize("name", list(VIS_SCENES))
def test_visible_binning_drops_only_invisible_pairs(name):
    """Mode 1 keeps every pair whose Gaussian reaches alpha >= 1/255 on an image pixel of the tile,
    and every pair it drops stays below (1/255) e^-0.05 on the whole tile (the stated margin)."""
    s = VIS_SCENES[name]()
    W, H = s["width"], s["height"]
    gx, gy = oracle.grid(W, H)
    pl0, rg0 = oracle.bin_tiles(s["means2d"], s["radii"], s["depths"], W, H)
    pl1, rg1 = oracle.bin_tiles(s["means2d"], s["radii"], s["depths"], W, H, s["conics"],
                                s["opacity"], oracle.BIN_VISIBLE)
    dropped = 0
    for t in range(gx * gy):
        full = pl0[rg0[t, 0]:rg0[t, 1]].tolist()
        kept = pl1[rg1[t, 0]:rg1[t, 1]].tolist()
        assert kept == [i for i in full if i in set(kept)]     # a subsequence, same order
        for i in set(full) - set(kept):
            amax = bf_tile_max_alpha(s, i, t % gx, t // gx)
            assert amax < TAU * math.exp(-0.05), (name, t, i, amax)
            dropped += 1
    assert dropped > 0.2 * len(pl0), (name, dropped, len(pl0))


def rect_min_q(m, conic, x0, x1, y0, y1):
    """Minimum of Q(p) = d^T Sigma^-1 d, d = m - p, over the closed rectangle [x0, x1] x [y0, y1]
    of pixel positions, and a point where it is reached: the mean itself when it lies inside,
    else the best of the four edge minima, each edge the 1D quadratic Q restricted to it minimised
    at its stationary point clamped to the edge (every edge is tried, not only those facing the
    mean)."""
    a, b, c = (float(v) for v in conic)
    mx, my = float(m[0]), float(m[1])
    if x0 <= mx <= x1 and y0 <= my <= y1:
        return 0.0, mx, my

    def q(px, py):
        dx, dy = mx - px, my - py
        return a * dx * dx + 2.0 * b * dx * dy + c * dy * dy

    best = (math.inf, 0.0, 0.0)
    for px in (x0, x1):                      # vertical edges: dQ/dpy = 0 at py = my + b dx / c
        py = min(max(my + b * (mx - px) / c, y0), y1)
        best = min(best, (q(px, py), px, py))
    for py in (y0, y1):                      # horizontal edges
        px = min(max(mx + b * (my - py) / a, x0), x1)
        best = min(best, (q(px, py), px, py))
    return best


def visibility_threshold(o):
    """2 (e ln 2 + m - 1) + 0.1 with 255 o = m 2^e, m in [1, 2), from numpy's frexp."""
    mant, ex = np.frexp(255.0 * float(o))
    return 2.0 * ((int(ex) - 1) * math.log(2.0) + (2.0 * float(mant) - 1.0)) + 0.1


@pytest.mark.parametrize("name", list(VIS_SCENES))
def test_visible_binning_matches_rectangle_minimum(name):
    """Mode 1 in both directions against an independent minimum of Q over each tile's pixel
    rectangle (clipped to the image): a kept pair has min Q <= theta (+ rounding), and a pair of the
    3-sigma square with min Q < theta (- rounding) and o >= fp32(1/255) is kept. The analytic
    minimum is cross-checked against Q on a 1/8-pixel grid of the rectangle."""
    s = VIS_SCENES[name]()
    W, H = s["width"], s["height"]
    gx, gy = oracle.grid(W, H)
    pl0, rg0 = oracle.bin_tiles(s["means2d"], s["radii"], s["depths"], W, H)
    pl1, rg1 = oracle.bin_tiles(s["means2d"], s["radii"], s["depths"], W, H, s["conics"],
                                s["opacity"], oracle.BIN_VISIBLE)
    tau32 = float(np.float32(1.0) / np.float32(255.0))
    checked = 0
    for t in range(gx * gy):
        tx, ty = t % gx, t // gx
        x0, y0 = 16.0 * tx, 16.0 * ty
        x1, y1 = min(x0 + 15.0, W - 1.0), min(y0 + 15.0, H - 1.0)
        kept = set(pl1[rg1[t, 0]:rg1[t, 1]].tolist())
        for i in pl0[rg0[t, 0]:rg0[t, 1]].tolist():
            o = float(s["opacity"][i])
            mq, qx, qy = rect_min_q(s["means2d"][i], s["conics"][i], x0, x1, y0, y1)
            if checked % 7 == 0:                 # the analytic minimum against a dense grid
                h = 0.125
                X, Y = np.meshgrid(np.arange(x0, x1 + 1e-9, h), np.arange(y0, y1 + 1e-9, h))
                a, b, c = (float(v) for v in s["conics"][i])
                mx, my = float(s["means2d"][i][0]), float(s["means2d"][i][1])
                dx, dy = mx - X, my - Y
                dense = float(np.min(a * dx * dx + 2 * b * dx * dy + c * dy * dy))
                # every grid point is in the rectangle: the minimum is not above any of them
                assert mq <= dense * (1 + 1e-12) + 1e-12, (name, t, i, mq, dense)
                # the grid point nearest the minimiser (within h / sqrt 2) bounds it from above:
                # Q(p* + v) <= Q(p*) + |grad Q(p*)| |v| + lmax |v|^2
                ex, ey = mx - qx, my - qy
                grad = 2.0 * math.hypot(a * ex + b * ey, b * ex + c * ey)
                lmax = 0.5 * (a + c) + math.hypot(0.5 * (a - c), b)
                v = h / math.sqrt(2.0)
                assert dense <= mq + grad * v + lmax * v * v + 1e-9, (name, t, i, mq, dense)
            checked += 1
            th = visibility_threshold(o)
            eps = 1e-9 * (1.0 + th)
            if i in kept:
                assert o >= tau32 and mq <= th + eps, (name, t, i, mq, th)
            elif o >= tau32:
                assert mq >= th - eps, (name, t, i, mq, th)
    assert checked > 0


@pytest.mark.parametrize("name", list(VIS_SCENES))
def test_visible_binning_keeps_images(name):
    """The forward over mode-1 lists equals the forward over the 3-sigma lists exactly (image and
    final T), and each pixel's last contributor is the same Gaussian."""
    s = VIS_SCENES[name]()
    W, H = s["width"], s["height"]
    gx, gy = oracle.grid(W, H)
    pl0, rg0 = oracle.bin_tiles(s["means2d"], s["radii"], s["depths"], W, H)
    pl1, rg1 = oracle.bin_tiles(s["means2d"], s["radii"], s["depths"], W, H, s["conics"],
                                s["opacity"], oracle.BIN_VISIBLE)
    args = (s["means2d"], s["conics"], s["opacity"], s["colors"], (0.2, 0.1, 0.3))
    r0 = oracle.forward(W, H, rg0, pl0, *args)
    r1 = oracle.forward(W, H, rg1, pl1, *args)
    assert np.array_equal(r0["image"], r1["image"]) and np.array_equal(r0["final_T"], r1["final_T"])
    for py in range(H):
        for px in range(W):
            t = (py // 16) * gx + px // 16
            l0, l1 = r0["last_contrib"][py, px], r1["last_contrib"][py, px]
            assert (l0 == 0) == (l1 == 0)
            if l0:
                assert pl0[rg0[t, 0] + l0 - 1] == pl1[rg1[t, 0] + l1 - 1]


def test_visible_binning_edge_cases():
    """Opacity below 1/255 emits nothing; a Gaussian visible only beyond the image's right edge is
    dropped from the partial edge tile; one centred on a tile is kept there."""
    W, H = 40, 20                                   # last tile column holds pixels 32..39 only
    s = gsinputs.stack_scene(3, 0.5, width=W, height=H, at=(8.0, 8.0))
    s["means2d"][1] = (46.0, 8.0)                   # 6 px right of the last pixel column
    s["conics"][1] = (4.0, 0.0, 4.0)                # sigma 0.5: alpha ~ 0.5 exp(-72) at x = 39
    s["radii"][1] = 8
    s["opacity"][2] = np.float32(1.0 / 255.0) * np.float32(0.999)
    s["radii"][2] = 4
    pl, rg = oracle.bin_tiles(s["means2d"], s["radii"], s["depths"], W, H, s["conics"],
                              s["opacity"], oracle.BIN_VISIBLE)
    assert 2 not in pl.tolist()
    assert 1 not in pl.tolist()
    gx, _ = oracle.grid(W, H)
    assert 0 in pl[rg[0, 0]:rg[0, 1]].tolist()
    pl0, _ = oracle.bin_tiles(s["means2d"], s["radii"], s["depths"], W, H)
    assert 1 in pl0.tolist() and 2 in pl0.tolist()   # the 3-sigma square does emit them
