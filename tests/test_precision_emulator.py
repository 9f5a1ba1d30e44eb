"""Precision emulator of the GEMM form (CPU only): how much accuracy the 16-bit operands of the
exponent product cost, and why the GPU path splits each coefficient into a high and a low term.

With tile-local coordinates (x_hat = x_g - x_c, x_bar = x_c - x_p, x_c the tile centre) the
exponent of Eq. (power rewritten) is P = v_g . v_p + k with the per-pixel basis
v_p = [x_bar^2, y_bar^2, x_bar y_bar, x_bar, y_bar], exact in FP16 and BF16 (x_bar is a
multiple of 1/2 in [-7.5, 7.5]), the per-Gaussian vector
v_g = [-A/2, -C/2, -B, -(A x_hat + B y_hat), -(C y_hat + B x_hat)] and the constant
k = -Q(x_hat, y_hat) / 2. Here v_g is rounded to 16 bits with one term (hi) or two
(hi + lo, lo scaled by 2^12 before rounding so that it stays normal in FP16), the products are
exact (as in an MFMA with FP32 accumulation), k is rounded to FP32, and the blend of Eq.
(volume-render) with the thresholds of Alg. 1 is evaluated in FP64 with exact and emulated
exponents over the same lists. The assertions state the error band of each scheme: one FP16 term
perturbs alpha by ~1e-3 relative (too much for gradients checked to 1e-3), one BF16 term fails
50 dB, and two terms in either format are far inside both bounds.
"""
import math

import numpy as np
import pytest

import gsinputs
import oracle

LOG2E = 1.0 / math.log(2.0)
TAU = float(np.float32(1.0) / np.float32(255.0))
T_STOP = float(np.float32(1e-4))
A_MAX = float(np.float32(0.99))


def round_bf16(x):
    """Round FP64 values to BF16 (round to nearest even on the FP32 bit pattern)."""
    f = np.asarray(x, np.float64).astype(np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def round_f16(x):
    return np.asarray(x, np.float64).astype(np.float16).astype(np.float64)


def split(v, fmt, terms):
    """v rounded to `terms` 16-bit terms of format `fmt` (the low term pre-scaled by 2^12)."""
    rnd = round_f16 if fmt == "fp16" else round_bf16
    hi = rnd(v)
    if terms == 1:
        return hi
    lo = rnd((v - hi) * 4096.0) / 4096.0
    if terms == 2:
        return hi + lo
    lo2 = rnd((v - hi - lo) * 2.0 ** 24) / 2.0 ** 24
    return hi + lo + lo2


def exponents(scene, ids, tile, gx, fmt=None, terms=0):
    """[len(ids)][256] exponents P for the tile's 256 pixels: exact (fmt None) or through the
    rounded GEMM form."""
    tx, ty = tile % gx, tile // gx
    xc, yc = 16 * tx + 7.5, 16 * ty + 7.5
    px = (16 * tx + np.arange(16))[None, :].repeat(16, 0).ravel().astype(np.float64)
    py = (16 * ty + np.arange(16))[:, None].repeat(16, 1).ravel().astype(np.float64)
    m = scene["means2d"][ids].astype(np.float64)
    c = scene["conics"][ids].astype(np.float64)
    A, B, C = c[:, 0], c[:, 1], c[:, 2]
    if fmt is None:
        dx = m[:, 0, None] - px[None, :]
        dy = m[:, 1, None] - py[None, :]
        return -0.5 * (A[:, None] * dx * dx + C[:, None] * dy * dy) - B[:, None] * dx * dy
    xh, yh = m[:, 0] - xc, m[:, 1] - yc
    xb, yb = xc - px, yc - py
    vg = np.stack([-A / 2, -C / 2, -B, -(A * xh + B * yh), -(C * yh + B * xh)], 1)
    vp = np.stack([xb * xb, yb * yb, xb * yb, xb, yb], 0)
    k = (-0.5 * (A * xh * xh + 2 * B * xh * yh + C * yh * yh)).astype(np.float32).astype(np.float64)
    return split(vg, fmt, terms) @ vp + k[:, None]


def render(scene, pl, rg, W, H, fmt=None, terms=0):
    """Image [3][H][W] and, over contributing pairs, the alphas (exact scheme's pairs order)."""
    gx, gy = oracle.grid(W, H)
    img = np.zeros((3, gy * 16, gx * 16))
    alphas = []
    for t in range(gx * gy):
        ids = pl[rg[t, 0]:rg[t, 1]].astype(np.int64)
        tx, ty = t % gx, t // gx
        if len(ids) == 0:
            continue
        P = exponents(scene, ids, t, gx, fmt, terms)
        o = scene["opacity"][ids].astype(np.float64)
        a = np.minimum(A_MAX, o[:, None] * np.exp(np.minimum(P, 0.0)))
        T = np.ones(256)
        acc = np.zeros((3, 256))
        live = np.ones(256, bool)
        col = scene["colors"][ids].astype(np.float64)
        for j in range(len(ids)):
            ok = live & (a[j] >= TAU)
            Tn = T * (1 - a[j])
            stop = ok & (Tn < T_STOP)
            live &= ~stop
            ok &= ~stop
            acc += np.where(ok, a[j] * T, 0.0)[None, :] * col[j][:, None]
            alphas.append(np.where(ok, a[j], 0.0))
            T = np.where(ok, Tn, T)
        img[:, 16 * ty:16 * ty + 16, 16 * tx:16 * tx + 16] = acc.reshape(3, 16, 16)
    return img[:, :H, :W], np.concatenate(alphas) if alphas else np.zeros(0)


def scene_c1_like():
    return gsinputs.make_scene("C1")


def scene_c2_sigma():
    return gsinputs.make_scene("C2", n=8000, width=128, height=128, seed=12)


@pytest.mark.parametrize("make", [scene_c1_like, scene_c2_sigma], ids=["C1", "C2-sigma-128"])
def test_gemm_rounding_error_bands(make):
    s = make()
    W, H = s["width"], s["height"]
    pl, rg = oracle.bin_tiles(s["means2d"], s["radii"], s["depths"], W, H)
    exact, a_ex = render(s, pl, rg, W, H)
    # the exact exponents reproduce the FP64 oracle's image
    ref = oracle.forward(W, H, rg, pl, s["means2d"], s["conics"], s["opacity"], s["colors"])
    np.testing.assert_allclose(exact, ref["image"], atol=1e-12)

    def measure(fmt, terms):
        img, a = render(s, pl, rg, W, H, fmt, terms)
        mse = float(np.mean((img - exact) ** 2))
        psnr = math.inf if mse == 0 else 10 * math.log10(1.0 / mse)
        # alpha error over the pairs both evaluations blend (same positions, the lists agree)
        n = min(len(a), len(a_ex))
        both = (a[:n] > 0) & (a_ex[:n] > 0)
        rel = np.linalg.norm((a[:n] - a_ex[:n])[both]) / np.linalg.norm(a_ex[:n][both])
        return psnr, rel

    p16_1, r16_1 = measure("fp16", 1)
    p16_2, r16_2 = measure("fp16", 2)
    pb_1, rb_1 = measure("bf16", 1)
    pb_2, rb_2 = measure("bf16", 2)
    print(f"fp16x1 {p16_1:.1f} dB {r16_1:.1e} | fp16x2 {p16_2:.1f} dB {r16_2:.1e} | "
          f"bf16x1 {pb_1:.1f} dB {rb_1:.1e} | bf16x2 {pb_2:.1f} dB {rb_2:.1e}")
    # one 16-bit term: FP16 passes 50 dB but perturbs alpha by ~1e-3 or more; BF16 fails 50 dB
    assert p16_1 >= 50.0 and r16_1 >= 1e-3
    assert pb_1 < 50.0
    # two terms: far inside the 50 dB and 1e-3 bounds in both formats
    assert p16_2 >= 100.0 and r16_2 <= 1e-5
    assert pb_2 >= 80.0 and rb_2 <= 1e-3


def test_basis_is_exact_in_16_bits():
    # x_bar, y_bar in {-7.5, ..., 7.5} and their squares and products are exact in FP16 and BF16
    xb = np.arange(16) - 7.5
    grid = np.concatenate([xb, xb * xb, np.outer(xb, xb).ravel()])
    np.testing.assert_array_equal(round_f16(grid), grid)
    np.testing.assert_array_equal(round_bf16(grid), grid)


def test_rounding_helpers():
    # round to nearest even at the BF16 boundary, and FP16 as numpy rounds it
    assert round_bf16(1.0 + 2.0 ** -8) == 1.0                   # halfway: to even
    assert round_bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6    # halfway: to even (up)
    assert round_bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    v = np.array([0.1, -3.3, 1e-3])
    assert np.all(np.abs(split(v, "fp16", 2) - v) <= 2.0 ** -22 * np.abs(v) + 1e-12)
