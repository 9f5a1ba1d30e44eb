"""Helpers shared by the GPU tests: upload a scene, run the library, compare with the oracle."""
from __future__ import annotations

import math
import sys

import numpy as np
import torch

import oracle
from paper_2604_02120_amd import api

# Tolerances (the derivation of each is written once, in the design notes' numerics section).
#
# Decision margins. The oracle reports per pixel the smallest relative distance of any of its
# skip (alpha vs 1/255) or stop (T' vs 1e-4) decisions to the threshold. A decision closer than the
# path's own error can go either way, so exact comparisons (last_contrib, the tight absolute bounds)
# cover only the pixels whose margin exceeds the path's bound:
#   fp32: alpha is off by <= 1.2e-6 relative (worst case over contributing pairs, compensated
#         exponent) and T' by the measured relative T error (check_plain asserts it stays below
#         MARGIN / 2), so 1e-5 covers both;
#   fp16: the hi + lo operands put the exponent within 4e-5 of the exact one (the precision
#         emulator's worst case), i.e. alpha within 4e-5 relative; 1e-4 covers it;
#   bf16: hi + lo leaves up to 3e-3 in the exponent (emulator), so 1e-2.
MARGIN = {"fp32": 1e-5, "fp16": 1e-4, "bf16": 1e-2}
PLAIN_ABS = 1e-5        # plain FP32 image and final_T, non-marginal pixels
# GEMM forms, per channel on non-marginal pixels: the alpha error (4e-5 / 3e-3 relative) times
# sum(alpha T c) <= 1, with a factor ~2 of room
GEMM_ABS = {"fp16": 1e-4, "bf16": 5e-3}
# Every pixel, every path: one flipped skip decision adds or removes a term alpha T c < 1/255 and
# rescales the rest of the pixel by (1 - alpha), a change below 2/255 = 7.8e-3; a flipped stop
# decision changes it by less than 2e-4
FLIP_ABS = 1e-2
MAX_EXCLUDED = 0.01     # at most 1% of pixels may be marginal (fp32, fp16)
# last_contrib on non-marginal pixels: exact for fp32 and fp16. For bf16 the exponent error grows
# with the Gaussian's offset from the tile centre and the transmittance error compounds over the
# contributors, so a few decisions beyond the 1e-2 margin still flip (3 of 2.07M pixels at 1080p):
# a fraction of 1e-5 of the region's pixels is allowed.
MAX_LAST_MISMATCH = {"fp16": 0.0, "bf16": 1e-5}
GEMM_PSNR = 50.0        # FP16/BF16 GEMM path vs FP64 oracle, all pixels
GEMM_GRAD = 1e-3        # normwise relative gradient error, GEMM path
PLAIN_GRAD = 1e-5       # normwise relative gradient error, plain FP32 path
# Two stress scenes take 5e-5 in the plain form:
#   clustered (saturated pixels, lists up to ~8700 entries): the transmittance that the backward
#     recovers by division, T_i = T_(i+1) / (1 - alpha_i), carries the FP32 rounding of every
#     opaque layer between the pixel's end and the pair; measured 2.9e-5 (means);
#   bigrects (sigma up to 64 px, footprints of up to ~600 tiles): each such Gaussian's gradient is
#     a sum of hundreds of per-tile partials of both signs in FP32; measured 3.2e-5 (conics), the
#     same with either reduction of the per-tile sums.
# The whole 4K frame (C5) has the same tail of large footprints (log-normal sigma): its conic
# gradient measures 2.7e-5, the same with and without reach culling.
PLAIN_GRAD_STRESS = 5e-5
STRESS_SCENES = ("clustered", "bigrects", "C5")


def plain_grad_bound(scene: str) -> float:
    return PLAIN_GRAD_STRESS if scene in STRESS_SCENES else PLAIN_GRAD


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def upload(scene: dict, dev) -> dict:
    out = {"width": scene["width"], "height": scene["height"]}
    for k in ("means2d", "conics", "opacity", "colors", "depths"):
        out[k] = torch.from_numpy(np.ascontiguousarray(scene[k], np.float32)).to(dev)
    out["radii"] = torch.from_numpy(np.ascontiguousarray(scene["radii"], np.int32)).to(dev)
    return out


def upload_bins(point_list, ranges, dev):
    pl = torch.from_numpy(np.ascontiguousarray(point_list).astype(np.int32)).to(dev)
    rg = torch.from_numpy(np.ascontiguousarray(ranges).astype(np.int32)).to(dev)
    return pl, rg


def gpu_forward(sd: dict, pl, rg, prec, bg=(0.0, 0.0, 0.0)):
    img, T, last = api.blend_forward(sd["means2d"], sd["conics"], sd["opacity"], sd["colors"], rg,
                                     pl, sd["width"], sd["height"], bg, prec)
    torch.cuda.synchronize()
    return img.cpu().numpy().astype(np.float64), T.cpu().numpy().astype(np.float64), \
        last.cpu().numpy()


def psnr(a: np.ndarray, b: np.ndarray) -> float:
    mse = float(np.mean((a - b) ** 2))
    return math.inf if mse == 0 else 10.0 * math.log10(1.0 / mse)


def _region(ref, mask):
    return np.ones(ref["final_T"].shape, bool) if mask is None else mask


def check_plain(ref: dict, img, T, last, label="", mask=None):
    """Plain FP32 path. Pixels whose every decision is further than MARGIN["fp32"] from its
    threshold must match in last_contrib exactly and in image / final_T within PLAIN_ABS; the
    relative final_T error there must stay below half that margin (the margin must exceed the
    error of the quantity the stop test compares); every pixel within FLIP_ABS."""
    region = _region(ref, mask)
    ok = region & (ref["margin"] > MARGIN["fp32"])
    frac_excluded = 1.0 - ok.sum() / max(region.sum(), 1)
    err_img = np.abs(img - ref["image"])[:, ok].max(initial=0.0)
    err_T = np.abs(T - ref["final_T"])[ok].max(initial=0.0)
    rel_T = (np.abs(T - ref["final_T"]) / ref["final_T"])[ok].max(initial=0.0)
    err_all = np.abs(img - ref["image"])[:, region].max(initial=0.0)
    mism = int((last != ref["last_contrib"])[ok].sum())
    say(f"  plain {label}: max|d image| {err_img:.3e}  max|d T| {err_T:.3e}  max rel d T "
        f"{rel_T:.3e}  last mismatches {mism}  excluded {frac_excluded:.2e}  all-pixel max|d| "
        f"{err_all:.3e}  psnr {psnr(img[:, region], ref['image'][:, region]):.1f} dB")
    assert frac_excluded < MAX_EXCLUDED
    assert mism == 0
    assert err_img <= PLAIN_ABS and err_T <= PLAIN_ABS
    assert rel_T <= 0.5 * MARGIN["fp32"]
    assert err_all <= FLIP_ABS
    return err_img


def check_gemm(ref: dict, img, T, last, prec, label="", mask=None):
    """GEMM form (fp16 / bf16): PSNR >= GEMM_PSNR over every pixel of the region; per channel,
    max |d| <= FLIP_ABS over every pixel and <= GEMM_ABS[prec] over the pixels whose decisions are
    further than MARGIN[prec] from their thresholds, where last_contrib must also match."""
    region = _region(ref, mask)
    d = np.abs(img - ref["image"])
    p = psnr(img[:, region], ref["image"][:, region])
    ok = region & (ref["margin"] > MARGIN[prec])
    frac_excluded = 1.0 - ok.sum() / max(region.sum(), 1)
    maxabs = [float(d[c][region].max(initial=0.0)) for c in range(3)]
    maxabs_ok = [float(d[c][ok].max(initial=0.0)) for c in range(3)]
    mism = int((last != ref["last_contrib"])[ok].sum())
    say(f"  gemm {prec} {label}: psnr {p:.1f} dB  max|d| per channel {maxabs}  non-marginal "
        f"{maxabs_ok} (excluded {frac_excluded:.2e}, last mismatches {mism})  "
        f"max|d T| {np.abs(T - ref['final_T'])[region].max(initial=0.0):.3e}")
    assert p >= GEMM_PSNR
    assert max(maxabs) <= FLIP_ABS
    assert max(maxabs_ok) <= GEMM_ABS[prec]
    assert mism <= MAX_LAST_MISMATCH[prec] * region.sum()
    return p


def normwise(a, b) -> float:
    d = np.linalg.norm(np.ravel(a) - np.ravel(b))
    n = np.linalg.norm(np.ravel(b))
    return float(d / n) if n > 0 else float(d)
