#!/usr/bin/env python3
"""Throughput of the differentiable Gaussian blend on one MI355X.

Workload (the headline configuration, the largest that the metric names): one 3840x2160 frame
of 3,000,000 projected 2D Gaussians (log-normal footprint, median sigma 3 px, opacity
Beta(2, 2) x 0.99; seeded synthetic stand-in for the paper's trained scenes), upstream gradient
dL/dimage ~ N(0, 1). One step is the whole hot path for that frame: tile binning (count,
duplicate, radix sort, ranges) + forward blend + backward blend, with inputs resident in HBM. The
GEMM form with BF16 hi+lo operands on MFMA (FP32 accumulate, FP32 transmittance and colour) is
the headline; the plain FP32 per-pixel form and the FP16 GEMM form are timed the same way.

Prints one JSON line. `value` = frame pixels / (forward + backward blend time), the metric's
fwd+bwd blend rate (binning is timed separately); `step_mpix_s` = frame pixels x steps / wall time
of the timed steps, binning included. Beside the headline the line carries: `roofline` (the
dominant kernel against the published FP32 vector peak, HBM traffic from the counters of the same
workload), `counters` (issue and bandwidth fractions from rocprofv3 counters), `paths` (every
precision), `visible_binning` (the same step with the opacity-aware tile extent), `pipeline_3d`
(a 1080p step preceded by projecting 1M 3D Gaussians), `batched_c4` (16 views in one launch per
direction, replayed from a hipGraph), `cpu_baseline` (the FP64 oracle on the host's cores, median
of 3 full frames) and `accuracy` (every path against that oracle).

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline] [--no-visible] [--no-pipeline]
                    [--no-batched]
    python bench.py --sweep            # LDS batch size and resolution sweeps
    python bench.py --pipeline-only    # the 3D leg alone
    python bench.py --config C2        # the same line for another workload (C2: 1920x1080, 1M;
                                       # C3: 1280x720, 500k)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

import gsinputs  # noqa: E402
from paper_2604_02120_amd import api, autotune  # noqa: E402

METRIC = "Mpix/s fwd+bwd blend, GEMM-form vs plain FP32 on 1 MI355X at ≥50 dB vs oracle"
# Published FP32 vector peak of the MI355X (packed FP32: 256 CUs x 4 SIMDs x 16 lanes x 2 (FMA)
# x 2 (packed) x 2.4 GHz). Packed FP32 is disabled in this build, so the reachable rate is half:
PEAK_FP32_TFLOPS = 157.3
PEAK_FP32_NONPACKED_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# Algorithmic operations per evaluated pair (unit counts of the blend, fixed in advance):
#   forward : 1 exp + ~11 VALU (GEMM form; the exponent's 12 MFMA flops not counted here) or
#             1 exp + ~20 VALU (plain form), per evaluation (E)
#   backward: 1 exp + 1 rcp + ~30 VALU per revisited evaluation (Eb)
OPS_PER_EVAL = {("forward", "gemm"): 12, ("forward", "plain"): 21, ("backward", "gemm"): 32,
                ("backward", "plain"): 32}
# A finer count from the definition (each add, multiply, compare, min, exp one operation):
#   forward : 16 per evaluated pair + 10 per blended pair
#   backward: 16 per revisited pair + 39 per blended pair
FLOPS = {"forward": (16, 10), "backward": (16, 39)}
COUNTS = os.path.join(ROOT, "tests", "golden", "workload_counts.json")
OPACITY_LAW = {"uniform": "U(0.05, 0.99)", "beta22": "Beta(2, 2) x 0.99"}
TRAFFIC = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2604_02120_amd", "csrc", "blend.hip")
PROJECT_SRC = os.path.join(ROOT, "paper_2604_02120_amd", "csrc", "project.hip")


def parse():
    p = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=10)
    p.add_argument("--config", default="C5", choices=["C2", "C3", "C5"])
    p.add_argument("--precs", default="bf16,fp32,fp16,fp32_scan",
                   help="comma list; the first is the headline")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--arrays", action="store_true",
                   help="blend from the four attribute arrays instead of packed records")
    p.add_argument("--no-batched", action="store_true",
                   help="skip the 16-view batched measurement")
    p.add_argument("--no-deterministic", action="store_true",
                   help="skip the deterministic backward's measurement")
    p.add_argument("--no-visible", action="store_true",
                   help="skip the step with visible-tile binning")
    p.add_argument("--no-pipeline", action="store_true",
                   help="skip the leg that starts from 3D Gaussians (projection + the step)")
    p.add_argument("--pipeline-only", action="store_true",
                   help="run only the leg that starts from 3D Gaussians and print its JSON object")
    p.add_argument("--sweep", action="store_true",
                   help="instead of the benchmark line: sensitivity sweeps of the LDS batch size "
                        "and of the resolution (1x, 2x, 3x), GEMM form vs plain FP32")
    p.add_argument("--reduce-study", action="store_true",
                   help="instead of the benchmark line: backward time with the per-Gaussian sums "
                        "reduced on the vector ALUs vs on the matrix cores, on the 1080p, 4K and "
                        "a dense-footprint scene")
    p.add_argument("--peaks", action="store_true",
                   help="instead of the benchmark line: attainable FP32 FMA, exp2 and FP16 MFMA "
                        "rates of this GPU from a microbenchmark, beside the published peaks")
    p.add_argument("--calib-copy-mib", type=int, default=0,
                   help="also run one device-to-device copy of this many MiB (a known-size "
                        "kernel for scaling HBM byte counters)")
    return p.parse_args()


class Frame:
    """Device buffers of one frame: inputs, binning workspace sized for the exact pair count,
    outputs and gradients."""

    def __init__(self, cfg, dev, bin_mode="rect", scene=None):
        self.bin_mode = bin_mode
        s = gsinputs.make_scene(cfg) if scene is None else scene
        self.scene = s
        self.W, self.H, self.n = s["width"], s["height"], len(s["radii"])
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
        self.means2d, self.conics, self.opacity = t(s["means2d"]), t(s["conics"]), t(s["opacity"])
        self.colors, self.depths, self.radii = t(s["colors"]), t(s["depths"]), t(s["radii"])
        self.dloss_np = gsinputs.make_dloss(self.W, self.H, cfg.dloss_seed if cfg else 1002)
        self.dloss = t(self.dloss_np)
        ws0 = api.BinWorkspace(self.n, 0, self.W, self.H, device=dev)
        self.pairs = int(api.bin_count(self.means2d, self.radii, self.W, self.H, ws0,
                                       conics=self.conics, opacity=self.opacity,
                                       mode=bin_mode).item())
        self.ws = api.BinWorkspace(self.n, self.pairs, self.W, self.H, device=dev)
        gx, gy = api.grid(self.W, self.H)
        self.point_list = torch.empty(self.pairs, dtype=torch.int32, device=dev)
        self.ranges = torch.empty((gx * gy, 2), dtype=torch.int32, device=dev)
        self.fwd_out = (torch.empty((3, self.H, self.W), device=dev),
                        torch.empty((self.H, self.W), device=dev),
                        torch.empty((self.H, self.W), dtype=torch.int32, device=dev))
        self.bwd_out = (torch.empty((self.n, 2), device=dev), torch.empty((self.n, 3), device=dev),
                        torch.empty((self.n,), device=dev), torch.empty((self.n, 3), device=dev))
        self.records = torch.empty((self.n, 12), device=dev)
        self.packed = True       # blend from packed records (the pack is timed with the forward)
        self.status = None

    @classmethod
    def from_scene(cls, scene, dev, bin_mode="rect"):
        return cls(None, dev, bin_mode, scene)

    def step(self, prec, ev=None):
        if ev is not None:
            ev[0].record()
        api.bin_count(self.means2d, self.radii, self.W, self.H, self.ws, conics=self.conics,
                      opacity=self.opacity, mode=self.bin_mode)
        self.status = api.bin_fill(self.means2d, self.radii, self.depths, self.W, self.H, self.ws,
                                   self.point_list, self.ranges, conics=self.conics,
                                   opacity=self.opacity, mode=self.bin_mode)
        if ev is not None:
            ev[1].record()
        if self.packed:
            api.pack_gaussians(self.means2d, self.conics, self.opacity, self.colors,
                               out=self.records)
            img, T, last = api.blend_forward_packed(self.records, self.ranges, self.point_list,
                                                    self.W, self.H, (0.0, 0.0, 0.0), prec,
                                                    out=self.fwd_out)
        else:
            img, T, last = api.blend_forward(self.means2d, self.conics, self.opacity, self.colors,
                                             self.ranges, self.point_list, self.W, self.H,
                                             (0.0, 0.0, 0.0), prec, out=self.fwd_out)
        if ev is not None:
            ev[2].record()
        if self.packed:
            api.blend_backward_packed(self.records, self.ranges, self.point_list, self.W, self.H,
                                      T, last, self.dloss, (0.0, 0.0, 0.0), prec, out=self.bwd_out)
        else:
            api.blend_backward(self.means2d, self.conics, self.opacity, self.colors, self.ranges,
                               self.point_list, self.W, self.H, T, last, self.dloss,
                               (0.0, 0.0, 0.0), prec, out=self.bwd_out)
        if ev is not None:
            ev[3].record()


def time_path(fr: Frame, prec: str, steps: int, warmup: int) -> dict:
    for _ in range(warmup):
        fr.step(prec)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        fr.step(prec, evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if int(fr.status.item()) != 0:
        raise RuntimeError("binning overflowed its capacity")
    bin_ms = [e[0].elapsed_time(e[1]) for e in evs]
    fwd_ms = [e[1].elapsed_time(e[2]) for e in evs]
    bwd_ms = [e[2].elapsed_time(e[3]) for e in evs]
    px = fr.W * fr.H
    r = {
        "ms_per_step": 1e3 * wall / steps,
        "mpix_s": px * steps / wall / 1e6,
        "bin_ms": float(np.mean(bin_ms)), "fwd_ms": float(np.mean(fwd_ms)),
        "bwd_ms": float(np.mean(bwd_ms)),
        "fwd_ms_p10_p90": [float(np.percentile(fwd_ms, 10)), float(np.percentile(fwd_ms, 90))],
        "bwd_ms_p10_p90": [float(np.percentile(bwd_ms, 10)), float(np.percentile(bwd_ms, 90))],
        "fwd_ms_median": float(np.median(fwd_ms)), "bwd_ms_median": float(np.median(bwd_ms)),
    }
    r["blend_mpix_s"] = px / ((r["fwd_ms"] + r["bwd_ms"]) * 1e-3) / 1e6
    return r


def time_batched(steps: int, warmup: int, dev) -> dict:
    """The multi-view workload: 16 views (854x480 / 1280x720 / 1920x1080 drawn with seed 4), 300k
    Gaussians each, FP16 GEMM form. One step = binning of every view + one persistent forward
    launch + one persistent backward launch, autotuned, replayed from a hipGraph. Also timed:
    the same step eagerly, and as a loop of single-view calls."""
    scenes = gsinputs.make_views()
    views = []
    for sc in scenes:
        d = {"width": sc["width"], "height": sc["height"]}
        for k in ("means2d", "conics", "opacity", "colors", "depths", "radii"):
            d[k] = torch.from_numpy(np.ascontiguousarray(sc[k])).to(dev)
        views.append(d)
    bv = api.BatchedViews(views, prec="fp16", tuning="auto")
    for i, v in enumerate(bv.views):
        v["dL_dimage"].copy_(torch.from_numpy(gsinputs.make_dloss(v["width"], v["height"], 500 + i)))
    px = bv.pixels()

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        a.record()
        for _ in range(steps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / steps, a.elapsed_time(b) / steps

    eager_wall, eager_ev = timed(lambda: bv.step(check=False))
    bv.check()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        bv.step()
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        bv.step()
    graph_wall, graph_ev = timed(graph.replay)

    def per_view_loop():
        for v in bv.views:
            W, H = v["width"], v["height"]
            api.bin_count(v["means2d"], v["radii"], W, H, v["ws"])
            api.bin_fill(v["means2d"], v["radii"], v["depths"], W, H, v["ws"], v["point_list"],
                         v["ranges"])
            img, T, last = api.blend_forward(v["means2d"], v["conics"], v["opacity"], v["colors"],
                                             v["ranges"], v["point_list"], W, H, (0.0, 0.0, 0.0),
                                             "fp16", out=(v["image"], v["final_T"], v["last_contrib"]))
            api.blend_backward(v["means2d"], v["conics"], v["opacity"], v["colors"], v["ranges"],
                               v["point_list"], W, H, T, last, v["dL_dimage"], (0.0, 0.0, 0.0),
                               "fp16", out=(v["dL_dmeans2d"], v["dL_dconics"], v["dL_dopacity"],
                                            v["dL_dcolors"]))
    loop_wall, loop_ev = timed(per_view_loop)
    # batched kernels alone (binning excluded), eager, for the blend-only rate
    def fwd_bwd():
        bv.forward()
        bv.backward()
    fb_wall, fb_ev = timed(fwd_bwd)
    del graph
    tune = {k: bv.tuning.get(k) for k in autotune.KEYS}
    trials = bv.tuning.get("trials")
    out = {"workload": "16 views from {854x480, 1280x720, 1920x1080} (seed 4), 300k Gaussians "
                       "each (seeds 400+v); step = bin all views + batched fwd + batched bwd",
           "views": len(bv.views), "pixels": px, "gaussians": sum(v["n"] for v in bv.views),
           "tuning": tune, "tuning_trials_ms": trials,
           "graph_ms_per_step": round(graph_ev, 4), "graph_mpix_s": round(px / graph_ev / 1e3, 2),
           "eager_ms_per_step": round(eager_ev, 4),
           "per_view_loop_ms_per_step": round(loop_ev, 4),
           "batched_blend_ms": round(fb_ev, 4), "batched_blend_mpix_s": round(px / fb_ev / 1e3, 2)}
    bv.close()
    return out


def time_deterministic(fr: Frame, prec: str, steps: int, warmup: int, head: dict) -> dict:
    """The deterministic backward on the headline frame (after a step, so binning, records and
    the forward's outputs are current): its time beside the atomic backward's, whether repeated
    runs are identical bit for bit, and its normwise distance from the atomic gradients."""
    img, T, last = fr.fwd_out
    ws = api.DetWorkspace(fr.n, fr.pairs, device=fr.records.device)
    outs = [tuple(torch.empty_like(x) for x in fr.bwd_out) for _ in range(2)]
    run = lambda o: api.blend_backward_deterministic(  # noqa: E731
        fr.records, fr.ranges, fr.point_list, fr.W, fr.H, T, last, fr.dloss, (0.0, 0.0, 0.0), prec,
        ws=ws, out=o)
    for _ in range(warmup):
        run(outs[0])
    torch.cuda.synchronize()
    ms = []
    for k in range(steps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        run(outs[k % 2])
        b.record()
        b.synchronize()
        ms.append(a.elapsed_time(b))
    run(outs[1])
    torch.cuda.synchronize()
    same = all(torch.equal(x, y) for x, y in zip(outs[0], outs[1]))
    atomic = [g.double() for g in fr.bwd_out]
    diff = max(float(torch.linalg.vector_norm(x.double() - y) / torch.linalg.vector_norm(y))
               for x, y in zip(outs[0], atomic))
    return {"precision": prec, "bwd_ms_median": round(float(np.median(ms)), 4),
            "atomic_bwd_ms": round(head["bwd_ms"], 4), "workspace_bytes": ws.nbytes,
            "bit_identical_across_runs": same, "max_normwise_vs_atomic": float(f"{diff:.3e}")}


def time_visible(scene, dev, prec: str, steps: int, warmup: int, head: dict, ref_out) -> dict:
    """The same step with binning mode "visible" (only tiles where alpha can reach 1/255): fewer
    pairs, the same images. Reported beside the headline, which bins with the 3-sigma square."""
    fr = Frame(None, dev, bin_mode="visible", scene=scene)
    r = time_path(fr, prec, steps, warmup)
    out = {"mode": "visible", "precision": prec, "pairs": fr.pairs,
           **{k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()},
           "speedup_vs_rect_binning": {"step": round(head["ms_per_step"] / r["ms_per_step"], 3),
                                       "blend": round(r["blend_mpix_s"] / head["blend_mpix_s"], 3)}}
    if ref_out is not None:       # the images must be those of the 3-sigma binning, bit for bit
        img, T, _ = (x.cpu().numpy() for x in fr.fwd_out)
        out["image_identical_to_rect_binning"] = bool(
            np.array_equal(img.astype(np.float64), ref_out[0]) and np.array_equal(T, ref_out[1]))
    return out


def time_pipeline(dev, prec: str, steps: int, warmup: int) -> dict:
    """The step preceded by preprocessing: 1,000,000 3D Gaussians (SH degree 3, 16 coefficients)
    seen by a 1920x1080 pinhole camera are projected (gsb_project), then binned, blended forward
    and backward as in the headline step. Reports each stage and the projection kernel against
    HBM bandwidth: it moves 40 + 12 * 16 bytes in and 40 bytes out per Gaussian."""
    s = gsinputs.make_scene3d(n=1_000_000, seed=7)
    t = {k: torch.from_numpy(np.ascontiguousarray(s[k], np.float32)).to(dev)
         for k in ("means3d", "scales", "quats", "sh", "opacity")}
    n, K = s["means3d"].shape[0], s["sh"].shape[1]
    cam = api.camera_struct(s["camera"].R, s["camera"].t, s["camera"].fx, s["camera"].fy,
                            s["camera"].cx, s["camera"].cy, s["camera"].width,
                            s["camera"].height, s["camera"].near)
    proj = (torch.empty((n, 2), device=dev), torch.empty((n, 3), device=dev),
            torch.empty((n,), device=dev), torch.empty((n,), dtype=torch.int32, device=dev),
            torch.empty((n, 3), device=dev))
    api.project(t["means3d"], t["scales"], t["quats"], t["sh"], cam, out=proj)
    m2, con, dep, rad, col = proj
    fr = Frame.from_scene({"width": s["camera"].width, "height": s["camera"].height,
                           "means2d": m2.cpu().numpy(), "conics": con.cpu().numpy(),
                           "opacity": s["opacity"], "colors": col.cpu().numpy(),
                           "depths": dep.cpu().numpy(), "radii": rad.cpu().numpy()}, dev)
    # the frame reads the projection's own buffers, which every step rewrites
    fr.means2d, fr.conics, fr.colors, fr.depths, fr.radii = m2, con, col, dep, rad

    def step(ev=None):
        if ev is not None:
            ev[0].record()
        api.project(t["means3d"], t["scales"], t["quats"], t["sh"], cam, out=proj)
        fr.step(prec, None if ev is None else ev[1:])

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if int(fr.status.item()) != 0:
        raise RuntimeError("binning overflowed its capacity")
    ms = lambda a, b: float(np.mean([e[a].elapsed_time(e[b]) for e in evs]))  # noqa: E731
    proj_ms = ms(0, 1)
    # the projection kernel alone: 20 launches captured in a graph and replayed, so that host
    # launch gaps stay out of the events
    reps = 20
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side), torch.cuda.graph(g, stream=side):
        for _ in range(reps):
            api.project(t["means3d"], t["scales"], t["quats"], t["sh"], cam, out=proj)
    torch.cuda.current_stream().wait_stream(side)
    g.replay()
    torch.cuda.synchronize()
    ge = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    kern = []
    for _ in range(5):
        ge[0].record()
        g.replay()
        ge[1].record()
        torch.cuda.synchronize()
        kern.append(ge[0].elapsed_time(ge[1]) / reps)
    kern_ms = float(np.median(kern))
    nbytes = n * (40 + 12 * K + 40)
    gbs = nbytes / (kern_ms * 1e-3) / 1e9
    ent = traffic_entry("P3D", "project", PROJECT_SRC)   # HBM bytes from the counters, if current
    traffic = ent["bytes_per_launch"] if ent else None
    return {"workload": "1M 3D Gaussians, SH degree 3, 1920x1080 camera", "precision": prec,
            "visible": int((rad > 0).sum().item()), "pairs": fr.pairs,
            "ms_per_step": round(1e3 * wall / steps, 4),
            "mpix_s": round(fr.W * fr.H * steps / wall / 1e6, 2),
            "project_ms": round(proj_ms, 4), "project_kernel_ms": round(kern_ms, 4),
            "bin_ms": round(ms(1, 2), 4),
            "fwd_ms": round(ms(2, 3), 4), "bwd_ms": round(ms(3, 4), 4),
            "project_roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": 8000.0,
                                 "unit": "GB/s", "frac": round(gbs / 8000.0, 4),
                                 "traffic": traffic, "bytes_per_gaussian": 40 + 12 * K + 40}}


def run_sweeps(dev, steps: int, warmup: int) -> dict:
    """Sensitivity sweeps on the 1080p scene: (1) forward and backward time per LDS batch size
    b (single-view plans with fixed launch shapes), (2) the same scene rendered at 1x, 2x and 3x
    resolution (means and axis lengths scaled), forward + backward blend time, each in the FP16
    GEMM form and the plain FP32 form (reach-culled, and as a full scan)."""
    def upload(sc):
        d = {"width": sc["width"], "height": sc["height"]}
        for k in ("means2d", "conics", "opacity", "colors", "depths", "radii"):
            d[k] = torch.from_numpy(np.ascontiguousarray(sc[k])).to(dev)
        return d

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        ms = []
        for _ in range(steps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            b.synchronize()
            ms.append(a.elapsed_time(b))
        return float(np.median(ms))

    out = {"batch": [], "resolution": []}
    base = gsinputs.make_scene("C2")
    view = upload(base)
    g = torch.from_numpy(gsinputs.make_dloss(base["width"], base["height"], 1002)).to(dev)
    for prec in ("fp16", "fp32", "fp32_scan"):
        for nb in (64, 128, 256):
            bv = api.BatchedViews([view], prec=prec,
                                  tuning={"batch_fwd": nb, "batch_bwd": nb, "launch": 1})
            bv.views[0]["dL_dimage"].copy_(g)
            bv.bin()
            out["batch"].append({"precision": prec, "b": nb, "fwd_ms": round(timed(bv.forward), 4),
                                 "bwd_ms": round(timed(bv.backward), 4)})
            bv.close()
    for scale in (1, 2, 3):
        sc = gsinputs.make_scene("C2", scale=float(scale))
        fr = Frame.from_scene(sc, dev)
        row = {"scale": scale, "width": sc["width"], "height": sc["height"], "pairs": fr.pairs}
        for prec in ("fp16", "fp32", "fp32_scan"):
            r = time_path(fr, prec, steps, warmup)
            row[prec] = {"fwd_ms": round(r["fwd_ms"], 4), "bwd_ms": round(r["bwd_ms"], 4),
                         "blend_mpix_s": round(r["blend_mpix_s"], 2)}
        for plain in ("fp32", "fp32_scan"):
            sfx = "" if plain == "fp32" else "_vs_full_scan"
            row["gemm_speedup_fwd" + sfx] = round(row[plain]["fwd_ms"] / row["fp16"]["fwd_ms"], 3)
            row["gemm_speedup_blend" + sfx] = round(
                row["fp16"]["blend_mpix_s"] / row[plain]["blend_mpix_s"], 3)
        out["resolution"].append(row)
        del fr
        torch.cuda.empty_cache()
    return out


# Large, overlapping footprints: most of a 16-Gaussian group is live in most wavefronts.
DENSE = gsinputs.SceneConfig("dense", 1920, 1080, 200_000, "loguniform", 4.0, 32.0, "uniform", 48)


def reduce_study(dev, steps: int, warmup: int) -> list:
    """Backward blend time with the per-Gaussian gradient sums reduced on the vector ALUs
    (bwd_reduce 0) and with the geometric sums as a matrix-core product (bwd_reduce 1), through
    one-view plans launched one block per tile, for each precision, on three scenes."""
    rows = []
    for name, cfg in (("C2", gsinputs.CONFIGS["C2"]), ("C5", gsinputs.CONFIGS["C5"]),
                      ("dense", DENSE)):
        sc = gsinputs.make_scene(cfg)
        d = {"width": sc["width"], "height": sc["height"]}
        for k in ("means2d", "conics", "opacity", "colors", "depths", "radii"):
            d[k] = torch.from_numpy(np.ascontiguousarray(sc[k])).to(dev)
        g = torch.from_numpy(gsinputs.make_dloss(sc["width"], sc["height"], 1002)).to(dev)
        for prec in ("bf16", "fp16", "fp32"):
            row = {"scene": name, "width": sc["width"], "height": sc["height"],
                   "gaussians": len(sc["radii"]), "precision": prec}
            for red, nb in ((0, 128), (1, 128), (1, 64)):
                bv = api.BatchedViews([d], prec=prec, tuning={"launch": 1, "batch_bwd": nb,
                                                               "bwd_reduce": red})
                bv.views[0]["dL_dimage"].copy_(g)
                bv.bin()
                bv.forward()
                for _ in range(warmup):
                    bv.backward()
                torch.cuda.synchronize()
                ms = []
                for _ in range(steps):
                    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    a.record()
                    bv.backward()
                    b.record()
                    b.synchronize()
                    ms.append(a.elapsed_time(b))
                row[f"bwd_ms_{'mfma' if red else 'valu'}_b{nb}"] = round(float(np.median(ms)), 4)
                row["pairs"] = bv.views[0]["pairs"]
                bv.close()
            rows.append(row)
        del d
        torch.cuda.empty_cache()
    return rows


def measure_peaks() -> dict:
    """Attainable issue rates from the microbenchmark library (libgsbpeaks.so): independent chains
    of FP32 FMA (not packed), of exp2 each followed by a multiply, and of
    v_mfma_f32_32x32x16_f16, over 8 blocks of 256 threads per compute unit."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2604_02120_amd", "libgsbpeaks.so"))
    lib.gsbpk_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                              ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double)]
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    out = {"compute_units": cus, "blocks": 8 * cus}
    simd_cycles = 4 * cus * 2.4e9          # SIMD-cycles per second at 2.4 GHz
    for which, name, iters in ((0, "fma_f32", 1 << 16), (1, "exp2_f32_plus_mul", 1 << 14),
                               (2, "mfma_f32_32x32x16_f16", 1 << 14)):
        ms, ops = ctypes.c_float(0.0), ctypes.c_double(0.0)
        if lib.gsbpk_run(which, 8 * cus, iters, ctypes.byref(ms), ctypes.byref(ops)) != 0:
            raise RuntimeError(f"microbenchmark {name} failed")
        rate = ops.value / (ms.value * 1e-3)
        r = {"ms": round(ms.value, 4), "ops": ops.value}
        if which == 0:
            r["tflops"] = round(2 * rate / 1e12, 2)
            r["published_tflops_packed"] = PEAK_FP32_TFLOPS
            r["wave64_instr_per_simd_cycle"] = round(rate / 64 / simd_cycles, 4)
        elif which == 1:
            r["exp2_per_s"] = rate
            r["wave64_exp2_per_simd_cycle"] = round(rate / 64 / simd_cycles, 4)
        else:
            r["tflops"] = round(rate * 32 * 32 * 16 * 2 / 1e12, 1)
            r["published_tflops_dense_fp16"] = 2500.0
        out[name] = r
    return out


def kernel_hash(src: str = None) -> str:
    """Hash of a kernel source's code with its comments and whitespace removed: counters taken
    from a kernel stay attached to it through edits of its comments, not through code changes."""
    text = open(src or KERNEL_SRC, encoding="utf-8").read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return hashlib.sha256(" ".join(text.split()).encode()).hexdigest()[:16]


def traffic_entry(config: str, kern: str, src: str = None):
    """Counter-derived entry of `kern` for workload `config` from profiles/traffic.json, if it
    was taken from the current kernel source (else None)."""
    if not os.path.exists(TRAFFIC):
        return None
    ent = json.load(open(TRAFFIC)).get(config, {}).get(kern)
    if ent and ent.get("kernel_sha") == kernel_hash(src):
        return ent
    return None


def roofline(res: dict, counts: dict, config: str, prec: str) -> dict:
    """ALU roofline of the dominant blend kernel (the slower of forward / backward): algorithmic
    operations per launch (the unit counts above x the oracle's evaluation counts) / the
    kernel's mean duration from HIP events over the timed steps, against the published FP32 peak.
    The measured HBM traffic is attached when counters of this workload and kernel source exist."""
    kern = "backward" if res["bwd_ms"] >= res["fwd_ms"] else "forward"
    form = "plain" if prec == "fp32" else "gemm"
    evals = counts["E"] if kern == "forward" else counts["Eb"]
    ops = OPS_PER_EVAL[(kern, form)] * evals
    ms = res["fwd_ms"] if kern == "forward" else res["bwd_ms"]
    achieved = ops / (ms * 1e-3) / 1e12
    per_pair, per_blend = FLOPS[kern]
    fine = per_pair * evals + per_blend * counts["K"]
    ent = traffic_entry(config, f"{kern}_{prec}")
    return {"bound": "alu", "kernel": f"blend_{kern}_{prec}", "achieved": round(achieved, 3),
            "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
            "traffic": ent["bytes_per_launch"] if ent else None,
            "ops_per_launch": ops,
            "ops_rule": f"{OPS_PER_EVAL[(kern, form)]} per evaluated pair x "
                        f"{'E' if kern == 'forward' else 'Eb'} = {evals}",
            "avg_ms": round(ms, 4),
            "frac_of_nonpacked_peak": round(achieved / PEAK_FP32_NONPACKED_TFLOPS, 4),
            "definition_ops_per_launch": fine,
            "definition_frac_of_nonpacked_peak":
                round(fine / (ms * 1e-3) / 1e12 / PEAK_FP32_NONPACKED_TFLOPS, 4)}


def device_info(dev) -> dict:
    p = torch.cuda.get_device_properties(dev)
    return {"name": p.name, "arch": p.gcnArchName.split(":")[0], "compute_units":
            p.multi_processor_count, "hbm_gib": round(p.total_memory / 2 ** 30, 1),
            "torch": torch.__version__, "hip": torch.version.hip}


def counter_fractions(config: str, prec: str) -> dict | None:
    """Fractions of the chip's rates for the blend kernels of `prec` on workload `config`, from
    the rocprofv3 counters in profiles/traffic.json, for kernels whose source is unchanged since
    the counters were taken."""
    if not os.path.exists(TRAFFIC):
        return None
    out = {"source": f"rocprofv3 --pmc over the {config} step, profiles/blend_{config.lower()}_*_pmc.md"}
    for kern in ("forward", "backward"):
        ent = traffic_entry(config, f"{kern}_{prec}")
        out[kern] = ent.get("fractions") if ent else None
    return out


# The paper's own figures, for orientation only: end-to-end forward render latency of the whole
# 3DGS pipeline on trained scenes (Table 2); the paper has no blend-only and no backward figure.
PAPER_CONTEXT = {
    "kind": "end-to-end forward render latency, trained scenes (Table 2); not comparable",
    "A100_mean_latency_ms": {"vanilla_3dgs": 5.36, "gemm_gs": 3.79, "speedup": 1.42},
    "H100_mean_speedup": 1.37,
}


def psnr(a, b) -> float:
    mse = float(np.mean((a - b) ** 2))
    return math.inf if mse == 0 else 10 * math.log10(1.0 / mse)


# Decision margins of the parity tests, per precision: a pixel is non-marginal when every skip /
# stop decision of the exact blend lies further than this (relative) from its threshold.
MARGIN = {"fp32": 1e-5, "fp16": 1e-4, "bf16": 1e-2}


def host_cpu() -> dict:
    """The host's CPU model (lscpu, else /proc/cpuinfo) and the cores this process may use."""
    model = None
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            if ln.startswith("Model name:"):
                model = ln.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    if model is None and os.path.exists("/proc/cpuinfo"):
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    return {"model": model, "nproc": len(os.sched_getaffinity(0))}


def cpu_baseline_and_accuracy(fr: Frame, gpu_results: dict, runs: int = 3) -> tuple[dict, dict]:
    """The FP64 oracle as it stands, on the host's cores, over the same full frame (bin + fwd +
    bwd), `runs` times (the median is the baseline), and the accuracy of every GPU path against
    it."""
    import oracle
    s = fr.scene
    W, H = fr.W, fr.H
    times = []
    for _ in range(runs):
        t0 = time.perf_counter()
        pl, rg = oracle.bin_tiles(s["means2d"], s["radii"], s["depths"], W, H)
        t1 = time.perf_counter()
        ref = oracle.forward(W, H, rg, pl, s["means2d"], s["conics"], s["opacity"], s["colors"])
        t2 = time.perf_counter()
        gref = oracle.backward(W, H, rg, pl, s["means2d"], s["conics"], s["opacity"], s["colors"],
                               fr.dloss_np)
        t3 = time.perf_counter()
        times.append((t3 - t0, t1 - t0, t2 - t1, t3 - t2))
    tot = sorted(times)[len(times) // 2]
    fb = float(np.median([t[2] + t[3] for t in times]))
    cpu = {"value": round(W * H / fb / 1e6, 4), "unit": "Mpix/s",
           "cores": oracle.threads(), "kind": "oracle",
           "sample": f"one full {W}x{H} frame of the same scene, {runs} runs, median: forward + "
                     f"backward blend in FP64 ({tot[2]:.1f} s + {tot[3]:.1f} s; binning "
                     f"{tot[1]:.1f} s more)",
           "step_mpix_s": round(W * H / tot[0] / 1e6, 4),
           "bin_s": round(tot[1], 3), "fwd_s": round(tot[2], 3), "bwd_s": round(tot[3], 3),
           "runs_s": [round(t[0], 3) for t in times], "host": host_cpu()}
    acc = {}
    for prec, out in gpu_results.items():
        img, T, last, grads = out
        d = np.abs(img - ref["image"])
        ok = ref["margin"] > MARGIN[prec]
        a = {"psnr_db": round(psnr(img, ref["image"]), 2),
             "max_abs_per_channel": [float(d[c].max()) for c in range(3)],
             "margin": MARGIN[prec], "nonmarginal_frac": round(float(ok.mean()), 5),
             "max_abs_nonmarginal_per_channel": [float(d[c][ok].max(initial=0.0))
                                                 for c in range(3)],
             "last_contrib_mismatch_nonmarginal": int((last != ref["last_contrib"])[ok].sum())}
        for k, g in zip(("dmeans2d", "dconics", "dopacity", "dcolors"), grads):
            e = np.linalg.norm((g - gref[k]).ravel()) / np.linalg.norm(gref[k].ravel())
            a[f"grad_rel_{k}"] = float(f"{e:.3e}")
        acc[prec] = a
    return cpu, acc


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    if args.sweep:
        print(json.dumps({"sweep": run_sweeps(dev, max(5, args.steps // 2), 2)}), flush=True)
        return
    if args.peaks:
        print(json.dumps({"peaks": measure_peaks()}), flush=True)
        return
    if args.reduce_study:
        print(json.dumps({"reduce_study": reduce_study(dev, max(5, args.steps // 2), 3)}),
              flush=True)
        return
    if args.calib_copy_mib:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.pipeline_only:
        print(json.dumps({"pipeline_3d": time_pipeline(dev, args.precs.split(",")[0], args.steps,
                                                       args.warmup)}), flush=True)
        return
    cfg = gsinputs.CONFIGS[args.config]
    fr = Frame(cfg, dev)
    fr.packed = not args.arrays
    counts = json.load(open(COUNTS))[args.config]
    precs = args.precs.split(",")
    results, outputs, scans = {}, {}, {}
    for prec in precs:
        results[prec] = time_path(fr, prec, args.steps, args.warmup)
        if not args.no_cpu_baseline:
            img, T, last = (x.cpu().numpy() for x in fr.fwd_out)
            grads = [g.cpu().numpy().astype(np.float64) for g in fr.bwd_out]
            # a full-scan path is compared with its culled path, not with the oracle
            (scans if prec.endswith("_scan") else outputs)[prec] = (
                img.astype(np.float64), T, last, grads)
    head = results[precs[0]]
    line = {
        "metric": METRIC, "value": round(head["blend_mpix_s"], 3), "unit": "Mpix/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp16": "f16+f32", "bf16": "bf16+f32", "fp32": "f32"}[precs[0]],
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {fr.W}x{fr.H}, {fr.n} projected Gaussians, "
                               f"log-normal sigma (median {cfg.sigma_a:g} px), opacity "
                               f"{OPACITY_LAW[cfg.opacity_law]}; step = bin + forward + backward; "
                               f"value = pixels / (forward + backward blend)",
                   "width": fr.W, "height": fr.H, "gaussians": fr.n, "pairs": fr.pairs,
                   "precision": precs[0], "parallelism": "single GPU"},
        "blend_mpix_s": round(head["blend_mpix_s"], 3),
        "step_mpix_s": round(head["mpix_s"], 3),
        "breakdown_ms": {k: round(head[k], 4) for k in ("bin_ms", "fwd_ms", "bwd_ms")},
        "roofline": roofline(head, counts, args.config, precs[0]),
        "counters": counter_fractions(args.config, precs[0]),
        "paths": {p: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()}
                  for p, r in results.items()},
        "paper_context": PAPER_CONTEXT,
        "device": device_info(dev),
    }
    if "fp32" in results and precs[0] != "fp32":
        line["speedup_vs_plain_fp32"] = {
            "step": round(results["fp32"]["ms_per_step"] / head["ms_per_step"], 3),
            "blend": round(head["blend_mpix_s"] / results["fp32"]["blend_mpix_s"], 3)}
    if "fp32_scan" in results:
        # the plain form without reach culling: every staged Gaussian evaluated at every pixel
        sc = results["fp32_scan"]
        fs = {"precision": "fp32 with GSB_FULL_SCAN",
              "blend_mpix_s": round(sc["blend_mpix_s"], 3),
              "fwd_ms": round(sc["fwd_ms"], 4), "bwd_ms": round(sc["bwd_ms"], 4)}
        if "fp32" in results:
            fs["reach_culling_speedup"] = {
                "fwd": round(sc["fwd_ms"] / results["fp32"]["fwd_ms"], 3),
                "bwd": round(sc["bwd_ms"] / results["fp32"]["bwd_ms"], 3)}
        if precs[0] not in ("fp32", "fp32_scan"):
            fs["gemm_speedup_blend"] = round(head["blend_mpix_s"] / sc["blend_mpix_s"], 3)
        if "fp32" in outputs and "fp32_scan" in scans:
            a, b = outputs["fp32"], scans["fp32_scan"]
            fs["forward_identical_to_culled"] = bool(all(np.array_equal(x, y)
                                                         for x, y in zip(a[:3], b[:3])))
            fs["grad_max_normwise_vs_culled"] = float(max(
                np.linalg.norm(x - y) / max(np.linalg.norm(x), 1e-300)
                for x, y in zip(a[3], b[3])))
        line["plain_full_scan"] = fs
    if not args.no_deterministic and fr.packed:
        fr.step(precs[0])
        torch.cuda.synchronize()
        line["deterministic_backward"] = time_deterministic(fr, precs[0], max(5, args.steps // 5),
                                                            2, head)
    if not args.no_visible:
        line["visible_binning"] = time_visible(fr.scene, dev, precs[0], args.steps, args.warmup,
                                               head, outputs.get(precs[0]))
    if not args.no_pipeline:
        line["pipeline_3d"] = time_pipeline(dev, precs[0], args.steps, args.warmup)
    if not args.no_batched:
        line["batched_c4"] = time_batched(max(5, args.steps // 2), 2, dev)
    if not args.no_cpu_baseline:
        line["cpu_baseline"], line["accuracy"] = cpu_baseline_and_accuracy(fr, outputs)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
