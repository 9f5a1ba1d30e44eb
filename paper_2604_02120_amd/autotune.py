"""Autotuner for the launch shape of batched (multi-view) blends.

For a ``api.BatchedViews`` it times the forward + backward launches for every candidate shape
(LDS batch size of each direction, resident blocks per compute unit, persistent or one block per
item, the backward's reduction on the vector ALUs or the matrix cores) and keeps the fastest.
Results are cached in a JSON file keyed by (GPU arch, precision, the views' sizes with Gaussian
counts rounded to powers of two), so a shape is measured once per workload family.

The cache file is ``$GSBLEND_TUNING_CACHE`` if set, else ``~/.cache/gsblend/tuning.json``.
"""
from __future__ import annotations

import json
import math
import os

import torch

BATCHES_FWD = (128, 256)
BATCHES_BWD = (64, 128, 256)
BLOCKS_PER_CU = (0, 2)          # persistent launches: 0 = as many as fit
# launch 0: persistent blocks pulling from the per-XCD queues; 1: one block per item.
# bwd_reduce 0: the backward's nine per-Gaussian sums by cross-lane adds; 1: its five geometric
# sums as a product with the pixel basis on the matrix cores (tried with one-block-per-item
# launches and LDS batches of 64 and 128, the shapes whose LDS keeps 4-5 blocks per CU).
CANDIDATES = ([dict(batch_fwd=f, batch_bwd=b, blocks_per_cu=c, launch=0, bwd_reduce=0)
               for f in BATCHES_FWD for b in BATCHES_BWD for c in BLOCKS_PER_CU] +
              [dict(batch_fwd=f, batch_bwd=b, blocks_per_cu=0, launch=1, bwd_reduce=0)
               for f in BATCHES_FWD for b in BATCHES_BWD] +
              [dict(batch_fwd=f, batch_bwd=b, blocks_per_cu=0, launch=1, bwd_reduce=1)
               for f in BATCHES_FWD for b in (64, 128)])
KEYS = ("batch_fwd", "batch_bwd", "blocks_per_cu", "launch", "bwd_reduce")


def cache_path() -> str:
    return os.environ.get("GSBLEND_TUNING_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "gsblend", "tuning.json"))


def workload_key(bv) -> str:
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    sizes = sorted((v["width"], v["height"], 1 << max(0, math.ceil(math.log2(max(v["n"], 1)))))
                   for v in bv.views)
    return json.dumps({"arch": arch, "prec": bv.prec, "views": sizes}, sort_keys=True)


def _load() -> dict:
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(data: dict) -> None:
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def measure(bv, tuning: dict, reps: int = 5, warmup: int = 2) -> float:
    """Median ms of one batched forward + backward with ``tuning`` (binning already done)."""
    bv._make_plan(tuning)
    for _ in range(warmup):
        bv.forward()
        bv.backward()
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        bv.forward()
        bv.backward()
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    times.sort()
    return times[len(times) // 2]


def tune(bv, candidates=None, reps: int = 5, use_cache: bool = True) -> dict:
    """Best shape for ``bv`` (also installed as its plan). Returns the chosen dict, with the
    measured ``ms`` of every candidate under ``"trials"``."""
    key = workload_key(bv)
    cache = _load() if use_cache else {}
    if use_cache and key in cache:
        best = cache[key]["best"]
        bv._make_plan(best)
        return dict(best)
    bv.bin()
    trials = []
    for cand in candidates or CANDIDATES:
        trials.append((measure(bv, cand, reps), cand))
    trials.sort(key=lambda t: t[0])
    best = dict(trials[0][1])
    bv._make_plan(best)
    if use_cache:
        cache[key] = {"best": best, "trials": [{"ms": ms, **c} for ms, c in trials]}
        _store(cache)
    out = dict(best)
    out["trials"] = [{"ms": round(ms, 4), **c} for ms, c in trials]
    return out
