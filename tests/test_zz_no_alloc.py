"""gsb_bin_noalloc (binning with the library-held workspace) against gsb_bin_count + gsb_bin_fill
with a caller workspace: the same pair count, point list and ranges bit for bit, on two calls in a
row, the second with a smaller input (the array keeps the first call's contents)."""
import numpy as np
import pytest
import torch

import gsinputs
from gpu_util import say, upload
from paper_2604_02120_amd import _lib, api

pytestmark = pytest.mark.gpu


def noalloc_bins(sd, capacity, mode="rect"):
    W, H = sd["width"], sd["height"]
    n = sd["radii"].shape[0]
    gx, gy = api.grid(W, H)
    dev = sd["means2d"].device
    pl = torch.full((max(capacity, 1),), -1, dtype=torch.int32, device=dev)
    rg = torch.full((gx * gy, 2), -1, dtype=torch.int32, device=dev)
    n_pairs = torch.full((1,), -1, dtype=torch.int64, device=dev)
    status = torch.full((1,), -1, dtype=torch.int32, device=dev)
    code, cp, op = api._bin_mode(mode, sd["conics"], sd["opacity"])
    _lib.gsb_bin_noalloc(sd["means2d"].data_ptr(), sd["radii"].data_ptr(), sd["depths"].data_ptr(),
                         n, W, H, pl.data_ptr(), capacity, rg.data_ptr(), n_pairs.data_ptr(),
                         status.data_ptr(), torch.cuda.current_stream().cuda_stream, cp, op, code)
    torch.cuda.synchronize()
    return pl, rg, int(n_pairs.item()), int(status.item())


def check_case(gpu, scene, mode, slack=1.1):
    sd = upload(scene, gpu)
    W, H = scene["width"], scene["height"]
    pl_ref, rg_ref = api.bin_tiles(sd["means2d"], sd["radii"], sd["depths"], W, H,
                                   conics=sd["conics"], opacity=sd["opacity"], mode=mode)
    torch.cuda.synchronize()
    P = pl_ref.numel()
    cap = int(P * slack) + 16                       # a bound chosen before the call
    need = _lib.gsb_bin_workspace_bytes(len(scene["radii"]), cap, W, H)
    say(f"[noalloc] {W}x{H} n={len(scene['radii'])} mode={mode} pairs={P} cap={cap} "
        f"workspace {need / 2**20:.1f} MiB")
    assert need <= _lib.GSB_NOALLOC_SCRATCH_BYTES
    pl, rg, n_pairs, status = noalloc_bins(sd, cap, mode)
    assert status == 0 and n_pairs == P
    assert torch.equal(rg, rg_ref)
    assert torch.equal(pl[:P], pl_ref)
    assert bool((pl[P:] == -1).all())               # nothing written past the pairs


def test_noalloc_equals_workspace_binning_twice(gpu):
    big = gsinputs.make_views()[0]                  # one 300k-Gaussian view of the multi-view set
    small = gsinputs.make_scene("C1")               # 64x64, 2000 Gaussians
    check_case(gpu, big, "rect")
    check_case(gpu, small, "rect")                  # smaller, after the larger call
    check_case(gpu, small, "visible")


def test_noalloc_capacity_and_size_limits(gpu):
    s = gsinputs.make_scene("C1")
    sd = upload(s, gpu)
    pl_ref, _ = api.bin_tiles(sd["means2d"], sd["radii"], sd["depths"], 64, 64)
    P = pl_ref.numel()
    _, _, n_pairs, status = noalloc_bins(sd, P // 2)
    assert status == _lib.GSB_ERR_CAPACITY and n_pairs == P
    # a workspace larger than the library's array is refused on the host, before any launch
    with pytest.raises(_lib.GsbError) as e:
        _lib.gsb_bin_noalloc(sd["means2d"].data_ptr(), sd["radii"].data_ptr(),
                             sd["depths"].data_ptr(), 1_000_000, 1920, 1080, sd["means2d"].data_ptr(),
                             10_000_000, sd["means2d"].data_ptr(), sd["means2d"].data_ptr(),
                             sd["means2d"].data_ptr(), 0)
    assert e.value.status == _lib.GSB_ERR_INVALID
