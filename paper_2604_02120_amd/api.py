"""Tensor-level calls on top of the C ABI: device memory and streams come from PyTorch, every
step of the work runs in libgsblend's kernels.

Tensors must be contiguous and on the current HIP device:
  means2d f32[n][2], conics f32[n][3] (A, B, C), opacity f32[n], colors f32[n][3],
  depths f32[n], radii i32[n]; point_list/ranges are i32 tensors holding u32 values.
"""
from __future__ import annotations

import torch

from . import _lib

TILE = 16


def grid(W: int, H: int) -> tuple[int, int]:
    return (W + TILE - 1) // TILE, (H + TILE - 1) // TILE


def _stream(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def _req(t: torch.Tensor, dtype, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} CUDA/HIP tensor")
    return t


def prec_code(prec) -> int:
    if isinstance(prec, str):
        return _lib.PRECISIONS[prec]
    return int(prec)


class BinWorkspace:
    """Device workspace of the binning calls, sized for (n, pair_capacity, W, H)."""

    def __init__(self, n: int, pair_capacity: int, W: int, H: int, device=None):
        self.n, self.capacity, self.W, self.H = n, pair_capacity, W, H
        self.nbytes = _lib.gsb_bin_workspace_bytes(n, pair_capacity, W, H)
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=device or "cuda")

    def ptr(self) -> int:
        return self.buf.data_ptr()


def bin_count(means2d, radii, W: int, H: int, ws: BinWorkspace, stream=None) -> torch.Tensor:
    """Device int64[1] pair count; the per-Gaussian offsets stay in ``ws``."""
    n = radii.shape[0]
    _req(means2d, torch.float32, "means2d")
    _req(radii, torch.int32, "radii")
    n_pairs = torch.empty(1, dtype=torch.int64, device=means2d.device)
    _lib.gsb_bin_count(means2d.data_ptr(), radii.data_ptr(), n, W, H, ws.ptr(), ws.nbytes,
                       n_pairs.data_ptr(), _stream(stream))
    return n_pairs


def bin_fill(means2d, radii, depths, W: int, H: int, ws: BinWorkspace, point_list, ranges,
             stream=None) -> torch.Tensor:
    """Fills point_list (i32[capacity]) and ranges (i32[gx*gy][2]); returns the device status."""
    n = radii.shape[0]
    _req(depths, torch.float32, "depths")
    _req(point_list, torch.int32, "point_list")
    _req(ranges, torch.int32, "ranges")
    status = torch.empty(1, dtype=torch.int32, device=means2d.device)
    _lib.gsb_bin_fill(means2d.data_ptr(), radii.data_ptr(), depths.data_ptr(), n, W, H, ws.ptr(),
                      ws.nbytes, point_list.data_ptr(), point_list.numel(), ranges.data_ptr(),
                      status.data_ptr(), _stream(stream))
    return status


def bin_tiles(means2d, radii, depths, W: int, H: int, stream=None):
    """Count, then fill with an exactly sized list. Returns (point_list i32[P], ranges
    i32[gx*gy][2]). Synchronises once to read the pair count."""
    n = radii.shape[0]
    ws0 = BinWorkspace(n, 0, W, H, device=means2d.device)
    n_pairs = int(bin_count(means2d, radii, W, H, ws0, stream).item())
    ws = BinWorkspace(n, n_pairs, W, H, device=means2d.device)
    ws.buf[: ws0.nbytes].copy_(ws0.buf)          # per-Gaussian offsets from the count
    gx, gy = grid(W, H)
    point_list = torch.empty(max(n_pairs, 1), dtype=torch.int32, device=means2d.device)
    ranges = torch.empty((gx * gy, 2), dtype=torch.int32, device=means2d.device)
    bin_fill(means2d, radii, depths, W, H, ws, point_list[:n_pairs] if n_pairs else point_list[:0],
             ranges, stream)
    return point_list[:n_pairs], ranges


def blend_forward(means2d, conics, opacity, colors, ranges, point_list, W: int, H: int,
                  bg=(0.0, 0.0, 0.0), prec="fp16", stream=None, out=None):
    """Returns (image f32[3][H][W], final_T f32[H][W], last_contrib i32[H][W])."""
    n = opacity.shape[0]
    for t, nm in ((means2d, "means2d"), (conics, "conics"), (opacity, "opacity"), (colors, "colors")):
        _req(t, torch.float32, nm)
    _req(ranges, torch.int32, "ranges")
    _req(point_list, torch.int32, "point_list")
    dev = means2d.device
    if out is None:
        out = (torch.empty((3, H, W), dtype=torch.float32, device=dev),
               torch.empty((H, W), dtype=torch.float32, device=dev),
               torch.empty((H, W), dtype=torch.int32, device=dev))
    image, final_T, last = out
    pl = point_list if point_list.numel() else ranges   # any valid device address for an empty list
    _lib.gsb_blend_forward(W, H, ranges.data_ptr(), pl.data_ptr(), means2d.data_ptr(),
                           conics.data_ptr(), opacity.data_ptr(), colors.data_ptr(), n, bg,
                           prec_code(prec), image.data_ptr(), final_T.data_ptr(), last.data_ptr(),
                           _stream(stream))
    return image, final_T, last


def blend_backward(means2d, conics, opacity, colors, ranges, point_list, W: int, H: int,
                   final_T, last_contrib, dL_dimage, bg=(0.0, 0.0, 0.0), prec="fp16",
                   stream=None, out=None):
    """Returns (dL_dmeans2d [n][2], dL_dconics [n][3], dL_dopacity [n], dL_dcolors [n][3])."""
    n = opacity.shape[0]
    _req(final_T, torch.float32, "final_T")
    _req(last_contrib, torch.int32, "last_contrib")
    _req(dL_dimage, torch.float32, "dL_dimage")
    dev = means2d.device
    if out is None:
        out = (torch.empty((n, 2), dtype=torch.float32, device=dev),
               torch.empty((n, 3), dtype=torch.float32, device=dev),
               torch.empty((n,), dtype=torch.float32, device=dev),
               torch.empty((n, 3), dtype=torch.float32, device=dev))
    dm, dc, do, dcol = out
    pl = point_list if point_list.numel() else ranges
    _lib.gsb_blend_backward(W, H, ranges.data_ptr(), pl.data_ptr(), means2d.data_ptr(),
                            conics.data_ptr(), opacity.data_ptr(), colors.data_ptr(), n, bg,
                            prec_code(prec), final_T.data_ptr(), last_contrib.data_ptr(),
                            dL_dimage.data_ptr(), dm.data_ptr(), dc.data_ptr(), do.data_ptr(),
                            dcol.data_ptr(), _stream(stream))
    return dm, dc, do, dcol
