"""Differentiable blend: torch.autograd.Function over gsb_blend_forward / gsb_blend_backward.

The binning (ranges, point_list) is an input and carries no gradient; final_T and last_contrib
are returned for inspection and are not differentiable.
"""
from __future__ import annotations

import torch

from . import api


class BlendFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, means2d, conics, opacity, colors, ranges, point_list, W, H, bg, prec):
        image, final_T, last = api.blend_forward(means2d, conics, opacity, colors, ranges,
                                                 point_list, W, H, bg, prec)
        ctx.save_for_backward(means2d, conics, opacity, colors, ranges, point_list, final_T, last)
        ctx.cfg = (W, H, tuple(float(v) for v in bg), prec)
        ctx.mark_non_differentiable(final_T, last)
        return image, final_T, last

    @staticmethod
    def backward(ctx, g_image, g_T, g_last):
        means2d, conics, opacity, colors, ranges, point_list, final_T, last = ctx.saved_tensors
        W, H, bg, prec = ctx.cfg
        dm, dc, do, dcol = api.blend_backward(means2d, conics, opacity, colors, ranges, point_list,
                                              W, H, final_T, last, g_image.contiguous(), bg, prec)
        return dm, dc, do, dcol, None, None, None, None, None, None


def blend(means2d, conics, opacity, colors, ranges, point_list, W: int, H: int,
          bg=(0.0, 0.0, 0.0), prec="fp16"):
    """image, final_T, last_contrib = blend(...); image is differentiable w.r.t. the attributes."""
    return BlendFunction.apply(means2d, conics, opacity, colors, ranges, point_list, W, H, bg, prec)
