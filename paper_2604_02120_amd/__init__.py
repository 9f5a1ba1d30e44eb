"""MI355X (gfx950) tile blending of projected 2D Gaussians with a GEMM-form exponent on MFMA
(GEMM-GS, arXiv 2604.02120), as a C-ABI library (``libgsblend.so``, declared in
``include/gsblend.h``) plus this thin binding.

* ``paper_2604_02120_amd._lib``     — ctypes functions with the C names (``gsb_*``).
* ``paper_2604_02120_amd.api``      — tensor-level projection of 3D Gaussians, bin / forward /
  backward, and ``BatchedViews`` (many views per launch).
* ``paper_2604_02120_amd.autotune`` — launch-shape autotuner for batched views.
* ``paper_2604_02120_amd.autograd`` — ``BlendFunction`` / ``blend`` for torch autograd.
* ``paper_2604_02120_amd.build``    — hipcc build of the library.
"""
from ._lib import (GSB_BF16_GEMM, GSB_FP16_GEMM, GSB_FP32_PLAIN, GsbError,  # noqa: F401
                   load)

__all__ = ["GsbError", "load", "GSB_FP32_PLAIN", "GSB_FP16_GEMM", "GSB_BF16_GEMM"]
