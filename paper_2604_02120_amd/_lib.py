"""ctypes binding of libgsblend.so: one Python function per C entry point, same names.

Argument marshalling only. Pointers are passed as integers (device addresses, e.g.
``tensor.data_ptr()``); ``stream`` is a hipStream_t as an integer (0 = default stream). A
non-zero status raises :class:`GsbError` carrying the library's message.

The library must have been built (``python -m paper_2604_02120_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsblend.so")

GSB_OK = 0
GSB_ERR_INVALID = 1
GSB_ERR_CAPACITY = 2
GSB_ERR_UNSUPPORTED = 3
GSB_ERR_HIP = 4
GSB_ERR_INTERNAL = 5
GSB_BIN_RECT = 0
GSB_BIN_VISIBLE = 1

GSB_FP32_PLAIN = 0
GSB_FP16_GEMM = 1
GSB_BF16_GEMM = 2
# OR'ed into a precision: evaluate every staged Gaussian at every pixel (no reach culling in the
# plain form; the GEMM forms always do)
GSB_FULL_SCAN = 0x100
PRECISIONS = {"fp32": GSB_FP32_PLAIN, "fp16": GSB_FP16_GEMM, "bf16": GSB_BF16_GEMM,
              "fp32_scan": GSB_FP32_PLAIN | GSB_FULL_SCAN}
GSB_LAUNCH_PERSISTENT = 0
GSB_LAUNCH_GRID = 1
GSB_REDUCE_VALU = 0
GSB_REDUCE_MFMA = 1

# every function declared in include/gsblend.h
EXPORTS = ("gsb_abi_version", "gsb_last_error", "gsb_project", "gsb_bin_workspace_bytes",
           "gsb_bin_count", "gsb_bin_fill", "gsb_bin_noalloc", "gsb_pack_gaussians",
           "gsb_blend_forward_packed", "gsb_blend_backward_packed",
           "gsb_backward_det_workspace_bytes", "gsb_blend_backward_deterministic",
           "gsb_blend_forward", "gsb_blend_backward", "gsb_plan_create",
           "gsb_plan_destroy", "gsb_blend_batched_forward", "gsb_blend_batched_backward")


class GsbCamera(ctypes.Structure):
    """struct gsb_camera: pinhole camera (host struct)."""
    _fields_ = [("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("near", ctypes.c_float)]


class GsbView(ctypes.Structure):
    """struct gsb_view: one view of a batched plan (device pointers as integers)."""
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("n", ctypes.c_int64),
                ("ranges", ctypes.c_void_p), ("point_list", ctypes.c_void_p),
                ("means2d", ctypes.c_void_p), ("conics", ctypes.c_void_p),
                ("opacity", ctypes.c_void_p), ("colors", ctypes.c_void_p),
                ("bg", ctypes.c_float * 3),
                ("image", ctypes.c_void_p), ("final_T", ctypes.c_void_p),
                ("last_contrib", ctypes.c_void_p), ("dL_dimage", ctypes.c_void_p),
                ("dL_dmeans2d", ctypes.c_void_p), ("dL_dconics", ctypes.c_void_p),
                ("dL_dopacity", ctypes.c_void_p), ("dL_dcolors", ctypes.c_void_p)]


class GsbTuning(ctypes.Structure):
    """struct gsb_tuning (zero fields take the library defaults)."""
    _fields_ = [("batch_fwd", ctypes.c_int32), ("batch_bwd", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("launch", ctypes.c_int32),
                ("bwd_reduce", ctypes.c_int32)]


class GsbError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"gsblend status {status}: {message}")
        self.status = status


_lib = None


def load() -> ctypes.CDLL:
    """Load libgsblend.so (once). Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2604_02120_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    P, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
    lib.gsb_abi_version.argtypes = []
    lib.gsb_abi_version.restype = i32
    lib.gsb_last_error.argtypes = []
    lib.gsb_last_error.restype = ctypes.c_char_p
    lib.gsb_project.argtypes = [P, P, P, P, i32, i32, i64, ctypes.POINTER(GsbCamera), P, P, P,
                                P, P, P]
    lib.gsb_bin_workspace_bytes.argtypes = [i64, i64, i32, i32, ctypes.POINTER(sz)]
    lib.gsb_bin_count.argtypes = [P, P, P, P, i32, i64, i32, i32, P, sz, P, P]
    lib.gsb_bin_fill.argtypes = [P, P, P, P, i32, P, i64, i32, i32, P, sz, P, i64, P, P, P]
    lib.gsb_bin_noalloc.argtypes = [P, P, P, P, i32, P, i64, i32, i32, P, i64, P, P, P, P]
    lib.gsb_pack_gaussians.argtypes = [P, P, P, P, i64, P, P]
    lib.gsb_blend_forward_packed.argtypes = [i32, i32, P, P, P, i64, P, i32, P, P, P, P]
    lib.gsb_blend_backward_packed.argtypes = [i32, i32, P, P, P, i64, P, i32, P, P, P, P, P, P,
                                              P, P]
    lib.gsb_backward_det_workspace_bytes.argtypes = [i64, i64, ctypes.POINTER(sz)]
    lib.gsb_blend_backward_deterministic.argtypes = [i32, i32, P, P, i64, P, i64, P, i32, P, P,
                                                     P, P, sz, P, P, P, P, P]
    lib.gsb_blend_forward.argtypes = [i32, i32, P, P, P, P, P, P, i64, P, i32, P, P, P, P]
    lib.gsb_blend_backward.argtypes = [i32, i32, P, P, P, P, P, P, i64, P, i32, P, P, P, P, P,
                                       P, P, P]
    lib.gsb_plan_create.argtypes = [ctypes.POINTER(GsbView), i32, i32, ctypes.POINTER(GsbTuning),
                                    ctypes.POINTER(ctypes.c_void_p)]
    lib.gsb_plan_destroy.argtypes = [P]
    lib.gsb_blend_batched_forward.argtypes = [P, P]
    lib.gsb_blend_batched_backward.argtypes = [P, P]
    for name in EXPORTS[2:]:
        getattr(lib, name).restype = i32
    _lib = lib
    return lib


def _check(status: int) -> None:
    if status != GSB_OK:
        raise GsbError(status, gsb_last_error())


def _bg(bg) -> ctypes.Array:
    if bg is None:
        return None
    b = (ctypes.c_float * 3)(*[float(v) for v in bg])
    return b


def gsb_abi_version() -> int:
    return int(load().gsb_abi_version())


def gsb_last_error() -> str:
    return load().gsb_last_error().decode()


def gsb_project(means3d: int, scales: int, quats: int, sh: int, sh_coeffs: int, sh_degree: int,
                n: int, camera: GsbCamera, means2d: int, conics: int, depths: int, radii: int,
                colors: int, stream: int = 0) -> None:
    _check(load().gsb_project(means3d, scales, quats, sh, sh_coeffs, sh_degree, n,
                              ctypes.byref(camera), means2d, conics, depths, radii, colors,
                              stream))


def gsb_bin_workspace_bytes(n: int, pair_capacity: int, W: int, H: int) -> int:
    out = ctypes.c_size_t(0)
    _check(load().gsb_bin_workspace_bytes(n, pair_capacity, W, H, ctypes.byref(out)))
    return int(out.value)


def gsb_bin_count(means2d: int, radii: int, n: int, W: int, H: int, ws: int, ws_bytes: int,
                  n_pairs_dev: int, stream: int = 0, conics: int = 0, opacity: int = 0,
                  mode: int = 0) -> None:
    _check(load().gsb_bin_count(means2d, radii, conics, opacity, mode, n, W, H, ws, ws_bytes,
                                n_pairs_dev, stream))


def gsb_bin_fill(means2d: int, radii: int, depths: int, n: int, W: int, H: int, ws: int,
                 ws_bytes: int, point_list: int, pair_capacity: int, ranges: int,
                 status_dev: int, stream: int = 0, conics: int = 0, opacity: int = 0,
                 mode: int = 0) -> None:
    _check(load().gsb_bin_fill(means2d, radii, conics, opacity, mode, depths, n, W, H, ws,
                               ws_bytes, point_list, pair_capacity, ranges, status_dev, stream))


def gsb_bin_noalloc(means2d: int, radii: int, depths: int, n: int, W: int, H: int,
                    point_list: int, pair_capacity: int, ranges: int, n_pairs_dev: int,
                    status_dev: int, stream: int = 0, conics: int = 0, opacity: int = 0,
                    mode: int = 0) -> None:
    _check(load().gsb_bin_noalloc(means2d, radii, conics, opacity, mode, depths, n, W, H,
                                  point_list, pair_capacity, ranges, n_pairs_dev, status_dev,
                                  stream))


GSB_NOALLOC_SCRATCH_BYTES = 64 << 20
GSB_RECORD_FLOATS = 12


def gsb_pack_gaussians(means2d: int, conics: int, opacity: int, colors: int, n: int,
                       records: int, stream: int = 0) -> None:
    _check(load().gsb_pack_gaussians(means2d, conics, opacity, colors, n, records, stream))


def gsb_blend_forward_packed(W: int, H: int, ranges: int, point_list: int, records: int, n: int,
                             bg, prec: int, image: int, final_T: int, last_contrib: int,
                             stream: int = 0) -> None:
    _check(load().gsb_blend_forward_packed(W, H, ranges, point_list, records, n, _bg(bg), prec,
                                           image, final_T, last_contrib, stream))


def gsb_blend_backward_packed(W: int, H: int, ranges: int, point_list: int, records: int, n: int,
                              bg, prec: int, final_T: int, last_contrib: int, dL_dimage: int,
                              dL_dmeans2d: int, dL_dconics: int, dL_dopacity: int,
                              dL_dcolors: int, stream: int = 0) -> None:
    _check(load().gsb_blend_backward_packed(W, H, ranges, point_list, records, n, _bg(bg), prec,
                                            final_T, last_contrib, dL_dimage, dL_dmeans2d,
                                            dL_dconics, dL_dopacity, dL_dcolors, stream))


def gsb_backward_det_workspace_bytes(n: int, pairs: int) -> int:
    out = ctypes.c_size_t(0)
    _check(load().gsb_backward_det_workspace_bytes(n, pairs, ctypes.byref(out)))
    return int(out.value)


def gsb_blend_backward_deterministic(W: int, H: int, ranges: int, point_list: int, pairs: int,
                                     records: int, n: int, bg, prec: int, final_T: int,
                                     last_contrib: int, dL_dimage: int, ws: int, ws_bytes: int,
                                     dL_dmeans2d: int, dL_dconics: int, dL_dopacity: int,
                                     dL_dcolors: int, stream: int = 0) -> None:
    _check(load().gsb_blend_backward_deterministic(
        W, H, ranges, point_list, pairs, records, n, _bg(bg), prec, final_T, last_contrib,
        dL_dimage, ws, ws_bytes, dL_dmeans2d, dL_dconics, dL_dopacity, dL_dcolors, stream))


def gsb_blend_forward(W: int, H: int, ranges: int, point_list: int, means2d: int, conics: int,
                      opacity: int, colors: int, n: int, bg, prec: int, image: int, final_T: int,
                      last_contrib: int, stream: int = 0) -> None:
    _check(load().gsb_blend_forward(W, H, ranges, point_list, means2d, conics, opacity, colors, n,
                                    _bg(bg), prec, image, final_T, last_contrib, stream))


def gsb_blend_backward(W: int, H: int, ranges: int, point_list: int, means2d: int, conics: int,
                       opacity: int, colors: int, n: int, bg, prec: int, final_T: int,
                       last_contrib: int, dL_dimage: int, dL_dmeans2d: int, dL_dconics: int,
                       dL_dopacity: int, dL_dcolors: int, stream: int = 0) -> None:
    _check(load().gsb_blend_backward(W, H, ranges, point_list, means2d, conics, opacity, colors,
                                     n, _bg(bg), prec, final_T, last_contrib, dL_dimage,
                                     dL_dmeans2d, dL_dconics, dL_dopacity, dL_dcolors, stream))


def gsb_plan_create(views, prec: int, tuning=None) -> int:
    """views: sequence of GsbView; tuning: GsbTuning or None. Returns the plan handle."""
    arr = (GsbView * max(len(views), 1))(*views)
    out = ctypes.c_void_p(0)
    tp = ctypes.byref(tuning) if tuning is not None else None
    _check(load().gsb_plan_create(arr, len(views), prec, tp, ctypes.byref(out)))
    return int(out.value)


def gsb_plan_destroy(plan: int) -> None:
    _check(load().gsb_plan_destroy(plan))


def gsb_blend_batched_forward(plan: int, stream: int = 0) -> None:
    _check(load().gsb_blend_batched_forward(plan, stream))


def gsb_blend_batched_backward(plan: int, stream: int = 0) -> None:
    _check(load().gsb_blend_batched_backward(plan, stream))
