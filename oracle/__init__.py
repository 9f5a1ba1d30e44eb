"""FP64 CPU oracle of the Gaussian blend (binning, forward, backward).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's CPU-baseline leg
may call this; the GPU library never does. It shares no code with the GPU library. The C source
(``gsoracle.c``) states what it computes and which reading of the paper it takes.

Inputs may be FP32 arrays (they are promoted exactly to FP64) or FP64 arrays (finite
differences). Outputs are FP64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gsoracle.c")
_LIB_PATH = os.path.join(_HERE, "libgsoracle.so")
TILE = 16

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain FP64: no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fno-fast-math",
                               "-ffp-contract=off", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        lib.orc_bin_count.argtypes = [P, P, P, P, i32, i64, i32, i32]
        lib.orc_bin_count.restype = i64
        lib.orc_bin.argtypes = [P, P, P, P, i32, P, i64, i32, i32, i64, P, P]
        lib.orc_bin.restype = i64
        lib.orc_bin_tile.argtypes = [P, P, P, P, i32, P, i64, i32, i32, i64, i64, P]
        lib.orc_bin_tile.restype = i64
        lib.orc_forward.argtypes = [i32, i32, P, P, P, P, P, P, P, P, P, P, P, P, P]
        lib.orc_forward.restype = None
        lib.orc_backward.argtypes = [i32, i32, P, P, P, P, P, P, P, i64, P, P, P, P, P]
        lib.orc_backward.restype = None
        lib.orc_sh_basis.argtypes = [P, i64, i32, P]
        lib.orc_sh_basis.restype = None
        lib.orc_project.argtypes = [P, P, P, P, i32, i32, i64, P, P, P, P, P, P, P, P]
        lib.orc_project.restype = None
        lib.orc_threads.restype = ctypes.c_int
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def threads() -> int:
    return int(_load().orc_threads())


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def grid(W: int, H: int) -> tuple[int, int]:
    return (W + TILE - 1) // TILE, (H + TILE - 1) // TILE


# Binning modes: 0 = every tile of the 3-sigma square (the rule of the method); 1 = only the tiles
# of that square on which the Gaussian can reach alpha >= 1/255 (the opacity-aware extent, a
# tighter binning that leaves images unchanged; rule in gsoracle.c).
BIN_RECT, BIN_VISIBLE = 0, 1


def _bin_args(means2d, radii, conics, opacity, mode):
    m = _f64(means2d)
    r = np.ascontiguousarray(radii, dtype=np.int32)
    if mode == BIN_RECT:
        return m, r, None, None
    if conics is None or opacity is None:
        raise ValueError("binning mode 1 needs conics and opacity")
    return m, r, _f64(conics), _f64(opacity)


def _p(a):
    return None if a is None else _ptr(a)


def bin_tiles(means2d, radii, depths, W: int, H: int, conics=None, opacity=None,
              mode: int = BIN_RECT) -> tuple[np.ndarray, np.ndarray]:
    """(point_list u32[P], ranges u32[n_tiles][2]) sorted by (tile, depth, index)."""
    lib = _load()
    m, r, c, o = _bin_args(means2d, radii, conics, opacity, mode)
    d = _f64(depths)
    n = r.shape[0]
    total = lib.orc_bin_count(_ptr(m), _ptr(r), _p(c), _p(o), mode, n, W, H)
    gx, gy = grid(W, H)
    point_list = np.zeros(max(total, 1), np.uint32)
    ranges = np.zeros((gx * gy, 2), np.uint32)
    got = lib.orc_bin(_ptr(m), _ptr(r), _p(c), _p(o), mode, _ptr(d), n, W, H, total,
                      _ptr(point_list), _ptr(ranges))
    assert got == total
    return point_list[:total], ranges


def bin_tile(means2d, radii, depths, W: int, H: int, t: int, conics=None, opacity=None,
             mode: int = BIN_RECT) -> np.ndarray:
    """Sorted list (u32) of tile t alone."""
    lib = _load()
    m, r, c, o = _bin_args(means2d, radii, conics, opacity, mode)
    d = _f64(depths)
    n = r.shape[0]
    k = lib.orc_bin_tile(_ptr(m), _ptr(r), _p(c), _p(o), mode, _ptr(d), n, W, H, t, 0, None)
    out = np.zeros(max(k, 1), np.uint32)
    lib.orc_bin_tile(_ptr(m), _ptr(r), _p(c), _p(o), mode, _ptr(d), n, W, H, t, k, _ptr(out))
    return out[:k]


def sampled_bins(means2d, radii, depths, W: int, H: int, tiles, conics=None, opacity=None,
                 mode: int = BIN_RECT) -> tuple[np.ndarray, np.ndarray]:
    """(point_list, ranges) in which only the given tiles hold their lists (every other tile is
    empty): the binning of a frame restricted to a sample of its tiles."""
    gx, gy = grid(W, H)
    ranges = np.zeros((gx * gy, 2), np.uint32)
    lists, pos = [], 0
    for t in sorted(int(t) for t in tiles):
        lst = bin_tile(means2d, radii, depths, W, H, t, conics, opacity, mode)
        ranges[t] = (pos, pos + len(lst)) if len(lst) else (0, 0)
        lists.append(lst)
        pos += len(lst)
    pl = np.concatenate(lists) if lists else np.zeros(0, np.uint32)
    return pl.astype(np.uint32), ranges


def forward(W: int, H: int, ranges, point_list, means2d, conics, opacity, colors,
            bg=(0.0, 0.0, 0.0)) -> dict[str, np.ndarray]:
    """image f64[3][H][W], final_T f64[H][W], last_contrib i32[H][W], n_eval i32[H][W],
    n_contrib i32[H][W], margin f64[H][W]."""
    lib = _load()
    rg = np.ascontiguousarray(ranges, dtype=np.uint32)
    pl = np.ascontiguousarray(point_list, dtype=np.uint32)
    if pl.size == 0:
        pl = np.zeros(1, np.uint32)
    m, c, o, col, b = _f64(means2d), _f64(conics), _f64(opacity), _f64(colors), _f64(bg)
    image = np.empty((3, H, W), np.float64)
    final_T = np.empty((H, W), np.float64)
    last = np.empty((H, W), np.int32)
    n_eval = np.empty((H, W), np.int32)
    n_contrib = np.empty((H, W), np.int32)
    margin = np.empty((H, W), np.float64)
    lib.orc_forward(W, H, _ptr(rg), _ptr(pl), _ptr(m), _ptr(c), _ptr(o), _ptr(col), _ptr(b),
                    _ptr(image), _ptr(final_T), _ptr(last), _ptr(n_eval), _ptr(n_contrib),
                    _ptr(margin))
    return {"image": image, "final_T": final_T, "last_contrib": last, "n_eval": n_eval,
            "n_contrib": n_contrib, "margin": margin}


def backward(W: int, H: int, ranges, point_list, means2d, conics, opacity, colors, dL_dimage,
             bg=(0.0, 0.0, 0.0)) -> dict[str, np.ndarray]:
    """Gradients of L = sum(dL_dimage * image): dmeans2d [N][2], dconics [N][3] (A, B, C),
    dopacity [N], dcolors [N][3]."""
    lib = _load()
    rg = np.ascontiguousarray(ranges, dtype=np.uint32)
    pl = np.ascontiguousarray(point_list, dtype=np.uint32)
    if pl.size == 0:
        pl = np.zeros(1, np.uint32)
    m, c, o, col, b = _f64(means2d), _f64(conics), _f64(opacity), _f64(colors), _f64(bg)
    g = _f64(dL_dimage)
    n = o.shape[0]
    out = {"dmeans2d": np.empty((n, 2)), "dconics": np.empty((n, 3)),
           "dopacity": np.empty(n), "dcolors": np.empty((n, 3))}
    lib.orc_backward(W, H, _ptr(rg), _ptr(pl), _ptr(m), _ptr(c), _ptr(o), _ptr(col), _ptr(b), n,
                     _ptr(g), _ptr(out["dmeans2d"]), _ptr(out["dconics"]), _ptr(out["dopacity"]),
                     _ptr(out["dcolors"]))
    return out


def render(scene: dict, bg=(0.0, 0.0, 0.0)) -> dict[str, np.ndarray]:
    """bin + forward of a scene dict (see ``gsinputs``)."""
    W, H = scene["width"], scene["height"]
    pl, rg = bin_tiles(scene["means2d"], scene["radii"], scene["depths"], W, H)
    out = forward(W, H, rg, pl, scene["means2d"], scene["conics"], scene["opacity"],
                  scene["colors"], bg)
    out["point_list"], out["ranges"] = pl, rg
    return out


def work_counts(fwd: dict, ranges) -> dict[str, int]:
    """E = per-pixel evaluations until stop (sum over pixels); Eb = list positions before each
    pixel's last contributor (sum; what the backward revisits); K = blended pairs; F = entries a
    tile must fetch (max over its pixels of the stop position, summed over tiles); P = pairs."""
    n_eval = fwd["n_eval"]
    H, W = n_eval.shape
    gx, gy = grid(W, H)
    pad = np.zeros((gy * TILE, gx * TILE), np.int64)
    pad[:H, :W] = n_eval
    F = int(pad.reshape(gy, TILE, gx, TILE).max(axis=(1, 3)).sum())
    rg = np.asarray(ranges, np.int64)
    return {"E": int(n_eval.astype(np.int64).sum()),
            "Eb": int(fwd["last_contrib"].astype(np.int64).sum()),
            "K": int(fwd["n_contrib"].astype(np.int64).sum()), "F": F,
            "P": int((rg[:, 1] - rg[:, 0]).sum())}


def camera_array(cam) -> np.ndarray:
    """[R(9), t(3), fx, fy, cx, cy, W, H, near] of a ``gsinputs.Camera``; every float rounded
    to FP32 first (the values the FP32 library receives)."""
    f = np.float32
    vals = [*np.ravel(cam.R), *cam.t, cam.fx, cam.fy, cam.cx, cam.cy]
    return np.array([*np.asarray(vals, f).astype(np.float64), cam.width, cam.height,
                     float(f(cam.near))], np.float64)


def sh_basis(dirs, deg: int) -> np.ndarray:
    """Real spherical harmonics (Condon-Shortley phase kept) of degree <= deg at directions
    dirs [n][3] (normalised inside): [n][(deg + 1)^2]."""
    lib = _load()
    d = _f64(dirs).reshape(-1, 3)
    out = np.empty((d.shape[0], (deg + 1) ** 2))
    lib.orc_sh_basis(_ptr(d), d.shape[0], deg, _ptr(out))
    return out


def project(scene3d: dict, sh_degree: int | None = None) -> dict[str, np.ndarray]:
    """Projection of 3D Gaussians to the screen in FP64 (rule in gsoracle.c): means2d, conics,
    depths, radii, colors, plus rad_real (3 sqrt(lmax) before the ceiling) and margin [n][3]
    (distance of the depth, det and screen-rectangle decisions from their thresholds: relative,
    relative, pixels; +inf where not reached). sh [n][K][3]; sh_degree defaults to the largest
    the stored K allows."""
    lib = _load()
    m, sc, q = _f64(scene3d["means3d"]), _f64(scene3d["scales"]), _f64(scene3d["quats"])
    sh = _f64(scene3d["sh"])
    n, K = m.shape[0], sh.shape[1]
    deg = int(round(np.sqrt(K))) - 1 if sh_degree is None else int(sh_degree)
    if not (0 <= deg <= 3 and (deg + 1) ** 2 <= K):
        raise ValueError(f"SH degree {deg} needs (deg + 1)^2 <= {K} coefficients, deg <= 3")
    cam = camera_array(scene3d["camera"])
    out = {"means2d": np.empty((n, 2)), "conics": np.empty((n, 3)), "depths": np.empty(n),
           "radii": np.empty(n, np.int32), "colors": np.empty((n, 3)), "rad_real": np.empty(n),
           "margin": np.empty((n, 3))}
    lib.orc_project(_ptr(m), _ptr(sc), _ptr(q), _ptr(sh), K, deg, n, _ptr(cam),
                    _ptr(out["means2d"]), _ptr(out["conics"]), _ptr(out["depths"]),
                    _ptr(out["radii"]), _ptr(out["colors"]), _ptr(out["rad_real"]),
                    _ptr(out["margin"]))
    return out
