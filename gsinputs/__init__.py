"""Seeded synthetic inputs for the Gaussian blend: projected 2D Gaussians and upstream gradients.

This module only draws inputs. It holds none of the blend's arithmetic: no exponent, no
compositing, no tile binning. Both the FP64 CPU oracle (in ``oracle/``) and the GPU library are
fed from here, so neither depends on the other.

What a scene is (the inputs of the blending stage of the paper, §2.1(a) and Alg. 1's fetched
attributes):

* ``means2d``  f32[N][2]  projected centre (x, y) in pixels; pixel (px, py) sits at integer coords.
* ``conics``   f32[N][3]  (A, B, C) of the inverse 2D covariance [[A, B], [B, C]] (Eq. alpha).
* ``opacity``  f32[N]     o_i.
* ``colors``   f32[N][3]  RGB c_i.
* ``depths``   f32[N]     view depth d_i > 0 (sorting key, §2.1(c)).
* ``radii``    i32[N]     screen radius r_i = ceil(3 * max(sigma1, sigma2)); 0 = not rendered.

The paper measures on trained scenes from Tanks & Temples, Deep Blending and Mip-NeRF 360
(Table 1). Those are not available here; these seeded scenes stand in for them with the same
resolutions / Gaussian counts and the heavy-tailed footprint laws stated in ``CONFIGS``.

Generation recipe (identical for every config): numpy ``default_rng(seed)`` (PCG64); full vectors
are drawn in the order x ~ U(0, W), y ~ U(0, H), theta ~ U(0, pi), sigma1, sigma2 (i.i.d. per
axis, config law), opacity (config law), rgb ~ U(0, 1) (N x 3), depth ~ U(1, 100). The conic is
R(theta) diag(sigma1^-2, sigma2^-2) R(theta)^T in FP64, rounded once to FP32; the radius is
computed in FP64 from the sigmas, never from the rounded conic.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = ["SceneConfig", "CONFIGS", "make_scene", "make_dloss", "make_views", "fd_subscene",
           "Camera", "make_scene3d", "look_at",
           "stack_scene"]

# log-normal sigma law: ln sigma ~ N(ln median, 0.932^2) has P(sigma > 64) = 1e-4 at median 2,
# i.e. "median 2 px, tail to 64 px"; clipped to [0.5, 64].
LOGNORMAL_SD = 0.932
SIGMA_MIN, SIGMA_MAX = 0.5, 64.0


@dataclasses.dataclass(frozen=True)
class SceneConfig:
    name: str
    width: int
    height: int
    n: int
    sigma_law: str            # "loguniform" (sigma in [lo, hi]) or "lognormal" (median)
    sigma_a: float            # loguniform lo, or lognormal median
    sigma_b: float            # loguniform hi (unused for lognormal)
    opacity_law: str          # "uniform" U(0.05, 0.99) or "beta22" Beta(2,2) * 0.99
    seed: int
    dloss_seed: int | None = None
    clustered: bool = False   # stress variant: means drawn around a few cluster centres

    @property
    def pixels(self) -> int:
        return self.width * self.height


# The five benchmark workloads, by size and law.
CONFIGS = {
    # 64x64, 2000 G, sigma log-uniform [0.5, 8]
    "C1": SceneConfig("C1", 64, 64, 2_000, "loguniform", 0.5, 8.0, "uniform", 1),
    # 1920x1080, 1e6 G, sigma log-normal median 2 px
    "C2": SceneConfig("C2", 1920, 1080, 1_000_000, "lognormal", 2.0, 0.0, "uniform", 2, 1002),
    # 1280x720, 5e5 G, as C2; dL/dimage ~ N(0, 1)
    "C3": SceneConfig("C3", 1280, 720, 500_000, "lognormal", 2.0, 0.0, "uniform", 3, 1003),
    # 3840x2160, 3e6 G, sigma log-normal median 3 px, opacity Beta(2,2)*0.99
    "C5": SceneConfig("C5", 3840, 2160, 3_000_000, "lognormal", 3.0, 0.0, "beta22", 5, 1005),
}

# Multi-view batch: 16 views whose resolution is drawn from this set with seed 4, 300k G each,
# view v drawn with seed 400 + v.
C4_RESOLUTIONS = ((854, 480), (1280, 720), (1920, 1080))
C4_VIEWS, C4_N, C4_DRAW_SEED = 16, 300_000, 4


def _sigmas(rng: np.random.Generator, cfg: SceneConfig, n: int) -> tuple[np.ndarray, np.ndarray]:
    if cfg.sigma_law == "loguniform":
        lo, hi = math.log(cfg.sigma_a), math.log(cfg.sigma_b)
        s1 = np.exp(rng.uniform(lo, hi, n))
        s2 = np.exp(rng.uniform(lo, hi, n))
    elif cfg.sigma_law == "lognormal":
        mu = math.log(cfg.sigma_a)
        s1 = np.clip(np.exp(rng.normal(mu, LOGNORMAL_SD, n)), SIGMA_MIN, SIGMA_MAX)
        s2 = np.clip(np.exp(rng.normal(mu, LOGNORMAL_SD, n)), SIGMA_MIN, SIGMA_MAX)
    else:
        raise ValueError(f"unknown sigma law {cfg.sigma_law!r}")
    return s1, s2


def _opacity(rng: np.random.Generator, cfg: SceneConfig, n: int) -> np.ndarray:
    if cfg.opacity_law == "uniform":
        return rng.uniform(0.05, 0.99, n)
    if cfg.opacity_law == "beta22":
        return rng.beta(2.0, 2.0, n) * 0.99
    raise ValueError(f"unknown opacity law {cfg.opacity_law!r}")


def conic_from_axes(theta: np.ndarray, s1: np.ndarray, s2: np.ndarray) -> np.ndarray:
    """(A, B, C) of R(theta) diag(s1^-2, s2^-2) R(theta)^T, FP64."""
    c, s = np.cos(theta), np.sin(theta)
    i1, i2 = 1.0 / (s1 * s1), 1.0 / (s2 * s2)
    a = c * c * i1 + s * s * i2
    b = c * s * (i1 - i2)
    cc = s * s * i1 + c * c * i2
    return np.stack([a, b, cc], axis=1)


def make_scene(cfg: SceneConfig | str, seed: int | None = None, *, n: int | None = None,
               width: int | None = None, height: int | None = None,
               depth_levels: int | None = None, scale: float = 1.0) -> dict[str, np.ndarray | int]:
    """Draw one scene. Overrides (n, width, height, seed) keep the config's laws.

    ``depth_levels`` quantises depth to that many distinct values (ties stress the sort's
    tie-break); ``None`` keeps continuous depth. ``scale`` renders the same draw at a
    ``scale`` times larger resolution: image size, means and axis lengths are multiplied by it.
    """
    if isinstance(cfg, str):
        cfg = CONFIGS[cfg]
    W = cfg.width if width is None else width
    H = cfg.height if height is None else height
    N = cfg.n if n is None else n
    rng = np.random.default_rng(cfg.seed if seed is None else seed)
    if cfg.clustered:
        k = max(1, N // 20_000)
        cx = rng.uniform(0, W, k)
        cy = rng.uniform(0, H, k)
        which = rng.integers(0, k, N)
        x = np.clip(cx[which] + rng.normal(0, 0.05 * W, N), 0, W - 1e-3)
        y = np.clip(cy[which] + rng.normal(0, 0.05 * H, N), 0, H - 1e-3)
    else:
        x = rng.uniform(0.0, W, N)
        y = rng.uniform(0.0, H, N)
    theta = rng.uniform(0.0, math.pi, N)
    s1, s2 = _sigmas(rng, cfg, N)
    opacity = _opacity(rng, cfg, N)
    rgb = rng.uniform(0.0, 1.0, (N, 3))
    depth = rng.uniform(1.0, 100.0, N)
    if depth_levels is not None:
        depth = 1.0 + np.floor((depth - 1.0) / 99.0 * depth_levels)
    if scale != 1.0:
        x, y, s1, s2 = x * scale, y * scale, s1 * scale, s2 * scale
        W, H = int(round(W * scale)), int(round(H * scale))
    conic = conic_from_axes(theta, s1, s2)
    radii = np.ceil(3.0 * np.maximum(s1, s2)).astype(np.int32)
    return {
        "width": int(W), "height": int(H),
        "means2d": np.stack([x, y], axis=1).astype(np.float32),
        "conics": conic.astype(np.float32),
        "opacity": opacity.astype(np.float32),
        "colors": rgb.astype(np.float32),
        "depths": depth.astype(np.float32),
        "radii": radii,
    }


def make_dloss(width: int, height: int, seed: int) -> np.ndarray:
    """Upstream gradient dL/dimage ~ N(0, 1), planar f32[3][H][W]."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((3, height, width)).astype(np.float32)


def make_views(n_views: int = C4_VIEWS, n: int = C4_N, draw_seed: int = C4_DRAW_SEED,
               scale: float = 1.0) -> list[dict]:
    """The multi-view batch: resolutions drawn from ``C4_RESOLUTIONS``; view v uses seed 400 + v.

    ``scale`` < 1 shrinks resolution and Gaussian count together (for quick tests).
    """
    rng = np.random.default_rng(draw_seed)
    picks = rng.integers(0, len(C4_RESOLUTIONS), n_views)
    base = SceneConfig("C4", 0, 0, n, "lognormal", 2.0, 0.0, "uniform", 0)
    views = []
    for v, p in enumerate(picks):
        W, H = C4_RESOLUTIONS[int(p)]
        W, H = max(1, int(round(W * scale))), max(1, int(round(H * scale)))
        nv = max(1, int(round(n * scale * scale)))
        views.append(make_scene(base, seed=400 + v, n=nv, width=W, height=H))
    return views


def fd_subscene(seed: int = 33) -> dict[str, np.ndarray | int]:
    """32x32, 200 Gaussians with the C1 laws, kept in FP64 (finite-difference checks)."""
    s = make_scene("C1", seed=seed, n=200, width=32, height=32)
    rng = np.random.default_rng(seed + 1)
    # FP64 copies with extra low-order bits so FD steps are not quantised by FP32 inputs.
    out = dict(s)
    for k in ("means2d", "conics", "opacity", "colors"):
        out[k] = s[k].astype(np.float64)
    out["means2d"] = out["means2d"] + rng.uniform(-1e-3, 1e-3, out["means2d"].shape)
    return out


def stack_scene(n: int, opacity: float, width: int = 16, height: int = 16,
                at: tuple[float, float] = (8.0, 8.0), sigma: float = 4.0) -> dict:
    """``n`` identical isotropic Gaussians centred on one pixel, depths 1..n (a hand-checkable
    stack)."""
    inv = 1.0 / (sigma * sigma)
    return {
        "width": width, "height": height,
        "means2d": np.tile(np.array([at], np.float32), (n, 1)),
        "conics": np.tile(np.array([[inv, 0.0, inv]], np.float32), (n, 1)),
        "opacity": np.full(n, opacity, np.float32),
        "colors": np.tile(np.array([[1.0, 0.5, 0.25]], np.float32), (n, 1)),
        "depths": np.arange(1, n + 1, dtype=np.float32),
        "radii": np.full(n, int(math.ceil(3 * sigma)), np.int32),
    }


# ----------------------------------------------------------------------------- 3D scenes
@dataclasses.dataclass(frozen=True)
class Camera:
    """Pinhole camera: world-to-camera rotation R (3x3, row-major) and translation t, focal
    lengths and principal point in pixels, image size, near plane."""
    R: tuple
    t: tuple
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    near: float = 0.2


def look_at(eye, target, up, fx, fy, width, height, near=0.2) -> Camera:
    """Camera at ``eye`` looking at ``target`` (+z forward, +y down in the image, +x right)."""
    eye, target, up = (np.asarray(v, np.float64) for v in (eye, target, up))
    z = target - eye
    z /= np.linalg.norm(z)
    x = np.cross(z, up)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z])
    t = -R @ eye
    return Camera(tuple(map(tuple, R.astype(np.float32).astype(np.float64))),
                  tuple(t.astype(np.float32).astype(np.float64)), float(fx), float(fy),
                  width / 2.0, height / 2.0, int(width), int(height), float(near))


def make_scene3d(n: int = 1_000_000, seed: int = 7, width: int = 1920, height: int = 1080,
                 sigma_px_median: float = 2.0, camera: Camera | None = None) -> dict:
    """3D Gaussians in front of a pinhole camera, drawn so that their projections resemble the
    2D scenes above: depth z ~ U(2, 20) along the view axis, image position uniform, per-axis 3D
    scale = (log-normal pixel sigma, median ``sigma_px_median``, sd 0.932, clipped to [0.5, 64])
    * z / f, a uniformly random rotation (normalised Gaussian quaternion), opacity U(0.05, 0.99),
    spherical-harmonic colour coefficients sh [n][16][3] (degree 3): band 0 U(-1.75, 1.75),
    bands 1-3 N(0, 0.15^2). The camera looks along +z from the origin unless one is given (then
    points are drawn in that camera's frame and mapped to world coordinates).
    Draw order: u, v, z, the three scales, quaternion (4), opacity, band 0 (3), bands 1-3 (45)."""
    cam = camera or Camera(((1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0)), (0.0, 0.0, 0.0),
                           1000.0, 1000.0, width / 2.0, height / 2.0, width, height, 0.2)
    rng = np.random.default_rng(seed)
    u = rng.uniform(0.0, cam.width, n)
    v = rng.uniform(0.0, cam.height, n)
    z = rng.uniform(2.0, 20.0, n)
    sig = np.clip(np.exp(rng.normal(math.log(sigma_px_median), 0.932, (n, 3))), 0.5, 64.0)
    q = rng.normal(0.0, 1.0, (n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    opacity = rng.uniform(0.05, 0.99, n)
    sh = np.empty((n, 16, 3))
    sh[:, 0, :] = rng.uniform(-1.75, 1.75, (n, 3))
    sh[:, 1:, :] = rng.normal(0.0, 0.15, (n, 15, 3))
    pc = np.stack([(u - cam.cx) / cam.fx * z, (v - cam.cy) / cam.fy * z, z], axis=1)
    R, t = np.asarray(cam.R), np.asarray(cam.t)
    pw = (pc - t) @ R                                  # camera -> world (R orthonormal)
    scales = sig * (z / cam.fx)[:, None]
    return {
        "camera": cam,
        "means3d": pw.astype(np.float32),
        "scales": scales.astype(np.float32),
        "quats": q.astype(np.float32),                 # (w, x, y, z)
        "opacity": opacity.astype(np.float32),
        "sh": sh.astype(np.float32),
    }
