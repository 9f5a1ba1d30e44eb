"""Pins of the oracle's preprocessing step (Sec. 2.1(a): 3D Gaussians + camera -> 2D Gaussians
and view-dependent colour) against what the mathematics fixes.

Independent constructions only: scipy's spherical harmonics and rotations, finite-difference
Jacobians of the pinhole map, numpy eigenvalues and inverses, closed forms of special cases,
and invariants of the projection under rigid motions.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy.special import sph_harm_y

import gsinputs
import oracle

F32 = np.float32


def scipy_real_sh(dirs, deg):
    """Real SH (Condon-Shortley phase kept) from scipy's complex ones: sqrt(2) Re Y_l^m for
    m > 0, Y_l^0, sqrt(2) Im Y_l^|m| for m < 0; order (l, m = -l..l)."""
    d = np.asarray(dirs, np.float64)
    d = d / np.linalg.norm(d, axis=1, keepdims=True)
    theta = np.arccos(np.clip(d[:, 2], -1.0, 1.0))
    phi = np.arctan2(d[:, 1], d[:, 0])
    cols = []
    for l in range(deg + 1):
        for m in range(-l, l + 1):
            y = sph_harm_y(l, abs(m), theta, phi)
            cols.append(np.sqrt(2) * y.real if m > 0 else (y.real if m == 0 else np.sqrt(2) * y.imag))
    return np.stack(cols, axis=1)


def one_camera(R=np.eye(3), t=(0.0, 0.0, 0.0), f=800.0, W=640, H=480, near=0.2):
    return gsinputs.Camera(tuple(map(tuple, np.asarray(R, np.float64))), tuple(t), f, f,
                           W / 2.0, H / 2.0, W, H, near)


def scene_of(cam, means, scales, quats=None, sh=None):
    n = len(means)
    if quats is None:
        quats = np.tile([1.0, 0.0, 0.0, 0.0], (n, 1))
    if sh is None:
        sh = np.zeros((n, 1, 3))
    return {"camera": cam, "means3d": np.asarray(means, np.float64),
            "scales": np.asarray(scales, np.float64), "quats": np.asarray(quats, np.float64),
            "sh": np.asarray(sh, np.float64)}


# ----------------------------------------------------------------------------- SH basis
def test_sh_basis_matches_scipy():
    rng = np.random.default_rng(0)
    d = rng.normal(size=(500, 3))
    d = np.vstack([d, [[0, 0, 1], [0, 0, -1], [1, 0, 0], [0, -1, 0]]])   # poles and axes
    for deg in range(4):
        np.testing.assert_allclose(oracle.sh_basis(d, deg), scipy_real_sh(d, deg), atol=1e-13)


def test_sh_basis_degree1_and_orthonormality():
    # band 1 is sqrt(3 / (4 pi)) (-y, z, -x) in this phase convention
    d = np.array([[0.3, -0.5, 0.8], [-1.0, 2.0, 0.5]])
    u = d / np.linalg.norm(d, axis=1, keepdims=True)
    c1 = math.sqrt(3.0 / (4.0 * math.pi))
    np.testing.assert_allclose(oracle.sh_basis(d, 1)[:, 1:],
                               c1 * np.stack([-u[:, 1], u[:, 2], -u[:, 0]], 1), atol=1e-15)
    # Gram matrix over the sphere: Gauss-Legendre in cos(theta) x uniform phi, exact for these
    # polynomial degrees
    ct, wt = np.polynomial.legendre.leggauss(12)
    nphi = 16
    phi = 2 * math.pi * np.arange(nphi) / nphi
    T, P = np.meshgrid(ct, phi, indexing="ij")
    st = np.sqrt(1 - T ** 2)
    dirs = np.stack([st * np.cos(P), st * np.sin(P), T], -1).reshape(-1, 3)
    w = (np.repeat(wt, nphi) * (2 * math.pi / nphi))
    Y = oracle.sh_basis(dirs, 3)
    np.testing.assert_allclose((Y * w[:, None]).T @ Y, np.eye(16), atol=1e-12)


# ----------------------------------------------------------------------------- projection
def test_project_on_axis_closed_form():
    # identity camera, isotropic Gaussian on the optical axis: Sigma2 = ((f s / z)^2 + 0.3) I,
    # the eigenvalue gap is 0 so lmax = v + sqrt(0.1)
    cam = one_camera()
    zs = np.array([0.5, 1.0, 3.0, 10.0])
    ss = np.array([0.001, 0.01, 0.05, 0.002])
    out = oracle.project(scene_of(cam, np.stack([0 * zs, 0 * zs, zs], 1), np.repeat(ss[:, None], 3, 1)))
    v = (800.0 * ss / zs) ** 2 + 0.3
    np.testing.assert_allclose(out["means2d"], np.tile([320.0, 240.0], (4, 1)), rtol=0, atol=1e-12)
    np.testing.assert_allclose(out["depths"], zs, rtol=1e-15)
    np.testing.assert_allclose(out["conics"], np.stack([1 / v, 0 * v, 1 / v], 1), rtol=1e-13, atol=1e-15)
    np.testing.assert_array_equal(out["radii"], np.ceil(3 * np.sqrt(v + math.sqrt(0.1))).astype(int))


def test_project_clamps_jacobian_outside_field_of_view():
    # isotropic Sigma3 = s^2 I, identity camera: Sigma2 = s^2 J J^T + 0.3 I with J's x/z replaced
    # by the clamp limit 1.3 W / (2 f) once |x/z| exceeds it (y/z stays inside)
    f, W, H, z, s = 800.0, 640, 480, 4.0, 0.8
    lim = 1.3 * W / (2 * f)
    for xz in (0.5 * lim, 1.5 * lim, -1.2 * lim):
        yz = 0.1
        out = oracle.project(scene_of(one_camera(f=f, W=W, H=H), [[xz * z, yz * z, z]], [[s, s, s]]))
        cx = min(lim, max(-lim, xz))
        k = (s * f / z) ** 2
        S2 = k * np.array([[1 + cx * cx, cx * yz], [cx * yz, 1 + yz * yz]]) + 0.3 * np.eye(2)
        assert out["radii"][0] > 0
        np.testing.assert_allclose(out["means2d"][0], [f * xz + W / 2, f * yz + H / 2], rtol=1e-14)
        inv = np.linalg.inv(S2)
        np.testing.assert_allclose(out["conics"][0], [inv[0, 0], inv[0, 1], inv[1, 1]], rtol=1e-12)


def look_at_frame(eye, target, up):
    """right, down, forward unit vectors of a look-at camera, built here independently."""
    fwd = np.asarray(target, float) - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    return right, down, fwd


def random_scene_in_view(n, seed, cam, eye, frame, depth=(1.0, 12.0), sh_deg=3):
    rng = np.random.default_rng(seed)
    right, down, fwd = frame
    d = rng.uniform(*depth, n)
    a = rng.uniform(-0.35, 0.35, n) * d * cam.width / cam.fx
    b = rng.uniform(-0.35, 0.35, n) * d * cam.height / cam.fy
    means = eye + d[:, None] * fwd + a[:, None] * right + b[:, None] * down
    scales = np.exp(rng.normal(np.log(0.02), 0.8, (n, 3)))
    q = rng.normal(size=(n, 4))
    sh = rng.normal(0, 0.4, (n, (sh_deg + 1) ** 2, 3))
    return scene_of(cam, means, scales, q, sh), d, a, b


def test_project_matches_pinhole_fd_jacobian_and_scipy_rotation():
    eye = np.array([1.0, -2.0, 0.5])
    target, up = np.array([0.2, 3.0, 1.0]), np.array([0.0, 0.0, 1.0])
    cam = gsinputs.look_at(eye, target, up, 900.0, 880.0, 800, 600)
    eye32 = -np.asarray(cam.R).T @ np.asarray(cam.t)        # centre of the rounded camera
    frame = [np.asarray(cam.R)[i] for i in range(3)]        # rows: the rounded right/down/fwd
    ref_frame = look_at_frame(eye, target, up)
    for u, v in zip(frame, ref_frame):                      # the rows are that frame
        np.testing.assert_allclose(u, v, atol=1e-7)
    sc, d, a, b = random_scene_in_view(300, 1, cam, eye32, frame)
    out = oracle.project(sc)
    assert (out["radii"] > 0).all()
    # means: a point a to the right and b below the axis at depth d lands at (cx + fx a / d, ...)
    np.testing.assert_allclose(out["means2d"], np.stack([cam.cx + cam.fx * a / d,
                                                         cam.cy + cam.fy * b / d], 1), atol=1e-6)
    # (the FP32-rounded rows are unit vectors to ~1e-7)
    np.testing.assert_allclose(out["depths"], d, rtol=3e-7)
    # covariance: finite-difference Jacobian of the world -> pixel map, scipy rotation of q
    R, t = np.asarray(cam.R), np.asarray(cam.t)

    def pix(m):
        p = R @ m + t
        return np.array([cam.fx * p[0] / p[2] + cam.cx, cam.fy * p[1] / p[2] + cam.cy])

    h = 1e-5
    for i in range(0, 300, 7):
        m = sc["means3d"][i]
        Jf = np.stack([(pix(m + h * e) - pix(m - h * e)) / (2 * h) for e in np.eye(3)], 1)
        q = sc["quats"][i]
        Rq = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        S3 = Rq @ np.diag(sc["scales"][i] ** 2) @ Rq.T
        S2 = Jf @ S3 @ Jf.T + 0.3 * np.eye(2)
        inv = np.linalg.inv(S2)
        np.testing.assert_allclose(out["conics"][i], [inv[0, 0], inv[0, 1], inv[1, 1]],
                                   rtol=2e-7, atol=2e-9 * np.abs(inv).max())
        ev = np.linalg.eigvalsh(S2)
        if (ev[1] - ev[0]) / 2 > math.sqrt(0.1) + 1e-6:      # off the sqrt(0.1) floor
            rr = 3 * math.sqrt(ev[1])
            np.testing.assert_allclose(out["rad_real"][i], rr, rtol=1e-7)
            if abs(rr - round(rr)) > 1e-5:
                assert out["radii"][i] == math.ceil(rr)


def test_project_colors_follow_view_direction():
    eye = np.array([0.0, 0.0, -3.0])
    cam = gsinputs.look_at(eye, [0.1, 0.2, 5.0], [0.0, -1.0, 0.0], 700.0, 700.0, 640, 480)
    eye32 = -np.asarray(cam.R).T @ np.asarray(cam.t)
    frame = [np.asarray(cam.R)[i] for i in range(3)]
    sc, *_ = random_scene_in_view(400, 2, cam, eye32, frame)
    out = oracle.project(sc)
    Y = scipy_real_sh(sc["means3d"] - eye32, 3)
    want = np.maximum(0.0, 0.5 + np.einsum("nk,nkc->nc", Y, sc["sh"]))
    np.testing.assert_allclose(out["colors"], want, atol=1e-12)
    assert 0.05 < (out["colors"] == 0).mean() < 0.6         # the clamp at 0 is exercised
    # a lower degree reads only the first (deg + 1)^2 coefficients of each stored row
    for deg in range(3):
        k = (deg + 1) ** 2
        sh2 = sc["sh"].copy()
        sh2[:, k:, :] = 123.0
        got = oracle.project(dict(sc, sh=sh2), sh_degree=deg)["colors"]
        want = np.maximum(0.0, 0.5 + np.einsum("nk,nkc->nc", Y[:, :k], sc["sh"][:, :k]))
        np.testing.assert_allclose(got, want, atol=1e-12)


def test_project_joint_rigid_motion_invariance():
    # moving the world by a rotation Q and translation s, and the camera with it
    # (R' = R Q^T, t' = t - R Q^T s), leaves every 2D output unchanged (degree-0 colour too)
    cam = gsinputs.look_at([0.5, 0.3, -2.0], [0.0, 0.0, 4.0], [0.0, 1.0, 0.0], 800.0, 800.0, 640, 480)
    eye32 = -np.asarray(cam.R).T @ np.asarray(cam.t)
    frame = [np.asarray(cam.R)[i] for i in range(3)]
    sc, *_ = random_scene_in_view(200, 3, cam, eye32, frame, sh_deg=0)
    base = oracle.project(sc)
    Qr = Rotation.from_euler("zyx", [0.7, -0.4, 1.9])
    Q, s = Qr.as_matrix(), np.array([3.0, -1.0, 2.0])
    R, t = np.asarray(cam.R), np.asarray(cam.t)
    cam2 = gsinputs.Camera(tuple(map(tuple, R @ Q.T)), tuple(t - R @ Q.T @ s), cam.fx, cam.fy,
                           cam.cx, cam.cy, cam.width, cam.height, cam.near)
    qs = sc["quats"]
    rots = Qr * Rotation.from_quat(np.stack([qs[:, 1], qs[:, 2], qs[:, 3], qs[:, 0]], 1))
    xyzw = rots.as_quat()
    sc2 = dict(sc, camera=cam2, means3d=sc["means3d"] @ Q.T + s,
               quats=np.stack([xyzw[:, 3], xyzw[:, 0], xyzw[:, 1], xyzw[:, 2]], 1))
    # the moved camera is rounded to FP32 like every camera: tolerances cover that rounding
    moved = oracle.project(sc2)
    np.testing.assert_array_equal(moved["radii"] > 0, base["radii"] > 0)
    np.testing.assert_allclose(moved["means2d"], base["means2d"], atol=5e-3)
    np.testing.assert_allclose(moved["depths"], base["depths"], rtol=1e-6)
    np.testing.assert_allclose(moved["conics"], base["conics"], rtol=2e-4, atol=1e-9)
    np.testing.assert_allclose(moved["colors"], base["colors"], atol=1e-12)


def test_project_culling():
    cam = one_camera(near=0.5)
    f, W, H = 800.0, 640, 480
    # depth: at or behind the near plane -> culled, just in front -> kept
    zs = [0.5 * (1 - 1e-7), 0.5, -3.0, 0.5 * (1 + 1e-6)]
    out = oracle.project(scene_of(cam, [[0.0, 0.0, z] for z in zs], [[0.01] * 3] * 4,
                                  sh=np.full((4, 1, 3), 1.0)))
    np.testing.assert_array_equal(out["radii"] > 0, [False, False, False, True])
    for k in ("means2d", "conics", "depths", "colors"):
        assert not out[k][:3].any()
    # off screen: kept iff the radius square meets a tile of the image (brute force over tiles)
    rng = np.random.default_rng(4)
    n = 400
    u = rng.uniform(-200, W + 200, n)
    v = rng.uniform(-200, H + 200, n)
    z = rng.uniform(1, 5, n)
    s = np.exp(rng.normal(np.log(0.01), 1.0, n))
    sc = scene_of(cam, np.stack([(u - W / 2) / f * z, (v - H / 2) / f * z, z], 1),
                  np.repeat(s[:, None], 3, 1))
    out = oracle.project(sc)
    gx, gy = (W + 15) // 16, (H + 15) // 16
    checked = 0
    for i in range(n):
        r = math.ceil(out["rad_real"][i])
        x, y = u[i], v[i]
        if out["margin"][i, 2] < 1e-6:
            continue
        hit = any(16 * tx <= x + r - 1 and 16 * (tx + 1) > x - r for tx in range(gx)) and \
            any(16 * ty <= y + r - 1 and 16 * (ty + 1) > y - r for ty in range(gy))
        assert (out["radii"][i] > 0) == hit, (i, x, y, r)
        checked += 1
    assert checked > 390 and 50 < (out["radii"] == 0).sum() < 350


def test_project_scene_generator_statistics():
    # the synthetic 3D scene projects to 2D Gaussians of the 2D scenes' size law
    sc = gsinputs.make_scene3d(n=20000, seed=5)
    out = oracle.project(sc)
    assert (out["radii"] > 0).mean() > 0.99
    ref = gsinputs.make_scene("C2", n=20000)
    assert 0.8 < np.median(out["radii"]) / np.median(ref["radii"]) < 1.3
