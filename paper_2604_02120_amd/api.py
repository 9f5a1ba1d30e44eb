"""Tensor-level calls on top of the C ABI: device memory and streams come from PyTorch, every
step of the work runs in libgsblend's kernels.

Tensors must be contiguous and on the current HIP device:
  means2d f32[n][2], conics f32[n][3] (A, B, C), opacity f32[n], colors f32[n][3],
  depths f32[n], radii i32[n]; point_list/ranges are i32 tensors holding u32 values;
  for the projection means3d f32[n][3], scales f32[n][3], quats f32[n][4] (w, x, y, z) and
  sh f32[n][K][3].
"""
from __future__ import annotations

import ctypes

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


def camera_struct(R, t, fx, fy, cx, cy, width, height, near=0.2) -> _lib.GsbCamera:
    """A gsb_camera from a world-to-camera rotation R (3x3, row-major) and translation t."""
    c = _lib.GsbCamera()
    flat = [float(v) for row in R for v in row]
    if len(flat) != 9 or len(t) != 3:
        raise ValueError("R must be 3x3 and t of length 3")
    c.R[:] = flat
    c.t[:] = [float(v) for v in t]
    c.fx, c.fy, c.cx, c.cy = float(fx), float(fy), float(cx), float(cy)
    c.width, c.height, c.near = int(width), int(height), float(near)
    return c


def _camera(cam) -> _lib.GsbCamera:
    if isinstance(cam, _lib.GsbCamera):
        return cam
    return camera_struct(cam.R, cam.t, cam.fx, cam.fy, cam.cx, cam.cy, cam.width, cam.height,
                         cam.near)


def project(means3d, scales, quats, sh, camera, sh_degree=None, stream=None, out=None):
    """Preprocessing: 3D Gaussians (means3d f32[n][3], scales f32[n][3], quats f32[n][4] as
    (w, x, y, z), sh f32[n][K][3]) seen by ``camera`` (a GsbCamera, or any object with R, t, fx,
    fy, cx, cy, width, height, near) -> (means2d [n][2], conics [n][3], depths [n], radii i32[n],
    colors [n][3]). sh_degree defaults to the largest that K coefficients hold."""
    for t_, nm in ((means3d, "means3d"), (scales, "scales"), (quats, "quats"), (sh, "sh")):
        _req(t_, torch.float32, nm)
    n = means3d.shape[0]
    if sh.dim() != 3 or sh.shape[0] != n or sh.shape[2] != 3:
        raise ValueError("sh must be [n][K][3]")
    K = sh.shape[1]
    deg = int(round(K ** 0.5)) - 1 if sh_degree is None else int(sh_degree)
    dev = means3d.device
    if out is None:
        out = (torch.empty((n, 2), dtype=torch.float32, device=dev),
               torch.empty((n, 3), dtype=torch.float32, device=dev),
               torch.empty((n,), dtype=torch.float32, device=dev),
               torch.empty((n,), dtype=torch.int32, device=dev),
               torch.empty((n, 3), dtype=torch.float32, device=dev))
    m2, con, dep, rad, col = out
    _lib.gsb_project(means3d.data_ptr(), scales.data_ptr(), quats.data_ptr(), sh.data_ptr(), K,
                     deg, n, _camera(camera), m2.data_ptr(), con.data_ptr(), dep.data_ptr(),
                     rad.data_ptr(), col.data_ptr(), _stream(stream))
    return m2, con, dep, rad, col


class BinWorkspace:
    """Device workspace of the binning calls, sized for (n, pair_capacity, W, H)."""

    def __init__(self, n: int, pair_capacity: int, W: int, H: int, device=None):
        self.n, self.capacity, self.W, self.H = n, pair_capacity, W, H
        self.nbytes = _lib.gsb_bin_workspace_bytes(n, pair_capacity, W, H)
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=device or "cuda")

    def ptr(self) -> int:
        return self.buf.data_ptr()


BIN_MODES = {"rect": _lib.GSB_BIN_RECT, "visible": _lib.GSB_BIN_VISIBLE}


def _bin_mode(mode, conics, opacity):
    """(mode code, conics ptr, opacity ptr) for the binning calls."""
    code = BIN_MODES[mode] if isinstance(mode, str) else int(mode)
    if code == _lib.GSB_BIN_RECT:
        return code, 0, 0
    if conics is None or opacity is None:
        raise ValueError("the 'visible' binning mode needs conics and opacity")
    _req(conics, torch.float32, "conics")
    _req(opacity, torch.float32, "opacity")
    return code, conics.data_ptr(), opacity.data_ptr()


def bin_count(means2d, radii, W: int, H: int, ws: BinWorkspace, stream=None, conics=None,
              opacity=None, mode="rect") -> torch.Tensor:
    """Device int64[1] pair count; the per-Gaussian offsets stay in ``ws``. ``mode``: "rect" (the
    3-sigma square) or "visible" (only tiles where alpha can reach 1/255; needs conics, opacity)."""
    n = radii.shape[0]
    _req(means2d, torch.float32, "means2d")
    _req(radii, torch.int32, "radii")
    code, cp, op = _bin_mode(mode, conics, opacity)
    n_pairs = torch.empty(1, dtype=torch.int64, device=means2d.device)
    _lib.gsb_bin_count(means2d.data_ptr(), radii.data_ptr(), n, W, H, ws.ptr(), ws.nbytes,
                       n_pairs.data_ptr(), _stream(stream), cp, op, code)
    return n_pairs


def bin_fill(means2d, radii, depths, W: int, H: int, ws: BinWorkspace, point_list, ranges,
             stream=None, conics=None, opacity=None, mode="rect") -> torch.Tensor:
    """Fills point_list (i32[capacity]) and ranges (i32[gx*gy][2]); returns the device status.
    ``mode`` (and conics/opacity) must be those of the preceding bin_count."""
    n = radii.shape[0]
    _req(depths, torch.float32, "depths")
    _req(point_list, torch.int32, "point_list")
    _req(ranges, torch.int32, "ranges")
    code, cp, op = _bin_mode(mode, conics, opacity)
    status = torch.empty(1, dtype=torch.int32, device=means2d.device)
    _lib.gsb_bin_fill(means2d.data_ptr(), radii.data_ptr(), depths.data_ptr(), n, W, H, ws.ptr(),
                      ws.nbytes, point_list.data_ptr(), point_list.numel(), ranges.data_ptr(),
                      status.data_ptr(), _stream(stream), cp, op, code)
    return status


def bin_tiles(means2d, radii, depths, W: int, H: int, stream=None, conics=None, opacity=None,
              mode="rect"):
    """Count, then fill with an exactly sized list. Returns (point_list i32[P], ranges
    i32[gx*gy][2]). Synchronises once to read the pair count."""
    n = radii.shape[0]
    ws0 = BinWorkspace(n, 0, W, H, device=means2d.device)
    n_pairs = int(bin_count(means2d, radii, W, H, ws0, stream, conics, opacity, mode).item())
    ws = BinWorkspace(n, n_pairs, W, H, device=means2d.device)
    ws.buf[: ws0.nbytes].copy_(ws0.buf)          # per-Gaussian offsets from the count
    gx, gy = grid(W, H)
    point_list = torch.empty(max(n_pairs, 1), dtype=torch.int32, device=means2d.device)
    ranges = torch.empty((gx * gy, 2), dtype=torch.int32, device=means2d.device)
    bin_fill(means2d, radii, depths, W, H, ws, point_list[:n_pairs] if n_pairs else point_list[:0],
             ranges, stream, conics, opacity, mode)
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


def pack_gaussians(means2d, conics, opacity, colors, stream=None, out=None) -> torch.Tensor:
    """The per-Gaussian records (f32[n][12], one 48-byte record per Gaussian) that the _packed
    blends read instead of the four arrays."""
    n = opacity.shape[0]
    for t, name in ((means2d, "means2d"), (conics, "conics"), (opacity, "opacity"),
                    (colors, "colors")):
        _req(t, torch.float32, name)
    rec = torch.empty((n, _lib.GSB_RECORD_FLOATS), dtype=torch.float32,
                      device=means2d.device) if out is None else out
    _req(rec, torch.float32, "records")
    _lib.gsb_pack_gaussians(means2d.data_ptr(), conics.data_ptr(), opacity.data_ptr(),
                            colors.data_ptr(), n, rec.data_ptr(), _stream(stream))
    return rec


def blend_forward_packed(records, ranges, point_list, W: int, H: int, bg=(0.0, 0.0, 0.0),
                         prec="fp16", stream=None, out=None):
    """As blend_forward, reading the Gaussians from pack_gaussians' records."""
    n = records.shape[0]
    _req(records, torch.float32, "records")
    dev = records.device
    img, T, last = out if out is not None else (
        torch.empty((3, H, W), dtype=torch.float32, device=dev),
        torch.empty((H, W), dtype=torch.float32, device=dev),
        torch.empty((H, W), dtype=torch.int32, device=dev))
    _lib.gsb_blend_forward_packed(W, H, ranges.data_ptr(), point_list.data_ptr(),
                                  records.data_ptr(), n, bg, prec_code(prec), img.data_ptr(),
                                  T.data_ptr(), last.data_ptr(), _stream(stream))
    return img, T, last


def blend_backward_packed(records, ranges, point_list, W: int, H: int, final_T, last_contrib,
                          dL_dimage, bg=(0.0, 0.0, 0.0), prec="fp16", stream=None, out=None):
    """As blend_backward, reading the Gaussians from pack_gaussians' records."""
    n = records.shape[0]
    _req(records, torch.float32, "records")
    dev = records.device
    dm, dc, do, dcol = out if out is not None else (
        torch.empty((n, 2), dtype=torch.float32, device=dev),
        torch.empty((n, 3), dtype=torch.float32, device=dev),
        torch.empty((n,), dtype=torch.float32, device=dev),
        torch.empty((n, 3), dtype=torch.float32, device=dev))
    _lib.gsb_blend_backward_packed(W, H, ranges.data_ptr(), point_list.data_ptr(),
                                   records.data_ptr(), n, bg, prec_code(prec), final_T.data_ptr(),
                                   last_contrib.data_ptr(), dL_dimage.data_ptr(), dm.data_ptr(),
                                   dc.data_ptr(), do.data_ptr(), dcol.data_ptr(), _stream(stream))
    return dm, dc, do, dcol


class DetWorkspace:
    """Device workspace of gsb_blend_backward_deterministic for n Gaussians and `pairs` list
    entries (a uint8 tensor, 256-byte aligned by the caching allocator)."""

    def __init__(self, n: int, pairs: int, device=None):
        self.n, self.pairs = n, pairs
        self.nbytes = _lib.gsb_backward_det_workspace_bytes(n, pairs)
        self.buf = torch.empty(max(self.nbytes, 1), dtype=torch.uint8, device=device)

    def ptr(self) -> int:
        p = self.buf.data_ptr()
        assert p % 256 == 0
        return p


def blend_backward_deterministic(records, ranges, point_list, W: int, H: int, final_T,
                                 last_contrib, dL_dimage, bg=(0.0, 0.0, 0.0), prec="fp16",
                                 ws: DetWorkspace = None, stream=None, out=None):
    """As blend_backward_packed, with every gradient sum in a fixed order: the result is
    identical bit for bit from run to run. ``ws`` is allocated when not given."""
    n = records.shape[0]
    pairs = point_list.numel()
    _req(records, torch.float32, "records")
    dev = records.device
    if ws is None or ws.n < n or ws.pairs < pairs:
        ws = DetWorkspace(n, pairs, device=dev)
    dm, dc, do, dcol = out if out is not None else (
        torch.empty((n, 2), dtype=torch.float32, device=dev),
        torch.empty((n, 3), dtype=torch.float32, device=dev),
        torch.empty((n,), dtype=torch.float32, device=dev),
        torch.empty((n, 3), dtype=torch.float32, device=dev))
    _lib.gsb_blend_backward_deterministic(
        W, H, ranges.data_ptr(), point_list.data_ptr(), pairs, records.data_ptr(), n, bg,
        prec_code(prec), final_T.data_ptr(), last_contrib.data_ptr(), dL_dimage.data_ptr(),
        ws.ptr(), ws.nbytes, dm.data_ptr(), dc.data_ptr(), do.data_ptr(), dcol.data_ptr(),
        _stream(stream))
    return dm, dc, do, dcol


class BatchedViews:
    """Many views blended by one persistent launch per direction (gsb_plan_*).

    ``scenes``: list of dicts of contiguous device tensors (means2d, conics, opacity, colors,
    depths, radii) plus ``width``/``height``. Each view's binning buffers are sized once, eagerly,
    from its exact pair count (times ``capacity_slack``), so that ``bin()``, ``forward()`` and
    ``backward()`` afterwards enqueue kernels only: the whole step can be captured in a hipGraph.
    ``tuning``: None (library defaults), a dict (batch_fwd, batch_bwd, blocks_per_cu, launch,
    bwd_reduce) or "auto" (``autotune.tune``). ``dL_dimage[v]`` is allocated here (zeros) for the caller to fill.
    """

    def __init__(self, scenes, prec="fp16", tuning=None, bg=(0.0, 0.0, 0.0),
                 capacity_slack: float = 1.0, stream=None, bin_mode="rect", bin_streams: int = 4):
        self.prec = prec_code(prec)
        self.bin_streams = max(1, int(bin_streams))
        self._side = None
        self.bin_mode = bin_mode
        self.bg = tuple(float(v) for v in bg)
        self.views = []
        for sc in scenes:
            W, H = sc["width"], sc["height"]
            n = sc["radii"].shape[0]
            dev = sc["means2d"].device
            ws0 = BinWorkspace(n, 0, W, H, device=dev)
            pairs = int(bin_count(sc["means2d"], sc["radii"], W, H, ws0, stream, sc["conics"],
                                  sc["opacity"], bin_mode).item())
            cap = max(1, int(pairs * capacity_slack))
            gx, gy = grid(W, H)
            v = dict(sc)
            v.update(
                n=n, pairs=pairs, ws=BinWorkspace(n, cap, W, H, device=dev),
                n_pairs=torch.zeros(1, dtype=torch.int64, device=dev),
                status=torch.zeros(1, dtype=torch.int32, device=dev),
                point_list=torch.empty(cap, dtype=torch.int32, device=dev),
                ranges=torch.empty((gx * gy, 2), dtype=torch.int32, device=dev),
                image=torch.empty((3, H, W), dtype=torch.float32, device=dev),
                final_T=torch.empty((H, W), dtype=torch.float32, device=dev),
                last_contrib=torch.empty((H, W), dtype=torch.int32, device=dev),
                dL_dimage=torch.zeros((3, H, W), dtype=torch.float32, device=dev),
                dL_dmeans2d=torch.empty((n, 2), dtype=torch.float32, device=dev),
                dL_dconics=torch.empty((n, 3), dtype=torch.float32, device=dev),
                dL_dopacity=torch.empty((n,), dtype=torch.float32, device=dev),
                dL_dcolors=torch.empty((n, 3), dtype=torch.float32, device=dev))
            self.views.append(v)
        self.plan = None
        if tuning == "auto":
            from . import autotune
            self._make_plan(None)
            tuning = autotune.tune(self)
        self.tuning = tuning
        self._make_plan(tuning)

    def _gsb_views(self):
        out = []
        for v in self.views:
            out.append(_lib.GsbView(
                v["width"], v["height"], v["n"], v["ranges"].data_ptr(), v["point_list"].data_ptr(),
                v["means2d"].data_ptr(), v["conics"].data_ptr(), v["opacity"].data_ptr(),
                v["colors"].data_ptr(), (ctypes.c_float * 3)(*self.bg), v["image"].data_ptr(),
                v["final_T"].data_ptr(), v["last_contrib"].data_ptr(), v["dL_dimage"].data_ptr(),
                v["dL_dmeans2d"].data_ptr(), v["dL_dconics"].data_ptr(),
                v["dL_dopacity"].data_ptr(), v["dL_dcolors"].data_ptr()))
        return out

    def _make_plan(self, tuning):
        if self.plan is not None:
            _lib.gsb_plan_destroy(self.plan)
            self.plan = None
        t = None
        if tuning:
            t = _lib.GsbTuning(int(tuning.get("batch_fwd", 0)), int(tuning.get("batch_bwd", 0)),
                               int(tuning.get("blocks_per_cu", 0)), int(tuning.get("launch", 0)),
                               int(tuning.get("bwd_reduce", 0)))
        self.plan = _lib.gsb_plan_create(self._gsb_views(), self.prec, t)

    def _bin_view(self, v, s: int):
        W, H = v["width"], v["height"]
        ws = v["ws"]
        code, cp, op = _bin_mode(self.bin_mode, v["conics"], v["opacity"])
        _lib.gsb_bin_count(v["means2d"].data_ptr(), v["radii"].data_ptr(), v["n"], W, H,
                           ws.ptr(), ws.nbytes, v["n_pairs"].data_ptr(), s, cp, op, code)
        _lib.gsb_bin_fill(v["means2d"].data_ptr(), v["radii"].data_ptr(),
                          v["depths"].data_ptr(), v["n"], W, H, ws.ptr(), ws.nbytes,
                          v["point_list"].data_ptr(), v["point_list"].numel(),
                          v["ranges"].data_ptr(), v["status"].data_ptr(), s, cp, op, code)

    def bin(self, stream=None):
        """Bins every view. One view's binning is a chain of small dependent kernels that leaves
        most of the GPU idle, so the views are spread over ``bin_streams`` side streams forked
        from the calling stream and joined back into it (event waits, which a hipGraph capture
        records as parallel branches)."""
        cur = torch.cuda.current_stream() if stream is None else stream
        k = min(self.bin_streams, len(self.views))
        if k <= 1:
            for v in self.views:
                self._bin_view(v, cur.cuda_stream)
            return
        if self._side is None:
            self._side = [torch.cuda.Stream(device=self.views[0]["means2d"].device)
                          for _ in range(self.bin_streams)]
        side = self._side[:k]
        for st in side:
            st.wait_stream(cur)
        # heaviest views first, dealt round-robin
        order = sorted(range(len(self.views)), key=lambda i: -self.views[i]["pairs"])
        for j, i in enumerate(order):
            self._bin_view(self.views[i], side[j % k].cuda_stream)
        for st in side:
            cur.wait_stream(st)

    def check(self):
        """Raises if the last binning of any view overflowed its pair capacity (or failed a
        device-side check). Synchronises on the status words; not for use under capture: a
        captured step replays with the capacities sized at construction."""
        for i, v in enumerate(self.views):
            st = int(v["status"].item())
            if st != _lib.GSB_OK:
                raise _lib.GsbError(st, f"view {i}: binning status {st} (pairs "
                                        f"{int(v['n_pairs'].item())}, capacity "
                                        f"{v['point_list'].numel()})")

    def forward(self, stream=None):
        _lib.gsb_blend_batched_forward(self.plan, _stream(stream))

    def backward(self, stream=None):
        _lib.gsb_blend_batched_backward(self.plan, _stream(stream))

    def step(self, stream=None, check: bool = True):
        """bin + forward + backward of every view. With ``check`` (and outside a hipGraph
        capture) the binning status words are read afterwards and an overflow raises."""
        self.bin(stream)
        self.forward(stream)
        self.backward(stream)
        if check and not torch.cuda.is_current_stream_capturing():
            self.check()

    def pixels(self) -> int:
        return sum(v["width"] * v["height"] for v in self.views)

    def close(self):
        if self.plan is not None:
            _lib.gsb_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
