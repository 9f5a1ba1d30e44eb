"""Host-side checks of the C ABI: the library loads, exports every declared function, and rejects
bad arguments before touching a device (these run without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_2604_02120_amd import _lib, build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsblend.h")


@pytest.fixture(scope="module", autouse=True)
def built():
    if not os.path.exists(_lib.LIB_PATH):
        build.build()
    _lib.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gsb_\w+)\s*\(", text)))


def test_header_declares_what_binding_exposes():
    assert declared_functions() == sorted(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_abi_version():
    assert _lib.gsb_abi_version() == 8


def test_project_validation_before_device():
    ok = 256   # non-null, 16-byte aligned fake address: validation fails before any use
    from paper_2604_02120_amd import api
    cam = api.camera_struct(((1, 0, 0), (0, 1, 0), (0, 0, 1)), (0, 0, 0), 500, 500, 32, 24, 64, 48)

    def bad(frag, *args, camera=cam):
        defaults = dict(means3d=ok, scales=ok, quats=ok, sh=ok, sh_coeffs=16, sh_degree=3, n=10)
        defaults.update(dict(args))
        with pytest.raises(_lib.GsbError) as e:
            _lib.gsb_project(defaults["means3d"], defaults["scales"], defaults["quats"],
                             defaults["sh"], defaults["sh_coeffs"], defaults["sh_degree"],
                             defaults["n"], camera, ok, ok, ok, ok, ok)
        assert e.value.status == _lib.GSB_ERR_INVALID and frag in str(e.value), str(e.value)

    bad("n = -1", ("n", -1))
    bad("n = ", ("n", 1 << 31))
    bad("sh_degree", ("sh_degree", 4))
    bad("sh_degree", ("sh_degree", -1))
    bad("sh_coeffs", ("sh_coeffs", 8))           # degree 3 needs 16
    bad("sh_coeffs", ("sh_coeffs", 17), ("sh_degree", 0))
    bad("non-null", ("means3d", 0))
    bad("16-byte", ("quats", ok + 4))
    bad("16-byte", ("sh", ok + 8))
    for field, val, frag in (("fx", 0.0, "focal"), ("fy", float("nan"), "focal"),
                             ("near", -1.0, "near"), ("width", 0, "image size"),
                             ("height", 70000, "image size")):
        c = api.camera_struct(((1, 0, 0), (0, 1, 0), (0, 0, 1)), (0, 0, 0), 500, 500, 32, 24, 64, 48)
        setattr(c, field, val)
        bad(frag, camera=c)
    with pytest.raises(_lib.GsbError) as e:     # camera = NULL
        _lib._check(_lib.load().gsb_project(ok, ok, ok, ok, 16, 3, 10, None, ok, ok, ok, ok, ok, 0))
    assert "camera" in str(e.value)


def test_no_oracle_in_library():
    # the product library must not contain or link the CPU oracle
    data = open(_lib.LIB_PATH, "rb").read()
    assert b"orc_forward" not in data and b"libgsoracle" not in data


@pytest.mark.parametrize("args,frag", [
    ((-1, 0, 16, 16), "n = -1"),
    ((10, -5, 16, 16), "pair_capacity"),
    ((10, 0, 0, 16), "image size"),
    ((10, 0, 16, 70000), "image size"),
])
def test_workspace_validation(args, frag):
    with pytest.raises(_lib.GsbError) as e:
        _lib.gsb_bin_workspace_bytes(*args)
    assert e.value.status == _lib.GSB_ERR_INVALID and frag in str(e.value)


def test_workspace_grows_with_capacity():
    a = _lib.gsb_bin_workspace_bytes(1000, 0, 64, 64)
    b = _lib.gsb_bin_workspace_bytes(1000, 100_000, 64, 64)
    assert b > a + 100_000 * 12   # two tile-key buffers and a value buffer per pair


def test_forward_validation_before_device():
    ok = 256  # a non-null, 8-byte aligned fake address: validation fails before any use
    cases = [
        ((0, 16, ok, ok, ok, ok, ok, ok, 1, (0, 0, 0), 0, ok, ok, ok), "image size"),
        ((16, 16, 0, ok, ok, ok, ok, ok, 1, (0, 0, 0), 0, ok, ok, ok), "ranges"),
        ((16, 16, ok + 4, ok, ok, ok, ok, ok, 1, (0, 0, 0), 0, ok, ok, ok), "aligned"),
        ((16, 16, ok, ok, 0, ok, ok, ok, 1, (0, 0, 0), 0, ok, ok, ok), "attribute"),
        ((16, 16, ok, ok, ok, ok, ok, ok, 1, None, 0, ok, ok, ok), "bg"),
        ((16, 16, ok, ok, ok, ok, ok, ok, 1, (0, 0, 0), 9, ok, ok, ok), "precision"),
        ((16, 16, ok, ok, ok, ok, ok, ok, 1, (0, 0, 0), 0x200, ok, ok, ok), "precision"),
        ((16, 16, ok, ok, ok, ok, ok, ok, 1, (0, 0, 0), 3 | _lib.GSB_FULL_SCAN, ok, ok, ok),
         "precision"),
        # the full-scan flag is accepted with every precision (validation reaches the outputs)
        ((16, 16, ok, ok, ok, ok, ok, ok, 1, (0, 0, 0), _lib.GSB_FULL_SCAN, 0, ok, ok), "output"),
        ((16, 16, ok, ok, ok, ok, ok, ok, 1, (0, 0, 0), 2 | _lib.GSB_FULL_SCAN, 0, ok, ok),
         "output"),
        ((16, 16, ok, ok, ok, ok, ok, ok, 1, (0, 0, 0), 1, 0, ok, ok), "output"),
    ]
    for args, frag in cases:
        with pytest.raises(_lib.GsbError) as e:
            _lib.gsb_blend_forward(*args)
        assert e.value.status == _lib.GSB_ERR_INVALID, args
        assert frag in str(e.value), (frag, str(e.value))


def test_backward_validation_before_device():
    ok = 256
    with pytest.raises(_lib.GsbError) as e:
        _lib.gsb_blend_backward(16, 16, ok, ok, ok, ok, ok, ok, 3, (0, 0, 0), 0, ok, ok, ok,
                                0, ok, ok, ok)
    assert e.value.status == _lib.GSB_ERR_INVALID and "gradient" in str(e.value)


def test_bin_validation_before_device():
    ok = 256
    need = _lib.gsb_bin_workspace_bytes(100, 0, 32, 32)
    with pytest.raises(_lib.GsbError) as e:
        _lib.gsb_bin_count(ok, ok, 100, 32, 32, ok, need - 1, ok)
    assert e.value.status == _lib.GSB_ERR_INVALID and "workspace" in str(e.value)
    with pytest.raises(_lib.GsbError) as e:
        _lib.gsb_bin_count(ok, ok, 100, 32, 32, ok + 8, need, ok)
    assert "256-byte" in str(e.value)
    need2 = _lib.gsb_bin_workspace_bytes(100, 50, 32, 32)
    with pytest.raises(_lib.GsbError) as e:
        _lib.gsb_bin_fill(ok, ok, ok, 100, 32, 32, ok, need2, 0, 50, ok, ok)
    assert "point_list" in str(e.value)


def test_last_error_is_thread_local():
    import threading
    with pytest.raises(_lib.GsbError):
        _lib.gsb_bin_workspace_bytes(-1, 0, 16, 16)
    seen = []
    t = threading.Thread(target=lambda: seen.append(_lib.gsb_last_error()))
    t.start(); t.join()
    assert seen == [""]
    assert "n = -1" in _lib.gsb_last_error()


def test_plan_validation_before_device():
    ok = 256
    with pytest.raises(_lib.GsbError) as e:
        _lib.gsb_plan_create([], 1)
    assert e.value.status == _lib.GSB_ERR_INVALID and "n_views" in str(e.value)
    v = _lib.GsbView(16, 16, 10, ok, ok, ok, ok, ok, ok, (0.0, 0.0, 0.0), ok, ok, ok, 0, ok, ok, ok, ok)
    with pytest.raises(_lib.GsbError) as e:
        _lib.gsb_plan_create([v], 1)
    assert e.value.status == _lib.GSB_ERR_INVALID and "dL_dimage" in str(e.value)
    bad = _lib.GsbView(0, 16, 10, ok, ok, ok, ok, ok, ok, (0.0, 0.0, 0.0), ok, ok, ok, ok, ok, ok, ok, ok)
    with pytest.raises(_lib.GsbError) as e:
        _lib.gsb_plan_create([bad], 1)
    assert "view 0" in str(e.value) and "image size" in str(e.value)
    with pytest.raises(_lib.GsbError) as e:
        _lib.gsb_plan_create([v], 7)
    assert "precision" in str(e.value)
    with pytest.raises(_lib.GsbError) as e:
        _lib.gsb_blend_batched_forward(0)
    assert "plan" in str(e.value)
    _lib.gsb_plan_destroy(0)     # NULL is allowed


def test_bin_mode_validation_before_device():
    ok = 256
    need = _lib.gsb_bin_workspace_bytes(100, 0, 32, 32)
    with pytest.raises(_lib.GsbError) as e:
        _lib.gsb_bin_count(ok, ok, 100, 32, 32, ok, need, ok, mode=7)
    assert e.value.status == _lib.GSB_ERR_INVALID and "binning mode" in str(e.value)
    with pytest.raises(_lib.GsbError) as e:
        _lib.gsb_bin_count(ok, ok, 100, 32, 32, ok, need, ok, conics=0, opacity=ok,
                           mode=_lib.GSB_BIN_VISIBLE)
    assert "conics and opacity" in str(e.value)
    need2 = _lib.gsb_bin_workspace_bytes(100, 50, 32, 32)
    with pytest.raises(_lib.GsbError) as e:
        _lib.gsb_bin_fill(ok, ok, ok, 100, 32, 32, ok, need2, ok, 50, ok, ok, conics=ok + 2,
                          opacity=ok, mode=_lib.GSB_BIN_VISIBLE)
    assert "aligned" in str(e.value)


def test_packed_validation_before_device():
    ok = 256   # a non-null, 16-byte aligned fake address: validation fails before any use
    cases = [
        (lambda: _lib.gsb_pack_gaussians(ok, ok, ok, ok, 10, ok + 8), "16-byte"),
        (lambda: _lib.gsb_pack_gaussians(ok, ok, ok, 0, 10, ok), "non-null"),
        (lambda: _lib.gsb_pack_gaussians(ok, ok, ok, ok, -1, ok), "n = -1"),
        (lambda: _lib.gsb_blend_forward_packed(16, 16, ok, ok, ok + 4, 1, (0, 0, 0), 0, ok, ok,
                                               ok), "16-byte"),
        (lambda: _lib.gsb_blend_forward_packed(16, 16, ok, ok, 0, 1, (0, 0, 0), 0, ok, ok, ok),
         "attribute"),
        (lambda: _lib.gsb_blend_forward_packed(16, 16, ok, ok, ok, 1, (0, 0, 0), 7, ok, ok, ok),
         "precision"),
        (lambda: _lib.gsb_blend_backward_packed(16, 16, ok, ok, ok, 1, (0, 0, 0), 0, ok, ok, 0,
                                                ok, ok, ok, ok), "dL_dimage"),
        (lambda: _lib.gsb_blend_backward_packed(16, 16, ok, ok, ok, 1, (0, 0, 0), 0, ok, ok, ok,
                                                ok + 4, ok, ok, ok), "8-byte"),
    ]
    for call, frag in cases:
        with pytest.raises(_lib.GsbError) as e:
            call()
        assert e.value.status == _lib.GSB_ERR_INVALID and frag in str(e.value), str(e.value)


def test_deterministic_validation_before_device():
    ok = 256
    assert _lib.gsb_backward_det_workspace_bytes(1000, 100_000) > 100_000 * 36
    with pytest.raises(_lib.GsbError) as e:
        _lib.gsb_backward_det_workspace_bytes(10, -1)
    assert e.value.status == _lib.GSB_ERR_INVALID and "pairs" in str(e.value)
    need = _lib.gsb_backward_det_workspace_bytes(1, 16)

    def call(ws=ok, ws_bytes=need, rec=ok, pairs=16):
        _lib.gsb_blend_backward_deterministic(16, 16, ok, ok, pairs, rec, 1, (0, 0, 0), 0, ok, ok,
                                              ok, ws, ws_bytes, ok, ok, ok, ok)
    for kwargs, frag in ((dict(ws_bytes=need - 1), "smaller"), (dict(ws=ok + 16), "256-byte"),
                         (dict(rec=ok + 8), "16-byte"), (dict(ws=0), "non-null"),
                         (dict(pairs=-2), "pairs")):
        with pytest.raises(_lib.GsbError) as e:
            call(**kwargs)
        assert e.value.status == _lib.GSB_ERR_INVALID and frag in str(e.value), str(e.value)
