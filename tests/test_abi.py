"""C ABI checks that need no GPU: the library loads, exports every function
include/gs.h declares, sizes plans, and rejects bad arguments synchronously
(before any HIP call)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gs.h")

from paper_2410_00486_amd import _lib as L  # noqa: E402


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    names = _declared_functions()
    assert len(names) >= 20
    lib = ctypes.CDLL(L.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding declares a signature for each of them
    assert set(names) <= set(L.SIGNATURES), set(names) - set(L.SIGNATURES)


def _plan(n=100, deg=0, views=((128, 96),), tile=(16, 16), lds=256, chunk=2, cap=1000):
    p = L.GsPlan()
    cfg = L.GsRasterCfg(tile[0], tile[1], chunk, lds, 0, 0.1)
    wh = (ctypes.c_int32 * (2 * len(views)))(*[v for pair in views for v in pair])
    st = L.lib().gs_plan_init(ctypes.byref(p), n, deg, len(views), wh, ctypes.byref(cfg), cap)
    return st, p


def test_plan_sizes_and_queries():
    st, p = _plan(n=2000, views=((128, 96), (33, 17)), cap=5000)
    assert st == L.GS_OK
    lib = L.lib()
    assert lib.gs_workspace_size(ctypes.byref(p)) > 2000 * 64
    assert lib.gs_plan_total_pixels(ctypes.byref(p)) == 128 * 96 + 33 * 17
    assert lib.gs_plan_pixel_offset(ctypes.byref(p), 1) == 128 * 96
    assert lib.gs_plan_pixel_offset(ctypes.byref(p), 2) == -1
    assert lib.gs_plan_total_tiles(ctypes.byref(p)) == 8 * 6 + 3 * 2
    for r in range(8):
        assert lib.gs_plan_ws_offset(ctypes.byref(p), r) % 256 == 0
    assert lib.gs_plan_ws_offset(ctypes.byref(p), 99) == -1


@pytest.mark.parametrize("kw,status", [
    (dict(tile=(32, 32)), L.GS_ERR_UNSUPPORTED),
    (dict(tile=(8, 16)), L.GS_ERR_UNSUPPORTED),
    (dict(deg=4), L.GS_ERR_UNSUPPORTED),
    (dict(lds=48), L.GS_ERR_UNSUPPORTED),
    (dict(chunk=0), L.GS_ERR_INVALID_ARG),
    (dict(n=-1), L.GS_ERR_INVALID_ARG),
    (dict(cap=0), L.GS_ERR_INVALID_ARG),
    (dict(views=((0, 10),)), L.GS_ERR_INVALID_ARG),
    (dict(views=((20000, 10),)), L.GS_ERR_INVALID_ARG),
])
def test_plan_rejects_bad_arguments(kw, status):
    st, _ = _plan(**kw)
    assert st == status
    assert len(L.lib().gs_last_error()) > 0


def test_entry_points_reject_bad_arguments_without_gpu():
    lib = L.lib()
    st, p = _plan()
    assert st == L.GS_OK
    pp = ctypes.byref(p)
    g = L.GsGaussians(None, None, None, None, None, 100, 0)
    # uninitialised plan, null workspace, null gaussian pointers, wrong n
    assert lib.gs_preprocess(ctypes.byref(L.GsPlan()), ctypes.byref(g), 1, 256, None) == L.GS_ERR_INVALID_ARG
    assert lib.gs_preprocess(pp, ctypes.byref(g), 1, None, None) == L.GS_ERR_INVALID_ARG
    assert lib.gs_preprocess(pp, ctypes.byref(g), 1, 256, None) == L.GS_ERR_INVALID_ARG
    g2 = L.GsGaussians(16, 16, 16, 16, 16, 99, 0)
    assert lib.gs_preprocess(pp, ctypes.byref(g2), 1, 256, None) == L.GS_ERR_INVALID_ARG
    g3 = L.GsGaussians(16, 16, 8, 16, 16, 100, 0)      # quats not 16-byte aligned
    assert lib.gs_preprocess(pp, ctypes.byref(g3), 1, 256, None) == L.GS_ERR_INVALID_ARG
    assert lib.gs_bin_sort(pp, 255, None) == L.GS_ERR_INVALID_ARG   # misaligned workspace
    assert lib.gs_render_fwd(pp, 256, 16, None, 16, 16, 16, None, None, None, None) == L.GS_ERR_INVALID_ARG
    assert lib.gs_render_fwd(pp, 256, 16, 16, 16, 16, 16, 16, None, None, None) == L.GS_ERR_INVALID_ARG
    grads = L.GsGaussianGrads(None, None, None, None, None)
    assert lib.gs_render_bwd(pp, ctypes.byref(g2), 16, 256, 16, 16, 16, 16, 16, None, None, None,
                             ctypes.byref(grads), None, None) == L.GS_ERR_INVALID_ARG
    assert lib.gs_sort_pairs(None, None, 0, 40, None, None) == L.GS_OK
    assert lib.gs_sort_pairs(16, 16, 10, 0, 256, None) == L.GS_ERR_INVALID_ARG
    assert lib.gs_sort_pairs(16, 16, 10, 65, 256, None) == L.GS_ERR_INVALID_ARG
    assert lib.gs_adam_step(None, 0, 1, 0.9, 0.999, 1e-15, 0.0, 0, None, None) == L.GS_OK
    grp = (L.GsParamGroup * 1)(L.GsParamGroup(8, 16, 16, 16, 10, 1e-3, 0))
    assert lib.gs_adam_step(grp, 1, 1, 0.9, 0.999, 1e-15, 0.0, 0, None, None) == L.GS_ERR_INVALID_ARG
    assert lib.gs_adam_step(grp, 1, 0, 0.9, 0.999, 1e-15, 0.0, 0, None, None) == L.GS_ERR_INVALID_ARG
    assert lib.gs_graph_create(None, None, None) == L.GS_ERR_INVALID_ARG
    # an iteration with Adam groups but no device step counter
    it = L.GsIteration()
    it.plan = ctypes.pointer(p)
    it.ws = 256
    it.adam_groups = ctypes.cast(grp, ctypes.POINTER(L.GsParamGroup))
    it.n_adam_groups = 1
    it.step_dev = None
    assert lib.gs_iteration_enqueue(ctypes.byref(it), None) == L.GS_ERR_INVALID_ARG
    assert b"step_dev" in lib.gs_last_error()
    # pose retraction and its tangent pull-back: null buffers, view count
    assert lib.gs_pose_retract(None, 16, 16, 1, None) == L.GS_ERR_INVALID_ARG
    assert lib.gs_pose_retract(16, 16, 16, 0, None) == L.GS_ERR_INVALID_ARG
    assert lib.gs_pose_tangent_vjp(16, None, 16, 1, None) == L.GS_ERR_INVALID_ARG
    assert lib.gs_pose_tangent_vjp(16, 16, 16, L.GS_MAX_VIEWS + 1, None) == L.GS_ERR_INVALID_ARG
    assert lib.gs_status_string(L.GS_ERR_HIP) == b"GS_ERR_HIP"


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(L, "LIB_PATH", "/nonexistent/libgs.so")
    monkeypatch.setattr(L, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        L.lib()


def test_python_plan_layout_without_gpu():
    from paper_2410_00486_amd import Plan
    p = Plan(1000, 3, [(640, 480), (320, 240)], tile=(16, 8), pair_capacity=12345)
    assert p.total_pixels == 640 * 480 + 320 * 240
    assert p.total_tiles == 40 * 60 + 20 * 30
    assert p.pixel_offsets == [0, 640 * 480]
    with pytest.raises(L.GsError):
        Plan(10, 0, [(64, 64)], tile=(4, 4))
