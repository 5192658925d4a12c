"""The C ABI without a GPU: the library loads, exports every declared symbol,
and its host-only planning validates arguments and lays out the workspace."""
import ctypes
import os
import re

import pytest

from paper_2503_07946_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sd7.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("lib7dgs.so is not built (run __graft_entry__.build())")
    return L.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sd7_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_function(lib):
    names = declared_functions()
    assert set(names) == set(L.EXPORTS), names
    for name in names:
        assert hasattr(lib, name)


def test_struct_sizes_match_the_header_layout():
    # sd7_view: 16 floats, 2 int32, t, d[3], 2 lambdas, bg[3], d_per_gaussian -> 112 bytes
    assert ctypes.sizeof(L.Sd7View) == 112
    assert ctypes.sizeof(L.Sd7Scene) == 64
    assert ctypes.sizeof(L.Sd7Frame) == 64 + 112 + 4 * 8 + 7 * 8 + 8 + 8   # outputs + padding


def test_constants_match_the_header():
    from paper_2503_07946_amd import serve
    defines = dict(re.findall(r"#define (SD7_[A-Z_]+) \(?(-?\d+)u?\)?", open(HEADER).read()))
    for name in ("SD7_MAX_FRAMES", "SD7_TILE", "SD7_PAIR_ROUND", "SD7_CNT_KEPT", "SD7_CNT_PAIRS",
                 "SD7_CNT_PAIR_BASE", "SD7_CNT_FLAGS", "SD7_CNT_NEEDED", "SD7_CNT_WORDS", "SD7_AGR_WEIGHTS",
                 "SD7_OUT_SLICED", "SD7_FLAG_PAIR_OVERFLOW", "SD7_FLAG_SORT_STALL"):
        assert int(defines[name]) == getattr(L, name), name
    assert serve.PAIR_ROUND == L.SD7_PAIR_ROUND


def _frame(n=100, W=64, H=48, ptr=0x1000):
    f = L.Sd7Frame()
    p = ctypes.c_void_p(ptr)
    f.scene = L.Sd7Scene(p, p, p, p, p, p, n)
    f.view.W, f.view.H = W, H
    f.view.fx = f.view.fy = 50.0
    f.image = f.final_T = f.last = p
    return f


def _plan(lib, frames, cap):
    arr = (L.Sd7Frame * len(frames))(*frames)
    lay = L.Sd7Layout()
    rc = lib.sd7_plan(arr, len(frames), cap, ctypes.byref(lay))
    return rc, lay


def test_plan_layout(lib):
    frames = [_frame(100, 64, 48), _frame(0, 17, 5), _frame(5000, 800, 800)]
    rc, lay = _plan(lib, frames, 123457)
    assert rc == L.SD7_OK
    assert lay.nframes == 3 and lay.n_total == 5100
    assert list(lay.g0[:3]) == [0, 100, 100]
    tiles = [4 * 3, 2 * 1, 50 * 50]
    assert lay.tiles_total == sum(tiles)
    assert list(lay.tile0[:3]) == [0, 12, 14]
    assert lay.tile_sort_passes == 2          # 2500 tiles -> 12 bits
    offs = [getattr(lay, k) for k in L._OFFS]
    assert all(o % 256 == 0 for o in offs)
    assert offs == sorted(offs) and lay.bytes >= offs[-1]
    assert lay.off_ranges - lay.off_pair_g >= 4 * 123457
    rc, lay1 = _plan(lib, [_frame(10, 16, 16)], 0)
    assert rc == L.SD7_OK and lay1.tile_sort_passes == 1


@pytest.mark.parametrize("mutate,msg", [
    (lambda fs: setattr(fs[0].view, "W", 0), "W="),
    (lambda fs: setattr(fs[0].view, "H", 16385), "H="),
    (lambda fs: setattr(fs[0].scene, "n", -1), "n="),
    (lambda fs: setattr(fs[0].scene, "L", None), "NULL scene"),
    (lambda fs: setattr(fs[0], "image", None), "NULL image"),
    (lambda fs: setattr(fs[0].view, "fx", 0.0), "focal"),
])
def test_plan_rejects_bad_frames(lib, mutate, msg):
    fs = [_frame()]
    mutate(fs)
    rc, _ = _plan(lib, fs, 1000)
    assert rc == L.SD7_EINVAL
    assert msg in lib.sd7_last_error().decode()


def test_plan_rejects_bad_counts(lib):
    rc, _ = _plan(lib, [_frame()], -5)
    assert rc == L.SD7_EINVAL
    rc, _ = _plan(lib, [_frame()], 1 << 31)
    assert rc == L.SD7_EINVAL
    arr = (L.Sd7Frame * 1)(_frame())
    lay = L.Sd7Layout()
    assert lib.sd7_plan(arr, 0, 10, ctypes.byref(lay)) == L.SD7_EINVAL
    assert lib.sd7_plan(arr, 65, 10, ctypes.byref(lay)) == L.SD7_EINVAL
    assert lib.sd7_plan(None, 1, 10, ctypes.byref(lay)) == L.SD7_EINVAL


def test_empty_scene_needs_no_pointers(lib):
    f = _frame(0)
    f.scene = L.Sd7Scene(None, None, None, None, None, None, 0)
    rc, lay = _plan(lib, [f], 0)
    assert rc == L.SD7_OK and lay.n_total == 0


def test_stage_calls_reject_null_context(lib):
    arr = (L.Sd7Frame * 1)(_frame())
    for name in L.STAGES:
        rc = getattr(lib, name)(None, arr, 1, 100, ctypes.c_void_p(0x100), 1 << 20, None)
        assert rc == L.SD7_EINVAL, name
