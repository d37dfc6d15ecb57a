"""The C-ABI library loads on a machine without a GPU, exports every entry
point that include/ih.h declares, and rejects bad arguments before touching
the device (no call here reaches a kernel)."""
import ctypes
import os
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
HEADER = ROOT / "include" / "ih.h"
# IH_LIBRARY may name another build of the same library (the sanitized
# builds of tests/test_host_checks.py run this file against theirs).
LIB = Path(os.environ.get("IH_LIBRARY", ROOT / "paper_1711_01919_amd" / "libih.so"))


def declared_functions():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(ih_[a-z0-9_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not LIB.exists():
        import paper_1711_01919_amd.build as b
        b.build()
    return ctypes.CDLL(str(LIB))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("ih_compute", "ih_query", "ih_query_device", "ih_status_str"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), f"{name} declared in ih.h but not exported"


def test_status_strings(lib):
    lib.ih_status_str.restype = ctypes.c_char_p
    for code, name in enumerate(["IH_OK", "IH_ERR_INVALID_ARG", "IH_ERR_RANGE", "IH_ERR_OOM", "IH_ERR_HIP",
                                 "IH_ERR_BUDGET", "IH_NOT_READY", "IH_ERR_UNKNOWN_TICKET", "IH_ERR_SHUTDOWN"]):
        assert lib.ih_status_str(code).decode() == name


def test_compute_rejects_bad_arguments_before_launch(lib):
    f = lib.ih_compute
    f.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    fake = 0x1000  # never dereferenced: validation fails first
    assert f(None, 4, 4, 8, fake, None) == 1
    assert f(fake, 4, 4, 8, None, None) == 1
    assert f(fake, 0, 4, 8, fake, None) == 1
    assert f(fake, 4, -1, 8, fake, None) == 1
    assert f(fake, 4, 4, 0, fake, None) == 1
    assert f(fake, 4, 4, 257, fake, None) == 1
    assert f(fake, 65536, 65536, 8, fake, None) == 2          # H*W = 2^32
    assert f(fake, 4, 4, 8, fake + 2, None) == 1              # misaligned output


def test_compute_noalloc_rejects_before_touching_the_device(lib):
    """Argument errors, and frames whose carries exceed the fixed array
    (IH_ERR_RANGE), come back before any HIP call."""
    f = lib.ih_compute_noalloc
    f.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    fake = 0x1000  # never dereferenced: validation fails first
    assert f(None, 4, 4, 8, fake, None) == 1
    assert f(fake, 4, 4, 8, None, None) == 1
    assert f(fake, 0, 4, 8, fake, None) == 1
    assert f(fake, 4, 4, 257, fake, None) == 1
    assert f(fake, 4, 4, 8, fake + 2, None) == 1
    assert f(fake, 65536, 65536, 8, fake, None) == 2           # H*W = 2^32
    assert f(fake, 2160, 3840, 256, fake, None) == 2           # carries beyond the array
    assert f(fake, 4320, 7680, 128, fake, None) == 2


class View(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("B", ctypes.c_int32), ("stream", ctypes.c_void_p)]


@pytest.mark.parametrize("name", ["ih_query", "ih_query_binmajor"])
def test_query_rejects_bad_rectangles_before_launch(lib, name):
    f = getattr(lib, name)
    f.argtypes = [ctypes.POINTER(View), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    v = View(0x1000, 10, 20, 4, None)
    for bad in ([0, 0, 20, 0], [-1, 0, 0, 0], [3, 0, 2, 0], [0, 5, 0, 4], [0, 0, 0, 10]):
        rects = (ctypes.c_int32 * 8)(0, 0, 19, 9, *bad)
        assert f(ctypes.byref(v), ctypes.addressof(rects), 2, 0x2000) == 1
    assert f(None, None, 1, 0x2000) == 1
    assert f(ctypes.byref(v), None, 0, None) == 0              # n = 0 is a no-op


def test_transfer_pipeline_rejects_bad_arguments_before_launch(lib):
    f = lib.ih_transfer_pipeline
    vp = ctypes.c_void_p
    f.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32,
                  ctypes.c_int32, ctypes.c_int32, vp]
    fake = 0x1000  # never dereferenced: validation fails first
    one = (vp * 1)(fake)
    null_entry = (vp * 2)(fake, None)
    two = (vp * 2)(fake, fake)
    assert f(None, one, 1, 4, 4, 8, 2, None) == 1
    assert f(one, None, 1, 4, 4, 8, 2, None) == 1
    assert f(one, one, 0, 4, 4, 8, 2, None) == 1               # no frames
    assert f(one, one, 1, 4, 4, 8, 0, None) == 1               # n_streams out of range
    assert f(one, one, 1, 4, 4, 8, 9, None) == 1
    assert f(one, one, 1, 0, 4, 8, 2, None) == 1               # bad shape
    assert f(one, one, 1, 4, 4, 300, 2, None) == 1
    assert f(one, one, 1, 65536, 65536, 8, 2, None) == 2       # H*W = 2^32
    assert f(two, null_entry, 2, 4, 4, 8, 2, None) == 1        # null output pointer


def test_compute_lut_rejects_bad_tables_before_launch(lib):
    f = lib.ih_compute_lut
    f.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                  ctypes.c_void_p, ctypes.c_void_p]
    fake = 0x1000  # never dereferenced: validation fails first
    good = (ctypes.c_uint8 * 256)(*[v * 4 // 256 for v in range(256)])
    too_big = (ctypes.c_uint8 * 256)(*([0] * 255 + [4]))
    decreasing_too_big = (ctypes.c_uint8 * 256)(*([5] * 128 + [0] * 128))
    assert f(fake, 4, 4, 4, None, fake, None) == 1
    assert f(None, 4, 4, 4, good, fake, None) == 1
    assert f(fake, 4, 4, 4, too_big, fake, None) == 1
    assert f(fake, 4, 4, 4, decreasing_too_big, fake, None) == 1
    assert f(fake, 0, 4, 4, good, fake, None) == 1
    assert f(fake, 4, 4, 4, good, fake + 2, None) == 1


def test_batch_plan_rejects_bad_tables_and_layouts_before_launch(lib):
    class FrameDesc(ctypes.Structure):
        _fields_ = [("frame", ctypes.c_void_p), ("out", ctypes.c_void_p), ("H", ctypes.c_int32),
                    ("W", ctypes.c_int32), ("B", ctypes.c_int32), ("lut", ctypes.c_void_p),
                    ("binmajor", ctypes.c_int32)]
    f = lib.ih_batch_plan_create
    f.argtypes = [ctypes.POINTER(FrameDesc), ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.POINTER(ctypes.c_void_p)]
    fake = 0x1000  # never dereferenced: validation fails first
    too_big = (ctypes.c_uint8 * 256)(*([0] * 255 + [8]))
    decreasing_too_big = (ctypes.c_uint8 * 256)(*([9] * 100 + [1] * 156))
    plan = ctypes.c_void_p()
    for table in (decreasing_too_big, too_big):
        d = (FrameDesc * 1)(FrameDesc(fake, fake, 4, 4, 8, ctypes.cast(table, ctypes.c_void_p), 0))
        assert f(d, 1, None, None, ctypes.byref(plan)) == 1
        assert not plan.value
    good = (ctypes.c_uint8 * 256)(*([0] * 256))
    for d in (FrameDesc(fake, fake, 4, 4, 8, None, 2),                                 # no such layout
              FrameDesc(fake, fake, 4, 4, 8, ctypes.cast(good, ctypes.c_void_p), 1)):  # bin-major with a table
        assert f((FrameDesc * 1)(d), 1, None, None, ctypes.byref(plan)) == 1
        assert not plan.value


def test_batch_options_rejected_before_launch(lib):
    """Carry schedule codes below -2 and tile branches outside 0..4 are argument
    errors, reported before any descriptor is read or device call made."""
    class Options(ctypes.Structure):
        _fields_ = [("autotune", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("tile_x", ctypes.c_int32),
                    ("tile_y", ctypes.c_int32), ("nontemporal", ctypes.c_int32), ("group_bytes", ctypes.c_int64),
                    ("carry_bands", ctypes.c_int32), ("tile_branches", ctypes.c_int32)]
    f = lib.ih_batch_plan_create
    f.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(Options), ctypes.c_void_p,
                  ctypes.POINTER(ctypes.c_void_p)]
    fake = 0x1000  # never dereferenced: validation fails first
    plan = ctypes.c_void_p()
    for bad in (Options(0, 1, 0, 0, -1, 0, -3, 0), Options(0, 1, 0, 0, -1, 0, -1, 5),
                Options(0, 1, 0, 0, -1, 0, -1, -1)):
        assert f(fake, 1, ctypes.byref(bad), None, ctypes.byref(plan)) == 1
        assert not plan.value
