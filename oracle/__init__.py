"""Integral-histogram oracle: TEST INFRASTRUCTURE, not product code.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports it and shares no code with it.

This module compiles ``ih_oracle.c`` with gcc into ``liboracle_ih.so`` and
wraps its functions for numpy arrays.  The arithmetic lives in the C file;
each function cites the passage of the paper it follows (Sec. 2.1 Eq. 1 and
Eq. 2, Sec. 2.2 Algorithm 1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
SRC = HERE / "ih_oracle.c"
LIB = HERE / "liboracle_ih.so"
CFLAGS = ["-O2", "-std=c99", "-fPIC", "-shared", "-Wall", "-Wextra"]

_u8p = ctypes.POINTER(ctypes.c_uint8)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64 = ctypes.c_int64


def compile_oracle(out: Path = LIB, source: Path = SRC) -> Path:
    """Compile the oracle with gcc.  ``source`` may name a patched copy of
    ih_oracle.c (the pin tests compile copies with one mistake planted)."""
    out = Path(out)
    cmd = ["gcc", *CFLAGS, str(source), "-o", str(out) + ".tmp"]
    subprocess.run(cmd, check=True, capture_output=True)
    os.replace(str(out) + ".tmp", out)
    return out


def compile_flags() -> str:
    return "gcc " + " ".join(CFLAGS)


class Oracle:
    """numpy-facing wrapper around one compiled oracle library."""

    def __init__(self, path: Path = LIB):
        path = Path(path)
        if not path.exists():
            compile_oracle(path)
        self.path = path
        lib = ctypes.CDLL(str(path))
        lib.ihref_Q.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
        lib.ihref_Q.restype = ctypes.c_uint32
        lib.ihref_integral_histogram.argtypes = [_u8p, _i64, _i64, _i64, _u32p]
        lib.ihref_integral_histogram.restype = ctypes.c_int
        lib.ihref_integral_histogram_binmajor.argtypes = [_u8p, _i64, _i64, _i64, _u32p]
        lib.ihref_integral_histogram_binmajor.restype = ctypes.c_int
        lib.ihref_integral_histogram_lut.argtypes = [_u8p, _i64, _i64, _i64, _u8p, _u32p]
        lib.ihref_integral_histogram_lut.restype = ctypes.c_int
        lib.ihref_integral_rows.argtypes = [_u8p, _i64, _i64, _i64, _i64, _i64, _u32p, _u32p]
        lib.ihref_integral_rows.restype = ctypes.c_int
        lib.ihref_row_by_definition.argtypes = [_u8p, _i64, _i64, _i64, _i64, _u32p]
        lib.ihref_row_by_definition.restype = ctypes.c_int
        lib.ihref_entry.argtypes = [_u8p, _i64, _i64, _i64, _i64, _i64]
        lib.ihref_entry.restype = ctypes.c_uint32
        lib.ihref_region_histogram.argtypes = [_u32p, _i64, _i64, _i64, _i32p, _i64, _u32p]
        lib.ihref_region_histogram.restype = ctypes.c_int64
        lib.ihref_rect_count.argtypes = [_u8p, _i64, _i64, _i64, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_int32, _u32p]
        lib.ihref_rect_count.restype = ctypes.c_int
        self.lib = lib

    # -- helpers -------------------------------------------------------
    @staticmethod
    def _frame(I):
        I = np.ascontiguousarray(I, dtype=np.uint8)
        if I.ndim != 2:
            raise ValueError("frame must be 2-D (H, W)")
        return I, I.ctypes.data_as(_u8p)

    # -- Sec. 2.1 binning function ------------------------------------
    def Q(self, v: int, B: int) -> int:
        return int(self.lib.ihref_Q(int(v), int(B)))

    # -- Eq. 1 via Algorithm 1 ----------------------------------------
    def integral_histogram(self, I, B: int) -> np.ndarray:
        I, p = self._frame(I)
        H, W = I.shape
        out = np.empty((H, W, B), dtype=np.uint32)
        rc = self.lib.ihref_integral_histogram(p, H, W, B, out.ctypes.data_as(_u32p))
        if rc != 0:
            raise ValueError("bad arguments")
        return out

    def integral_histogram_binmajor(self, I, B: int) -> np.ndarray:
        """Eq. 1 per bin plane, stored bin-major: shape (B, H, W)."""
        I, p = self._frame(I)
        H, W = I.shape
        out = np.empty((B, H, W), dtype=np.uint32)
        rc = self.lib.ihref_integral_histogram_binmajor(p, H, W, B, out.ctypes.data_as(_u32p))
        if rc != 0:
            raise ValueError("bad arguments")
        return out

    def integral_histogram_lut(self, I, B: int, lut) -> np.ndarray:
        """Eq. 1 with bin membership from a 256-entry table (bin of value v = lut[v])."""
        I, p = self._frame(I)
        H, W = I.shape
        lut = np.ascontiguousarray(lut, dtype=np.uint8)
        if lut.shape != (256,):
            raise ValueError("lut must hold 256 entries")
        out = np.zeros((H, W, B), dtype=np.uint32)
        rc = self.lib.ihref_integral_histogram_lut(p, H, W, B, lut.ctypes.data_as(_u8p), out.ctypes.data_as(_u32p))
        if rc != 0:
            raise ValueError("bad arguments")
        return out

    def integral_rows(self, I, B: int, y_begin: int, y_end: int, prev_row=None) -> np.ndarray:
        I, p = self._frame(I)
        H, W = I.shape
        out = np.empty((y_end - y_begin, W, B), dtype=np.uint32)
        if prev_row is not None:
            prev_row = np.ascontiguousarray(prev_row, dtype=np.uint32).reshape(W, B)
            pp = prev_row.ctypes.data_as(_u32p)
        else:
            pp = None
        rc = self.lib.ihref_integral_rows(p, H, W, B, y_begin, y_end, pp, out.ctypes.data_as(_u32p))
        if rc != 0:
            raise ValueError("bad arguments")
        return out

    def iter_row_blocks(self, I, B: int, rows_per_block: int):
        """Yield (y_begin, block) over the whole frame, carrying the last row."""
        H = I.shape[0]
        prev = None
        for y0 in range(0, H, rows_per_block):
            y1 = min(H, y0 + rows_per_block)
            blk = self.integral_rows(I, B, y0, y1, prev)
            prev = blk[-1]
            yield y0, blk

    def row_by_definition(self, I, B: int, y: int) -> np.ndarray:
        I, p = self._frame(I)
        H, W = I.shape
        out = np.empty((W, B), dtype=np.uint32)
        rc = self.lib.ihref_row_by_definition(p, H, W, B, y, out.ctypes.data_as(_u32p))
        if rc != 0:
            raise ValueError("bad arguments")
        return out

    def entry(self, I, B: int, x: int, y: int, b: int) -> int:
        I, p = self._frame(I)
        return int(self.lib.ihref_entry(p, I.shape[1], B, x, y, b))

    # -- Eq. 2 ----------------------------------------------------------
    def region_histogram(self, IH: np.ndarray, rects) -> np.ndarray:
        IH = np.ascontiguousarray(IH, dtype=np.uint32)
        H, W, B = IH.shape
        rects = np.ascontiguousarray(rects, dtype=np.int32).reshape(-1, 4)
        out = np.zeros((rects.shape[0], B), dtype=np.uint32)
        bad = self.lib.ihref_region_histogram(IH.ctypes.data_as(_u32p), H, W, B,
                                              rects.ctypes.data_as(_i32p), rects.shape[0],
                                              out.ctypes.data_as(_u32p))
        if bad:
            raise ValueError(f"rectangle {bad - 1} is outside the frame")
        return out

    def rect_count(self, I, B: int, rect) -> np.ndarray:
        I, p = self._frame(I)
        H, W = I.shape
        out = np.zeros(B, dtype=np.uint32)
        x0, y0, x1, y1 = (int(v) for v in rect)
        if self.lib.ihref_rect_count(p, H, W, B, x0, y0, x1, y1, out.ctypes.data_as(_u32p)) != 0:
            raise ValueError("rectangle outside the frame")
        return out


_default = None


def get() -> Oracle:
    """The default (mistake-free) oracle, compiled on first use and again
    whenever its source is newer than the built library."""
    global _default
    if _default is None:
        if not LIB.exists() or LIB.stat().st_mtime < SRC.stat().st_mtime:
            compile_oracle(LIB)
        _default = Oracle(LIB)
    return _default
