"""ctypes binding of libih.so (C ABI in include/ih.h).

Argument marshalling only: tensors supply device pointers, torch streams
supply hipStream_t handles, and every computation runs in the library's HIP
kernels.  Importing this module raises ImportError when libih.so has not been
built; there is no fallback of any kind.
"""
from __future__ import annotations

import ctypes
import os
from pathlib import Path

import numpy as np
import torch

# IH_LIBRARY may name another build of the same library (for A/B timing).
LIB_PATH = Path(os.environ.get("IH_LIBRARY", Path(__file__).resolve().with_name("libih.so")))

IH_OK = 0
STATUS = {
    0: "IH_OK", 1: "IH_ERR_INVALID_ARG", 2: "IH_ERR_RANGE", 3: "IH_ERR_OOM", 4: "IH_ERR_HIP",
    5: "IH_ERR_BUDGET", 6: "IH_NOT_READY", 7: "IH_ERR_UNKNOWN_TICKET", 8: "IH_ERR_SHUTDOWN",
}


class IHError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)}: {detail}")


class Rect(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_int32), ("y0", ctypes.c_int32),
                ("x1", ctypes.c_int32), ("y1", ctypes.c_int32)]


class View(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("B", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class PhaseTimes(ctypes.Structure):
    _fields_ = [("agg_ms", ctypes.c_double), ("scan_ms", ctypes.c_double),
                ("tile_ms", ctypes.c_double), ("frames", ctypes.c_uint64)]


class FrameDesc(ctypes.Structure):
    _fields_ = [("frame", ctypes.c_void_p), ("out", ctypes.c_void_p), ("H", ctypes.c_int32),
                ("W", ctypes.c_int32), ("B", ctypes.c_int32), ("lut", ctypes.c_void_p), ("binmajor", ctypes.c_int32)]


class BatchOptions(ctypes.Structure):
    _fields_ = [("autotune", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("tile_x", ctypes.c_int32),
                ("tile_y", ctypes.c_int32), ("nontemporal", ctypes.c_int32), ("group_bytes", ctypes.c_int64),
                ("carry_bands", ctypes.c_int32), ("tile_branches", ctypes.c_int32)]


class FrameSchedule(ctypes.Structure):
    _fields_ = [("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32), ("nontemporal", ctypes.c_int32),
                ("carry_bands", ctypes.c_int32), ("group", ctypes.c_int32)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("frames", ctypes.c_int64), ("entries", ctypes.c_int64), ("kernel_launches", ctypes.c_int32),
                ("tile_launches", ctypes.c_int32), ("graph", ctypes.c_int32), ("groups", ctypes.c_int32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_slots", ctypes.c_int32),
                ("n_hip_streams", ctypes.c_int32), ("max_batch", ctypes.c_int32), ("retain", ctypes.c_int32),
                ("pinned_bytes", ctypes.c_uint64)]


class Timing(ctypes.Structure):
    _fields_ = [("t_submit_ns", ctypes.c_uint64), ("t_admit_ns", ctypes.c_uint64), ("t_done_ns", ctypes.c_uint64)]


class ServerCounters(ctypes.Structure):
    _fields_ = [("pending", ctypes.c_int64), ("admitted", ctypes.c_int64), ("retained", ctypes.c_int64),
                ("device_bytes_used", ctypes.c_uint64), ("device_bytes_peak", ctypes.c_uint64),
                ("budget_blocked", ctypes.c_uint64)]


class PipelineStats(ctypes.Structure):
    _fields_ = [("wall_ms", ctypes.c_double), ("frames_per_s", ctypes.c_double), ("h2d_ms", ctypes.c_double),
                ("kernel_ms", ctypes.c_double), ("d2h_ms", ctypes.c_double)]


def _load() -> ctypes.CDLL:
    if not LIB_PATH.exists():
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1711_01919_amd.build`")
    lib = ctypes.CDLL(str(LIB_PATH))
    vp, i32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t
    lib.ih_compute.argtypes = [vp, i32, i32, i32, vp, vp]
    lib.ih_compute_binmajor.argtypes = [vp, i32, i32, i32, vp, vp]
    lib.ih_write_reference.argtypes = [vp, i32, i32, i32, i32, i32, vp]
    lib.ih_write_reference.restype = ctypes.c_int
    lib.ih_compute_binmajor.restype = ctypes.c_int
    lib.ih_compute_lut.argtypes = [vp, i32, i32, i32, vp, vp, vp]
    lib.ih_compute_lut.restype = ctypes.c_int
    lib.ih_compute_noalloc.argtypes = [vp, i32, i32, i32, vp, vp]
    lib.ih_compute_noalloc.restype = ctypes.c_int
    lib.ih_query.argtypes = [ctypes.POINTER(View), vp, sz, vp]
    lib.ih_query_device.argtypes = [ctypes.POINTER(View), vp, sz, vp, vp]
    lib.ih_query_binmajor.argtypes = [ctypes.POINTER(View), vp, sz, vp]
    lib.ih_query_binmajor_device.argtypes = [ctypes.POINTER(View), vp, sz, vp, vp]
    for f in (lib.ih_compute, lib.ih_query, lib.ih_query_device, lib.ih_query_binmajor,
              lib.ih_query_binmajor_device):
        f.restype = ctypes.c_int
    lib.ih_profile_enable.argtypes = [ctypes.c_int]
    lib.ih_profile_enable.restype = ctypes.c_int
    lib.ih_profile_read.argtypes = [ctypes.POINTER(PhaseTimes)]
    lib.ih_profile_read.restype = ctypes.c_int
    lib.ih_batch_plan_create.argtypes = [ctypes.POINTER(FrameDesc), sz, ctypes.POINTER(BatchOptions), vp,
                                         ctypes.POINTER(vp)]
    lib.ih_batch_plan_launch.argtypes = [vp, vp]
    lib.ih_batch_plan_destroy.argtypes = [vp]
    lib.ih_batch_plan_info.argtypes = [vp, ctypes.POINTER(BatchInfo)]
    lib.ih_batch_plan_frame_tile.argtypes = [vp, sz, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                             ctypes.POINTER(i32)]
    lib.ih_batch_plan_frame_schedule.argtypes = [vp, sz, ctypes.POINTER(FrameSchedule)]
    for f in (lib.ih_batch_plan_create, lib.ih_batch_plan_launch, lib.ih_batch_plan_destroy,
              lib.ih_batch_plan_info, lib.ih_batch_plan_frame_tile, lib.ih_batch_plan_frame_schedule):
        f.restype = ctypes.c_int
    lib.ih_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
    lib.ih_submit.argtypes = [vp, i32, vp, i32, i32, i32, vp, sz, ctypes.POINTER(ctypes.c_uint64)]
    lib.ih_submit_lut.argtypes = [vp, i32, vp, i32, i32, i32, vp, vp, sz, ctypes.POINTER(ctypes.c_uint64)]
    lib.ih_poll.argtypes = [vp, ctypes.c_uint64, vp, ctypes.POINTER(Timing)]
    lib.ih_server_query_latest.argtypes = [vp, i32, vp, sz, vp, ctypes.POINTER(ctypes.c_uint64)]
    lib.ih_server_stats.argtypes = [vp, ctypes.POINTER(ServerCounters)]
    lib.ih_server_destroy.argtypes = [vp]
    lib.ih_server_hold.argtypes = [vp, i32]
    for f in (lib.ih_server_create, lib.ih_submit, lib.ih_submit_lut, lib.ih_poll, lib.ih_server_query_latest,
              lib.ih_server_stats, lib.ih_server_destroy, lib.ih_server_hold):
        f.restype = ctypes.c_int
    lib.ih_transfer_pipeline.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), sz, i32, i32, i32, i32,
                                         ctypes.POINTER(PipelineStats)]
    lib.ih_transfer_pipeline.restype = ctypes.c_int
    lib.ih_status_str.argtypes = [ctypes.c_int]
    lib.ih_status_str.restype = ctypes.c_char_p
    lib.ih_last_error.restype = ctypes.c_char_p
    lib.ih_version.restype = ctypes.c_char_p
    return lib


lib = _load()


def _check(st: int, where: str):
    if st != IH_OK:
        raise IHError(st, where, lib.ih_last_error().decode())


def _stream_handle(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else int(t.data_ptr())


def empty_ih(H: int, W: int, B: int, device="cuda") -> torch.Tensor:
    return torch.empty((H, W, B), dtype=torch.uint32, device=device)


def compute(frame: torch.Tensor, B: int, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Integral histogram (H, W, B) uint32 of a (H, W) uint8 device frame."""
    if frame.dtype != torch.uint8 or frame.dim() != 2 or not frame.is_cuda or not frame.is_contiguous():
        raise ValueError("frame must be a contiguous 2-D uint8 CUDA tensor")
    H, W = frame.shape
    if out is None:
        out = empty_ih(H, W, B, frame.device)
    elif out.dtype != torch.uint32 or not out.is_contiguous() or out.numel() < H * W * B:
        raise ValueError("out must be a contiguous uint32 tensor with H*W*B elements")
    _check(lib.ih_compute(_ptr(frame), H, W, B, _ptr(out), _stream_handle(stream)), "ih_compute")
    return out


def compute_noalloc(frame: torch.Tensor, B: int, out: torch.Tensor, stream=None) -> torch.Tensor:
    """ih_compute_noalloc: as compute(), into a caller-given out, with the
    carries in the library's fixed per-GPU array (the call allocates no
    device memory)."""
    if frame.dtype != torch.uint8 or frame.dim() != 2 or not frame.is_cuda or not frame.is_contiguous():
        raise ValueError("frame must be a contiguous 2-D uint8 CUDA tensor")
    H, W = frame.shape
    if out.dtype != torch.uint32 or not out.is_cuda or not out.is_contiguous() or out.numel() < H * W * B:
        raise ValueError("out must be a contiguous uint32 CUDA tensor with H*W*B elements")
    _check(lib.ih_compute_noalloc(_ptr(frame), H, W, int(B), _ptr(out), _stream_handle(stream)),
           "ih_compute_noalloc")
    return out


def compute_binmajor(frame: torch.Tensor, B: int, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """ih_compute_binmajor: the integral histogram in the bin-major layout,
    a (B, H, W) uint32 tensor."""
    if frame.dtype != torch.uint8 or frame.dim() != 2 or not frame.is_cuda or not frame.is_contiguous():
        raise ValueError("frame must be a contiguous 2-D uint8 CUDA tensor")
    H, W = frame.shape
    if out is None:
        out = torch.empty((B, H, W), dtype=torch.uint32, device=frame.device)
    elif out.dtype != torch.uint32 or not out.is_cuda or not out.is_contiguous() or out.numel() < H * W * B:
        raise ValueError("out must be a contiguous uint32 CUDA tensor with B*H*W elements")
    _check(lib.ih_compute_binmajor(_ptr(frame), H, W, int(B), _ptr(out), _stream_handle(stream)),
           "ih_compute_binmajor")
    return out


def compute_lut(frame: torch.Tensor, B: int, lut, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """ih_compute_lut: the integral histogram with bins given by a table
    (pixel value v counts in bin lut[v]; 256 entries below B, in any order)."""
    if frame.dtype != torch.uint8 or frame.dim() != 2 or not frame.is_cuda or not frame.is_contiguous():
        raise ValueError("frame must be a contiguous 2-D uint8 CUDA tensor")
    table = np.ascontiguousarray(lut, dtype=np.uint8)
    if table.shape != (256,):
        raise ValueError("lut must hold 256 entries")
    H, W = frame.shape
    if out is None:
        out = torch.empty((H, W, B), dtype=torch.uint32, device=frame.device)
    elif out.dtype != torch.uint32 or not out.is_cuda or not out.is_contiguous() or out.numel() < H * W * B:
        raise ValueError("out must be a contiguous uint32 CUDA tensor with H*W*B elements")
    _check(lib.ih_compute_lut(_ptr(frame), H, W, int(B), table.ctypes.data, _ptr(out), _stream_handle(stream)),
           "ih_compute_lut")
    return out


def write_reference(out: torch.Tensor, tile, stream=None) -> None:
    """ih_write_reference on an (H, W, B) uint32 device tensor (B <= 64)."""
    if out.dtype != torch.uint32 or out.dim() != 3 or not out.is_cuda or not out.is_contiguous():
        raise ValueError("out must be a contiguous (H, W, B) uint32 CUDA tensor")
    H, W, B = out.shape
    _check(lib.ih_write_reference(_ptr(out), H, W, B, int(tile[0]), int(tile[1]), _stream_handle(stream)),
           "ih_write_reference")


def compute_raw(frame_ptr: int, H: int, W: int, B: int, out_ptr: int, stream=None) -> int:
    """Direct pass-through of ih_compute (status code returned, not raised)."""
    return lib.ih_compute(frame_ptr, H, W, B, out_ptr, _stream_handle(stream))


def _view(ih: torch.Tensor, stream) -> View:
    if ih.dtype != torch.uint32 or ih.dim() != 3 or not ih.is_cuda or not ih.is_contiguous():
        raise ValueError("ih must be a contiguous (H, W, B) uint32 CUDA tensor")
    H, W, B = ih.shape
    return View(_ptr(ih), H, W, B, _stream_handle(stream))


def query(ih: torch.Tensor, rects, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Region histograms (n, B) for host rectangles {x0, y0, x1, y1} (inclusive)."""
    rects = np.ascontiguousarray(rects, dtype=np.int32).reshape(-1, 4)
    v = _view(ih, stream)
    n = rects.shape[0]
    if out is None:
        out = torch.empty((n, ih.shape[2]), dtype=torch.uint32, device=ih.device)
    _check(lib.ih_query(ctypes.byref(v), rects.ctypes.data, n, _ptr(out)), "ih_query")
    return out


def query_device(ih: torch.Tensor, rects_dev: torch.Tensor, out: torch.Tensor | None = None,
                 bad_count: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Region histograms for rectangles already on the device ((n, 4) int32)."""
    if rects_dev.dtype != torch.int32 or not rects_dev.is_cuda or not rects_dev.is_contiguous():
        raise ValueError("rects_dev must be a contiguous int32 CUDA tensor of shape (n, 4)")
    v = _view(ih, stream)
    n = rects_dev.numel() // 4
    if out is None:
        out = torch.empty((n, ih.shape[2]), dtype=torch.uint32, device=ih.device)
    _check(lib.ih_query_device(ctypes.byref(v), _ptr(rects_dev), n, _ptr(out), _ptr(bad_count)),
           "ih_query_device")
    return out


def _view_binmajor(ih: torch.Tensor, stream) -> View:
    if ih.dtype != torch.uint32 or ih.dim() != 3 or not ih.is_cuda or not ih.is_contiguous():
        raise ValueError("ih must be a contiguous (B, H, W) uint32 CUDA tensor")
    B, H, W = ih.shape
    return View(_ptr(ih), H, W, B, _stream_handle(stream))


def query_binmajor(ih: torch.Tensor, rects, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """ih_query_binmajor: region histograms (n, B) from a bin-major (B, H, W)
    integral histogram, for host rectangles {x0, y0, x1, y1} (inclusive)."""
    rects = np.ascontiguousarray(rects, dtype=np.int32).reshape(-1, 4)
    v = _view_binmajor(ih, stream)
    n = rects.shape[0]
    if out is None:
        out = torch.empty((n, ih.shape[0]), dtype=torch.uint32, device=ih.device)
    _check(lib.ih_query_binmajor(ctypes.byref(v), rects.ctypes.data, n, _ptr(out)), "ih_query_binmajor")
    return out


def query_binmajor_device(ih: torch.Tensor, rects_dev: torch.Tensor, out: torch.Tensor | None = None,
                          bad_count: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """ih_query_binmajor_device: as query_binmajor, rectangles on the device."""
    if rects_dev.dtype != torch.int32 or not rects_dev.is_cuda or not rects_dev.is_contiguous():
        raise ValueError("rects_dev must be a contiguous int32 CUDA tensor of shape (n, 4)")
    v = _view_binmajor(ih, stream)
    n = rects_dev.numel() // 4
    if out is None:
        out = torch.empty((n, ih.shape[0]), dtype=torch.uint32, device=ih.device)
    _check(lib.ih_query_binmajor_device(ctypes.byref(v), _ptr(rects_dev), n, _ptr(out), _ptr(bad_count)),
           "ih_query_binmajor_device")
    return out


class BatchPlan:
    """A batched integral-histogram plan over (frame, out) device tensor pairs.

    The tensors must stay alive and in place while the plan exists; the plan
    keeps references to them."""

    def __init__(self, frames, outs, bins, autotune=False, use_graph=True, tile=None,
                 nontemporal=-1, stream=None, group_bytes=0, luts=None, binmajor=None, carry_bands=-1,
                 tile_branches=0):
        """group_bytes > 0 pipelines the plan in groups of about that many
        output bytes (see ih_batch_options in include/ih.h).  luts: None, or
        per frame None (uniform bins) or a 256-entry bin table.  binmajor:
        None, or per frame whether its output takes the (B, H, W) layout.
        carry_bands: -1 as chosen, 0 reduce-then-scan, K >= 1 the fused carry
        schedule with K tile bands per carry band, -2 prefix counts.
        tile_branches: 0 as chosen, 1 tile-pass launches one after another,
        2..4 spread over that many graph branches."""
        if not (len(frames) == len(outs) == len(bins)) or len(frames) == 0:
            raise ValueError("frames, outs and bins must be equally long and non-empty")
        tables = [None] * len(frames) if luts is None else [
            None if t is None else np.ascontiguousarray(t, dtype=np.uint8) for t in luts]
        if len(tables) != len(frames) or any(t is not None and t.shape != (256,) for t in tables):
            raise ValueError("luts must give one 256-entry table (or None) per frame")
        layouts = [False] * len(frames) if binmajor is None else [bool(x) for x in binmajor]
        if len(layouts) != len(frames):
            raise ValueError("binmajor must give one flag per frame")
        descs = (FrameDesc * len(frames))()
        for k, (f, o, b) in enumerate(zip(frames, outs, bins)):
            if f.dtype != torch.uint8 or f.dim() != 2 or not f.is_cuda or not f.is_contiguous():
                raise ValueError(f"frame {k} must be a contiguous 2-D uint8 CUDA tensor")
            H, W = f.shape
            if o.dtype != torch.uint32 or not o.is_cuda or not o.is_contiguous() or o.numel() < H * W * b:
                raise ValueError(f"out {k} must be a contiguous uint32 CUDA tensor with H*W*B elements")
            descs[k] = FrameDesc(_ptr(f), _ptr(o), H, W, int(b),
                                 None if tables[k] is None else tables[k].ctypes.data, 1 if layouts[k] else 0)
        tx, ty = tile if tile else (0, 0)
        opt = BatchOptions(1 if autotune else 0, 1 if use_graph else 0, tx, ty, int(nontemporal),
                           int(group_bytes), int(carry_bands), int(tile_branches))
        h = ctypes.c_void_p()
        _check(lib.ih_batch_plan_create(descs, len(frames), ctypes.byref(opt), _stream_handle(stream),
                                        ctypes.byref(h)), "ih_batch_plan_create")
        self._h = h
        self._keep = (list(frames), list(outs))

    def launch(self, stream=None):
        _check(lib.ih_batch_plan_launch(self._h, _stream_handle(stream)), "ih_batch_plan_launch")

    def info(self) -> dict:
        i = BatchInfo()
        _check(lib.ih_batch_plan_info(self._h, ctypes.byref(i)), "ih_batch_plan_info")
        return {"frames": i.frames, "entries": i.entries, "kernel_launches": i.kernel_launches,
                "tile_launches": i.tile_launches, "graph": bool(i.graph), "groups": i.groups}

    def frame_tile(self, k: int):
        tx, ty, nt = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib.ih_batch_plan_frame_tile(self._h, k, ctypes.byref(tx), ctypes.byref(ty), ctypes.byref(nt)),
               "ih_batch_plan_frame_tile")
        return tx.value, ty.value, bool(nt.value)

    def frame_schedule(self, k: int) -> dict:
        sc = FrameSchedule()
        _check(lib.ih_batch_plan_frame_schedule(self._h, k, ctypes.byref(sc)), "ih_batch_plan_frame_schedule")
        return {"tile": (sc.tile_x, sc.tile_y), "nontemporal": bool(sc.nontemporal),
                "carry_bands": sc.carry_bands, "group": sc.group}

    def close(self):
        if self._h:
            _check(lib.ih_batch_plan_destroy(self._h), "ih_batch_plan_destroy")
            self._h = None
            self._keep = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


IH_NOT_READY = 6


class Server:
    """Serving loop over host frames and rectangles (ih_server_* in ih.h)."""

    def __init__(self, budget_bytes: int, max_slots: int = 64, n_hip_streams: int = 4,
                 max_batch: int = 16, retain: bool = False, pinned_bytes: int = 0):
        cfg = ServerConfig(int(budget_bytes), max_slots, n_hip_streams, max_batch, 1 if retain else 0,
                           int(pinned_bytes))
        h = ctypes.c_void_p()
        _check(lib.ih_server_create(ctypes.byref(cfg), ctypes.byref(h)), "ih_server_create")
        self._h = h
        self._shape = {}

    def submit(self, stream_id: int, frame: np.ndarray, B: int, rects=None, lut=None) -> int:
        """ih_submit, or ih_submit_lut when a 256-entry bin table is given."""
        frame = np.ascontiguousarray(frame, dtype=np.uint8)
        if frame.ndim != 2:
            raise ValueError("frame must be 2-D")
        H, W = frame.shape
        r = np.ascontiguousarray(rects if rects is not None else np.zeros((0, 4)), dtype=np.int32).reshape(-1, 4)
        t = ctypes.c_uint64()
        rp = r.ctypes.data if len(r) else None
        if lut is None:
            _check(lib.ih_submit(self._h, stream_id, frame.ctypes.data, H, W, B, rp, len(r), ctypes.byref(t)),
                   "ih_submit")
        else:
            table = np.ascontiguousarray(lut, dtype=np.uint8)
            if table.shape != (256,):
                raise ValueError("lut must hold 256 entries")
            _check(lib.ih_submit_lut(self._h, stream_id, frame.ctypes.data, H, W, B, table.ctypes.data, rp,
                                     len(r), ctypes.byref(t)), "ih_submit_lut")
        self._shape[t.value] = (len(r), B)
        return t.value

    def poll(self, ticket: int):
        """(hists, timing) when finished, None while not ready; raises on failure."""
        nq, B = self._shape.get(ticket, (0, 1))
        out = np.empty((nq, B), dtype=np.uint32)
        tm = Timing()
        st = lib.ih_poll(self._h, ticket, out.ctypes.data if nq else None, ctypes.byref(tm))
        if st == IH_NOT_READY:
            return None
        self._shape.pop(ticket, None)
        _check(st, "ih_poll")
        return out, {"t_submit_ns": tm.t_submit_ns, "t_admit_ns": tm.t_admit_ns, "t_done_ns": tm.t_done_ns}

    def poll_status(self, ticket: int) -> int:
        """Raw status of ih_poll (collects the ticket when finished)."""
        return lib.ih_poll(self._h, ticket, None, None)

    def wait(self, ticket: int, timeout_s: float = 60.0, sleep_s: float = 1e-4):
        import time
        t_end = time.monotonic() + timeout_s
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            if time.monotonic() > t_end:
                raise TimeoutError(f"ticket {ticket} not finished after {timeout_s} s")
            time.sleep(sleep_s)

    def query_latest(self, stream_id: int, rects, B: int):
        r = np.ascontiguousarray(rects, dtype=np.int32).reshape(-1, 4)
        out = np.empty((len(r), B), dtype=np.uint32)
        t = ctypes.c_uint64()
        _check(lib.ih_server_query_latest(self._h, stream_id, r.ctypes.data, len(r), out.ctypes.data,
                                          ctypes.byref(t)), "ih_server_query_latest")
        return out, t.value

    def stats(self) -> dict:
        c = ServerCounters()
        _check(lib.ih_server_stats(self._h, ctypes.byref(c)), "ih_server_stats")
        return {"pending": c.pending, "admitted": c.admitted, "retained": c.retained,
                "device_bytes_used": c.device_bytes_used, "device_bytes_peak": c.device_bytes_peak,
                "budget_blocked": c.budget_blocked}

    def hold(self, on: bool = True):
        _check(lib.ih_server_hold(self._h, 1 if on else 0), "ih_server_hold")

    def close(self):
        if self._h:
            _check(lib.ih_server_destroy(self._h), "ih_server_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _host_ptr(a) -> int:
    """Address of a C-contiguous host buffer (numpy array or CPU tensor)."""
    if isinstance(a, torch.Tensor):
        if a.is_cuda or not a.is_contiguous():
            raise ValueError("host buffers must be contiguous CPU tensors")
        return a.data_ptr()
    if not (isinstance(a, np.ndarray) and a.flags.c_contiguous):
        raise ValueError("host buffers must be C-contiguous numpy arrays or CPU tensors")
    return a.ctypes.data


def transfer_pipeline(frames, outs, B: int, n_streams: int = 2) -> dict:
    """ih_transfer_pipeline: host frames (H x W uint8 each, one shape) to host
    integral histograms (H x W x B uint32 each), copies and kernels of
    consecutive frames overlapped on n_streams streams.  Returns the timing."""
    if len(frames) == 0 or len(frames) != len(outs):
        raise ValueError("frames and outs must be equally long and non-empty")
    H, W = frames[0].shape
    for f, o in zip(frames, outs):
        if tuple(f.shape) != (H, W) or f.dtype not in (np.uint8, torch.uint8):
            raise ValueError(f"every frame must be a {H}x{W} uint8 array")
        n_el = o.numel() if isinstance(o, torch.Tensor) else o.size
        if o.dtype not in (np.uint32, torch.uint32) or n_el < H * W * B:
            raise ValueError("every output must be a uint32 buffer of H*W*B elements")
    n = len(frames)
    fp = (ctypes.c_void_p * n)(*[_host_ptr(f) for f in frames])
    op = (ctypes.c_void_p * n)(*[_host_ptr(o) for o in outs])
    st = PipelineStats()
    _check(lib.ih_transfer_pipeline(fp, op, n, H, W, int(B), int(n_streams), ctypes.byref(st)),
           "ih_transfer_pipeline")
    return {"wall_ms": st.wall_ms, "frames_per_s": st.frames_per_s, "h2d_ms": st.h2d_ms,
            "kernel_ms": st.kernel_ms, "d2h_ms": st.d2h_ms}


def profile_enable(on: bool = True):
    """Start (clearing totals) or stop per-phase event timing of ih_compute."""
    _check(lib.ih_profile_enable(1 if on else 0), "ih_profile_enable")


def profile_read() -> dict:
    """Summed per-phase event durations (ms) since profile_enable(True)."""
    t = PhaseTimes()
    _check(lib.ih_profile_read(ctypes.byref(t)), "ih_profile_read")
    return {"agg_ms": t.agg_ms, "scan_ms": t.scan_ms, "tile_ms": t.tile_ms, "frames": int(t.frames)}


def version() -> str:
    return lib.ih_version().decode()
