"""Thin Python binding of libpat (C ABI in include/pat.h).

Argument marshalling only: every step of the path runs in the HIP library.
Tensors must be CUDA (HIP) tensors on the context's device, contiguous, of the
documented dtype; the current torch stream is passed to the library unless a
stream is given.  Importing this module does not need a GPU, but creating a
context does, and a missing libpat.so raises immediately.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpat.so")

NOALLOC_SCRATCH_BYTES = 16 << 20  # PAT_NOALLOC_SCRATCH_BYTES
PAT_OK, PAT_EINVAL, PAT_ENOMEM, PAT_EDEVICE, PAT_EBUSY, PAT_ENOTFOUND, PAT_ETIMEOUT, PAT_ENOCONV = 0, -1, -2, -3, -4, -5, -6, -7
TABLE_F32, TABLE_Q16, TABLE_R16, TABLE_F32X4 = 0, 1, 2, 3
SIG_F32, SIG_F16 = 0, 1

EXPORTED = [
    "pat_last_error", "pat_version", "pat_ctx_create", "pat_ctx_destroy", "pat_ctx_reserve",
    "pat_backproject_scratch_bytes", "pat_eikonal_tables", "pat_eikonal_tables_o2", "pat_eikonal_tables_3d",
    "pat_eikonal_last_stats", "pat_eikonal_update_eval", "pat_table_to_fixed", "pat_table_to_q16", "pat_table_to_r16", "pat_table_r16_bytes",
    "pat_table_to_x4", "pat_table_x4_bytes",
    "pat_tile_order", "pat_tile_order_3d", "pat_filter", "pat_backproject", "pat_backproject_noalloc",
    "pat_backproject_const",
    "pat_backproject_const_3d",
    "pat_server_create", "pat_server_create_ex", "pat_server_destroy", "pat_server_add_map", "pat_server_add_map_3d",
    "pat_server_map_state", "pat_server_remove_map", "pat_server_submit", "pat_server_wait", "pat_server_stats",
    "pat_server_reset_stats", "pat_server_hold",
]
MAP_BUILDING, MAP_READY, MAP_FAILED, MAP_EVICTED = 0, 1, 2, 3


class PatError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libpat error {code}: {msg}")
        self.code = code


class ServerConfig(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("table_fmt", C.c_int), ("max_batch", C.c_int),
                ("max_inflight", C.c_int), ("max_slots", C.c_int)]


class ServerStats(C.Structure):
    _fields_ = [("frames_submitted", C.c_int64), ("frames_done", C.c_int64), ("frames_refused", C.c_int64),
                ("batches", C.c_int64), ("builds", C.c_int64), ("evictions", C.c_int64),
                ("mean_batch_frames", C.c_double), ("frames_per_s", C.c_double), ("gathers_per_s", C.c_double),
                ("latency_p50_us", C.c_double), ("latency_p99_us", C.c_double), ("latency_max_us", C.c_double),
                ("bytes_budget", C.c_uint64), ("bytes_used", C.c_uint64), ("bytes_tables", C.c_uint64),
                ("maps_ready", C.c_int), ("maps_building", C.c_int), ("queue_depth", C.c_int),
                ("inflight_batches", C.c_int)]


class EikonalStats(C.Structure):
    _fields_ = [("rounds", C.c_int64), ("tile_visits", C.c_int64), ("guard_hits", C.c_int64),
                ("sweeps", C.c_int64), ("lsb_seconds", C.c_double), ("seconds", C.c_double)]


_lib = None


def lib() -> C.CDLL:
    """Load libpat.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1501_03869_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dbl, sz = C.c_void_p, C.c_int, C.c_int64, C.c_double, C.c_size_t
        L.pat_last_error.restype = C.c_char_p
        L.pat_last_error.argtypes = []
        L.pat_version.restype = i32
        L.pat_ctx_create.argtypes = [i32, C.POINTER(vp)]
        L.pat_ctx_destroy.argtypes = [vp]
        L.pat_ctx_reserve.argtypes = [vp, i32, i32, i32]
        L.pat_backproject_scratch_bytes.argtypes = [i32, i32, i32]
        L.pat_backproject_scratch_bytes.restype = sz
        L.pat_eikonal_tables.argtypes = [vp, vp, i32, i32, dbl, vp, i32, vp, i32, vp, vp]
        L.pat_eikonal_tables_o2.argtypes = [vp, vp, i32, i32, dbl, vp, i32, vp, i32, vp, vp]
        L.pat_eikonal_tables_3d.argtypes = [vp, vp, i32, i32, i32, dbl, vp, i32, vp, i32, vp, vp]
        L.pat_eikonal_last_stats.argtypes = [vp, C.POINTER(EikonalStats)]
        L.pat_eikonal_update_eval.argtypes = [vp, vp, i32, i32, vp, vp]
        L.pat_table_to_fixed.argtypes = [vp, vp, i32, i32, dbl, dbl, i32, vp, vp]
        L.pat_table_to_q16.argtypes = [vp, vp, i64, dbl, dbl, i32, vp, vp]
        L.pat_table_to_r16.argtypes = [vp, vp, i32, i32, dbl, dbl, i32, vp, vp]
        L.pat_table_r16_bytes.argtypes = [i32, i32]
        L.pat_table_r16_bytes.restype = sz
        L.pat_table_to_x4.argtypes = [vp, vp, i32, i32, vp, vp]
        L.pat_table_x4_bytes.argtypes = [i32, i32]
        L.pat_table_x4_bytes.restype = sz
        L.pat_tile_order.argtypes = [i32, i32, vp, i32, i32, i32, vp]
        L.pat_tile_order_3d.argtypes = [i32, i32, i32, vp, i32, i32, i32, i32, vp]
        L.pat_filter.argtypes = [vp, vp, i32, i32, dbl, dbl, vp, vp]
        L.pat_backproject.argtypes = [vp, vp, i32, vp, i32, i32, vp, vp, i32, i32, i32, dbl, dbl, i32, vp, vp]
        L.pat_backproject_noalloc.argtypes = L.pat_backproject.argtypes
        L.pat_backproject_const.argtypes = [vp, i32, i32, dbl, dbl, vp, i32, vp, i32, vp, i32, i32, vp, vp, i32, i32,
                                            dbl, dbl, vp, vp]
        L.pat_backproject_const_3d.argtypes = [vp, i32, i32, i32, dbl, dbl, vp, i32, vp, i32, vp, i32, i32, vp, vp,
                                               i32, i32, dbl, dbl, vp, vp]
        L.pat_server_create.argtypes = [vp, sz, C.POINTER(vp)]
        L.pat_server_create_ex.argtypes = [vp, C.POINTER(ServerConfig), C.POINTER(vp)]
        L.pat_server_destroy.argtypes = [vp]
        L.pat_server_add_map.argtypes = [vp, vp, i32, i32, dbl, vp, i32, vp, i32, dbl, dbl, i32, C.POINTER(i32)]
        L.pat_server_add_map_3d.argtypes = [vp, vp, i32, i32, i32, dbl, vp, i32, vp, i32, dbl, dbl, i32, C.POINTER(i32)]
        L.pat_server_map_state.argtypes = [vp, i32, C.POINTER(i32)]
        L.pat_server_remove_map.argtypes = [vp, i32]
        L.pat_server_submit.argtypes = [vp, i32, vp, i32, C.c_float, i32, C.POINTER(C.c_uint64)]
        L.pat_server_wait.argtypes = [vp, C.c_uint64, vp, i32]
        L.pat_server_stats.argtypes = [vp, C.POINTER(ServerStats)]
        L.pat_server_reset_stats.argtypes = [vp]
        L.pat_server_hold.argtypes = [vp, i32]
        _lib = L
    return _lib


def check(rc: int) -> None:
    if rc != PAT_OK:
        raise PatError(rc, lib().pat_last_error().decode(errors="replace"))


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(stream):
    import torch
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _need(t, dtype, name):
    import torch
    if t is None:
        return
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Context:
    """Owns a pat_ctx on one HIP device."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        check(lib().pat_ctx_create(int(device), C.byref(h)))
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            lib().pat_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reserve(self, S: int, P: int, F: int = 1):
        """Pre-allocate gather scratch for calls of these sizes (graph capture)."""
        check(lib().pat_ctx_reserve(self.h, int(S), int(P), int(F)))

    # ------------------------------------------------------------------ tables
    def eikonal_tables(self, speed, h: float, sensors: np.ndarray, pix, table=None, stream=None):
        """speed: float32 [ny][nx] device; sensors: host float64 [S][2]; pix: int32 [P] device."""
        import torch
        _need(speed, torch.float32, "speed")
        _need(pix, torch.int32, "pix")
        ny, nx = speed.shape
        sxy = np.ascontiguousarray(sensors, dtype=np.float64)
        if sxy.ndim != 2 or sxy.shape[1] != 2:
            raise ValueError("sensors must be [S][2]")
        S, P = sxy.shape[0], pix.shape[0]
        if table is None:
            table = torch.empty((S, P), dtype=torch.float32, device=speed.device)
        _need(table, torch.float32, "table")
        check(lib().pat_eikonal_tables(self.h, _ptr(speed), nx, ny, float(h), sxy.ctypes.data, S, _ptr(pix), P,
                                       _ptr(table), _stream(stream)))
        return table

    def eikonal_tables_o2(self, speed, h: float, sensors: np.ndarray, pix, table=None, stream=None):
        """Second-order fast-marching tables (the paper's scheme); arguments as eikonal_tables."""
        import torch
        _need(speed, torch.float32, "speed")
        _need(pix, torch.int32, "pix")
        ny, nx = speed.shape
        sxy = np.ascontiguousarray(sensors, dtype=np.float64)
        if sxy.ndim != 2 or sxy.shape[1] != 2:
            raise ValueError("sensors must be [S][2]")
        S, P = sxy.shape[0], pix.shape[0]
        if table is None:
            table = torch.empty((S, P), dtype=torch.float32, device=speed.device)
        _need(table, torch.float32, "table")
        check(lib().pat_eikonal_tables_o2(self.h, _ptr(speed), nx, ny, float(h), sxy.ctypes.data, S, _ptr(pix), P,
                                          _ptr(table), _stream(stream)))
        return table

    def eikonal_tables_3d(self, speed, h: float, sensors: np.ndarray, vox, table=None, stream=None):
        """speed: float32 [nz][ny][nx] device; sensors: host float64 [S][3]; vox: int32 [P] device."""
        import torch
        _need(speed, torch.float32, "speed")
        _need(vox, torch.int32, "vox")
        nz, ny, nx = speed.shape
        sxyz = np.ascontiguousarray(sensors, dtype=np.float64)
        if sxyz.ndim != 2 or sxyz.shape[1] != 3:
            raise ValueError("sensors must be [S][3]")
        S, P = sxyz.shape[0], vox.shape[0]
        if table is None:
            table = torch.empty((S, P), dtype=torch.float32, device=speed.device)
        _need(table, torch.float32, "table")
        check(lib().pat_eikonal_tables_3d(self.h, _ptr(speed), nx, ny, nz, float(h), sxyz.ctypes.data, S, _ptr(vox),
                                          P, _ptr(table), _stream(stream)))
        return table

    def eikonal_stats(self) -> dict:
        st = EikonalStats()
        check(lib().pat_eikonal_last_stats(self.h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in EikonalStats._fields_}

    def table_to_q16(self, table, dt: float, N: int, t0: float = 0.0, out=None, stream=None):
        """16.16 sample-index table (pat_table_to_fixed) of a float32 [S][P] table, as int32 bits."""
        import torch
        _need(table, torch.float32, "table")
        if out is None:
            out = torch.empty(table.shape, dtype=torch.int32, device=table.device)
        _need(out, torch.int32, "out")
        if table.dim() == 2:
            S, P = table.shape
            check(lib().pat_table_to_fixed(self.h, _ptr(table), S, P, float(t0), float(dt), int(N), _ptr(out),
                                           _stream(stream)))
        else:
            check(lib().pat_table_to_q16(self.h, _ptr(table), table.numel(), float(t0), float(dt), int(N),
                                         _ptr(out), _stream(stream)))
        return out

    def table_to_r16(self, table, dt: float, N: int, t0: float = 0.0, stream=None) -> "R16Table":
        """Tile-relative 16-bit form of a float32 [S][P] table (see pat_table_to_r16)."""
        import torch
        _need(table, torch.float32, "table")
        S, P = table.shape
        buf = torch.empty(int(lib().pat_table_r16_bytes(S, P)), dtype=torch.uint8, device=table.device)
        check(lib().pat_table_to_r16(self.h, _ptr(table), S, P, float(t0), float(dt), int(N), _ptr(buf),
                                     _stream(stream)))
        return R16Table(buf, S, P)

    def table_to_x4(self, table, stream=None) -> "X4Table":
        """Four sensors interleaved per ROI position (see pat_table_to_x4)."""
        import torch
        _need(table, torch.float32, "table")
        S, P = table.shape
        buf = torch.empty(((S + 3) // 4, P, 4), dtype=torch.float32, device=table.device)
        check(lib().pat_table_to_x4(self.h, _ptr(table), S, P, _ptr(buf), _stream(stream)))
        return X4Table(buf, S, P)

    # ------------------------------------------------------------------ frames
    def filter(self, p, dt: float, t0: float = 0.0, out=None, stream=None):
        import torch
        _need(p, torch.float32, "p")
        N = p.shape[-1]
        rows = p.numel() // N if N else 0
        if out is None:
            out = torch.empty_like(p)
        _need(out, torch.float32, "out")
        check(lib().pat_filter(self.h, _ptr(p), rows, N, float(t0), float(dt), _ptr(out), _stream(stream)))
        return out

    def backproject(self, table, sig, dt: float, t0: float = 0.0, *, filtered: bool = True, w=None,
                    frame_scale=None, out=None, stream=None, noalloc: bool = False):
        """table: [S][P] float32 seconds or int32 (16.16 bits), or an R16Table / X4Table from
        table_to_r16 / table_to_x4; sig: [S][N] or [F][S][N] float32/float16.
        noalloc: call pat_backproject_noalloc (gather scratch from the device's fixed array); `out` must then
        be given, so that the call allocates nothing."""
        import torch
        if noalloc and out is None:
            raise ValueError("noalloc needs a preallocated out")
        S, P = table.shape
        if isinstance(table, R16Table):
            tfmt = TABLE_R16
            _need(table.buf, torch.uint8, "table")
        elif isinstance(table, X4Table):
            tfmt = TABLE_F32X4
            _need(table.buf, torch.float32, "table")
        else:
            tfmt = TABLE_Q16 if table.dtype == torch.int32 else TABLE_F32
            _need(table, torch.int32 if tfmt == TABLE_Q16 else torch.float32, "table")
        single = sig.dim() == 2
        F = 1 if single else sig.shape[0]
        N = sig.shape[-1]
        if sig.shape[-2] != S:
            raise ValueError("signal and table sensor counts differ")
        sfmt = SIG_F16 if sig.dtype == torch.float16 else SIG_F32
        _need(sig, torch.float16 if sfmt == SIG_F16 else torch.float32, "sig")
        _need(w, torch.float32, "w")
        _need(frame_scale, torch.float32, "frame_scale")
        if out is None:
            out = torch.empty((P,) if single else (F, P), dtype=torch.float32, device=table.device)
        _need(out, torch.float32, "out")
        fn = lib().pat_backproject_noalloc if noalloc else lib().pat_backproject
        check(fn(self.h, _ptr(table), tfmt, _ptr(sig), sfmt, 1 if filtered else 0, _ptr(frame_scale), _ptr(w), S, P,
                 N, float(t0), float(dt), F, _ptr(out), _stream(stream)))
        return out

    def backproject_const_3d(self, nx: int, ny: int, nz: int, h: float, c: float, sensors: np.ndarray, vox, sig,
                             dt: float, t0: float = 0.0, *, filtered: bool = True, w=None, frame_scale=None, out=None,
                             stream=None):
        """Conventional back projection on a 3-D grid (straight-ray delays |x - s| / c)."""
        import torch
        _need(vox, torch.int32, "vox")
        sxyz = np.ascontiguousarray(sensors, dtype=np.float64)
        if sxyz.ndim != 2 or sxyz.shape[1] != 3:
            raise ValueError("sensors must be [S][3]")
        S, P = sxyz.shape[0], vox.shape[0]
        single = sig.dim() == 2
        F = 1 if single else sig.shape[0]
        N = sig.shape[-1]
        if sig.shape[-2] != S:
            raise ValueError("signal and sensor counts differ")
        sfmt = SIG_F16 if sig.dtype == torch.float16 else SIG_F32
        _need(sig, torch.float16 if sfmt == SIG_F16 else torch.float32, "sig")
        _need(w, torch.float32, "w")
        _need(frame_scale, torch.float32, "frame_scale")
        if out is None:
            out = torch.empty((P,) if single else (F, P), dtype=torch.float32, device=sig.device)
        _need(out, torch.float32, "out")
        check(lib().pat_backproject_const_3d(self.h, int(nx), int(ny), int(nz), float(h), float(c), sxyz.ctypes.data,
                                             S, _ptr(vox), P, _ptr(sig), sfmt, 1 if filtered else 0,
                                             _ptr(frame_scale), _ptr(w), N, F, float(t0), float(dt), _ptr(out),
                                             _stream(stream)))
        return out

    def backproject_const(self, nx: int, ny: int, h: float, c: float, sensors: np.ndarray, pix, sig, dt: float,
                          t0: float = 0.0, *, filtered: bool = True, w=None, frame_scale=None, out=None, stream=None):
        """Conventional back projection with straight-ray delays |x - s| / c."""
        import torch
        _need(pix, torch.int32, "pix")
        sxy = np.ascontiguousarray(sensors, dtype=np.float64)
        S, P = sxy.shape[0], pix.shape[0]
        single = sig.dim() == 2
        F = 1 if single else sig.shape[0]
        N = sig.shape[-1]
        if sig.shape[-2] != S:
            raise ValueError("signal and sensor counts differ")
        sfmt = SIG_F16 if sig.dtype == torch.float16 else SIG_F32
        _need(sig, torch.float16 if sfmt == SIG_F16 else torch.float32, "sig")
        _need(w, torch.float32, "w")
        _need(frame_scale, torch.float32, "frame_scale")
        if out is None:
            out = torch.empty((P,) if single else (F, P), dtype=torch.float32, device=sig.device)
        _need(out, torch.float32, "out")
        check(lib().pat_backproject_const(self.h, int(nx), int(ny), float(h), float(c), sxy.ctypes.data, S,
                                          _ptr(pix), P, _ptr(sig), sfmt, 1 if filtered else 0, _ptr(frame_scale),
                                          _ptr(w), N, F, float(t0), float(dt), _ptr(out), _stream(stream)))
        return out


class X4Table:
    """A PAT_TABLE_F32X4 table: the float32 [ceil(S/4)][P][4] device buffer and
    the S x P shape of the table it interleaves."""

    def __init__(self, buf, S: int, P: int):
        self.buf, self.shape = buf, (int(S), int(P))

    @property
    def device(self):
        return self.buf.device

    def data_ptr(self) -> int:
        return self.buf.data_ptr()

    def is_contiguous(self) -> bool:
        return True

    def table(self):
        """The [S][P] view of the same delays (a copy)."""
        S, P = self.shape
        return self.buf.permute(0, 2, 1).reshape(-1, P)[:S].contiguous()


class R16Table:
    """A PAT_TABLE_R16 table: the device buffer and its S x P shape.  offsets()
    and headers() view the two arrays the buffer holds."""

    def __init__(self, buf, S: int, P: int):
        self.buf, self.shape = buf, (int(S), int(P))

    @property
    def device(self):
        return self.buf.device

    def data_ptr(self) -> int:
        return self.buf.data_ptr()

    def is_contiguous(self) -> bool:
        return True

    def offsets(self):
        S, P = self.shape
        return self.buf[: 2 * S * P].view(_torch().int16).view(S, P)

    def headers(self):
        S, P = self.shape
        off = (2 * S * P + 255) // 256 * 256
        return self.buf[off: off + 4 * S * ((P + 31) // 32)].view(_torch().int32).view(S, (P + 31) // 32)


def _torch():
    import torch
    return torch


def tile_order(nx: int, ny: int, pix: np.ndarray, tile_w: int = 16, tile_h: int = 16) -> np.ndarray:
    """Host helper: ROI node indices in tile-major order."""
    src = np.ascontiguousarray(pix, dtype=np.int32)
    out = np.empty_like(src)
    check(lib().pat_tile_order(nx, ny, src.ctypes.data, src.shape[0], tile_w, tile_h, out.ctypes.data))
    return out


def tile_order_3d(nx: int, ny: int, nz: int, vox: np.ndarray, tile_w: int = 4, tile_h: int = 4,
                  tile_d: int = 2) -> np.ndarray:
    """Host helper: ROI voxel indices in tile-major order (3-D)."""
    src = np.ascontiguousarray(vox, dtype=np.int32)
    out = np.empty_like(src)
    check(lib().pat_tile_order_3d(nx, ny, nz, src.ctypes.data, src.shape[0], tile_w, tile_h, tile_d,
                                  out.ctypes.data))
    return out


def eikonal_update_eval(nbr, F, dims: int, stream=None):
    """The tables' local update alone (pat_eikonal_update_eval): nbr int32
    [n][3] device tensor of neighbour minima as uint32 bits, F int32 [n]
    slowness units; returns int32 [n] (uint32 bits) on the same device."""
    torch = _torch()
    _need(nbr, torch.int32, "nbr")
    _need(F, torch.int32, "F")
    if nbr.dim() != 2 or nbr.shape[1] != 3 or F.shape != (nbr.shape[0],):
        raise ValueError("nbr must be [n][3] and F [n]")
    out = torch.empty(F.shape, dtype=torch.int32, device=F.device)
    check(lib().pat_eikonal_update_eval(_ptr(nbr), _ptr(F), int(F.shape[0]), dims, _ptr(out), _stream(stream)))
    return out


def backproject_scratch_bytes(S: int, P: int, F: int = 1) -> int:
    return int(lib().pat_backproject_scratch_bytes(S, P, F))


class Server:
    """Frame server (resident tables, continuous mixed-geometry batching)."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int = 0, table_fmt: int = TABLE_F32, sig_fmt: int = SIG_F32,
                 max_batch: int = 0, max_inflight: int = 0, max_slots: int = 0, budget_only: bool = False):
        """sig_fmt is the default format of submitted frames (submit may override
        it per frame).  budget_only: create through pat_server_create (HBM budget
        only, float32 tables, defaults for the rest)."""
        h = C.c_void_p()
        if budget_only:
            check(lib().pat_server_create(ctx.h, C.c_size_t(int(hbm_budget_bytes)), C.byref(h)))
        else:
            cfg = ServerConfig(int(hbm_budget_bytes), int(table_fmt), int(max_batch), int(max_inflight),
                               int(max_slots))
            check(lib().pat_server_create_ex(ctx.h, C.byref(cfg), C.byref(h)))
        self.h = h
        self.sig_fmt = sig_fmt
        self._geo = {}

    def close(self):
        if getattr(self, "h", None):
            check(lib().pat_server_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_map(self, speed: np.ndarray, h: float, sensors: np.ndarray, pix: np.ndarray, n_samples: int, dt: float,
                t0: float = 0.0) -> int:
        c = np.ascontiguousarray(speed, dtype=np.float32)
        ny, nx = c.shape
        sxy = np.ascontiguousarray(sensors, dtype=np.float64)
        px = np.ascontiguousarray(pix, dtype=np.int32)
        mid = C.c_int()
        check(lib().pat_server_add_map(self.h, c.ctypes.data, nx, ny, float(h), sxy.ctypes.data, sxy.shape[0],
                                       px.ctypes.data, px.shape[0], float(t0), float(dt), int(n_samples),
                                       C.byref(mid)))
        self._geo[mid.value] = (sxy.shape[0], px.shape[0], int(n_samples))
        return mid.value

    def add_map_3d(self, speed: np.ndarray, h: float, sensors: np.ndarray, vox: np.ndarray, n_samples: int,
                   dt: float, t0: float = 0.0) -> int:
        c = np.ascontiguousarray(speed, dtype=np.float32)
        nz, ny, nx = c.shape
        sxyz = np.ascontiguousarray(sensors, dtype=np.float64)
        if sxyz.ndim != 2 or sxyz.shape[1] != 3:
            raise ValueError("sensors must be [S][3]")
        px = np.ascontiguousarray(vox, dtype=np.int32)
        mid = C.c_int()
        check(lib().pat_server_add_map_3d(self.h, c.ctypes.data, nx, ny, nz, float(h), sxyz.ctypes.data, sxyz.shape[0],
                                          px.ctypes.data, px.shape[0], float(t0), float(dt), int(n_samples),
                                          C.byref(mid)))
        self._geo[mid.value] = (sxyz.shape[0], px.shape[0], int(n_samples))
        return mid.value

    def map_state(self, map_id: int) -> int:
        st = C.c_int()
        check(lib().pat_server_map_state(self.h, int(map_id), C.byref(st)))
        return st.value

    def remove_map(self, map_id: int):
        check(lib().pat_server_remove_map(self.h, int(map_id)))

    def submit(self, map_id: int, frame: np.ndarray, scale: float = 1.0, nonblocking: bool = False,
               sig_fmt: int | None = None) -> int:
        fmt = self.sig_fmt if sig_fmt is None else int(sig_fmt)
        want = np.float16 if fmt == SIG_F16 else np.float32
        f = np.ascontiguousarray(frame, dtype=want)
        if map_id in self._geo:  # unknown ids are reported by the library
            S, P, N = self._geo[map_id]
            if f.shape != (S, N):
                raise ValueError(f"frame must be {(S, N)}, got {f.shape}")
        t = C.c_uint64()
        check(lib().pat_server_submit(self.h, int(map_id), f.ctypes.data, fmt, C.c_float(scale),
                                      1 if nonblocking else 0, C.byref(t)))
        return t.value

    def wait(self, ticket: int, map_id: int | None = None, P: int | None = None, timeout_ms: int = -1):
        if P is None:
            P = self._geo[map_id][1]
        out = np.empty(P, dtype=np.float32)
        check(lib().pat_server_wait(self.h, C.c_uint64(ticket), out.ctypes.data, int(timeout_ms)))
        return out

    def stats(self) -> dict:
        st = ServerStats()
        check(lib().pat_server_stats(self.h, C.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def reset_stats(self):
        check(lib().pat_server_reset_stats(self.h))

    def hold(self, on: bool = True):
        """Queue submitted frames without launching them until hold(False)."""
        check(lib().pat_server_hold(self.h, 1 if on else 0))
