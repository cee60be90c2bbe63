"""ctypes front end of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: the plain, slow definition of fast-marching back
projection that the GPU library is checked against.  Only the tests, the
smoke check and the benchmark's CPU-baseline leg may import this module.  It
shares no code with the GPU library and does not import it.

Every function converts its inputs to float64 (float32 inputs convert exactly)
and returns float64 results, except the 16.16 table, which is uint32.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_fp = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_u8 = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_i32 = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u32 = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_u16 = np.ctypeslib.ndpointer(dtype=np.uint16, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (FP64, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fPIC",
                               "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        L.orc_fmm.argtypes = [C.c_int, C.c_int, C.c_double, _dp, _u8, _dp, C.POINTER(C.c_long)]
        L.orc_fmm.restype = C.c_int
        L.orc_seed.argtypes = [C.c_int, C.c_int, C.c_double, _dp, C.c_double, C.c_double, C.c_double, _u8, _dp]
        L.orc_seed.restype = C.c_int
        L.orc_tables.argtypes = [C.c_int, C.c_int, C.c_double, _fp, _dp, C.c_int, _i32, C.c_long, _dp, C.c_int]
        L.orc_tables.restype = C.c_int
        L.orc_fmm2.argtypes = [C.c_int, C.c_int, C.c_double, _dp, _u8, _dp, C.POINTER(C.c_long), C.c_int,
                               C.c_void_p]
        L.orc_fmm2.restype = C.c_int
        L.orc_tables2.argtypes = [C.c_int, C.c_int, C.c_double, _fp, _dp, C.c_int, _i32, C.c_long, _dp, C.c_int]
        L.orc_tables2.restype = C.c_int
        L.orc_tables_const.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, _dp, C.c_int, _i32, C.c_long, _dp]
        L.orc_tables_const.restype = C.c_int
        L.orc_tables_const3.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, _dp, C.c_int, _i32,
                                        C.c_long, _dp]
        L.orc_tables_const3.restype = C.c_int
        L.orc_filter.argtypes = [_dp, C.c_long, C.c_int, C.c_double, C.c_double, _dp]
        L.orc_filter.restype = None
        L.orc_gather.argtypes = [_dp, _dp, C.c_void_p, C.c_int, C.c_long, C.c_int, C.c_int, C.c_double,
                                 C.c_double, _dp, C.c_int]
        L.orc_gather.restype = None
        L.orc_table_to_q16.argtypes = [_fp, C.c_long, C.c_double, C.c_double, C.c_int, _u32]
        L.orc_table_to_q16.restype = None
        L.orc_gather_q16.argtypes = [_u32, _dp, C.c_void_p, C.c_int, C.c_long, C.c_int, C.c_int, _dp, C.c_int]
        L.orc_gather_q16.restype = None
        L.orc_table_to_r16.argtypes = [_fp, C.c_int, C.c_long, C.c_double, C.c_double, C.c_int, _u16, _u32]
        L.orc_table_to_r16.restype = None
        L.orc_r16_to_q16.argtypes = [_u16, _u32, C.c_int, C.c_long, _u32]
        L.orc_r16_to_q16.restype = None
        L.orc_fmm3.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, _dp, _u8, _dp, C.POINTER(C.c_long)]
        L.orc_fmm3.restype = C.c_int
        L.orc_seed3.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, _dp, C.c_double, C.c_double, C.c_double,
                                C.c_double, _u8, _dp]
        L.orc_seed3.restype = C.c_int
        L.orc_tables3.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, _fp, _dp, C.c_int, _i32, C.c_long, _dp,
                                  C.c_int]
        L.orc_tables3.restype = C.c_int
        L.orc_max_threads.argtypes = []
        L.orc_max_threads.restype = C.c_int
        _lib = L
    return _lib


def max_threads() -> int:
    return int(lib().orc_max_threads())


def fmm(slow: np.ndarray, frozen: np.ndarray, T0: np.ndarray, h: float):
    """Fast marching on a [ny][nx] slowness grid from an arbitrary frozen set.

    frozen: bool [ny][nx]; T0: the frozen nodes' values.  Returns (T, pops)."""
    ny, nx = slow.shape
    T = np.ascontiguousarray(T0, dtype=np.float64).copy()
    pops = C.c_long(0)
    rc = lib().orc_fmm(nx, ny, float(h), np.ascontiguousarray(slow, dtype=np.float64),
                       np.ascontiguousarray(frozen, dtype=np.uint8), T, C.byref(pops))
    if rc:
        raise MemoryError("orc_fmm")
    return T, int(pops.value)


def fmm2(slow: np.ndarray, frozen: np.ndarray, T0: np.ndarray, h: float, order: int = 2,
         with_order: bool = False):
    """Fast marching with the paper's second-order one-sided differences
    (order=2) or the first-order update (order=1).  Returns (T, pops), or
    (T, pops, accepted) with the flat node indices in acceptance order when
    with_order is set."""
    ny, nx = slow.shape
    T = np.ascontiguousarray(T0, dtype=np.float64).copy()
    pops = C.c_long(0)
    acc = np.full(nx * ny, -1, dtype=np.int32)
    rc = lib().orc_fmm2(nx, ny, float(h), np.ascontiguousarray(slow, dtype=np.float64),
                        np.ascontiguousarray(frozen, dtype=np.uint8), T, C.byref(pops), int(order),
                        acc.ctypes.data if with_order else None)
    if rc:
        raise MemoryError("orc_fmm2")
    if with_order:
        return T, int(pops.value), acc[:int(pops.value)].copy()
    return T, int(pops.value)


def seed(slow: np.ndarray, h: float, sx: float, sy: float, r0: float | None = None):
    """Point-source initial condition (frozen mask, T with frozen values set)."""
    ny, nx = slow.shape
    fr = np.zeros((ny, nx), dtype=np.uint8)
    T = np.full((ny, nx), np.inf)
    c = lib().orc_seed(nx, ny, float(h), np.ascontiguousarray(slow, dtype=np.float64), float(sx), float(sy),
                       float(2.0 * h if r0 is None else r0), fr, T)
    if c < 0:
        raise ValueError("source outside the grid")
    return fr.astype(bool), T


def travel_time_map(speed: np.ndarray, h: float, sx: float, sy: float) -> np.ndarray:
    """Full first-arrival map [ny][nx] (seconds) from one point source."""
    slow = 1.0 / np.asarray(speed, dtype=np.float64)
    fr, T0 = seed(slow, h, sx, sy)
    T, _ = fmm(slow, fr, T0, h)
    return T


def tables(speed: np.ndarray, h: float, sensors: np.ndarray, pix: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """Delay table T[S][P] (seconds, float64): one fast-marching solve per sensor."""
    speed = np.ascontiguousarray(speed, dtype=np.float32)
    ny, nx = speed.shape
    sxy = np.ascontiguousarray(sensors, dtype=np.float64)
    pix = np.ascontiguousarray(pix, dtype=np.int32)
    S, P = sxy.shape[0], pix.shape[0]
    out = np.empty((S, P), dtype=np.float64)
    rc = lib().orc_tables(nx, ny, float(h), speed, sxy, S, pix, P, out, int(nthreads))
    if rc == -1:
        raise ValueError("orc_tables: invalid input")
    if rc:
        raise MemoryError("orc_tables")
    return out


def tables2(speed: np.ndarray, h: float, sensors: np.ndarray, pix: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """Delay table T[S][P] from the second-order fast marching (orc_fmm2)."""
    speed = np.ascontiguousarray(speed, dtype=np.float32)
    ny, nx = speed.shape
    sxy = np.ascontiguousarray(sensors, dtype=np.float64)
    pix = np.ascontiguousarray(pix, dtype=np.int32)
    S, P = sxy.shape[0], pix.shape[0]
    out = np.empty((S, P), dtype=np.float64)
    rc = lib().orc_tables2(nx, ny, float(h), speed, sxy, S, pix, P, out, int(nthreads))
    if rc == -1:
        raise ValueError("orc_tables2: invalid input")
    if rc:
        raise MemoryError("orc_tables2")
    return out


def tables_const(nx: int, ny: int, h: float, c: float, sensors: np.ndarray, pix: np.ndarray) -> np.ndarray:
    """Straight-ray delays |x - s| / c of the conventional back projection."""
    sxy = np.ascontiguousarray(sensors, dtype=np.float64)
    pix = np.ascontiguousarray(pix, dtype=np.int32)
    out = np.empty((sxy.shape[0], pix.shape[0]), dtype=np.float64)
    if lib().orc_tables_const(int(nx), int(ny), float(h), float(c), sxy, sxy.shape[0], pix, pix.shape[0], out):
        raise ValueError("orc_tables_const: invalid input")
    return out


def tables_const3(nx: int, ny: int, nz: int, h: float, c: float, sensors: np.ndarray, vox: np.ndarray) -> np.ndarray:
    """Straight-ray delays |x - s| / c on a 3-D grid; sensors [S][3]."""
    sxyz = np.ascontiguousarray(sensors, dtype=np.float64)
    vox = np.ascontiguousarray(vox, dtype=np.int32)
    out = np.empty((sxyz.shape[0], vox.shape[0]), dtype=np.float64)
    if lib().orc_tables_const3(int(nx), int(ny), int(nz), float(h), float(c), sxyz, sxyz.shape[0], vox,
                               vox.shape[0], out):
        raise ValueError("orc_tables_const3: invalid input")
    return out


def filt(p: np.ndarray, dt: float, t0: float = 0.0) -> np.ndarray:
    """UBP filter b = p - t dp/dt along the last axis."""
    p = np.ascontiguousarray(p, dtype=np.float64)
    N = p.shape[-1]
    out = np.empty_like(p)
    lib().orc_filter(p, p.size // N, N, float(t0), float(dt), out)
    return out


def _weights(w, S):
    if w is None:
        return None, None
    w = np.ascontiguousarray(w, dtype=np.float64)
    assert w.shape == (S,)
    return w, w.ctypes.data_as(C.c_void_p)


def gather(T: np.ndarray, b: np.ndarray, dt: float, t0: float = 0.0, w=None, nthreads: int = 0) -> np.ndarray:
    """img[..][p] = sum_s w_s * lerp(b_s, (T[s][p]-t0)/dt).  b is [S][N] or [F][S][N]."""
    T = np.ascontiguousarray(T, dtype=np.float64)
    S, P = T.shape
    b = np.ascontiguousarray(b, dtype=np.float64)
    single = b.ndim == 2
    bb = b[None] if single else b
    F, S2, N = bb.shape
    assert S2 == S
    keep, wp = _weights(w, S)
    out = np.empty((F, P), dtype=np.float64)
    lib().orc_gather(T, np.ascontiguousarray(bb), wp, S, P, N, F, float(t0), float(dt), out, int(nthreads))
    del keep
    return out[0] if single else out


def table_to_q16(T: np.ndarray, dt: float, N: int, t0: float = 0.0) -> np.ndarray:
    """16.16 fixed-point fractional sample index of a float32 delay table."""
    T = np.ascontiguousarray(T, dtype=np.float32)
    q = np.empty(T.shape, dtype=np.uint32)
    lib().orc_table_to_q16(T, T.size, float(t0), float(dt), int(N), q)
    return q


def table_to_r16(T: np.ndarray, dt: float, N: int, t0: float = 0.0):
    """Tile-relative 16-bit form of a float32 delay table: (off uint16 [S][P],
    hdr uint32 [S][ceil(P/32)])."""
    T = np.ascontiguousarray(T, dtype=np.float32)
    S, P = T.shape
    off = np.empty((S, P), dtype=np.uint16)
    hdr = np.empty((S, (P + 31) // 32), dtype=np.uint32)
    lib().orc_table_to_r16(T, S, P, float(t0), float(dt), int(N), off, hdr)
    return off, hdr


def r16_to_q16(off: np.ndarray, hdr: np.ndarray) -> np.ndarray:
    """The 16.16 table a tile-relative 16-bit table stands for."""
    off = np.ascontiguousarray(off, dtype=np.uint16)
    hdr = np.ascontiguousarray(hdr, dtype=np.uint32)
    S, P = off.shape
    assert hdr.shape == (S, (P + 31) // 32)
    q = np.empty((S, P), dtype=np.uint32)
    lib().orc_r16_to_q16(off, hdr, S, P, q)
    return q


def gather_q16(q: np.ndarray, b: np.ndarray, w=None, nthreads: int = 0) -> np.ndarray:
    """Gather from a 16.16 delay table; b is [S][N] or [F][S][N]."""
    q = np.ascontiguousarray(q, dtype=np.uint32)
    S, P = q.shape
    b = np.ascontiguousarray(b, dtype=np.float64)
    single = b.ndim == 2
    bb = b[None] if single else b
    F, S2, N = bb.shape
    assert S2 == S
    keep, wp = _weights(w, S)
    out = np.empty((F, P), dtype=np.float64)
    lib().orc_gather_q16(q, np.ascontiguousarray(bb), wp, S, P, N, F, out, int(nthreads))
    del keep
    return out[0] if single else out


def backproject(T: np.ndarray, p: np.ndarray, dt: float, t0: float = 0.0, w=None, nthreads: int = 0) -> np.ndarray:
    """Full back projection of raw signals: filter, then gather."""
    return gather(T, filt(p, dt, t0), dt, t0, w, nthreads)


# ----------------------------------------------------------------------------- 3-D

def fmm3(slow: np.ndarray, frozen: np.ndarray, T0: np.ndarray, h: float):
    """Fast marching on a [nz][ny][nx] slowness grid from a frozen set.  Returns (T, pops)."""
    nz, ny, nx = slow.shape
    T = np.ascontiguousarray(T0, dtype=np.float64).copy()
    pops = C.c_long(0)
    rc = lib().orc_fmm3(nx, ny, nz, float(h), np.ascontiguousarray(slow, dtype=np.float64),
                        np.ascontiguousarray(frozen, dtype=np.uint8), T, C.byref(pops))
    if rc:
        raise MemoryError("orc_fmm3")
    return T, int(pops.value)


def seed3(slow: np.ndarray, h: float, sx: float, sy: float, sz: float, r0: float | None = None):
    """3-D point-source initial condition (frozen mask, T with frozen values set)."""
    nz, ny, nx = slow.shape
    fr = np.zeros((nz, ny, nx), dtype=np.uint8)
    T = np.full((nz, ny, nx), np.inf)
    c = lib().orc_seed3(nx, ny, nz, float(h), np.ascontiguousarray(slow, dtype=np.float64), float(sx), float(sy),
                        float(sz), float(2.0 * h if r0 is None else r0), fr, T)
    if c < 0:
        raise ValueError("source outside the grid")
    return fr.astype(bool), T


def travel_time_map3(speed: np.ndarray, h: float, sx: float, sy: float, sz: float) -> np.ndarray:
    """Full 3-D first-arrival map [nz][ny][nx] (seconds) from one point source."""
    slow = 1.0 / np.asarray(speed, dtype=np.float64)
    fr, T0 = seed3(slow, h, sx, sy, sz)
    T, _ = fmm3(slow, fr, T0, h)
    return T


def tables3(speed: np.ndarray, h: float, sensors: np.ndarray, pix: np.ndarray, nthreads: int = 0) -> np.ndarray:
    """3-D delay table T[S][P] (seconds, float64); speed [nz][ny][nx], sensors [S][3]."""
    speed = np.ascontiguousarray(speed, dtype=np.float32)
    nz, ny, nx = speed.shape
    sxyz = np.ascontiguousarray(sensors, dtype=np.float64)
    pix = np.ascontiguousarray(pix, dtype=np.int32)
    S, P = sxyz.shape[0], pix.shape[0]
    out = np.empty((S, P), dtype=np.float64)
    rc = lib().orc_tables3(nx, ny, nz, float(h), speed, sxyz, S, pix, P, out, int(nthreads))
    if rc == -1:
        raise ValueError("orc_tables3: invalid input")
    if rc:
        raise MemoryError("orc_tables3")
    return out
