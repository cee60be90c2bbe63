"""A-priori error bounds of the reduced-precision back projections (test helper).

The FP64 reference is the back projection of Section II-C on the raw samples
p: the central-difference UBP filter b[n] = p[n] - t_n (p[n+1] - p[n-1]) /
(2 dt) (one-sided at both ends), read at u = (T - t0)/dt with linear
interpolation, summed over sensors.  A GPU form differs from it by
  - delays off by at most `quant` samples (16.16 rounding 2^-17, the 16-bit
    tile form 2^-(k+1), or the FP32 decode of float seconds),
  - samples rounded to binary16 after division by a per-frame scale,
  - FP32 arithmetic in the filter, the interpolation and the sum over S.
Each is bounded per pixel from the definition; nothing here comes from the
GPU path.
"""
from __future__ import annotations

import numpy as np


def ubp_filter(p: np.ndarray, dt: float, t0: float = 0.0) -> np.ndarray:
    """b = p - t dp/dt with central differences, one-sided at the ends (FP64)."""
    N = p.shape[-1]
    t = t0 + dt * np.arange(N, dtype=np.float64)
    d = np.empty_like(p, dtype=np.float64)
    d[..., 1:-1] = (p[..., 2:] - p[..., :-2]) / (2.0 * dt)
    d[..., 0] = (p[..., 1] - p[..., 0]) / dt
    d[..., -1] = (p[..., -1] - p[..., -2]) / dt
    return p - t * d


def gather_error_bound(T: np.ndarray, p: np.ndarray, dt: float, quant, fp16_scale: float | None = None,
                       w: np.ndarray | None = None, t0: float = 0.0, filtered: bool = False) -> np.ndarray:
    """Per-pixel bound of |img - img_FP64(T, p)| for one frame.

    T: FP64 delays [S][P] (seconds); p: FP64 samples [S][N], raw (the filter
    is part of the gather) or, with filtered, already b; quant: the largest
    delay error in samples, scalar or [S][P] (< 1); fp16_scale: the frame's
    binary16 scale, or None for FP32 samples."""
    S, N = p.shape
    P = T.shape[1]
    w = np.ones(S) if w is None else np.abs(np.asarray(w, np.float64))
    quant = np.broadcast_to(np.asarray(quant, np.float64), (S, P))
    u = (T - t0) / dt
    valid = np.isfinite(u) & (u >= 0) & (u <= N - 1)
    # invalid delays near an end take that end's interval
    uq = np.where(np.isfinite(u), np.clip(u, 0.0, N - 1.0), 0.0)
    n = np.minimum(np.floor(uq).astype(np.int64), N - 2)
    rows = np.arange(S)[:, None]
    b = p if filtered else ubp_filter(p, dt, t0)
    # interval slopes |b[m+1] - b[m]|; a delay off by < 1 sample may fall in
    # the interval below or above its own
    slope = np.abs(np.diff(b, axis=1))
    s3 = np.maximum(np.maximum(slope[rows, n], slope[rows, np.maximum(n - 1, 0)]),
                    slope[rows, np.minimum(n + 1, N - 2)])
    term = quant * s3
    bmax = np.maximum(np.abs(b[rows, n]), np.abs(b[rows, n + 1]))
    # a delay within quant of either end of the record may be taken as valid
    # on one side and not on the other: its whole contribution
    edge = np.isfinite(u) & ((np.abs(u) <= quant) | (np.abs(u - (N - 1)) <= quant))
    term = np.where(edge, np.maximum(term, bmax + quant * s3), term)
    if fp16_scale is not None:
        # binary16 rounding of p / scale: relative 2^-11, absolute 2^-25 (half
        # the subnormal spacing), times the scale
        dp = 2.0 ** -11 * np.abs(p) + 2.0 ** -25 * float(fp16_scale)
        k = np.abs(t0 / dt + np.arange(N, dtype=np.float64)) * (0.0 if filtered else 0.5)
        db = np.empty_like(dp)
        db[:, 1:-1] = dp[:, 1:-1] + k[1:-1] * (dp[:, 2:] + dp[:, :-2])
        db[:, 0] = dp[:, 0] + 2 * k[0] * (dp[:, 1] + dp[:, 0])
        db[:, -1] = dp[:, -1] + 2 * k[-1] * (dp[:, -1] + dp[:, -2])
        lo, hi = np.maximum(n - 1, 0), np.minimum(n + 2, N - 1)
        term = term + np.maximum.reduce([db[rows, lo], db[rows, n], db[rows, n + 1], db[rows, hi]])
    # FP32 arithmetic: each gather is a few rounded operations on four taps
    # with coefficients up to (n + 1)/2 + 1, and the sum over S sensors adds
    # S - 1 more roundings of partial sums bounded by the sum of magnitudes
    lo, hi = np.maximum(n - 1, 0), np.minimum(n + 2, N - 1)
    taps = np.abs(p[rows, lo]) + np.abs(p[rows, n]) + np.abs(p[rows, n + 1]) + np.abs(p[rows, hi])
    mag = (1.0 + (0.0 if filtered else 0.5) * (np.abs(t0 / dt) + n + 1)) * taps
    wv = w[:, None] * (valid | edge)
    return (wv * term).sum(0) + 2.0 ** -24 * (S + 8) * (wv * mag).sum(0)


def f32_decode_quant(T: np.ndarray, dt: float, t0: float = 0.0) -> np.ndarray:
    """Delay error (samples) of decoding float32 seconds as u = T (1/dt) - t0/dt
    in FP32 with 1/dt split into two floats: a few ulps of u."""
    u = np.abs((T - t0) / dt)
    return np.where(np.isfinite(u), 4.0 * 2.0 ** -24 * (u + abs(t0 / dt) + 1.0), 0.0)


def fp16_frames(p: np.ndarray):
    """Per-frame scale max|p|/2^14, the binary16 codes, and their exact values."""
    F = p.shape[0]
    scale = (np.abs(p).reshape(F, -1).max(1) / 2.0 ** 14).astype(np.float32)
    scale[scale == 0] = 1.0
    h = (p / scale[:, None, None]).astype(np.float16)
    return scale, h, h.astype(np.float64) * scale.astype(np.float64)[:, None, None]


def straight_ray_quant(nx: int, ny: int, h: float, c: float, sensors: np.ndarray, pix: np.ndarray, dt: float,
                       t0: float = 0.0) -> np.ndarray:
    """Delay error (samples) of the straight-ray delay |x - s| / c evaluated in
    FP32 from node positions x0 + i h and float32 sensor positions: a few
    roundings of each coordinate, of the distance and of the product with
    1/c, then the FP32 decode."""
    i, j = pix % nx, pix // nx
    x0, y0 = 0.5 * (nx - 1) * h, 0.5 * (ny - 1) * h
    dpx = 2.0 ** -22 * (x0 + i * h)
    dpy = 2.0 ** -22 * (y0 + j * h)
    ds = 2.0 ** -22 * (np.abs(sensors[:, 0]) + np.abs(sensors[:, 1]))
    d = np.hypot((i * h - x0)[None, :] - sensors[:, :1], (j * h - y0)[None, :] - sensors[:, 1:2])
    T = d / c
    dT = (dpx[None, :] + dpy[None, :] + ds[:, None]) / c + 8.0 * 2.0 ** -24 * T
    return dT / dt + f32_decode_quant(T, dt, t0)
