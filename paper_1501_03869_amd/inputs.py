"""Seeded synthetic inputs for the photoacoustic back-projection workloads.

This module only draws and lays out inputs: speed-of-sound maps, ring sensor
positions, region-of-interest pixel lists, absorber phantoms and the N-shaped
pressure pulses that stand in for measured sensor signals.  It contains none of
the method's arithmetic (no eikonal update, no filter, no gather).  Travel
times needed to place the synthetic pulses are passed in by the caller.

The workloads stand in for the paper's CT-derived monkey skull and its k-Wave
simulated signals (Section III, "Numerical simulation"), which are not
available: a skull annulus between brain tissue and water-like coupling medium,
a ring array of point sensors, and a vascular phantom.  Speeds follow the
values the paper quotes for brain (1540 m/s) and skull (2200-3000 m/s,
Introduction and Section III).

Grid convention: node (i, j), i along x, flat index k = j*nx + i, located at
x_i = (i - (nx-1)/2) h, y_j = (j - (ny-1)/2) h; the grid centre is the centre of
the sensor ring.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Seed offsets: speed map 1000+cfg, phantom / absorbers 2000+frame,
# noise 3000+frame, Poisson arrivals 4000.
SEED_MAP = 1000
SEED_PHANTOM = 2000
SEED_NOISE = 3000
SEED_ARRIVALS = 4000

PULSE_SIGMA = 50e-9  # seconds, width of the Gaussian-derivative N-pulse


@dataclasses.dataclass
class Geometry:
    """One imaging geometry: speed map, sensors, ROI and sampling."""
    name: str
    nx: int
    ny: int
    h: float                 # metres
    speed: np.ndarray        # float32 [ny][nx], m/s
    sensors: np.ndarray      # float64 [S][2], metres, grid-centred
    pix: np.ndarray          # int32 [P], node indices j*nx+i
    n_samples: int
    dt: float                # seconds
    t0: float = 0.0          # time of the first sample (laser pulse at t=0)

    @property
    def S(self) -> int:
        return int(self.sensors.shape[0])

    @property
    def P(self) -> int:
        return int(self.pix.shape[0])


def node_coords(nx: int, ny: int, h: float):
    """Return (x[nx], y[ny]) node coordinates in metres (grid-centred)."""
    x = (np.arange(nx, dtype=np.float64) - (nx - 1) / 2.0) * h
    y = (np.arange(ny, dtype=np.float64) - (ny - 1) / 2.0) * h
    return x, y


def radius_map(nx: int, ny: int, h: float) -> np.ndarray:
    x, y = node_coords(nx, ny, h)
    return np.hypot(x[None, :], y[:, None])


def ring_sensors(S: int, R: float) -> np.ndarray:
    """S point sensors evenly on a circle of radius R (metres), k = 0..S-1."""
    k = np.arange(S, dtype=np.float64)
    ang = 2.0 * np.pi * k / S
    return np.stack([R * np.cos(ang), R * np.sin(ang)], axis=1)


def disk_pixels(nx: int, ny: int, h: float, r: float, inclusive: bool = False) -> np.ndarray:
    """Row-major node indices of the nodes with radius < r (<= r if inclusive)."""
    rad = radius_map(nx, ny, h)
    m = rad <= r if inclusive else rad < r
    return np.flatnonzero(m.ravel()).astype(np.int32)


def _smooth_field(rng: np.random.Generator, nx: int, ny: int, h: float, ell: float) -> np.ndarray:
    """White noise filtered by a Gaussian kernel of std ell/sqrt(2).

    The resulting covariance is proportional to exp(-r^2 / (2 ell^2))."""
    from scipy.ndimage import gaussian_filter
    w = rng.standard_normal((ny, nx))
    return gaussian_filter(w, sigma=(ell / math.sqrt(2.0)) / h, mode="wrap")


def annulus_speed_small(nx=128, ny=128, h=0.25e-3, c_bg=1540.0, c_skull=2800.0,
                        r_in=12e-3, thick=6e-3) -> np.ndarray:
    """Homogeneous background with a constant-speed centred skull annulus."""
    rad = radius_map(nx, ny, h)
    c = np.full((ny, nx), c_bg, dtype=np.float64)
    c[(rad >= r_in) & (rad < r_in + thick)] = c_skull
    return c.astype(np.float32)


def skull_speed(seed: int, nx: int, ny: int, h: float, r_brain=16.5e-3, r_skull=23.5e-3,
                ell=2e-3, c_brain=1540.0, brain_var=0.02, c_lo=2200.0, c_hi=3000.0,
                c_out=1540.0) -> np.ndarray:
    """Brain disk with +-2% smooth variation, skull annulus 2200..3000 m/s from a
    smooth random field (correlation length ell), coupling medium outside."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rad = radius_map(nx, ny, h)
    brain = rad < r_brain
    skull = (rad >= r_brain) & (rad < r_skull)
    u = _smooth_field(rng, nx, ny, h, ell)
    v = _smooth_field(rng, nx, ny, h, ell)
    us = u[skull]
    u = (u - us.min()) / (us.max() - us.min())
    v = v / np.abs(v[brain]).max()
    c = np.full((ny, nx), c_out, dtype=np.float64)
    c[brain] = c_brain * (1.0 + brain_var * v[brain])
    c[skull] = c_lo + (c_hi - c_lo) * u[skull]
    return c.astype(np.float32)


def config(name: str) -> Geometry:
    """Geometry of a named workload.

    small  : 128^2, h=0.25 mm, annulus 12..18 mm at 2800 m/s, 64 sensors at
             15.5 mm, 1024 samples at 20 MHz, all 16384 pixels.
    paper  : 256^2, h=0.2 mm, random skull 16.5..23.5 mm, 512 sensors at
             24.5 mm, 2048 samples at 25 MHz, 21336 pixels inside r<16.5 mm.
    large  : 1024^2, h=0.05 mm, same physical geometry, 1024 sensors,
             4096 samples at 40 MHz, 823592 pixels inside r<=25.6 mm.
    serve_a: 128^2 small geometry with 128 sensors.
    serve_c: 512^2, h=0.1 mm, paper geometry, 512 sensors, 85564 pixels.
    tiny   : 24^2 quick-test geometry (homogeneous with a thin skull).
    """
    if name == "small":
        nx = ny = 128
        h = 0.25e-3
        return Geometry(name, nx, ny, h, annulus_speed_small(nx, ny, h), ring_sensors(64, 15.5e-3),
                        np.arange(nx * ny, dtype=np.int32), 1024, 50e-9)
    if name == "serve_a":
        nx = ny = 128
        h = 0.25e-3
        return Geometry(name, nx, ny, h, annulus_speed_small(nx, ny, h), ring_sensors(128, 15.5e-3),
                        np.arange(nx * ny, dtype=np.int32), 1024, 50e-9)
    if name == "paper":
        nx = ny = 256
        h = 0.2e-3
        return Geometry(name, nx, ny, h, skull_speed(SEED_MAP + 2, nx, ny, h), ring_sensors(512, 24.5e-3),
                        disk_pixels(nx, ny, h, 16.5e-3), 2048, 40e-9)
    if name == "large":
        nx = ny = 1024
        h = 0.05e-3
        return Geometry(name, nx, ny, h, skull_speed(SEED_MAP + 3, nx, ny, h), ring_sensors(1024, 24.5e-3),
                        disk_pixels(nx, ny, h, 25.6e-3, inclusive=True), 4096, 25e-9)
    if name == "serve_c":
        nx = ny = 512
        h = 0.1e-3
        return Geometry(name, nx, ny, h, skull_speed(SEED_MAP + 5, nx, ny, h), ring_sensors(512, 24.5e-3),
                        disk_pixels(nx, ny, h, 16.5e-3), 2048, 40e-9)
    if name == "tiny":
        nx = ny = 24
        h = 0.5e-3
        c = annulus_speed_small(nx, ny, h, r_in=4e-3, thick=1.5e-3)
        return Geometry(name, nx, ny, h, c, ring_sensors(8, 5.0e-3), np.arange(nx * ny, dtype=np.int32), 256, 50e-9)
    raise KeyError(name)


def perturb_speed(speed: np.ndarray, seed: int, frac: float = 0.017, mean_frac: float | None = None,
                  min_speed: float = 2000.0) -> np.ndarray:
    """Speed map with uncorrelated Gaussian errors added at the skull nodes
    (speed >= min_speed): standard deviation frac * max(speed), mean
    mean_frac * max(speed) (mean_frac defaults to frac).  The paper's
    robustness study concerns errors in the skull sound speed and quotes 1.7 %
    for both figures (Section III)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    top = float(np.max(speed))
    mu = top * (frac if mean_frac is None else mean_frac)
    noise = mu + top * frac * rng.standard_normal(speed.shape)
    out = speed.astype(np.float64) + np.where(speed >= min_speed, noise, 0.0)
    return out.astype(np.float32)


def paper_like_speed(seed: int, nx: int, ny: int, h: float) -> np.ndarray:
    """A fresh seeded skull map with the paper-scale generator (new maps in serving)."""
    return skull_speed(seed, nx, ny, h)


# ----------------------------------------------------------------------------- phantoms

def point_absorbers(seed: int, nx: int, ny: int, h: float, count=8, r_max=10e-3):
    """count absorbers uniform in the disk r < r_max, snapped to the nearest node.

    Returns (node index int64[count], amplitude float64[count] in U[0.5, 1])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rr = r_max * np.sqrt(rng.random(count))
    th = 2.0 * np.pi * rng.random(count)
    amp = 0.5 + 0.5 * rng.random(count)
    x0 = -(nx - 1) / 2.0 * h
    y0 = -(ny - 1) / 2.0 * h
    i = np.floor((rr * np.cos(th) - x0) / h + 0.5).astype(np.int64)
    j = np.floor((rr * np.sin(th) - y0) / h + 0.5).astype(np.int64)
    return j * nx + i, amp


def segment_phantom(seed: int, nx: int, ny: int, h: float, count=40, r_max=15.5e-3,
                    width_px=(1.0, 2.0)):
    """Vascular stand-in: count line segments with endpoints uniform in r < r_max
    and widths U[1,2] pixels, value 1.  Returns (node index int64[K], value[K])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x, y = node_coords(nx, ny, h)
    X, Y = np.meshgrid(x, y)
    mask = np.zeros((ny, nx), dtype=bool)
    for _ in range(count):
        r = r_max * np.sqrt(rng.random(2))
        t = 2.0 * np.pi * rng.random(2)
        ax, ay = r[0] * math.cos(t[0]), r[0] * math.sin(t[0])
        bx, by = r[1] * math.cos(t[1]), r[1] * math.sin(t[1])
        w = (width_px[0] + (width_px[1] - width_px[0]) * rng.random()) * h
        dx, dy = bx - ax, by - ay
        L2 = dx * dx + dy * dy
        s = np.clip(((X - ax) * dx + (Y - ay) * dy) / max(L2, 1e-30), 0.0, 1.0)
        d = np.hypot(X - (ax + s * dx), Y - (ay + s * dy))
        mask |= d <= 0.5 * w
    k = np.flatnonzero(mask.ravel()).astype(np.int64)
    return k, np.ones(k.shape[0], dtype=np.float64)


# ----------------------------------------------------------------------------- signals

def npulse_signals(src_delay: np.ndarray, src_amp: np.ndarray, src_dist: np.ndarray,
                   n_samples: int, dt: float, t0: float = 0.0, sigma: float = PULSE_SIGMA,
                   spreading: float = 0.5) -> np.ndarray:
    """Sum of Gaussian-derivative N-pulses, one per (sensor, source).

    src_delay[S][K]: arrival time of source k at sensor s (seconds, supplied by
    the caller); src_amp[K]; src_dist[S][K]: source-sensor distance in metres
    (for the r[mm]^-spreading amplitude decay: 1/2 cylindrical in 2-D, 1
    spherical in 3-D).  Pulse: A r^-spreading (-tau/sigma) exp(1/2 -
    tau^2/(2 sigma^2)), tau = t - delay, whose peak magnitude is
    A r^-spreading.  Only +-5 sigma around each arrival is evaluated.
    Returns float32 [S][n_samples]."""
    S, K = src_delay.shape
    out = np.zeros((S, n_samples), dtype=np.float64)
    half = int(math.ceil(5.0 * sigma / dt)) + 1
    offs = np.arange(-half, half + 1)
    for s in range(S):
        d = src_delay[s]
        ok = np.isfinite(d)
        if not ok.any():
            continue
        d = d[ok]
        a = src_amp[ok] * (src_dist[s][ok] * 1e3) ** -spreading
        n0 = np.floor((d - t0) / dt).astype(np.int64)
        idx = n0[:, None] + offs[None, :]
        tau = (t0 + idx * dt) - d[:, None]
        val = a[:, None] * (-tau / sigma) * np.exp(0.5 - tau * tau / (2.0 * sigma * sigma))
        good = (idx >= 0) & (idx < n_samples)
        out[s] += np.bincount(idx[good], weights=val[good], minlength=n_samples)
    return out.astype(np.float32)


def source_distances(geo: Geometry, src_nodes: np.ndarray) -> np.ndarray:
    """|x_k - s| in metres, [S][K]."""
    x, y = node_coords(geo.nx, geo.ny, geo.h)
    xs = x[src_nodes % geo.nx]
    ys = y[src_nodes // geo.nx]
    return np.hypot(xs[None, :] - geo.sensors[:, 0:1], ys[None, :] - geo.sensors[:, 1:2])


def frame_parts(geo: Geometry, table: np.ndarray, frame: int = 0, phantom: str = "segments"):
    """The inputs of one synthetic frame: the phantom's arrival times at every
    sensor (read from the table's columns), amplitudes and source-sensor
    distances.  The phantom's nodes must lie inside the ROI (true for the
    built-in geometries)."""
    if phantom == "points":
        nodes, amp = point_absorbers(SEED_PHANTOM + frame, geo.nx, geo.ny, geo.h)
    else:
        nodes, amp = segment_phantom(SEED_PHANTOM + frame, geo.nx, geo.ny, geo.h,
                                     r_max=min(15.5e-3, 0.45 * geo.nx * geo.h))
    col = np.full(geo.nx * geo.ny, -1, dtype=np.int64)
    col[geo.pix] = np.arange(geo.P)
    c = col[nodes]
    keep = c >= 0
    nodes, amp, c = nodes[keep], amp[keep], c[keep]
    delay = np.asarray(table[:, c], dtype=np.float64)
    return delay, amp, source_distances(geo, nodes)


def frame_from_parts(parts, n_samples: int, dt: float, t0: float = 0.0, frame: int = 0,
                     noise_snr_db: float | None = None) -> np.ndarray:
    """p[S][N] from frame_parts: N-pulses, plus white Gaussian noise at the
    given SNR (seed SEED_NOISE + frame) if requested."""
    delay, amp, dist = parts
    p = npulse_signals(delay, amp, dist, n_samples, dt, t0)
    if noise_snr_db is not None:
        rng = np.random.Generator(np.random.PCG64(SEED_NOISE + frame))
        rms = float(np.sqrt(np.mean(p.astype(np.float64) ** 2)))
        sd = rms / (10.0 ** (noise_snr_db / 20.0))
        p = (p + sd * rng.standard_normal(p.shape)).astype(np.float32)
    return p


def frame_for(geo: Geometry, table: np.ndarray, frame: int = 0, noise_snr_db: float | None = None,
              phantom: str = "segments") -> np.ndarray:
    """One synthetic frame p[S][N] for the given delay table T[S][P] (seconds).

    The phantom's nodes must lie inside the ROI (true for the built-in
    geometries); their travel times are read from the table's columns."""
    return frame_from_parts(frame_parts(geo, table, frame, phantom), geo.n_samples, geo.dt, geo.t0, frame,
                            noise_snr_db)


def random_table(seed: int, S: int, P: int, n_samples: int, dt: float, t0: float = 0.0,
                 frac_out: float = 0.0) -> np.ndarray:
    """Random delays in seconds (float32 [S][P]) spread over the sample window,
    with an optional fraction placed outside it (negative, past the end or +inf)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.random((S, P)) * (n_samples - 1)
    T = t0 + u * dt
    if frac_out > 0:
        m = rng.random((S, P)) < frac_out
        kind = rng.integers(0, 3, size=(S, P))
        T = np.where(m & (kind == 0), t0 - dt * (1 + rng.random((S, P))), T)
        T = np.where(m & (kind == 1), t0 + dt * (n_samples - 1) * (1.0 + 0.01 + rng.random((S, P))), T)
        T = np.where(m & (kind == 2), np.inf, T)
    return T.astype(np.float32)


def random_signals(seed: int, S: int, N: int, F: int = 1) -> np.ndarray:
    """Gaussian white-noise sensor signals, float32 [F][S][N] (or [S][N] if F == 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = rng.standard_normal((F, S, N)).astype(np.float32)
    return p[0] if F == 1 else p


def poisson_arrivals(rate_hz: float, duration_s: float, seed: int = SEED_ARRIVALS) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process of the given rate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(rate_hz * duration_s * 1.5) + 16
    t = np.cumsum(rng.exponential(1.0 / rate_hz, size=n))
    return t[t < duration_s]


# ----------------------------------------------------------------------------- 3-D

@dataclasses.dataclass
class Geometry3:
    """A 3-D imaging geometry: node-centred grid [nz][ny][nx], sensors on a sphere."""
    name: str
    nx: int
    ny: int
    nz: int
    h: float                 # metres
    speed: np.ndarray        # float32 [nz][ny][nx], m/s
    sensors: np.ndarray      # float64 [S][3], metres, grid-centred
    pix: np.ndarray          # int32 [P], voxel indices (l*ny + j)*nx + i
    n_samples: int
    dt: float
    t0: float = 0.0

    @property
    def S(self) -> int:
        return int(self.sensors.shape[0])

    @property
    def P(self) -> int:
        return int(self.pix.shape[0])


def node_coords3(nx: int, ny: int, nz: int, h: float):
    """(x[nx], y[ny], z[nz]) node coordinates in metres (grid-centred)."""
    x, y = node_coords(nx, ny, h)
    z = (np.arange(nz, dtype=np.float64) - (nz - 1) / 2.0) * h
    return x, y, z


def radius_map3(nx: int, ny: int, nz: int, h: float) -> np.ndarray:
    x, y, z = node_coords3(nx, ny, nz, h)
    return np.sqrt(z[:, None, None] ** 2 + y[None, :, None] ** 2 + x[None, None, :] ** 2)


def sphere_sensors(S: int, R: float) -> np.ndarray:
    """S sensors on a sphere of radius R (Fibonacci lattice), [S][3] metres."""
    k = np.arange(S, dtype=np.float64) + 0.5
    zc = 1.0 - 2.0 * k / S
    rho = np.sqrt(np.maximum(0.0, 1.0 - zc * zc))
    phi = np.pi * (3.0 - math.sqrt(5.0)) * k
    return R * np.stack([rho * np.cos(phi), rho * np.sin(phi), zc], axis=1)


def ball_voxels(nx: int, ny: int, nz: int, h: float, r: float) -> np.ndarray:
    """Row-major voxel indices with radius < r."""
    return np.flatnonzero(radius_map3(nx, ny, nz, h).ravel() < r).astype(np.int32)


def head_speed3(seed: int, n: int, h: float, r_brain=11e-3, r_skull=14e-3, ell=2e-3, c_brain=1540.0,
                brain_var=0.02, c_lo=2200.0, c_hi=3000.0, c_out=1540.0) -> np.ndarray:
    """3-D analogue of skull_speed: brain ball with +-2 % smooth variation, skull
    shell 2200..3000 m/s from a smooth random field, coupling medium outside."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.Generator(np.random.PCG64(seed))
    rad = radius_map3(n, n, n, h)
    brain = rad < r_brain
    skull = (rad >= r_brain) & (rad < r_skull)
    sig = (ell / math.sqrt(2.0)) / h
    u = gaussian_filter(rng.standard_normal((n, n, n)), sigma=sig, mode="wrap")
    v = gaussian_filter(rng.standard_normal((n, n, n)), sigma=sig, mode="wrap")
    us = u[skull]
    u = (u - us.min()) / (us.max() - us.min())
    v = v / np.abs(v[brain]).max()
    c = np.full((n, n, n), c_out, dtype=np.float64)
    c[brain] = c_brain * (1.0 + brain_var * v[brain])
    c[skull] = c_lo + (c_hi - c_lo) * u[skull]
    return c.astype(np.float32)


def config3(name: str) -> Geometry3:
    """Named 3-D geometries.

    tiny3 : 20^3, h = 0.5 mm, random medium 1400..3000 m/s, 6 sensors inside
            the grid, all voxels.
    head3 : 64^3, h = 0.5 mm, brain ball r < 11 mm, skull shell 11..14 mm,
            256 sensors on a sphere r = 15 mm, 1024 samples at 20 MHz,
            the voxels with r < 11 mm."""
    if name == "tiny3":
        n, h = 20, 0.5e-3
        rng = np.random.Generator(np.random.PCG64(SEED_MAP + 30))
        speed = rng.uniform(1400.0, 3000.0, size=(n, n, n)).astype(np.float32)
        sens = rng.uniform(-4e-3, 4e-3, size=(6, 3))
        return Geometry3(name, n, n, n, h, speed, sens, np.arange(n ** 3, dtype=np.int32), 512, 5e-8)
    if name == "head3":
        n, h = 64, 0.5e-3
        return Geometry3(name, n, n, n, h, head_speed3(SEED_MAP + 31, n, h), sphere_sensors(256, 15e-3),
                         ball_voxels(n, n, n, h, 11e-3), 1024, 5e-8)
    raise KeyError(name)


def source_distances3(geo: Geometry3, src_nodes: np.ndarray) -> np.ndarray:
    """|x_k - s| in metres, [S][K]."""
    x, y, z = node_coords3(geo.nx, geo.ny, geo.nz, geo.h)
    i = src_nodes % geo.nx
    j = (src_nodes // geo.nx) % geo.ny
    l = src_nodes // (geo.nx * geo.ny)
    d = np.stack([x[i], y[j], z[l]], axis=1)  # [K][3]
    return np.linalg.norm(d[None, :, :] - geo.sensors[:, None, :], axis=2)


def frame_for3(geo: Geometry3, table: np.ndarray, frame: int = 0, count: int = 8) -> np.ndarray:
    """One synthetic 3-D frame p[S][N]: count point absorbers at random ROI
    voxels (amplitudes U[0.5, 1]), N-pulses with spherical (1/r) spreading,
    arrival times from the table's columns."""
    rng = np.random.Generator(np.random.PCG64(SEED_PHANTOM + 100 + frame))
    c = rng.choice(geo.P, size=min(count, geo.P), replace=False)
    amp = 0.5 + 0.5 * rng.random(c.size)
    nodes = geo.pix[c].astype(np.int64)
    delay = np.asarray(table, dtype=np.float64)[:, c]
    return npulse_signals(delay, amp, source_distances3(geo, nodes), geo.n_samples, geo.dt, geo.t0, spreading=1.0)
