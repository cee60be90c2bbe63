"""The wave-window gather (k_bp_win) against the FP64 oracle.

pat_backproject takes this kernel for float32, 16.16 and 16-bit tile-relative
tables (not the interleaved form) above 128 MiB, for a single frame with at
least 131072 columns or for several frames that fill the GPU (the 1024^2
precision study runs it at full size).  Here the PAT_GATHER_FORCE=win hook
sends smaller shapes to it, so that the oracle checks every pixel:
  - a smooth table (the small geometry's fast-marching delays, tile-ordered
    ROI), where nearly every gather reads the wave's LDS window;
  - random delays with some outside the record, where nearly every gather
    misses the window and takes the global-memory path;
  - a 128-sample record (the window is the whole record) with delays at both
    ends, where the filter is one-sided;
with float32 and binary16 frames, raw and pre-filtered input, weights, one to
three frames per launch, and column counts that leave a ragged last group
(odd counts also misalign the 16-bit rows)."""
import numpy as np
import pytest

from paper_1501_03869_amd import inputs

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-4


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.fixture(scope="module")
def ctx():
    from paper_1501_03869_amd import pat
    c = pat.Context(0)
    yield c
    c.close()


@pytest.fixture()
def force_win(monkeypatch):
    monkeypatch.setenv("PAT_GATHER_FORCE", "win")


@pytest.fixture(scope="module")
def smooth(orc):
    from paper_1501_03869_amd import pat
    geo = inputs.config("small")
    geo.pix = pat.tile_order(geo.nx, geo.ny, geo.pix, 32, 32)
    T = orc.tables(geo.speed, geo.h, geo.sensors, geo.pix).astype(np.float32)
    frames = np.stack([inputs.frame_for(geo, T, f) for f in range(3)])
    return geo, T, frames


def _fp16(p3):
    F = p3.shape[0]
    scale = (np.abs(p3).reshape(F, -1).max(1) / 2.0 ** 14).astype(np.float32)
    h = (p3 / scale[:, None, None]).astype(np.float16)
    return scale, h, h.astype(np.float64) * scale.astype(np.float64)[:, None, None]


def _run(ctx, orc, T, p3, dt, t0, tfmt, sig, filtered, w):
    """GPU gather of frames p3 [F][S][N] (raw, or b when filtered) through the
    given table form, and the oracle's image of the same inputs."""
    F, S, N = p3.shape
    if sig == "f16":
        scale, h, vals = _fp16(p3)
        sigd, sc = dev(h if F > 1 else h[0]), dev(scale)
    else:
        vals = p3.astype(np.float64)
        sigd, sc = dev(p3 if F > 1 else p3[0]), None
    b = vals if filtered else orc.filt(vals, dt, t0)
    wd = None if w is None else dev(w)
    w64 = None if w is None else w.astype(np.float64)
    if tfmt == "q16":
        tab = ctx.table_to_q16(dev(T), dt, N, t0)
        ref = orc.gather_q16(orc.table_to_q16(T, dt, N, t0), b, w64)
    elif tfmt == "r16":
        # the oracle gathers the 16.16 table its own 16-bit encoding stands for
        tab = ctx.table_to_r16(dev(T), dt, N, t0)
        ref = orc.gather_q16(orc.r16_to_q16(*orc.table_to_r16(T, dt, N, t0)), b, w64)
    else:
        tab = dev(T)
        ref = orc.gather(T.astype(np.float64), b, dt, t0, w64)
    got = ctx.backproject(tab, sigd, dt, t0, filtered=filtered, w=wd, frame_scale=sc).cpu().numpy()
    return got.reshape(ref.shape), ref


@pytest.mark.parametrize("tfmt,sig,filtered,weights,F", [
    ("f32", "f32", False, False, 1),
    ("f32", "f32", False, True, 3),
    ("f32", "f16", False, False, 2),
    ("f32", "f32", True, False, 1),
    ("f32", "f16", True, True, 1),
    ("q16", "f32", False, False, 1),
    ("q16", "f16", False, True, 3),
    ("q16", "f32", True, False, 2),
    ("r16", "f32", False, False, 1),
    ("r16", "f16", False, True, 2),
    ("r16", "f16", True, False, 1),
])
def test_smooth_table(ctx, orc, smooth, force_win, tfmt, sig, filtered, weights, F):
    geo, T, frames = smooth
    p3 = frames[:F]
    if filtered:
        p3 = orc.filt(p3.astype(np.float64), geo.dt).astype(np.float32)
    w = np.random.default_rng(3).uniform(0.5, 1.5, geo.S).astype(np.float32) if weights else None
    got, ref = _run(ctx, orc, T, p3, geo.dt, 0.0, tfmt, sig, filtered, w)
    err = rel_l2(got, ref)
    print(f"[win] small geometry {tfmt} {sig} filtered={filtered} weights={weights} F={F}: rel L2 {err:.3e}",
          flush=True)
    assert err <= IMG_TOL


@pytest.mark.parametrize("S,P,N,F,tfmt,sig,filtered,t0", [
    (37, 4099, 300, 2, "f32", "f32", False, 0.0),
    (37, 4099, 300, 1, "q16", "f16", False, 0.0),
    (13, 1037, 1024, 3, "f32", "f16", True, 2.5e-7),
    (64, 777, 256, 1, "q16", "f32", True, 0.0),
    (37, 4099, 300, 2, "r16", "f32", False, 0.0),
    (13, 1037, 1024, 1, "r16", "f16", False, 2.5e-7),
])
def test_random_delays(ctx, orc, force_win, S, P, N, F, tfmt, sig, filtered, t0):
    dt = 4e-8
    T = inputs.random_table(100 + S, S, P, N, dt, t0, frac_out=0.1)
    p = inputs.random_signals(101 + S, S, N, F)
    p3 = p if F > 1 else p[None]
    w = np.random.default_rng(4).uniform(0.5, 1.5, S).astype(np.float32)
    got, ref = _run(ctx, orc, T, p3, dt, t0, tfmt, sig, filtered, w)
    err = rel_l2(got, ref)
    print(f"[win] random delays S={S} P={P} N={N} F={F} {tfmt} {sig} filtered={filtered}: rel L2 {err:.3e}",
          flush=True)
    assert err <= IMG_TOL


@pytest.mark.parametrize("tfmt,sig", [("f32", "f32"), ("q16", "f16"), ("r16", "f32")])
def test_record_ends(ctx, orc, force_win, tfmt, sig):
    # N = 128: the window is the whole record; delays within a few samples of
    # either end, exactly at 0 and N-1, and just outside (a power-of-two
    # sample period makes the whole-sample delays exact in float32 seconds,
    # so that both sides see the same end samples as inside the record)
    S, P, N, dt = 24, 1000, 128, 2.0 ** -24
    rng = np.random.default_rng(5)
    u = np.where(rng.random((S, P)) < 0.5, rng.uniform(0, 3, (S, P)), rng.uniform(N - 4, N - 1, (S, P)))
    u[:, ::97] = 0.0
    u[:, 5::97] = N - 1
    u[:, 11::97] = -1e-3
    u[:, 17::97] = N - 1 + 1e-3
    T = (u * dt).astype(np.float32)
    p = inputs.random_signals(6, S, N)
    got, ref = _run(ctx, orc, T, p[None], dt, 0.0, tfmt, sig, False, None)
    err = rel_l2(got, ref)
    print(f"[win] record ends {tfmt} {sig}: rel L2 {err:.3e}", flush=True)
    assert err <= IMG_TOL


def test_same_as_the_other_kernels_and_reproducible(ctx, smooth, monkeypatch):
    geo, T, frames = smooth
    Td, pd = dev(T), dev(frames[0])
    monkeypatch.delenv("PAT_GATHER_FORCE", raising=False)
    other = ctx.backproject(Td, pd, geo.dt, filtered=False).cpu().numpy()
    monkeypatch.setenv("PAT_GATHER_FORCE", "win")
    a = ctx.backproject(Td, pd, geo.dt, filtered=False).cpu().numpy()
    b = ctx.backproject(Td, pd, geo.dt, filtered=False).cpu().numpy()
    print(f"[win] against the split-sensor kernel: rel L2 {rel_l2(a, other):.3e}", flush=True)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    assert rel_l2(a, other) <= 1e-5


@pytest.mark.parametrize("S,P,N,F,tfmt,sig", [
    (1, 256, 128, 1, "f32", "f32"),     # one sensor, exactly one group of 256 columns
    (2, 257, 130, 2, "f32", "f16"),     # a last group with one column
    (5, 511, 300, 5, "q16", "f32"),     # more waves than sensors would fill: one sensor per wave
    (3, 1280, 256, 3, "r16", "f16"),    # whole groups only, three frames
])
def test_small_shapes(ctx, orc, force_win, S, P, N, F, tfmt, sig):
    dt = 5e-8
    # delays inside the record with a compact spread per group, as a tile-ordered ROI gives
    rng = np.random.default_rng(200 + S)
    base = rng.uniform(2.0, N - 70.0, (S, 1))
    u = base + rng.uniform(0.0, 60.0, (S, P))
    T = (u * dt).astype(np.float32)
    p = inputs.random_signals(201 + S, S, N, F)
    p3 = p if F > 1 else p[None]
    got, ref = _run(ctx, orc, T, p3, dt, 0.0, tfmt, sig, False, None)
    err = rel_l2(got, ref)
    print(f"[win] small shape S={S} P={P} N={N} F={F} {tfmt} {sig}: rel L2 {err:.3e}", flush=True)
    assert err <= IMG_TOL


@pytest.mark.parametrize("F,sig,tfmt,filtered,weights", [
    (3, "f32", "f32", False, False),
    (5, "f16", "q16", False, False),
    (4, "f32", "r16", False, False),
    (4, "f16", "f32", True, True),     # pre-filtered FP16 frames with weights, 4 per wave
    (2, "f32", "q16", True, False),    # pre-filtered FP32 frames, 2 per wave
    (6, "f32", "f32", False, True),    # raw frames with weights; a last block of 2 past F
])
def test_frames_sharing_table_reads(ctx, orc, F, sig, tfmt, filtered, weights):
    # a table larger than the 256 MB Infinity Cache (520 x 140000 float32
    # entries, 291 MB): each wave decodes its delays once for 2 (F = 2, 3) or
    # 4 frames, the last block holding frames past F that are not stored
    S, P, N, dt = 520, 140000, 512, 4e-8
    rng = np.random.default_rng(300 + F)
    base = rng.uniform(2.0, N - 150.0, (S, 1))
    u = base + np.tile(np.linspace(0.0, 100.0, 256), P // 256 + 1)[:P][None, :] + rng.uniform(0.0, 8.0, (S, P))
    T = (u * dt).astype(np.float32)
    assert T.nbytes > (256 << 20)
    p = inputs.random_signals(301 + F, S, N, F)
    if filtered:
        p = orc.filt(p.astype(np.float64), dt).astype(np.float32)
    w = np.random.default_rng(302 + F).uniform(0.5, 1.5, S).astype(np.float32) if weights else None
    got, ref = _run(ctx, orc, T, p, dt, 0.0, tfmt, sig, filtered, w)
    err = rel_l2(got, ref)
    print(f"[win] frames sharing table reads F={F} {tfmt} {sig} filtered={filtered} weights={weights}: "
          f"rel L2 {err:.3e}", flush=True)
    assert err <= IMG_TOL
