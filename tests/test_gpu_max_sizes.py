"""Back projection (Section II-C) at the largest column counts each gather
path takes, against the FP64 oracle on sampled pixels.

The limits come from the kernels' 32-bit buffer offsets:
  - the wave-window kernel takes P < 2^29 (a table row of 4 P bytes);
  - the split-sensor kernel takes P < 2^26 (a step's 8 table rows);
  - past that, a shape the wave-window kernel does not take (here N < 128)
    goes to the LDS-windowed kernel, whose offsets are 64-bit.
The delay tables are made on the device (tile-like ramps over runs of 256
columns, a fixed jitter, and delays before, after and outside the record in
the last columns), and the oracle gathers about 4000 sampled columns: the
first ones, the ragged tail and random ones between."""
import numpy as np
import pytest

from paper_1501_03869_amd import inputs

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-4


@pytest.fixture(scope="module")
def ctx():
    from paper_1501_03869_amd import pat
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = pat.Context(0)
    yield c
    c.close()


def device_table(S, P, N, dt, seed):
    """float32 [S][P] seconds on the device."""
    rng = np.random.default_rng(seed)
    base = rng.uniform(4.0, N - 60.0, S)
    col = torch.arange(P, dtype=torch.int32, device="cuda")
    u = (col % 256).float() * (40.0 / 256) + (col % 97).float() * (1.0 / 97)
    T = torch.empty((S, P), dtype=torch.float32, device="cuda")
    for s in range(S):
        T[s] = (u + float(base[s])) * dt
    del col, u
    T[:, P - 40:P - 25] = -3.0 * dt          # before the record
    T[:, P - 25:P - 10] = (N + 5.0) * dt     # after it
    T[:, P - 10:P - 5] = (N - 1.0) * dt      # the last sample
    T[:, P - 2] = float("inf")
    return T


def sample_columns(P, seed):
    rng = np.random.default_rng(seed)
    idx = np.concatenate([np.arange(300), np.arange(P - 600, P), rng.integers(0, P, 3000)])
    return np.unique(idx).astype(np.int64)


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def check(ctx, orc, T, tab, S, P, N, dt, sig_fmt, weights, seed, label):
    p = inputs.random_signals(seed, S, N)
    idx = sample_columns(P, seed)
    Ts = T[:, torch.from_numpy(idx).cuda()].double().cpu().numpy()
    w = np.random.default_rng(seed + 1).uniform(0.5, 1.5, S).astype(np.float32) if weights else None
    wd = None if w is None else torch.from_numpy(w).cuda()
    if sig_fmt == "f16":
        scale = np.float32(np.abs(p).max() / 2.0 ** 14)
        h = (p / scale).astype(np.float16)
        vals = h.astype(np.float64) * np.float64(scale)
        sig, sc = torch.from_numpy(h).cuda(), torch.tensor([scale], dtype=torch.float32, device="cuda")
    else:
        vals = p.astype(np.float64)
        sig, sc = torch.from_numpy(p).cuda(), None
    img = ctx.backproject(tab, sig, dt, 0.0, filtered=False, w=wd, frame_scale=sc)
    got = img.reshape(-1)[torch.from_numpy(idx).cuda()].cpu().numpy()
    ref = orc.gather(Ts, orc.filt(vals, dt), dt, 0.0, None if w is None else w.astype(np.float64))
    err = rel_l2(got, ref)
    tail = rel_l2(got[-600:], ref[-600:])
    print(f"[max sizes] {label}: S={S} P={P} N={N} {sig_fmt}: {len(idx)} sampled columns rel L2 {err:.3e}, "
          f"last 600 {tail:.3e}", flush=True)
    assert err <= IMG_TOL and tail <= IMG_TOL


def test_wave_window_at_its_column_limit(ctx, orc):
    # 2 x (2^29 - 7) float32 delays, 4.3 GB: the largest P the wave-window kernel takes
    S, P, N, dt = 2, (1 << 29) - 7, 128, 4e-8
    T = device_table(S, P, N, dt, 41)
    check(ctx, orc, T, T, S, P, N, dt, "f32", True, 41, "wave-window kernel")


def test_split_sensor_at_its_column_limit(ctx, orc):
    # interleaved table of 8 sensors x (2^26 - 5) columns: the largest P the
    # split-sensor kernel takes, with FP16 records
    S, P, N, dt = 8, (1 << 26) - 5, 64, 4e-8
    T = device_table(S, P, N, dt, 42)
    tab = ctx.table_to_x4(T)
    check(ctx, orc, T, tab, S, P, N, dt, "f16", False, 42, "split-sensor kernel, interleaved table")


def test_windowed_kernel_past_the_split_sensor_limit(ctx, orc):
    # 4 x (2^26 + 3) columns with 64-sample records: too short for the
    # wave-window kernel and past the split-sensor kernel's offsets
    S, P, N, dt = 4, (1 << 26) + 3, 64, 4e-8
    T = device_table(S, P, N, dt, 43)
    check(ctx, orc, T, T, S, P, N, dt, "f32", True, 43, "LDS-windowed kernel")
