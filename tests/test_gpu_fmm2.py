"""Second-order fast-marching tables on the GPU (the paper's scheme, one
map per wave in heap order, FP64) against the oracle's second-order
marcher: the float32 tables are the oracle's times rounded once."""
import numpy as np
import pytest
import torch

from paper_1501_03869_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1501_03869_amd import pat
    c = pat.Context(0)
    yield c
    c.close()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _compare(ctx, orc, speed, h, sens, pix, label):
    got = ctx.eikonal_tables_o2(dev(speed), h, sens, dev(pix))
    torch.cuda.synchronize()
    st = ctx.eikonal_stats()
    got = got.cpu().numpy()
    ref = orc.tables2(speed, h, sens, pix)
    ref32 = ref.astype(np.float32)
    same = float(np.mean(got == ref32))
    rel = float((np.abs(got.astype(np.float64) - ref)[ref > 0] / ref[ref > 0]).max())
    print(f"[fmm2] {label}: S={len(sens)} P={len(pix)} equal to the rounded oracle times: {same:.6f}, "
          f"max rel {rel:.3e}, {st['seconds']:.3f} s", flush=True)
    assert np.all(got[ref == 0] == 0)
    assert rel <= 1e-7
    assert same == 1.0


@pytest.mark.parametrize("name", ["tiny", "small", "paper"])
def test_tables_o2_match_oracle(ctx, orc, name):
    geo = inputs.config(name)
    _compare(ctx, orc, geo.speed, geo.h, geo.sensors, geo.pix, name)


def test_tables_o2_ragged_random_medium(ctx, orc):
    rng = np.random.default_rng(44)
    nx, ny, h = 45, 70, 0.3e-3
    c = rng.uniform(1400, 3200, size=(ny, nx)).astype(np.float32)
    x, y = inputs.node_coords(nx, ny, h)
    sens = np.array([[x[0], y[0]], [x[-1], y[-1]], [x[-1], y[0]], [0.0, 0.0], [x[3] + 0.37 * h, y[40] - 0.2 * h],
                     [x[-1], 0.1 * h], [x[1], y[1]]])
    pix = rng.permutation(nx * ny)[: nx * ny - 17].astype(np.int32)
    _compare(ctx, orc, c, h, sens, pix, "ragged")


def test_tables_o2_closer_to_straight_rays(ctx, orc):
    # homogeneous medium: the second-order times lie closer to |x - s| / c
    # than the first-order ones (GPU tables of both schemes)
    n, h, c = 129, 0.1e-3, 1500.0
    speed = np.full((n, n), c, np.float32)
    x, y = inputs.node_coords(n, n, h)
    sens = np.array([[x[5], y[60]], [0.0, 0.0], [x[100], y[17]]])
    pix = np.arange(n * n, dtype=np.int32)
    t2 = ctx.eikonal_tables_o2(dev(speed), h, sens, dev(pix)).cpu().numpy().astype(np.float64)
    t1 = ctx.eikonal_tables(dev(speed), h, sens, dev(pix)).cpu().numpy().astype(np.float64)
    X, Y = x[pix % n], y[pix // n]
    for s in range(len(sens)):
        exact = np.hypot(X - sens[s, 0], Y - sens[s, 1]) / c
        far = exact > 5 * h / c
        e1 = float((np.abs(t1[s] - exact)[far] / exact[far]).mean())
        e2 = float((np.abs(t2[s] - exact)[far] / exact[far]).mean())
        print(f"[fmm2] sensor {s}: mean rel error first order {e1:.3e}, second order {e2:.3e}", flush=True)
        assert e2 < 0.5 * e1


def test_tables_o2_rejects_bad_input(ctx):
    from paper_1501_03869_amd import pat
    geo = inputs.config("tiny")
    bad = geo.speed.copy()
    bad[1, 1] = np.nan
    with pytest.raises(pat.PatError):
        ctx.eikonal_tables_o2(dev(bad), geo.h, geo.sensors, dev(geo.pix))
    with pytest.raises(pat.PatError):
        ctx.eikonal_tables_o2(dev(geo.speed), geo.h, geo.sensors * 10, dev(geo.pix))
    with pytest.raises(pat.PatError):
        ctx.eikonal_tables_o2(dev(geo.speed), geo.h, geo.sensors, dev(np.array([geo.speed.size], np.int32)))


@pytest.mark.parametrize("entries,name", [(0, "tiny"), (8, "tiny"), (300, "small")])
def test_trial_set_in_device_memory(ctx, orc, entries, name, monkeypatch):
    # the trial set of a map lives in LDS up to a capacity and in device
    # memory beyond it; the paper geometry's sets (a few hundred entries)
    # stay in LDS, so lower the capacity to run the device-memory part (all
    # of it, most of it, and the largest sets of the 128^2 geometry, about
    # 340 entries, just past it): the tables must not change
    monkeypatch.setenv("PAT_FMM2_LDS_ENTRIES", str(entries))
    geo = inputs.config(name)
    _compare(ctx, orc, geo.speed, geo.h, geo.sensors, geo.pix, f"{name}, {entries} trial entries in LDS")
