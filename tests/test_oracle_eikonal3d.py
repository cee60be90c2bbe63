"""Pins of the 3-D eikonal oracle (6-neighbour first-order Godunov fast
marching) against facts that do not come from the oracle itself: the 2-D
oracle on a one-layer grid, exact straight rays along axes, a plane wave's
prefix sum, Dijkstra bounds from scipy, symmetry, convergence to |x - s| / c
and the update's own quadratic at every node."""
import math

import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import dijkstra

from paper_1501_03869_amd import inputs


def _grid_graph3(slow, h, scale):
    nz, ny, nx = slow.shape
    n = slow.size
    idx = np.arange(n).reshape(nz, ny, nx)
    rows, cols, w = [], [], []
    for ax in range(3):
        a = np.take(idx, np.arange(idx.shape[ax] - 1), axis=ax).ravel()
        b = np.take(idx, np.arange(1, idx.shape[ax]), axis=ax).ravel()
        fa, fb = slow.ravel()[a], slow.ravel()[b]
        # an edge into node m costs scale * f_m * h (the update's own step)
        rows += [a, b]
        cols += [b, a]
        w += [scale * fb * h, scale * fa * h]
    return coo_matrix((np.concatenate(w), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n)).tocsr()


def _godunov3_textbook(a, b, c, fh):
    """Largest root of sum over the upwind sides of (T - v)^2 = fh^2, taking
    sides in increasing order while the root stays above the next value."""
    v = sorted([a, b, c])
    if math.isinf(v[0]):
        return math.inf
    for k in (1, 2, 3):
        vs = v[:k]
        if any(math.isinf(x) for x in vs):
            break
        s1, s2 = sum(vs), sum(x * x for x in vs)
        disc = s1 * s1 - k * (s2 - fh * fh)
        t = (s1 + math.sqrt(max(disc, 0.0))) / k
        if k == 3 or t <= v[k]:
            return t
    return v[0] + fh


def test_single_layer_equals_2d_oracle(orc):
    # nz = 1: every z-neighbour is missing, so the 3-D marcher must reproduce
    # the (separately pinned) 2-D marcher bit for bit
    rng = np.random.default_rng(5)
    speed2 = rng.uniform(1400.0, 3000.0, size=(23, 31))
    slow2 = 1.0 / speed2
    h = 1e-4
    fr2, T02 = orc.seed(slow2, h, 2.3e-4, -3.1e-4)
    T2, _ = orc.fmm(slow2, fr2, T02, h)
    fr3, T03 = orc.seed3(slow2[None], h, 2.3e-4, -3.1e-4, 0.0)
    assert np.array_equal(fr3[0], fr2)
    T3, _ = orc.fmm3(slow2[None], fr3, T03, h)
    assert np.array_equal(T3[0], T2)


def test_axes_are_exact_and_symmetric(orc):
    # homogeneous cube, source on the centre node: along each axis the update
    # is one-sided, so T = distance * f exactly; the map is invariant under
    # permutations of the axes bit for bit, and under mirror images to the
    # last bits (heap ties are broken by index, which a mirror reverses, so a
    # node may keep a few-ulp-smaller value from an earlier partial update)
    n, h, c = 17, 1e-3, 1500.0
    speed = np.full((n, n, n), c)
    T = orc.travel_time_map3(speed, h, 0.0, 0.0, 0.0)
    m = n // 2
    for k in range(n):
        d = abs(k - m) * h / c
        assert T[m, m, k] == pytest.approx(d, rel=1e-15, abs=1e-20)
        assert T[m, k, m] == T[m, m, k] and T[k, m, m] == T[m, m, k]
    for perm in [(0, 2, 1), (1, 0, 2), (2, 1, 0), (1, 2, 0)]:
        assert np.array_equal(np.transpose(T, perm), T)
    for M in (T[::-1], T[:, ::-1], T[:, :, ::-1]):
        np.testing.assert_allclose(M, T, rtol=1e-15, atol=0)


def test_plane_wave_prefix_sum(orc):
    # a frozen plane z = 0 in a medium that varies with z only: T(l) is the
    # prefix sum of f(l') h over the layers above it
    nz, ny, nx, h = 13, 6, 7, 2e-4
    cz = np.linspace(1400.0, 2900.0, nz)
    speed = np.broadcast_to(cz[:, None, None], (nz, ny, nx)).copy()
    slow = 1.0 / speed
    fr = np.zeros((nz, ny, nx), bool)
    fr[0] = True
    T0 = np.zeros((nz, ny, nx))
    T, _ = orc.fmm3(slow, fr, T0, h)
    expect = np.concatenate([[0.0], np.cumsum(h / cz[1:])])
    for l in range(nz):
        assert np.allclose(T[l], expect[l], rtol=1e-14, atol=0)


def test_dijkstra_bounds_and_quadratic(orc):
    # random medium: Dijkstra with steps f h / sqrt(3) <= T <= Dijkstra with
    # steps f h (the update's increment lies in [f h / sqrt(3), f h]); every
    # non-frozen node satisfies the Godunov quadratic of its final neighbours
    rng = np.random.default_rng(9)
    nz, ny, nx, h = 9, 11, 10, 1e-4
    speed = rng.uniform(1400.0, 3000.0, size=(nz, ny, nx))
    slow = 1.0 / speed
    fr, T0 = orc.seed3(slow, h, 1.1e-4, -0.7e-4, 0.3e-4)
    T, pops = orc.fmm3(slow, fr, T0, h)
    assert pops == slow.size - fr.sum()
    src = np.flatnonzero(fr.ravel())
    up = dijkstra(_grid_graph3(slow, h, 1.0), indices=src, min_only=True) + 0.0
    lo = dijkstra(_grid_graph3(slow, h, 1.0 / math.sqrt(3.0)), indices=src, min_only=True)
    # Dijkstra distances start from 0 at the frozen nodes; add the largest
    # frozen value to the upper bound, nothing to the lower one
    assert np.all(T.ravel() <= up + T0[fr].max() * (1 + 1e-12) + 1e-18)
    assert np.all(T.ravel() >= lo - 1e-18)
    for k in np.flatnonzero(~fr.ravel()):
        l, j, i = np.unravel_index(k, T.shape)

        def nb(ll, jj, ii):
            if 0 <= ll < nz and 0 <= jj < ny and 0 <= ii < nx and T[ll, jj, ii] < T[l, j, i]:
                return T[ll, jj, ii]
            return math.inf
        a = min(nb(l, j, i - 1), nb(l, j, i + 1))
        b = min(nb(l, j - 1, i), nb(l, j + 1, i))
        c = min(nb(l - 1, j, i), nb(l + 1, j, i))
        assert T[l, j, i] == pytest.approx(_godunov3_textbook(a, b, c, slow[l, j, i] * h), rel=1e-12)


def test_homogeneous_converges_to_straight_rays(orc):
    # first-order scheme: the error against |x - s| / c on the same physical
    # cube shrinks as h halves
    L, c = 4e-3, 1500.0
    errs = []
    for n in (11, 21, 41):
        h = L / (n - 1)
        T = orc.travel_time_map3(np.full((n, n, n), c), h, 0.0, 0.0, 0.0)
        x, y, z = inputs.node_coords3(n, n, n, h)
        exact = np.sqrt(z[:, None, None] ** 2 + y[None, :, None] ** 2 + x[None, None, :] ** 2) / c
        far = exact > 1e-3 / c
        rel = np.abs(T - exact)[far] / exact[far]
        errs.append((rel.max(), rel.mean()))
    # measured: max 12.6 / 12.2 / 9.2 %, mean 8.6 / 6.8 / 4.7 % (the
    # first-order scheme's error is largest on the diagonals near the source)
    assert errs[0][0] > errs[1][0] > errs[2][0] and errs[0][1] > errs[1][1] > errs[2][1]
    assert errs[2][0] < 0.1 and errs[2][1] < 0.05


def test_tables3_match_maps_and_reject(orc):
    geo = inputs.config3("tiny3")
    T = orc.tables3(geo.speed, geo.h, geo.sensors, geo.pix)
    for s in (0, 3):
        m = orc.travel_time_map3(geo.speed, geo.h, *geo.sensors[s])
        assert np.array_equal(T[s], m.ravel()[geo.pix])
    with pytest.raises(ValueError):
        orc.tables3(geo.speed, geo.h, np.array([[1.0, 0.0, 0.0]]), geo.pix)
    with pytest.raises(ValueError):
        orc.tables3(geo.speed, geo.h, geo.sensors, np.array([geo.speed.size], np.int32))


def test_const3_straight_rays(orc):
    # the conventional back projection's 3-D straight-ray table: a one-layer
    # grid gives the (pinned) 2-D straight-ray table bit for bit, exchanging
    # axes permutes it, and the fast-marching table of a homogeneous cube lies
    # above it within the first-order scheme's error
    n, h, c = 21, 0.3e-3, 1500.0
    x, y, z = inputs.node_coords3(n, n, n, h)
    rng = np.random.default_rng(12)
    sens = np.stack([rng.uniform(x[0], x[-1], 3), rng.uniform(y[0], y[-1], 3), rng.uniform(z[0], z[-1], 3)], 1)
    vox = rng.permutation(n ** 3)[:2000].astype(np.int32)
    T = orc.tables_const3(n, n, n, h, c, sens, vox)
    # one layer
    x2, y2 = inputs.node_coords(n, 17, h)
    s2 = np.stack([rng.uniform(x2[0], x2[-1], 4), rng.uniform(y2[0], y2[-1], 4)], 1)
    pix = np.arange(n * 17, dtype=np.int32)
    T2 = orc.tables_const(n, 17, h, c, s2, pix)
    T1 = orc.tables_const3(n, 17, 1, h, c, np.concatenate([s2, np.zeros((4, 1))], 1), pix)
    assert np.array_equal(T1, T2)
    # axis exchange x <-> z: node (i, j, l) -> (l, j, i), sensor (sx, sy, sz) -> (sz, sy, sx)
    i, j, l = vox % n, (vox // n) % n, vox // (n * n)
    Tp = orc.tables_const3(n, n, n, h, c, sens[:, ::-1].copy(), (i * n + j) * n + l)
    np.testing.assert_allclose(Tp, T, rtol=1e-15, atol=0)
    # homogeneous fast marching from nodes (sensors snapped to nodes)
    snap = np.stack([x[np.abs(x[:, None] - sens[:, 0]).argmin(0)], y[np.abs(y[:, None] - sens[:, 1]).argmin(0)],
                     z[np.abs(z[:, None] - sens[:, 2]).argmin(0)]], 1)
    Ts = orc.tables_const3(n, n, n, h, c, snap, vox)
    Fm = orc.tables3(np.full((n, n, n), c, np.float32), h, snap, vox)
    far = Ts > 5 * h / c
    assert np.all(Fm >= Ts * (1 - 1e-12))
    assert ((Fm - Ts)[far] / Ts[far]).max() < 0.15
    with pytest.raises(ValueError):
        orc.tables_const3(n, n, n, h, -1.0, sens, vox)
    with pytest.raises(ValueError):
        orc.tables_const3(n, n, n, h, c, sens, np.array([n ** 3], np.int32))
