"""Pins of the oracle's second-order fast marching (the paper's scheme,
Section II-B, after Sethian): with first-order updates it is the (pinned)
first-order marcher bit for bit; a quadratic arrival-time field with an
exact two-node boundary band is reproduced exactly (second-order one-sided
differences are exact on quadratics, first-order ones only on linear fields);
a point source
converges to straight rays faster than with the first-order update; and a
transposed problem gives the transposed map."""
import math

import numpy as np
import pytest

from paper_1501_03869_amd import inputs


def test_order1_is_first_order_marcher(orc):
    rng = np.random.default_rng(3)
    for shape in ((23, 31), (40, 17)):
        slow = 1.0 / rng.uniform(1400.0, 3000.0, size=shape)
        fr, T0 = orc.seed(slow, 1e-4, 0.3e-4, -0.2e-4)
        T1, p1 = orc.fmm(slow, fr, T0, 1e-4)
        T2, p2 = orc.fmm2(slow, fr, T0, 1e-4, order=1)
        assert np.array_equal(T1, T2) and p1 == p2


def _quadratic_front(n, h, c0, a, b, g):
    # T = (a x + b y + g (x^2 + y^2)) / c0 from the lower-left corner (x, y >= 0),
    # an arrival-time field whose slowness |grad T| is sampled at the nodes;
    # its gradient points into the grid, so the upwind nodes of every node are
    # those at -x and -y.  The first two rows and columns are frozen at the
    # exact values.
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x)
    exact = (a * X + b * Y + g * (X * X + Y * Y)) / c0
    slow = np.hypot(a + 2 * g * X, b + 2 * g * Y) / c0
    fr = np.zeros((n, n), bool)
    fr[:2, :] = True
    fr[:, :2] = True
    return exact, slow, fr


def test_quadratic_front_exact_to_second_order(orc):
    # second-order one-sided differences are exact on quadratics, so the
    # marcher reproduces a quadratic arrival-time field to rounding; the
    # first-order update is exact only on linear fields
    n, h, c0 = 41, 0.25e-3, 1500.0
    for a, b, g in ((1.0, 0.0, 0.0), (0.8, 0.6, 0.0), (1.0, 0.3, 40.0), (0.2, 1.0, 25.0), (0.6, 0.6, 60.0)):
        exact, slow, fr = _quadratic_front(n, h, c0, a, b, g)
        T2, _ = orc.fmm2(slow, fr, np.where(fr, exact, np.inf), h, order=2)
        T1, _ = orc.fmm2(slow, fr, np.where(fr, exact, np.inf), h, order=1)
        err2 = np.abs(T2 - exact).max() / exact.max()
        err1 = np.abs(T1 - exact).max() / exact.max()
        assert err2 < 1e-12, (a, b, g, err2)
        if g > 0:
            assert err1 > 1e-4, (a, b, g, err1)


def test_point_source_converges_faster_than_first_order(orc):
    L, c = 6e-3, 1500.0
    errs = {1: [], 2: []}
    for n in (31, 61, 121):
        h = L / (n - 1)
        slow = np.full((n, n), 1.0 / c)
        fr, T0 = orc.seed(slow, h, 0.0, 0.0)
        x, y = inputs.node_coords(n, n, h)
        exact = np.hypot(x[None, :], y[:, None]) / c
        far = exact > 1e-3 / c
        for order in (1, 2):
            T, _ = orc.fmm2(slow, fr, T0, h, order=order)
            errs[order].append(float((np.abs(T - exact)[far] / exact[far]).mean()))
    assert errs[2][0] > errs[2][1] > errs[2][2]
    assert all(e2 < e1 for e1, e2 in zip(errs[1], errs[2]))
    # halving h shrinks the second-order error by more than the first-order one
    assert errs[2][2] / errs[2][1] < errs[1][2] / errs[1][1]


def test_transpose(orc):
    rng = np.random.default_rng(5)
    speed = rng.uniform(1400.0, 3000.0, size=(29, 29))
    slow = 1.0 / speed
    fr, T0 = orc.seed(slow, 1e-4, 0.37e-4, -0.81e-4)
    T, _ = orc.fmm2(slow, fr, T0, 1e-4)
    frt, T0t = orc.seed(slow.T.copy(), 1e-4, -0.81e-4, 0.37e-4)
    Tt, _ = orc.fmm2(slow.T.copy(), frt, T0t, 1e-4)
    np.testing.assert_allclose(Tt.T, T, rtol=1e-13, atol=0)


def test_tables2_are_maps(orc):
    geo = inputs.config("tiny")
    T = orc.tables2(geo.speed, geo.h, geo.sensors, geo.pix)
    slow = 1.0 / geo.speed.astype(np.float64)
    for s in (0, 2):
        fr, T0 = orc.seed(slow, geo.h, *geo.sensors[s])
        m, _ = orc.fmm2(slow, fr, T0, geo.h)
        assert np.array_equal(T[s], m.ravel()[geo.pix])


# ---------------------------------------------------------------------------
# Hand-worked examples (tests/golden/fmm2_hand_examples.json): every branch of
# the second-order update evaluated by hand from its definition, and a whole
# march traced pop by pop.

def _golden():
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "fmm2_hand_examples.json")) as f:
        return json.load(f)


def test_hand_single_updates(orc):
    g = _golden()["single_update"]
    nx, ny, h = g["nx"], g["ny"], g["h"]
    for case in g["cases"]:
        slow = np.full((ny, nx), g["default_slowness"])
        for i, j, f in case["slowness"]:
            slow[j, i] = f
        fr = np.ones((ny, nx), bool)
        T0 = np.full((ny, nx), g["default_frozen"])
        for i, j, t in case["frozen"]:
            T0[j, i] = t
        for i, j in case["free"]:
            fr[j, i] = False
            T0[j, i] = np.inf
        T, pops = orc.fmm2(slow, fr, T0, h, order=2)
        assert pops == len(case["free"]), case["name"]
        for i, j, t in case["expect"]:
            assert T[j, i] == pytest.approx(t, rel=1e-14), (case["name"], T[j, i], t)
        # frozen nodes keep their values
        assert np.array_equal(T[fr], T0[fr]), case["name"]


def test_hand_march(orc):
    g = _golden()["march"]
    slow = np.array(g["slowness"], dtype=np.float64)
    fr = np.zeros_like(slow, dtype=bool)
    T0 = np.full(slow.shape, np.inf)
    for i, j, t in g["frozen"]:
        fr[j, i] = True
        T0[j, i] = t
    T, pops, acc = orc.fmm2(slow, fr, T0, g["h"], order=2, with_order=True)
    np.testing.assert_allclose(T, np.array(g["expect_T"]), rtol=1e-14, atol=0)
    assert acc.tolist() == g["expect_accept_order"]
    assert pops == slow.size - fr.sum()


# ---------------------------------------------------------------------------
# Replay property: the march is re-run in the oracle's own acceptance order,
# with every candidate update recomputed here from the definition (textbook
# quadratic root in extended precision, both branch conditions written out),
# and checked value by value.  At every pop the accepted node must also be the
# smallest trial node (ties by index), as the heap order requires.

_LD = np.longdouble


def _axis_def(T, known, i, j, di, dj, nx, ny):
    """(c, b) of one axis, or None without an accepted neighbour on it."""
    best = None
    for sgn in (-1, 1):  # on equal values the lower-index side is kept
        ii, jj = i + sgn * di, j + sgn * dj
        if 0 <= ii < nx and 0 <= jj < ny and known[jj, ii]:
            if best is None or T[jj, ii] < best[0]:
                best = (T[jj, ii], sgn)
    if best is None:
        return None, False
    t1, sgn = best
    i2, j2 = i + 2 * sgn * di, j + 2 * sgn * dj
    if 0 <= i2 < nx and 0 <= j2 < ny and known[j2, i2]:
        t2 = T[j2, i2]
        if t2 <= t1:  # ordered: second-order one-sided difference
            return (_LD(9) / 4, (4 * _LD(t1) - _LD(t2)) / 3), False
        return (_LD(1), _LD(t1)), True  # T2 > T1: first order
    return (_LD(1), _LD(t1)), False


def _update_def(T, known, i, j, fh, stats):
    ny, nx = known.shape
    tx, fx = _axis_def(T, known, i, j, 1, 0, nx, ny)
    ty, fy = _axis_def(T, known, i, j, 0, 1, nx, ny)
    stats["t2_gt_t1"] += fx + fy
    terms = [t for t in (tx, ty) if t is not None]
    if not terms:
        return np.inf
    fh = _LD(fh)
    one = [b + fh / np.sqrt(c) for c, b in terms]
    if len(terms) == 2:
        (c1, b1), (c2, b2) = terms
        A = c1 + c2
        B = -2 * (c1 * b1 + c2 * b2)
        C = c1 * b1 * b1 + c2 * b2 * b2 - fh * fh
        disc = B * B - 4 * A * C
        if disc >= 0:
            r = (-B + np.sqrt(disc)) / (2 * A)
            if r >= b1 and r >= b2:
                stats["two_axis"] += 1
                return float(r)
            stats["rejected"] += 1
    return float(min(one))


def _replay(slow, fr, T0, h, T, acc, stats):
    ny, nx = slow.shape
    known = fr.copy()
    cur = np.where(fr, T0, np.inf)
    trial = np.zeros_like(fr)

    def compute(m):
        j, i = divmod(m, nx)
        return _update_def(cur, known, i, j, slow[j, i] * h, stats)

    for m in range(nx * ny):  # nodes next to the frozen set start as trial
        j, i = divmod(m, nx)
        if fr[j, i]:
            continue
        if any(0 <= i + a < nx and 0 <= j + b < ny and fr[j + b, i + a]
               for a, b in ((-1, 0), (1, 0), (0, -1), (0, 1))):
            trial[j, i] = True
            cur[j, i] = compute(m)
    for k in acc:
        j, i = divmod(int(k), nx)
        assert trial[j, i] and not known[j, i]
        # the popped node is the smallest trial value, ties by index
        tv = np.where(trial & ~known, cur, np.inf)
        smaller = (tv < cur[j, i] * (1 - 1e-13))
        assert not smaller.any(), (int(k), cur[j, i], tv.min())
        assert cur[j, i] == pytest.approx(T[j, i], rel=1e-12), (int(k), cur[j, i], T[j, i])
        known[j, i] = True
        for a, b in ((-1, 0), (1, 0), (0, -1), (0, 1)):
            ii, jj = i + a, j + b
            if 0 <= ii < nx and 0 <= jj < ny and not known[jj, ii]:
                t = compute(jj * nx + ii)
                if t < cur[jj, ii]:
                    cur[jj, ii] = t
                    trial[jj, ii] = True
    assert known.all()


def test_replay_point_sources(orc):
    rng = np.random.default_rng(11)
    stats = {"t2_gt_t1": 0, "two_axis": 0, "rejected": 0}
    for shape in ((13, 17), (20, 9), (16, 16)):
        slow = rng.uniform(0.5, 2.0, size=shape)
        ny, nx = shape
        sx, sy = rng.uniform(-0.4 * (nx - 1), 0.4 * (nx - 1)), rng.uniform(-0.4 * (ny - 1), 0.4 * (ny - 1))
        fr, T0 = orc.seed(slow, 1.0, sx, sy)
        fr = fr.astype(bool)
        T, pops, acc = orc.fmm2(slow, fr, T0, 1.0, order=2, with_order=True)
        assert pops == fr.size - fr.sum()
        _replay(slow, fr, T0, 1.0, T, acc, stats)
    assert stats["t2_gt_t1"] > 0 and stats["rejected"] > 0 and stats["two_axis"] > 0, stats


def test_replay_scattered_frozen_values(orc):
    # frozen nodes at random values (not a physical field) drive the update
    # through every branch many times: T2 > T1 fallbacks, rejected two-axis
    # roots and accepted ones
    rng = np.random.default_rng(12)
    stats = {"t2_gt_t1": 0, "two_axis": 0, "rejected": 0}
    for shape in ((12, 14), (17, 10)):
        slow = rng.uniform(0.5, 2.0, size=shape)
        fr = rng.random(shape) < 0.3
        T0 = np.where(fr, rng.uniform(0.0, 6.0, size=shape), np.inf)
        T, pops, acc = orc.fmm2(slow, fr, T0, 1.0, order=2, with_order=True)
        _replay(slow, fr, T0, 1.0, T, acc, stats)
    assert stats["t2_gt_t1"] > 20 and stats["rejected"] > 20 and stats["two_axis"] > 20, stats
