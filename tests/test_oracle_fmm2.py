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
