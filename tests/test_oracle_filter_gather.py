"""Pins of the oracle's filter b = p - t dp/dt and its back-projection gather
(Section II-C, Eq. BP): polynomial closed forms, convergence to the analytic
filtered pulse, hand-evaluated examples, numpy's own linear interpolation as
brute force, and the focusing of a synthetic point absorber."""
import json
import math
import os

import numpy as np
import pytest

from paper_1501_03869_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_filter_affine_exact(orc):
    # p = alpha + beta t with t0 = 0: the difference quotient is beta at every
    # sample (ends included), so b = alpha everywhere.
    N, dt = 37, 4e-8
    t = np.arange(N) * dt
    alpha, beta = 0.7, -3.1e6
    b = orc.filt(alpha + beta * t, dt, 0.0)
    np.testing.assert_allclose(b, alpha, rtol=0, atol=1e-13)


def test_filter_quadratic_interior(orc):
    # p = alpha + beta t + gamma t^2: the central difference is exact for a
    # quadratic, so b = alpha - gamma t^2 inside; the one-sided ends are off by
    # gamma t dt.
    N, dt, t0 = 50, 2e-8, 3e-7
    t = t0 + np.arange(N) * dt
    alpha, beta, gamma = 1.3, 2e6, -4e12
    b = orc.filt(alpha + beta * t + gamma * t * t, dt, t0)
    np.testing.assert_allclose(b[1:-1], alpha - gamma * t[1:-1] ** 2, rtol=1e-9, atol=1e-12)
    assert b[0] == pytest.approx(alpha - gamma * t[0] ** 2 - gamma * t[0] * dt, rel=1e-8)
    assert b[-1] == pytest.approx(alpha - gamma * t[-1] ** 2 + gamma * t[-1] * dt, rel=1e-8)


def test_filter_converges_second_order(orc):
    # analytic N-pulse p(t) = -(tau/s) exp(1/2 - tau^2/(2 s^2)); its exact
    # filtered form is p - t p'.  The sampled filter must converge as dt^2.
    s, tc, T = 50e-9, 1.0e-6, 2.0e-6

    def pulse(t):
        tau = t - tc
        return -(tau / s) * np.exp(0.5 - tau * tau / (2 * s * s))

    def dpulse(t):
        tau = t - tc
        return -(1.0 / s) * (1 - tau * tau / (s * s)) * np.exp(0.5 - tau * tau / (2 * s * s))

    errs = []
    for dt in (10e-9, 5e-9, 2.5e-9, 1.25e-9):
        N = int(round(T / dt)) + 1
        t = np.arange(N) * dt
        b = orc.filt(pulse(t), dt, 0.0)
        exact = pulse(t) - t * dpulse(t)
        errs.append(np.abs(b - exact)[1:-1].max() / np.abs(exact).max())
    for a, c in zip(errs, errs[1:]):
        assert 3.6 < a / c < 4.4


def test_gather_hand_examples(orc):
    g = json.load(open(os.path.join(GOLD, "gather_hand_examples.json")))
    b = np.array(g["b"])[None, :]
    T = np.array([[float(c["T"]) for c in g["cases"]]])
    img = orc.gather(T.reshape(1, -1), b, g["dt"], g["t0"])
    for k, c in enumerate(g["cases"]):
        assert img[k] == pytest.approx(c["value"], rel=1e-12, abs=1e-15), c["why"]


def test_gather_affine_closed_form(orc):
    # if every sensor's signal is affine in time, linear interpolation is exact:
    # img[p] = sum_s w_s (u_s + v_s T[s][p]) over in-range delays.
    rng = np.random.default_rng(3)
    S, P, N, dt, t0 = 7, 300, 64, 5e-8, 1e-7
    u, v = rng.normal(size=S), rng.normal(size=S) * 1e6
    t = t0 + np.arange(N) * dt
    b = u[:, None] + v[:, None] * t[None, :]
    w = rng.uniform(0.5, 2.0, size=S)
    T = inputs.random_table(5, S, P, N, dt, t0, frac_out=0.2).astype(np.float64)
    inr = np.isfinite(T) & (T >= t0) & (T <= t0 + (N - 1) * dt)
    expect = np.where(inr, w[:, None] * (u[:, None] + v[:, None] * np.where(inr, T, 0)), 0).sum(0)
    img = orc.gather(T, b, dt, t0, w)
    np.testing.assert_allclose(img, expect, rtol=1e-12, atol=1e-12)


def test_gather_matches_numpy_interp(orc):
    # brute force: numpy's piecewise-linear interpolation, zero outside the record
    rng = np.random.default_rng(4)
    S, P, N, F, dt, t0 = 5, 97, 33, 3, 1e-7, -2e-7
    b = rng.normal(size=(F, S, N))
    w = rng.normal(size=S)
    T = inputs.random_table(9, S, P, N, dt, t0, frac_out=0.3).astype(np.float64)
    T[0, :4] = t0 + np.array([0, N - 1, 0.5, N - 1.5]) * dt  # both ends exactly
    img = orc.gather(T, b, dt, t0, w)
    ref = np.zeros((F, P))
    grid = t0 + np.arange(N) * dt
    for f in range(F):
        for s in range(S):
            x = T[s]
            val = np.interp(np.where(np.isfinite(x), x, 0.0), grid, b[f, s], left=0.0, right=0.0)
            val = np.where(np.isfinite(x) & (x >= grid[0]) & (x <= grid[-1]), val, 0.0)
            ref[f] += w[s] * val
    np.testing.assert_allclose(img, ref, rtol=1e-9, atol=1e-12)
    # a single frame gives the same as the batch
    np.testing.assert_array_equal(orc.gather(T, b[1], dt, t0, w), img[1])
    # thread count never changes the (sensor-ordered) sum
    np.testing.assert_array_equal(orc.gather(T, b, dt, t0, w, nthreads=1), img)


def test_q16_encoding(orc):
    # exactly representable delays: q = u * 65536 exactly; q >> 16 is the sample
    # and the low half the fraction; out-of-range and non-finite map to the sentinel.
    dt, N = 2.0 ** -24, 150
    t0 = 16 * dt  # (16 + u) * 2^16 < 2^24: every delay below is exact in float32
    rng = np.random.default_rng(5)
    qn = rng.integers(0, (N - 1) * 65536 + 1, size=1000).astype(np.uint64)
    T = (t0 + qn.astype(np.float64) / 65536.0 * dt).astype(np.float32)
    assert np.array_equal(T.astype(np.float64), t0 + qn / 65536.0 * dt)  # exact in float32
    q = orc.table_to_q16(T.reshape(10, 100), dt, N, t0).ravel()
    assert np.array_equal(q.astype(np.uint64), qn)
    bad = np.array([t0 - dt * 1e-3, t0 + (N - 1 + 1e-3) * dt, np.inf, -np.inf, np.nan], np.float32)
    assert np.all(orc.table_to_q16(bad[None, :], dt, N, t0) == 0xFFFFFFFF)
    # general delays: quantisation error at most half an LSB (2^-17 sample)
    T2 = inputs.random_table(6, 4, 500, 4096, 25e-9)
    q2 = orc.table_to_q16(T2, 25e-9, 4096)
    u = T2.astype(np.float64) / 25e-9
    assert np.abs(q2 / 65536.0 - u).max() <= 2.0 ** -17 * (1 + 1e-9)
    # the 16.16 gather equals the seconds gather on exactly representable delays
    b = rng.normal(size=(1, N))
    Tq = T[None, :]
    np.testing.assert_allclose(orc.gather_q16(q[None, :], b), orc.gather(Tq, b, dt, t0), rtol=1e-13, atol=1e-13)


def test_point_absorbers_focus(orc):
    # End to end on the small annulus geometry: signals synthesised from 8 point
    # absorbers at the oracle's own travel times.  At an absorber every sensor
    # reads the filtered pulse at its zero crossing, where b = t A e^(1/2)/(s sqrt r)
    # > 0, so the image peaks there and its value is close to that coherent sum.
    # Sampled at 10 ns (5 samples per pulse width) so the difference quotient
    # resolves the pulse.
    geo = inputs.config("small")
    sub = geo.sensors[::2]  # 32 sensors keep this quick
    dt, N = 10e-9, 5120
    T = orc.tables(geo.speed, geo.h, sub, geo.pix)
    nodes, amp = inputs.point_absorbers(inputs.SEED_PHANTOM, geo.nx, geo.ny, geo.h)
    dist = inputs.source_distances(inputs.Geometry(geo.name, geo.nx, geo.ny, geo.h, geo.speed, sub, geo.pix,
                                                   N, dt), nodes)
    p = inputs.npulse_signals(T[:, nodes], amp, dist, N, dt)
    img = orc.backproject(T, p, dt).reshape(geo.ny, geo.nx)
    others = np.zeros(geo.nx * geo.ny, bool)
    others[nodes] = True
    others = others.reshape(geo.ny, geo.nx)
    sig = inputs.PULSE_SIGMA
    for q, (k, a) in enumerate(zip(nodes, amp)):
        j, i = divmod(int(k), geo.nx)
        sl = (slice(max(j - 2, 0), j + 3), slice(max(i - 2, 0), i + 3))
        patch = np.where(others[sl], -np.inf, img[sl])
        assert img[j, i] > patch.max()
        coherent = (T[:, k] * a * math.exp(0.5) / (sig * np.sqrt(dist[:, q] * 1e3))).sum()
        assert img[j, i] == pytest.approx(coherent, rel=0.1)
    # a flipped filter sign (b = p + t dp/dt) would make these peaks negative
    assert img.ravel()[nodes].min() > 0
