// The first-order upwind (Godunov) update of the travel-time tables
// (Section II-B), exact in integer arithmetic on uint32 fixed-point times.
//
// With the upwind neighbour minima n_k along each axis and the node's
// slowness times the grid step in whole fixed-point units,
// F = round(h / (c lsb)), the continuous update solves
// sum_k max(T - n_k, 0)^2 = F^2.  Here T is that root rounded to the nearest
// unit (halves up), which is the largest integer T with
//   G(T) = sum_k max(2 (T - n_k) - 1, 0)^2  <=  4 F^2,
// since G is increasing in T.  G falls when a neighbour rises, so the update
// is monotone in every neighbour: raising one never lowers the result.
// Relaxation that only lowers values, started from "not reached", therefore
// ends at the greatest fixed point of the update whatever the order of the
// node updates, and the tables do not depend on the workgroup schedule.
//
// The roots are closed forms in integer square roots (a <= b <= c the sorted
// neighbours, d = b - a, e = c - a):
//   one-sided    a + F                                         if a + F <= b,
//   two-sided    a + floor((d + 1 + isqrt(2F^2 - d^2)) / 2)     if that is <= c,
//   three-sided  max(c, a + floor((2 (d + e) + 3 + isqrt(4w)) / 6)),
//                w = (d + e)^2 - 3 (d^2 + e^2 - F^2),
// each the largest T allowed by the terms active at it: a square root in
// [r, r + 1) (or 2 sqrt(w) in [r, r + 1)) leaves the floor's argument in an
// interval with no integer inside.  F <= 2^23 keeps every square below 2^52.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pat_eik {

constexpr uint32_t EIK_INF = 0xFFFFFFFFu;

// floor(sqrt(z)) from an estimate r within 16 of it (r, z < 2^52) and
// z_lo = z mod 2^32: the residual z - r^2 is then below 2^31 in magnitude, so
// 32-bit wrapping arithmetic gives it exactly, and each step moves r by one
// while keeping it (r^2 needs only its low 32 bits).  R24: r < 2^24, whose
// estimates here are usually within a unit.  Otherwise (roots up to 2^25,
// estimates off by up to about ten) one Newton step on the exact residual,
// r + floor(res / (2r + 1)), first brings r within a unit.  One step down and
// one up are then taken as selects, and the loops run only where a lane is
// still off.
template <bool R24>
__device__ __forceinline__ uint32_t isqrt_fix(uint32_t z_lo, uint32_t r) {
    auto sq = [](uint32_t x) { return R24 ? __umul24(x, x) : x * x; };
    int32_t res = (int32_t)(z_lo - sq(r));
    if constexpr (!R24) {
        r += (uint32_t)(int32_t)floorf((float)res * __builtin_amdgcn_rcpf((float)(2u * r + 1u)));
        res = (int32_t)(z_lo - sq(r));
    }
    const bool dn = res < 0 && r > 0;
    r -= dn ? 1u : 0u;
    res += dn ? 2 * (int32_t)r + 1 : 0;
    const bool up = res > 2 * (int32_t)r;
    res -= up ? 2 * (int32_t)r + 1 : 0;
    r += up ? 1u : 0u;
    if (res < 0 || res > 2 * (int32_t)r) {
        while (res < 0 && r > 0) {
            --r;
            res += 2 * (int32_t)r + 1;
        }
        while (res > 2 * (int32_t)r) {
            ++r;
            res -= 2 * (int32_t)r - 1;
        }
    }
    return r;
}

// 2F^2 and 3F^2 as floats, the estimates' constants per node
__device__ __forceinline__ float eik_f2(uint32_t F) {
    const float f = (float)F;
    return 2.0f * f * f;
}
__device__ __forceinline__ float eik_f3(uint32_t F) {
    const float f = (float)F;
    return 3.0f * f * f;
}

// 2-D: a, b the upwind minima along x and y; F2 = 2F^2 as a float (exact
// while 2F^2 < 2^24, else within a relative 2^-24), kept per node by the
// caller.
// z = 2F^2 - d^2 lies in [F^2, 2F^2] for the two-sided root, its float
// estimate is within a relative 2^-23 and the hardware square root within a
// unit of the last place, so the estimate of isqrt(z) < 2^24 is within a few
// units.  Without branches: the two-sided root is evaluated for every node
// and selected, so that a wave does not split between the cases.
__device__ __forceinline__ uint32_t godunov2_int(uint32_t a, uint32_t b, uint32_t F, float F2) {
    const uint32_t m = min(a, b), M = max(a, b);
    const uint32_t d = M - m;
    const bool two = M != EIK_INF && d < F;
    const uint32_t dc = two ? d : 0u;
    const uint32_t z_lo = 2u * __umul24(F, F) - __umul24(dc, dc);
    const float fd = (float)dc;
    const uint32_t r = isqrt_fix<true>(z_lo, (uint32_t)__builtin_amdgcn_sqrtf(fmaf(-fd, fd, F2)));
    const uint32_t inc = two ? (dc + 1u + r) >> 1 : F;
    // m + inc, held below "not reached"
    const uint32_t t = m + inc;
    const uint32_t sat = t < m ? EIK_INF - 1 : min(t, EIK_INF - 1);
    return m == EIK_INF ? EIK_INF : sat;
}

// 3-D: a, b, c the upwind minima along x, y and z, F2 and F3 = 2F^2 and
// 3F^2 as floats.  Where the three-axis root applies, d <= e < F, so its
// discriminant w = 3F^2 - d^2 - e^2 - (e - d)^2 (the form above, rewritten)
// is at least F^2: the float estimate of 4w is within a relative 2^-21 and
// that of isqrt(4w) < 2^25 within a few units.  The one- and two-axis roots
// are selected as in 2-D; the three-axis root is taken only by the lanes
// that need it.
__device__ __forceinline__ uint32_t godunov3_int(uint32_t a, uint32_t b, uint32_t c, uint32_t F, float F2,
                                                 float F3) {
    uint32_t t;
    t = min(a, b); b = max(a, b); a = t;
    t = min(b, c); c = max(b, c); b = t;
    t = min(a, b); b = max(a, b); a = t;
    const uint32_t d = b - a, e = c - a;
    const bool two = b != EIK_INF && d < F;
    const uint32_t dc = two ? d : 0u;
    const uint32_t z_lo = 2u * __umul24(F, F) - __umul24(dc, dc);
    const float fd = (float)dc;
    const uint32_t r2 = isqrt_fix<true>(z_lo, (uint32_t)__builtin_amdgcn_sqrtf(fmaf(-fd, fd, F2)));
    const uint32_t inc2 = (dc + 1u + r2) >> 1;
    // the two-sided root passes c: then e < inc2 <= F
    const bool three = two && c != EIK_INF && inc2 > e;
    uint32_t inc = two ? inc2 : F;
    if (three) {
        const uint32_t g = e - dc;
        const uint32_t w4_lo = 4u * (3u * __umul24(F, F) - __umul24(dc, dc) - __umul24(e, e) - __umul24(g, g));
        const float fe = (float)e, fg = (float)g;
        const float w4_est = 4.0f * fmaf(-fg, fg, fmaf(-fe, fe, fmaf(-fd, fd, F3)));
        const uint32_t r3 = isqrt_fix<false>(w4_lo, (uint32_t)__builtin_amdgcn_sqrtf(w4_est));
        inc = max(e, (2u * (dc + e) + 3u + r3) / 6u);
    }
    const uint32_t s = a + inc;
    const uint32_t sat = s < a ? EIK_INF - 1 : min(s, EIK_INF - 1);
    return a == EIK_INF ? EIK_INF : sat;
}

}  // namespace pat_eik
