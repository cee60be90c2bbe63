// Device helpers shared by the back-projection kernels: delay decoding for
// both table formats, signal loads for both sample formats, and the UBP
// filter on three neighbouring samples.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include "pat.h"

namespace pat_gather {

struct DelayF32 {
    static constexpr bool kR16 = false;
    static constexpr bool kX4 = false;
    float inv_hi, inv_lo, off;  // u = T * (inv_hi + inv_lo) + off
    float umax;                 // N - 1
    __device__ __forceinline__ bool decode(float T, int N, int &n, float &a) const {
        const float u = fmaf(T, inv_hi, fmaf(T, inv_lo, off));
        if (!(u >= 0.0f && u <= umax)) return false;  // also rejects NaN and inf
        n = min((int)u, N - 2);
        a = u - (float)n;
        return true;
    }
    __device__ __forceinline__ bool decode(uint32_t bits, int N, int &n, float &a) const {
        return decode(__uint_as_float(bits), N, n, a);
    }
    // The same decoding without branches: n and a are computed for every
    // lane (from u clamped to 0 when the delay does not contribute).
    __device__ __forceinline__ bool decode_bf(uint32_t bits, int N, int &n, float &a) const {
        const float T = __uint_as_float(bits);
        const float u = fmaf(T, inv_hi, fmaf(T, inv_lo, off));
        const bool ok = u >= 0.0f && u <= umax;  // also rejects NaN and inf
        const float uc = ok ? u : 0.0f;
        n = min((int)uc, N - 2);
        a = uc - (float)n;
        return ok;
    }
    // The split-sensor kernel's decoding computes u with one FMA,
    // u = T * (1/dt)_f32 - t0/dt: the dropped term T * inv_lo is at most
    // u * 2^-25, about half an ulp of u, so u stays within about 1 ulp.
    __device__ __forceinline__ float u1(float T) const { return fmaf(T, inv_hi, off); }
    // The same decoding without branches (split-sensor kernel, general
    // path): n and a are computed for every lane (from u clamped to 0 when
    // the delay does not contribute).
    __device__ __forceinline__ bool decode_bf1(uint32_t bits, int N, int &n, float &a) const {
        const float u = u1(__uint_as_float(bits));
        const bool ok = u >= 0.0f && u <= umax;  // also rejects NaN and inf
        const float uc = ok ? u : 0.0f;
        n = min((int)uc, N - 2);
        a = uc - (float)n;
        return ok;
    }
    // Fast-path decoding for an integer range lo <= u < hi (lo >= 0): u is
    // clamped to [lo, hi) (median of three against lo and the float just
    // below hi), n = floor and a = fraction of the clamped value, so
    // lo <= n <= hi-1 for every lane and n, a are exact where u lies in the
    // range.  Returns whether it does (the clamp changed nothing; never for
    // NaN or inf).
    __device__ __forceinline__ bool decode_in(uint32_t bits, int lo, int hi, int &n, float &a) const {
        const float u = u1(__uint_as_float(bits));
        const float below_hi = __uint_as_float(__float_as_uint((float)hi) - 1u);
        const float uc = __builtin_amdgcn_fmed3f(u, (float)lo, below_hi);
        n = (int)uc;
        a = uc - (float)n;
        return uc == u;
    }
    // Window-relative, branch-free decoding for an LDS window that starts at
    // sample an: idx = floor(u) - an and a = frac(u) with u' = u - an computed
    // directly (the anchor folds into the offset, so u' keeps more fraction
    // bits than u).  ok: the delay contributes; idx and a are 0 when not ok.
    struct Win { float off, lo, hi; };
    __device__ __forceinline__ Win window(int an) const {
        Win w;
        w.off = off - (float)an;
        w.lo = -(float)an;
        w.hi = umax - (float)an;
        return w;
    }
    __device__ __forceinline__ bool decode_win(uint32_t bits, const Win &w, int &idx, float &a) const {
        const float T = __uint_as_float(bits);
        float u = fmaf(T, inv_hi, fmaf(T, inv_lo, w.off));
        const bool ok = u >= w.lo && u <= w.hi;
        u = ok ? u : 0.0f;
        idx = (int)floorf(u);
        a = u - floorf(u);
        return ok;
    }
};

struct DelayQ16 {
    static constexpr bool kR16 = false;
    static constexpr bool kX4 = false;
    __device__ __forceinline__ bool decode(uint32_t q, int N, int &n, float &a) const {
        if (q == 0xFFFFFFFFu) return false;
        n = (int)(q >> 16);
        a = (float)(q & 0xFFFFu) * (1.0f / 65536.0f);
        if (n > N - 2) {  // only u = N-1 exactly: end of the last interval
            n = N - 2;
            a = 1.0f;
        }
        return true;
    }
    __device__ __forceinline__ bool decode_bf(uint32_t q, int N, int &n, float &a) const {
        const bool ok = q != 0xFFFFFFFFu;
        const int n0 = (int)(q >> 16);
        const bool last = n0 > N - 2;  // only u = N-1 exactly
        n = last ? N - 2 : n0;
        a = last ? 1.0f : (float)(q & 0xFFFFu) * (1.0f / 65536.0f);
        return ok;
    }
    __device__ __forceinline__ bool decode_bf1(uint32_t q, int N, int &n, float &a) const {
        return decode_bf(q, N, n, a);
    }
    __device__ __forceinline__ bool decode_in(uint32_t q, int lo, int hi, int &n, float &a) const {
        const int n0 = (int)(q >> 16);  // the sentinel gives 65535 >= hi
        n = min(max(n0, lo), hi - 1);
        a = (float)(q & 0xFFFFu) * (1.0f / 65536.0f);
        return (uint32_t)(n0 - lo) < (uint32_t)(hi - lo);
    }
    struct Win { int an; };
    __device__ __forceinline__ Win window(int an) const { return Win{ an }; }
    __device__ __forceinline__ bool decode_win(uint32_t q, const Win &w, int &idx, float &a) const {
        const bool ok = q != 0xFFFFFFFFu;
        idx = ok ? (int)(q >> 16) - w.an : 0;
        a = ok ? (float)(q & 0xFFFFu) * (1.0f / 65536.0f) : 0.0f;
        return ok;
    }
};

// Tile-relative 16-bit delays: an offset per entry and a header
// (b << 16) | (16 - k) per sensor and 32-entry tile stand for the 16.16 value
// (b << 16) + (off << (16 - k)); offset 0xFFFF is the sentinel.  Decoding
// then proceeds as for 16.16 tables.
struct DelayR16 : DelayQ16 {
    static constexpr bool kR16 = true;
    __device__ __forceinline__ static uint32_t to_q16(uint32_t off, uint32_t hdr) {
        return off == 0xFFFFu ? 0xFFFFFFFFu : (hdr & 0xFFFF0000u) + (off << (hdr & 31u));
    }
};

// Float32 seconds with four sensors interleaved per ROI position
// (PAT_TABLE_F32X4, [ceil(S/4)][P][4]): decoded as DelayF32; one 16-byte
// load gives a lane the delays of four sensors at its pixel.
struct DelayF32X4 : DelayF32 {
    static constexpr bool kX4 = true;
};

// Workgroups are dealt to the 8 XCDs round-robin by workgroup index, each
// XCD with its own L2.  A tile's table row segment generally straddles cache
// lines shared with the neighbouring tiles, so neighbouring tiles are kept on
// one XCD: launch slot b (8 * ceil(T/8) slots) runs tile x*q + min(x, r) + k
// of the T tiles (x = b % 8, k = b / 8, T = 8q + r), i.e. XCD x takes one
// contiguous run of tiles; -1 for the at most 7 slots with no tile.
__device__ __forceinline__ int xcd_tile(int b, int T) {
    const int q = T >> 3, r = T & 7, x = b & 7, k = b >> 3;
    return k < q + (x < r ? 1 : 0) ? x * q + min(x, r) + k : -1;
}

__host__ __device__ inline int xcd_slots(int T) { return (T + 7) & ~7; }

template <int SFMT>
__device__ __forceinline__ float load_sig(const void *sig, long i, float scale) {
    if constexpr (SFMT == PAT_SIG_F32) {
        return static_cast<const float *>(sig)[i];
    } else {
        return __half2float(static_cast<const __half *>(sig)[i]) * scale;
    }
}

// b[n] = p[n] - (n + t0/dt) * 0.5 * (p[n+1] - p[n-1]); one-sided at both ends.
__device__ __forceinline__ float ubp(float pm, float p0, float pp, int n, int N, float t0dt) {
    float d = pp - pm;
    if (n == 0) d = 2.0f * (pp - p0);
    if (n == N - 1) d = 2.0f * (p0 - pm);
    return p0 - ((float)n + t0dt) * (0.5f * d);
}

template <int SFMT, bool FILTERED>
__device__ __forceinline__ float sample_b(const void *sig, long row, int n, int N, float sc, float t0dt) {
    if constexpr (FILTERED) {
        return load_sig<SFMT>(sig, row + n, sc);
    } else {
        const float pm = load_sig<SFMT>(sig, row + max(n - 1, 0), sc);
        const float p0 = load_sig<SFMT>(sig, row + n, sc);
        const float pp = load_sig<SFMT>(sig, row + min(n + 1, N - 1), sc);
        return ubp(pm, p0, pp, n, N, t0dt);
    }
}


}  // namespace pat_gather
