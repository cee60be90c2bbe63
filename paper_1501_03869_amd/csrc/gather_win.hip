// Back projection of frames with many ROI positions: one wave per run of
// consecutive table columns (PPL per lane) and a run of sensors, the signal
// read from a window in the wave's own slice of LDS.
//
// The sum is the delay-and-sum of Section II-C: the UBP-filtered signal
// b = p - t dp/dt of every sensor, read at the position's delay with linear
// interpolation, weighted and summed over sensors.  Per sensor a wave
//   - loads its 64 * PPL delays (16-byte loads, one contiguous run of the
//     table row) and decodes them to sample positions,
//   - starts a 128-sample window just below the smallest of them (a
//     wave-wide minimum by DPP and one lane read), and tests once per lane
//     whether all of the lane's positions fall inside it (a per-lane minimum
//     and maximum),
//   - loads those 128 samples, two per lane, evaluates the filter on them
//     (central differences, the neighbouring samples taken from the adjacent
//     lanes by DPP wave shifts) and writes them to its LDS slice,
//   - reads b[n], b[n+1] of every gather from the window: with no further
//     tests when every lane's positions fit, else each position is tested.
// So 64 * PPL gathers cost PPL/4 + 1 vector-memory loads per lane, against
// 5 per 256 gathers in the split-sensor kernel, where every lane loads its own
// taps.  A delay whose interval is not inside the window (the delays of the
// wave's positions spread over more than about 124 samples, or the record's
// first and last samples, where the filter is one-sided) is gathered from
// global memory instead, with the general-path arithmetic of the other
// kernels (a wave with a delay that does not contribute takes the tested
// path too).
//
// Table loads of sensor i+D and the window of sensor i+LW are in flight while
// sensor i is summed.  The waves of a workgroup take disjoint runs of the
// sensors, and their partial sums are added in LDS in wave order, so results
// are reproducible run to run.  Several frames share one launch, each
// pixel group's frames on one XCD, so that their table rows are read from
// HBM about once.
#include <mutex>
#include <type_traits>

#include "gather_common.h"
#include "pat_internal.h"

using namespace pat_gather;

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

constexpr int WN_WIN = 128;              // window samples, two per lane
constexpr int WN_MAXW = 16;              // waves per workgroup
constexpr int WN_RSRC_W3 = 0x00020000;   // buffer descriptor word 3: raw 32-bit dwords

__device__ __forceinline__ __amdgpu_buffer_rsrc_t wrsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, WN_RSRC_W3);
}

// DPP lane moves (all 64 lanes active): CTRL 0xB1 / 0x4E swap lanes within
// quads, 0x141 mirrors each half-row of 8, 0x140 each row of 16; 0x138 shifts
// the wave right by one lane (lane l reads lane l-1) and 0x130 left (lane l
// reads lane l+1); lanes with no source read 0.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}

// Minimum of v over the 64 lanes, wave-uniform: within rows of 16 by lane
// swaps and mirrors, then row 1 takes row 0's and row 3 row 2's (0x142:
// lane 15 of each row broadcast to the next), row 2 and 3 lane 31's (0x143),
// and lane 63 holds the result.
__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
    v = min(v, dpp<0xB1>(v));
    v = min(v, dpp<0x4E>(v));
    v = min(v, dpp<0x141>(v));
    v = min(v, dpp<0x140>(v));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x142, 0xA, 0xF, false));
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x143, 0xC, 0xF, false));
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// floor(u) of a float32 u >= 0 from its bit pattern, in integer operations
// (wave-uniform values stay in scalar registers); patterns of 2^24 and above,
// negative values, NaN and infinities give INT_MAX.
__device__ __forceinline__ int floor_bits(uint32_t m) {
    const int e = (int)(m >> 23) - 127;
    if (e < 0) return 0;
    if (e > 23) return 0x7FFFFFFF;
    return (int)(((m & 0x7FFFFFu) | 0x800000u) >> (23 - e));
}

// Bit pattern of the float32 value of an integer 0 <= k < 2^24, in integer
// operations.
__device__ __forceinline__ uint32_t float_bits(uint32_t k) {
    if (k == 0) return 0u;
    const int e = 31 - __builtin_clz(k);
    return ((uint32_t)(e + 127) << 23) | ((k << (23 - e)) & 0x7FFFFFu);
}

__device__ __forceinline__ float wh2f(uint32_t bits16) {
    return __half2float(__ushort_as_half((unsigned short)bits16));
}

// One sensor's table entries for a lane's PPL columns, as loaded.  Float32
// and 16.16 tables: one dword per column.  16-bit tile-relative tables: the
// offsets two per dword and the header of the lane's 32-column tile (the
// group that ends past P: one offset and one header per column, since its
// clamped columns may fall in another tile).
template <class Delay, int PPL, bool LAST>
struct TabStage {
    static constexpr bool R = Delay::kR16;
    static constexpr int NW = R ? (LAST ? PPL : PPL / 2) : PPL;
    static constexpr int NH = R ? (LAST ? PPL : 1) : 1;
    uint32_t w[NW];
    uint32_t h[NH];
    // the k-th column's entry as the decoding takes it: float32 bits, or a
    // 16.16 index
    __device__ __forceinline__ uint32_t val(int k) const {
        if constexpr (!R) {
            return w[k];
        } else {
            const uint32_t off = LAST ? w[k] : (w[k >> 1] >> (16 * (k & 1))) & 0xFFFFu;
            return DelayR16::to_q16(off, LAST ? h[k] : h[0]);
        }
    }
};

template <class Delay, int SFMT, bool FILTERED, bool HAS_W, int PPL, int D, int LW, int FPW>
__global__ void __launch_bounds__(64 * WN_MAXW)
    k_bp_win(const uint32_t *__restrict__ tab, const void *__restrict__ sig, const float *__restrict__ scale,
             const float *__restrict__ w, int S, int P, int N, int F, int spw, Delay dec, float t0dt,
             float *__restrict__ img) {
    static_assert(PPL % 4 == 0 && D % LW == 0 && D >= 2 * LW, "pipeline shape");
    constexpr int PIX = 64 * PPL;
    // [waves][FPW][PIX]: a wave's window of each of its frames, then its
    // partial sums
    extern __shared__ float wl[];
    constexpr bool kF32T = std::is_base_of<DelayF32, Delay>::value;
    constexpr bool F16 = SFMT == PAT_SIG_F16;
    constexpr uint32_t esz = F16 ? 2 : 4;
    // launch slot -> (group, block of FPW frames), frame blocks fastest: an
    // XCD runs the frames of a group together, so their table rows are read
    // from HBM about once; a wave decodes each table entry once for its FPW
    // frames
    const int groups = (P + PIX - 1) / PIX;
    const int FB = (F + FPW - 1) / FPW;
    const int gf = xcd_tile(blockIdx.x, groups * FB);
    if (gf < 0) return;
    const int g = gf / FB, fb = gf - g * FB;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = blockDim.x >> 6;
    const int pb = g * PIX;
    const int c0 = pb + PPL * lane;  // this lane's first column
    const int s_begin = wv * spw;
    const int ns = min(S, s_begin + spw) - s_begin;
    // frame fb * FPW + q of the block (q < FPW); frames past F repeat the
    // last one and are not stored
    const char *sigf[FPW];
    float *wwin[FPW];
    float acc2[FPW][PPL];
#pragma unroll
    for (int q = 0; q < FPW; ++q) {
        sigf[q] = static_cast<const char *>(sig) + (size_t)min(fb * FPW + q, F - 1) * S * N * esz;
        wwin[q] = wl + (wv * FPW + q) * PIX;
#pragma unroll
        for (int k = 0; k < PPL; ++k) acc2[q][k] = 0.0f;
    }

    // LAST: the group that ends past P, whose lanes load each column on its
    // own (columns past P read column P-1 and are not stored)
    auto body = [&](auto last_tag) {
        constexpr bool LAST = decltype(last_tag)::value;
        using TS = TabStage<Delay, PPL, LAST>;
        // 16-bit tables: offsets [S][P] at byte 0, headers [S][tiles] after them
        const int tiles = (P + 31) / 32;
        const uint16_t *off16 = reinterpret_cast<const uint16_t *>(tab);
        const uint32_t *hdr32 =
            reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(tab) + pat_r16_hdr_offset(S, P));
        auto tload = [&](int i, TS &t) {
            const int s = s_begin + min(i, ns - 1);
            if constexpr (Delay::kR16) {
                const __amdgpu_buffer_rsrc_t ro = wrsrc(off16 + (size_t)s * P, (uint32_t)P * 2u);
                const __amdgpu_buffer_rsrc_t rh = wrsrc(hdr32 + (size_t)s * tiles, (uint32_t)tiles * 4u);
                if constexpr (LAST) {
#pragma unroll
                    for (int k = 0; k < PPL; ++k) {
                        const uint32_t c = (uint32_t)min(c0 + k, P - 1);
                        t.w[k] = __builtin_amdgcn_raw_buffer_load_b16(ro, c * 2u, 0, 0);
                        t.h[k] = __builtin_amdgcn_raw_buffer_load_b32(rh, (c >> 5) * 4u, 0, 0);
                    }
                } else {
                    static_assert(PPL == 4 || PPL == 8, "16-bit entries per lane");
                    if constexpr (PPL == 4) {
                        const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(ro, (uint32_t)c0 * 2u, 0, 0);
                        t.w[0] = v[0];
                        t.w[1] = v[1];
                    } else {
                        const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(ro, (uint32_t)c0 * 2u, 0, 0);
                        t.w[0] = v[0]; t.w[1] = v[1]; t.w[2] = v[2]; t.w[3] = v[3];
                    }
                    t.h[0] = __builtin_amdgcn_raw_buffer_load_b32(rh, (uint32_t)(c0 >> 5) * 4u, 0, 0);
                }
            } else {
                const __amdgpu_buffer_rsrc_t r = wrsrc(tab + (size_t)s * P, (uint32_t)P * 4u);
                if constexpr (LAST) {
#pragma unroll
                    for (int k = 0; k < PPL; ++k)
                        t.w[k] = __builtin_amdgcn_raw_buffer_load_b32(r, (uint32_t)min(c0 + k, P - 1) * 4u, 0, 0);
                } else {
#pragma unroll
                    for (int j = 0; j < PPL / 4; ++j) {
                        const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, (uint32_t)c0 * 4u, 16 * j, 0);
                        t.w[4 * j] = v[0]; t.w[4 * j + 1] = v[1]; t.w[4 * j + 2] = v[2]; t.w[4 * j + 3] = v[3];
                    }
                }
            }
        };
        // window-relative range of n whose b[n], b[n+1] the window holds
        constexpr int LO = FILTERED ? 0 : 1;
        constexpr int HI = FILTERED ? WN_WIN - 1 : WN_WIN - 2;  // n < r0 + HI
        // One sensor decoded for its sum: x = the sample position u of every
        // column (float32 tables, as bits; u = T/dt - t0/dt with one FMA, as
        // in the split-sensor kernel) or its 16.16 index; r0 = the window's
        // first sample: the smallest sample index of the wave's delays, less
        // the filter's lower neighbour (even for FP16 records); ok = every
        // delay of the wave lies in the window (wave-uniform).  Positions are
        // compared as bit patterns: for non-negative float32 values and 16.16
        // indices that is their order, and negative values, NaN and the 16.16
        // sentinel sort last.
        struct Prep {
            uint32_t x[PPL];
            int r0, ok;
        };
        auto prep = [&](const TS &t, Prep &pr) {
            uint32_t kmin = 0xFFFFFFFFu, kmax = 0u;
#pragma unroll
            for (int k = 0; k < PPL; ++k) {
                uint32_t x = t.val(k);
                if constexpr (kF32T) x = __float_as_uint(dec.u1(__uint_as_float(x)));
                pr.x[k] = x;
                kmin = min(kmin, x);
                kmax = max(kmax, x);
            }
            const uint32_t m = wave_min(kmin);
            // (no contributing delay in the wave: the window at the record's end)
            const int n = kF32T ? floor_bits(m) : (int)(m >> 16);
            int r0 = min(n, N) - LO;
            if constexpr (F16) r0 &= ~1;
            r0 = max(0, min(r0, N - WN_WIN));
            uint32_t lo, hi;
            if constexpr (kF32T) {
                lo = float_bits((uint32_t)(r0 + LO));
                hi = float_bits((uint32_t)(r0 + HI));
            } else {
                lo = (uint32_t)(r0 + LO) << 16;
                hi = (uint32_t)(r0 + HI) << 16;
            }
            pr.r0 = r0;
            pr.ok = (__builtin_amdgcn_ballot_w64(kmin < lo) | __builtin_amdgcn_ballot_w64(kmax >= hi)) == 0;
        };
        auto wload = [&](int i, int r0, int q) -> u32x2 {
            const int s = s_begin + min(i, ns - 1);
            const __amdgpu_buffer_rsrc_t r = wrsrc(sigf[q] + (size_t)s * N * esz, (uint32_t)N * esz);
            const uint32_t off = (uint32_t)(r0 + 2 * lane) * esz;
            if constexpr (F16) {
                u32x2 v;
                v[0] = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
                v[1] = 0u;
                return v;
            } else {
                return __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
            }
        };
        // b[r0 + 2l], b[r0 + 2l + 1] into the lane's two window slots (raw
        // input: valid in slots 1 .. 126, lanes 0 and 63 lack a neighbour)
        const float t0h = 0.5f * t0dt;
        auto wstore = [&](const u32x2 &v, int r0, int q) {
            float p0, p1;
            if constexpr (F16) {
                p0 = wh2f(v[0] & 0xFFFFu);
                p1 = wh2f(v[0] >> 16);
            } else {
                p0 = __uint_as_float(v[0]);
                p1 = __uint_as_float(v[1]);
            }
            float b0 = p0, b1 = p1;
            if constexpr (!FILTERED) {
                const float pm = __uint_as_float(dpp<0x138>(__float_as_uint(p1)));  // p[r0 + 2l - 1]
                const float pn = __uint_as_float(dpp<0x130>(__float_as_uint(p0)));  // p[r0 + 2l + 2]
                const float k0 = fmaf((float)(r0 + 2 * lane), 0.5f, t0h);           // (j + t0/dt) / 2
                b0 = fmaf(-k0, p1 - pm, p0);
                b1 = fmaf(-(k0 + 0.5f), pn - p0, p1);
            }
            reinterpret_cast<float2 *>(wwin[q])[lane] = make_float2(b0, b1);
        };
        auto gather = [&](const Prep &pr, int i, int fq) {
            const int s = s_begin + i;
            float ws = 1.0f;
            if constexpr (HAS_W) ws = w[s];
            const int r0 = pr.r0;
            const float *wb = wwin[fq] - r0;  // wb[n]: b[n] for n in the window
            float (&acc)[PPL] = acc2[fq];
            if (pr.ok) {
                // every delay in the window: no tests
#pragma unroll
                for (int k = 0; k < PPL; ++k) {
                    int n;
                    float a;
                    if constexpr (kF32T) {
                        const float u = __uint_as_float(pr.x[k]);
                        n = (int)u;
                        a = __builtin_amdgcn_fractf(u);
                    } else {
                        n = (int)(pr.x[k] >> 16);
                        a = (float)(pr.x[k] & 0xFFFFu) * (1.0f / 65536.0f);
                    }
                    const float b0 = wb[n], b1 = wb[n + 1];
                    const float v = fmaf(a, b1 - b0, b0);
                    if constexpr (HAS_W) {
                        acc[k] = fmaf(ws, v, acc[k]);
                    } else {
                        acc[k] += v;
                    }
                }
                return;
            }
            // some delay of the wave lies outside the window: each is tested,
            // those outside read their taps from global memory
            bool in[PPL];
            uint64_t anymiss = 0;
            const float flo = (float)(r0 + LO), fhi = __uint_as_float(__float_as_uint((float)(r0 + HI)) - 1u);
#pragma unroll
            for (int k = 0; k < PPL; ++k) {
                int n;
                float a;
                if constexpr (kF32T) {
                    const float u = __uint_as_float(pr.x[k]);
                    const float uc = __builtin_amdgcn_fmed3f(u, flo, fhi);
                    in[k] = uc == u;
                    n = (int)uc;
                    a = __builtin_amdgcn_fractf(uc);
                } else {
                    const int n0 = (int)(pr.x[k] >> 16);
                    in[k] = (uint32_t)(n0 - r0 - LO) < (uint32_t)(HI - LO);
                    n = min(max(n0, r0 + LO), r0 + HI - 1);
                    a = (float)(pr.x[k] & 0xFFFFu) * (1.0f / 65536.0f);
                }
                const float b0 = wb[n], b1 = wb[n + 1];
                const float v = fmaf(a, b1 - b0, b0);
                if constexpr (HAS_W) {
                    acc[k] = in[k] ? fmaf(ws, v, acc[k]) : acc[k];  // v may be NaN where not in
                } else {
                    acc[k] += in[k] ? v : 0.0f;
                }
                anymiss |= __builtin_amdgcn_ballot_w64(!in[k]);
            }
            if (anymiss == 0) return;
            // delays outside the window (or not contributing): taps from
            // global memory, the filter one-sided at both ends of the record
            const __amdgpu_buffer_rsrc_t r = wrsrc(sigf[fq] + (size_t)s * N * esz, (uint32_t)N * esz);
            auto tap = [&](int m) -> float {
                if constexpr (F16) return wh2f(__builtin_amdgcn_raw_buffer_load_b16(r, (uint32_t)m * 2u, 0, 0));
                else return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (uint32_t)m * 4u, 0, 0));
            };
#pragma unroll
            for (int k = 0; k < PPL; ++k) {
                if (in[k]) continue;
                int n;
                float a;
                if constexpr (kF32T) {
                    const float u = __uint_as_float(pr.x[k]);
                    if (!(u >= 0.0f && u <= dec.umax)) continue;  // does not contribute (also NaN)
                    n = min((int)u, N - 2);
                    a = u - (float)n;
                } else {
                    if (!dec.decode_bf(pr.x[k], N, n, a)) continue;
                }
                float b0, b1;
                if constexpr (FILTERED) {
                    b0 = tap(n);
                    b1 = tap(n + 1);
                } else {
                    const float pm = tap(max(n - 1, 0)), p0 = tap(n), p1 = tap(n + 1), p2 = tap(min(n + 2, N - 1));
                    const float k0 = fmaf((float)n, 0.5f, t0h);
                    const float d0 = n == 0 ? 2.0f * (p1 - p0) : p1 - pm;
                    const float d1 = n + 1 == N - 1 ? 2.0f * (p1 - p0) : p2 - p0;
                    b0 = fmaf(-k0, d0, p0);
                    b1 = fmaf(-(k0 + 0.5f), d1, p1);
                }
                acc[k] = fmaf(ws, fmaf(a, b1 - b0, b0), acc[k]);
            }
        };

        // Rings: table loads of D sensors, decoded sensors and windows of LW.
        // Iteration i filters and stores window i, decodes sensor i+LW and
        // issues its window, sums sensor i from its window and issues the
        // table loads of sensor i+D.  Loads past the wave's sensors re-read
        // its last records.
        TS T[D];
        u32x2 Wr[LW][FPW];
        Prep X[LW];
        // prologue in the loop's issue order (window j, then the table of
        // sensor D - LW + j), so that the loop's first waits are its steady ones
#pragma unroll
        for (int j = 0; j < D - LW; ++j) tload(j, T[j]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < LW; ++j) {
            prep(T[j], X[j]);
#pragma unroll
            for (int q = 0; q < FPW; ++q) Wr[j][q] = wload(j, X[j].r0, q);
            __builtin_amdgcn_sched_barrier(0);
            tload(D - LW + j, T[D - LW + j]);
            __builtin_amdgcn_sched_barrier(0);
        }
        // whole blocks of D iterations (one loop state for the compiler's
        // waits); iterations past the last sensor sum nothing
        const int nsr = (ns + D - 1) / D * D;
        for (int base = 0; base < nsr; base += D) {
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const int i = base + k;
#pragma unroll
                for (int q = 0; q < FPW; ++q) wstore(Wr[k % LW][q], X[k % LW].r0, q);
                Prep nx;
                prep(T[(k + LW) % D], nx);
#pragma unroll
                for (int q = 0; q < FPW; ++q) Wr[k % LW][q] = wload(i + LW, nx.r0, q);
                if (i < ns) {
#pragma unroll
                    for (int q = 0; q < FPW; ++q) gather(X[k % LW], i, q);
                }
                X[k % LW] = nx;
                tload(i + D, T[k]);
            }
        }
    };
    if (ns > 0) {
        if (pb + PIX > P) body(std::true_type{});
        else body(std::false_type{});
    }

    // partial sums of the wave's frames in their own LDS slices (its windows
    // are no longer read), then wave 0 adds the waves' sums in wave order
#pragma unroll
    for (int q = 0; q < FPW; ++q) {
        const int f = fb * FPW + q;
        const float sc = (F16 && scale) ? scale[min(f, F - 1)] : 1.0f;  // filter and interpolation are linear
        if (nw == 1) {
            if (f < F) {
                float *out = img + (size_t)f * P;
#pragma unroll
                for (int k = 0; k < PPL; ++k)
                    if (c0 + k < P) out[c0 + k] = acc2[q][k] * sc;
            }
        } else {
#pragma unroll
            for (int k = 0; k < PPL; ++k) wwin[q][PPL * lane + k] = acc2[q][k] * sc;
        }
    }
    if (nw == 1) return;
    __syncthreads();
    if (wv == 0) {
#pragma unroll
        for (int q = 0; q < FPW; ++q) {
            const int f = fb * FPW + q;
            if (f >= F) continue;
            float *out = img + (size_t)f * P;
#pragma unroll
            for (int k = 0; k < PPL; ++k) {
                float sum = 0.0f;
                for (int m = 0; m < nw; ++m) sum += wl[(m * FPW + q) * PIX + PPL * lane + k];
                if (c0 + k < P) out[c0 + k] = sum;
            }
        }
    }
}

}  // namespace

namespace {

// Columns per lane, table loads and windows in flight per wave: the fastest
// of the shapes measured on the 1024^2 workload (4 columns per lane with the
// table 4, 6 or 8 sensors ahead and the window 1, 2 or 3 ahead; 8 columns
// per lane), 622-636 us against 632-670 us for the others.
constexpr int WN_PPL = 4, WN_D = 4, WN_LW = 2;
// Waves per compute unit the launch aims at: 24 (6 per SIMD) did best on the
// 1024^2 workload and on its first 256K and 512K columns; 12 was 5-17 %
// slower there.
constexpr long WN_WAVES_PER_CU = 24;
constexpr int WN_PIX = 64 * WN_PPL;

struct WinShape {
    int groups, waves, spw;
};

// Waves per workgroup: about per_cu waves per compute unit over the launch,
// and never more than keep every workgroup resident at once
// (blocks_per_cu(W) * CUs >= groups * F); sensors split evenly.
template <class BlocksPerCu>
WinShape win_shape(int S, int P, int F, int cus, long per_cu, BlocksPerCu blocks_per_cu) {
    WinShape s;
    s.groups = (P + WN_PIX - 1) / WN_PIX;
    const long wgs = (long)s.groups * std::max(F, 1);
    int W = 1;
    for (int cand = WN_MAXW; cand >= 1; --cand) {
        if ((long)blocks_per_cu(cand) * cus >= wgs) { W = cand; break; }
    }
    const long target = (per_cu * cus + wgs / 2) / wgs;
    W = (int)std::max(1L, std::min<long>(W, target));
    W = std::min(W, std::max(S, 1));
    s.spw = (std::max(S, 1) + W - 1) / W;
    s.waves = (std::max(S, 1) + s.spw - 1) / s.spw;
    return s;
}

template <class Delay, int SFMT, bool FILTERED, bool HAS_W, int FPW>
int launch_win_fpw(int S, int P, int F, const uint32_t *tab, const void *sig, const float *scale, const float *w,
                   int N, Delay dec, float t0dt, float *img, hipStream_t st) {
    auto kern = k_bp_win<Delay, SFMT, FILTERED, HAS_W, WN_PPL, WN_D, WN_LW, FPW>;
    // occupancy per block size, computed once per kernel and device
    static std::mutex mu;
    static int cache_dev = -1, cache_cus = 0, cache_bpc[WN_MAXW + 1];
    int dev = 0;
    PAT_HIP(hipGetDevice(&dev));
    const int FB = (F + FPW - 1) / FPW;
    WinShape sh;
    {
        std::lock_guard<std::mutex> lk(mu);
        if (cache_dev != dev) {
            PAT_HIP(hipDeviceGetAttribute(&cache_cus, hipDeviceAttributeMultiprocessorCount, dev));
            for (int W = 1; W <= WN_MAXW; ++W)
                PAT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&cache_bpc[W], kern, 64 * W,
                                                                     (size_t)W * FPW * WN_PIX * sizeof(float)));
            cache_dev = dev;
        }
        sh = win_shape(S, P, FB, cache_cus, WN_WAVES_PER_CU, [&](int W) { return cache_bpc[W]; });
    }
    const dim3 grid(xcd_slots(sh.groups * FB));
    kern<<<grid, dim3(64 * sh.waves), (size_t)sh.waves * FPW * WN_PIX * sizeof(float), st>>>(
        tab, sig, scale, w, S, P, N, F, sh.spw, dec, t0dt, img);
    PAT_HIP(hipGetLastError());
    return PAT_OK;
}

// Frames per wave: a table larger than the 256 MB Infinity Cache streams
// from HBM for every pass over it, so a wave that reads and decodes it once
// for 4 frames (2 for 2-3 frames) gains most: 16 frames on the 1024^2
// workload take 0.22 ms per frame against 0.36 with one frame per wave.  A
// table that the cache partly holds gains less than the extra registers
// cost (16 or 64 frames on the 512^2 serving map: 1 frame per wave is
// within 5 % of the best), so it keeps one.
template <class Delay, int SFMT, bool FILTERED, bool HAS_W>
int launch_win_one(int S, int P, int F, const uint32_t *tab, const void *sig, const float *scale, const float *w,
                   int N, Delay dec, float t0dt, float *img, hipStream_t st, size_t table_bytes) {
    if (F >= 2 && table_bytes > PAT_INFINITY_CACHE_BYTES) {
        if (F >= 4)
            return launch_win_fpw<Delay, SFMT, FILTERED, HAS_W, 4>(S, P, F, tab, sig, scale, w, N, dec, t0dt, img, st);
        return launch_win_fpw<Delay, SFMT, FILTERED, HAS_W, 2>(S, P, F, tab, sig, scale, w, N, dec, t0dt, img, st);
    }
    return launch_win_fpw<Delay, SFMT, FILTERED, HAS_W, 1>(S, P, F, tab, sig, scale, w, N, dec, t0dt, img, st);
}

template <class Delay, int SFMT>
int launch_win(bool filtered, int S, int P, int F, const uint32_t *tab, const void *sig, const float *scale,
               const float *w, int N, Delay dec, float t0dt, float *img, hipStream_t st, size_t tb) {
    if (w)
        return filtered ? launch_win_one<Delay, SFMT, true, true>(S, P, F, tab, sig, scale, w, N, dec, t0dt, img, st, tb)
                        : launch_win_one<Delay, SFMT, false, true>(S, P, F, tab, sig, scale, w, N, dec, t0dt, img, st, tb);
    return filtered ? launch_win_one<Delay, SFMT, true, false>(S, P, F, tab, sig, scale, w, N, dec, t0dt, img, st, tb)
                    : launch_win_one<Delay, SFMT, false, false>(S, P, F, tab, sig, scale, w, N, dec, t0dt, img, st, tb);
}

}  // namespace

bool pat_win_preferred(int P, int F, size_t table_bytes) {
    if (table_bytes <= PAT_CACHED_TABLE_BYTES) return false;
    if (P >= PAT_WIN_MIN_P) return true;
    // several frames on the 512^2 serving map (175 MB table, 335 groups):
    // 64 frames 24 against 31 us per frame for the batched kernel
    return F >= 2 && (long long)((P + WN_PIX - 1) / WN_PIX) * F >= 8LL * 256;
}

bool pat_win_eligible(int table_fmt, int sig_fmt, int S, int P, int N, int F, const void *sig) {
    if (table_fmt != PAT_TABLE_F32 && table_fmt != PAT_TABLE_Q16 && table_fmt != PAT_TABLE_R16) return false;
    if (S <= 0 || F <= 0 || N < WN_WIN || P < WN_PIX || P >= (1 << 29)) return false;
    if ((long long)((P + WN_PIX - 1) / WN_PIX) * F + 8 >= (1ll << 31)) return false;
    if ((uintptr_t)sig % 4 != 0) return false;
    if (sig_fmt == PAT_SIG_F16 && N % 2 != 0) return false;
    return true;
}

int pat_launch_backproject_win(const void *table, int table_fmt, const void *sig, int sig_fmt, int sig_is_filtered,
                               const float *frame_scale, const float *w, int S, int P, int N, int F, double t0,
                               double dt, float *img, hipStream_t st) {
    const float t0dt = (float)(t0 / dt);
    const bool filt = sig_is_filtered != 0;
    const uint32_t *tab = static_cast<const uint32_t *>(table);
    const size_t tb = table_fmt == PAT_TABLE_R16 ? pat_r16_bytes(S, P) : (size_t)S * P * 4;
    if (table_fmt == PAT_TABLE_F32) {
        DelayF32 d;
        const double inv = 1.0 / dt;
        d.inv_hi = (float)inv;
        d.inv_lo = (float)(inv - (double)d.inv_hi);
        d.off = (float)(-t0 / dt);
        d.umax = (float)(N - 1);
        return sig_fmt == PAT_SIG_F32
                   ? launch_win<DelayF32, PAT_SIG_F32>(filt, S, P, F, tab, sig, frame_scale, w, N, d, t0dt, img, st, tb)
                   : launch_win<DelayF32, PAT_SIG_F16>(filt, S, P, F, tab, sig, frame_scale, w, N, d, t0dt, img, st, tb);
    }
    if (table_fmt == PAT_TABLE_R16) {
        DelayR16 d;
        return sig_fmt == PAT_SIG_F32
                   ? launch_win<DelayR16, PAT_SIG_F32>(filt, S, P, F, tab, sig, frame_scale, w, N, d, t0dt, img, st, tb)
                   : launch_win<DelayR16, PAT_SIG_F16>(filt, S, P, F, tab, sig, frame_scale, w, N, d, t0dt, img, st, tb);
    }
    DelayQ16 d;
    return sig_fmt == PAT_SIG_F32
               ? launch_win<DelayQ16, PAT_SIG_F32>(filt, S, P, F, tab, sig, frame_scale, w, N, d, t0dt, img, st, tb)
               : launch_win<DelayQ16, PAT_SIG_F16>(filt, S, P, F, tab, sig, frame_scale, w, N, d, t0dt, img, st, tb);
}
