// Batched back projection: F frames that share one delay table, read once.
//
// The delay of a (pixel, sensor) pair is decoded once and reused for 16
// frames: the linear interpolation of the filtered signal is folded into four
// coefficients on the raw samples n-1 .. n+2 (or two on b[n], b[n+1] when the
// signals are already filtered), so per frame a gather is one or two LDS reads
// and four (two) FMAs.  Raw FP16 samples stay FP16 in LDS, stored as
// overlapping pairs (s[j], s[j+1]) so that the four taps are two aligned
// 32-bit reads; the per-frame FP16 scale is applied once to the finished sum.
//
// Work decomposition: a 256-thread workgroup owns 256 consecutive table
// columns (one pixel per thread; tile-major ROI order makes them a compact
// patch), 16 frames and a group of sensors.  For every sensor it stages, per
// frame, a 272-sample window around the delay of its first pixel (16-byte
// vector copies, double-buffered, one barrier per sensor).  Delays outside the
// window fall back to global loads of the same taps.  Sensor groups are summed
// in fixed order by the last workgroup to finish.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <algorithm>

#include "gather_common.h"
#include "pat_internal.h"

namespace {

using namespace pat_gather;

constexpr int BB_THREADS = 256;
constexpr int BB_FB = 16;                   // frames per workgroup
constexpr int BB_WS = 272;                  // staged samples per (sensor, frame)
constexpr int BB_NPROBE = 8;                // window probes per sensor: every 32nd pixel
constexpr int BB_MARGIN = 40;               // window start below the smallest probed delay
constexpr int BB_CHUNKS = BB_WS / 8;        // 8-sample copies per (sensor, frame)
constexpr int BB_RESIDENT = 256 * 4;          // workgroups resident at once (35 KiB of LDS each)

struct BbShape {
    int chunks, fgroups, groups, spg;
};

BbShape bb_shape(int S, int P, int F) {
    BbShape s;
    s.chunks = (P + BB_THREADS - 1) / BB_THREADS;
    s.fgroups = (F + BB_FB - 1) / BB_FB;
    const long base = (long)s.chunks * s.fgroups;
    const int S1 = std::max(S, 1);
    // as many sensor groups as fit in one wave of resident workgroups (at most 8)
    int G = (int)std::min<long>(std::max<long>(1, BB_RESIDENT / base), std::min(S1, 8));
    G = std::max(G, 1);
    s.spg = (S1 + G - 1) / G;
    s.groups = (S1 + s.spg - 1) / s.spg;
    return s;
}

__device__ __forceinline__ float lo_h(uint32_t d) { return __half2float(__ushort_as_half((unsigned short)(d & 0xFFFFu))); }
__device__ __forceinline__ float hi_h(uint32_t d) { return __half2float(__ushort_as_half((unsigned short)(d >> 16))); }

__device__ __forceinline__ int floor8(int x) { return (x >> 3) << 3; }

// Raw sample i (clamped into the record) as float, unscaled.
template <int SFMT>
__device__ __forceinline__ float raw_at(const void *sig, long row, int i, int N) {
    i = min(max(i, 0), N - 1);
    if constexpr (SFMT == PAT_SIG_F32) return static_cast<const float *>(sig)[row + i];
    else return __half2float(static_cast<const __half *>(sig)[row + i]);
}

// Eight window samples s[i0 .. i0+7] of one (sensor, frame) row (plus s[i0+8]
// for FP16, whose pairs overlap), loaded into registers; indices outside the
// record are clamped to it.
struct Raw8 {
    uint4 q;      // FP16: 8 halves; FP32: samples 0..3
    uint4 q2;     // FP32: samples 4..7
    uint32_t h8;  // FP16: sample 8
};

template <int SFMT>
__device__ __forceinline__ void load8(const void *sig, long row, int i0, int N, Raw8 &r) {
    if constexpr (SFMT == PAT_SIG_F16) {
        const unsigned short *h = static_cast<const unsigned short *>(sig) + row;
        if (i0 >= 0 && i0 + 8 < N) {
            r.q = *reinterpret_cast<const uint4 *>(h + i0);
            r.h8 = h[i0 + 8];
        } else {
            uint32_t v[9];
#pragma unroll
            for (int m = 0; m < 9; ++m) v[m] = h[min(max(i0 + m, 0), N - 1)];
            r.q.x = v[0] | (v[1] << 16);
            r.q.y = v[2] | (v[3] << 16);
            r.q.z = v[4] | (v[5] << 16);
            r.q.w = v[6] | (v[7] << 16);
            r.h8 = v[8];
        }
    } else {
        const float *x = static_cast<const float *>(sig) + row;
        if (i0 >= 0 && i0 + 8 <= N) {
            r.q = *reinterpret_cast<const uint4 *>(x + i0);
            r.q2 = *reinterpret_cast<const uint4 *>(x + i0 + 4);
        } else {
            uint32_t v[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) v[m] = __float_as_uint(x[min(max(i0 + m, 0), N - 1)]);
            r.q = make_uint4(v[0], v[1], v[2], v[3]);
            r.q2 = make_uint4(v[4], v[5], v[6], v[7]);
        }
    }
}

// Store eight loaded samples at dst: FP32 as is; FP16 as the overlapping pairs
// (s[j], s[j+1]) for j = i0 .. i0+7.
template <int SFMT>
__device__ __forceinline__ void store8(const Raw8 &r, uint32_t *dst) {
    if constexpr (SFMT == PAT_SIG_F16) {
        uint4 e, o;
        e.x = r.q.x;
        e.y = __builtin_amdgcn_alignbyte(r.q.y, r.q.x, 2);
        e.z = r.q.y;
        e.w = __builtin_amdgcn_alignbyte(r.q.z, r.q.y, 2);
        o.x = r.q.z;
        o.y = __builtin_amdgcn_alignbyte(r.q.w, r.q.z, 2);
        o.z = r.q.w;
        o.w = (r.q.w >> 16) | (r.h8 << 16);
        reinterpret_cast<uint4 *>(dst)[0] = e;
        reinterpret_cast<uint4 *>(dst)[1] = o;
    } else {
        reinterpret_cast<uint4 *>(dst)[0] = r.q;
        reinterpret_cast<uint4 *>(dst)[1] = r.q2;
    }
}

// Interpolation coefficients on the taps n-1, n, n+1, n+2 (raw) or n, n+1
// (filtered, c0 = c3 = 0) of lerp(b, n + a) times w, with
// b[i] = p[i] - (i + t0/dt) (p[i+1] - p[i-1]) / 2, one-sided at i = 0, N-1.
template <bool FILTERED>
__device__ __forceinline__ void coeffs(int n, float a, float w, int N, float t0dt, float (&c)[4]) {
    const float wa = w * a, wb = w - wa;  // w * alpha, w * (1 - alpha)
    if constexpr (FILTERED) {
        c[0] = 0.0f; c[1] = wb; c[2] = wa; c[3] = 0.0f;
    } else {
        const float tn = (float)n + t0dt, tn1 = tn + 1.0f;
        float e0 = 0.5f * tn, e1 = 1.0f, e2 = -0.5f * tn;        // b[n] on n-1, n, n+1
        if (n == 0) { e0 = 0.0f; e1 = 1.0f + tn; e2 = -tn; }
        float f0 = 0.5f * tn1, f1 = 1.0f, f2 = -0.5f * tn1;      // b[n+1] on n, n+1, n+2
        if (n + 1 == N - 1) { f0 = tn1; f1 = 1.0f - tn1; f2 = 0.0f; }
        c[0] = wb * e0;
        c[1] = fmaf(wb, e1, wa * f0);
        c[2] = fmaf(wb, e2, wa * f1);
        c[3] = wa * f2;
    }
}

template <class Delay, int SFMT, bool FILTERED>
__global__ void __launch_bounds__(BB_THREADS) k_bp_batch(const uint32_t *__restrict__ tab, const void *__restrict__ sig,
                                                         const float *__restrict__ scale, const float *__restrict__ w,
                                                         int S, int P, int N, int F, int spg, int G, Delay dec,
                                                         float t0dt, float *__restrict__ part,
                                                         float *__restrict__ img, unsigned int *__restrict__ done) {
    __shared__ __align__(16) uint32_t win[2][BB_FB][BB_WS];
    __shared__ unsigned int is_last;

    const int tid = threadIdx.x;
    const int c = blockIdx.x, fg = blockIdx.y, g = blockIdx.z;
    const int pbase = c * BB_THREADS;
    const int p = pbase + tid;
    const bool pix_ok = p < P;
    const int f0 = fg * BB_FB;
    const int nf = min(BB_FB, F - f0);
    const int s_begin = g * spg;
    const int s_end = min(S, s_begin + spg);

    float acc[BB_FB];
#pragma unroll
    for (int f = 0; f < BB_FB; ++f) acc[f] = 0.0f;

    // window start for sensor s: 8-aligned, BB_MARGIN samples below the
    // smallest delay of every 32nd pixel of the workgroup (a scalar min over
    // the raw 32-bit delay codes, whose order is the order of the delays;
    // non-contributing codes sort last)
    auto probe = [&](int s) -> uint32_t {
        uint32_t m = 0xFFFFFFFFu;
        if (s < s_end) {
#pragma unroll
            for (int q = 0; q < BB_NPROBE; ++q)
                m = min(m, tab[(long)s * P + min(pbase + q * (BB_THREADS / BB_NPROBE), P - 1)]);
        }
        return m;
    };
    auto anchor_of = [&](uint32_t pr) -> int {
        int n;
        float a;
        return dec.decode(pr, N, n, a) ? floor8(n - BB_MARGIN - 1) : 0;
    };
    constexpr int NSLOT = (BB_FB * BB_CHUNKS + BB_THREADS - 1) / BB_THREADS;
    Raw8 rr[NSLOT];
    // window loads of sensor s into registers, all issued together
    auto stage_load = [&](int s, int A) {
#pragma unroll
        for (int r = 0; r < NSLOT; ++r) {
            const int idx = tid + r * BB_THREADS;
            if (idx < nf * BB_CHUNKS) {
                const int f = idx / BB_CHUNKS, k = idx % BB_CHUNKS;
                load8<SFMT>(sig, ((long)(f0 + f) * S + s) * N, A + 8 * k, N, rr[r]);
            }
        }
    };
    auto stage_store = [&](int buf) {
#pragma unroll
        for (int r = 0; r < NSLOT; ++r) {
            const int idx = tid + r * BB_THREADS;
            if (idx < nf * BB_CHUNKS) {
                const int f = idx / BB_CHUNKS, k = idx % BB_CHUNKS;
                store8<SFMT>(rr[r], &win[buf][f][8 * k]);
            }
        }
    };

    // pipeline: while sensor s is gathered from LDS, the window loads of s+1,
    // its delays and the probe of s+2 are in flight
    int A = 0;
    uint32_t pr1 = 0xFFFFFFFFu;
    uint32_t tcur = 0xFFFFFFFFu;
    if (s_begin < s_end) {
        A = anchor_of(probe(s_begin));
        stage_load(s_begin, A);
        tcur = pix_ok ? tab[(long)s_begin * P + p] : 0xFFFFFFFFu;
        pr1 = probe(s_begin + 1);
        stage_store(0);
    }
    __syncthreads();

    for (int s = s_begin; s < s_end; ++s) {
        const int buf = (s - s_begin) & 1;
        const bool more = s + 1 < s_end;
        uint32_t tnext = 0xFFFFFFFFu, pr2 = 0xFFFFFFFFu;
        int Anext = A;
        if (more) {
            Anext = anchor_of(pr1);
            stage_load(s + 1, Anext);
            tnext = pix_ok ? tab[(long)(s + 1) * P + p] : 0xFFFFFFFFu;
            pr2 = probe(s + 2);
        }
        int n;
        float a;
        if (dec.decode(tcur, N, n, a)) {
            float cf[4];
            coeffs<FILTERED>(n, a, w ? w[s] : 1.0f, N, t0dt, cf);
            const int j = n - 1 - A;
            if ((unsigned)j <= (unsigned)(BB_WS - 4)) {
                // all taps of the 16 frames first, so the LDS reads overlap
                uint32_t d0[BB_FB], d1[BB_FB], d2[BB_FB], d3[BB_FB];
#pragma unroll
                for (int f = 0; f < BB_FB; ++f) {
                    const uint32_t *wf = &win[buf][f][j];
                    if constexpr (SFMT == PAT_SIG_F16) {
                        if constexpr (FILTERED) {
                            d0[f] = wf[1];
                        } else {
                            d0[f] = wf[0];
                            d1[f] = wf[2];
                        }
                    } else {
                        if constexpr (FILTERED) {
                            d1[f] = wf[1];
                            d2[f] = wf[2];
                        } else {
                            d0[f] = wf[0];
                            d1[f] = wf[1];
                            d2[f] = wf[2];
                            d3[f] = wf[3];
                        }
                    }
                }
#pragma unroll
                for (int f = 0; f < BB_FB; ++f) {
                    if constexpr (SFMT == PAT_SIG_F16) {
                        if constexpr (FILTERED) {
                            acc[f] = fmaf(cf[1], lo_h(d0[f]), fmaf(cf[2], hi_h(d0[f]), acc[f]));
                        } else {
                            acc[f] = fmaf(cf[0], lo_h(d0[f]), fmaf(cf[1], hi_h(d0[f]),
                                     fmaf(cf[2], lo_h(d1[f]), fmaf(cf[3], hi_h(d1[f]), acc[f]))));
                        }
                    } else {
                        if constexpr (FILTERED) {
                            acc[f] = fmaf(cf[1], __uint_as_float(d1[f]), fmaf(cf[2], __uint_as_float(d2[f]), acc[f]));
                        } else {
                            acc[f] = fmaf(cf[0], __uint_as_float(d0[f]), fmaf(cf[1], __uint_as_float(d1[f]),
                                     fmaf(cf[2], __uint_as_float(d2[f]), fmaf(cf[3], __uint_as_float(d3[f]), acc[f]))));
                        }
                    }
                }
            } else {
                for (int f = 0; f < nf; ++f) {
                    const long row = ((long)(f0 + f) * S + s) * N;
                    const float x0 = raw_at<SFMT>(sig, row, n - 1, N), x1 = raw_at<SFMT>(sig, row, n, N);
                    const float x2 = raw_at<SFMT>(sig, row, n + 1, N), x3 = raw_at<SFMT>(sig, row, n + 2, N);
                    if constexpr (FILTERED) acc[f] = fmaf(cf[1], x1, fmaf(cf[2], x2, acc[f]));
                    else acc[f] = fmaf(cf[0], x0, fmaf(cf[1], x1, fmaf(cf[2], x2, fmaf(cf[3], x3, acc[f]))));
                }
            }
        }
        if (more) stage_store(buf ^ 1);
        tcur = tnext;
        A = Anext;
        pr1 = pr2;
        __syncthreads();
    }

    // finished sums (FP16 frames carry their scale)
    float outv[BB_FB];
#pragma unroll
    for (int f = 0; f < BB_FB; ++f) {
        const float sc = (SFMT == PAT_SIG_F16 && scale && f < nf) ? scale[f0 + f] : 1.0f;
        outv[f] = acc[f] * sc;
    }
    if (G == 1) {
        if (pix_ok)
            for (int f = 0; f < nf; ++f) img[(long)(f0 + f) * P + p] = outv[f];
        return;
    }
    if (pix_ok)
        for (int f = 0; f < nf; ++f) part[((long)g * F + f0 + f) * P + p] = outv[f];
    __threadfence();
    __syncthreads();
    if (tid == 0) {
        const unsigned int prev = atomicAdd(&done[(long)fg * gridDim.x + c], 1u);
        is_last = (prev == (unsigned)(G - 1)) ? 1u : 0u;
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    if (pix_ok) {
        for (int f = 0; f < nf; ++f) {
            float sum = 0.0f;
            for (int gg = 0; gg < G; ++gg) sum += __builtin_nontemporal_load(part + ((long)gg * F + f0 + f) * P + p);
            img[(long)(f0 + f) * P + p] = sum;
        }
    }
    if (tid == 0) done[(long)fg * gridDim.x + c] = 0u;
}

}  // namespace

size_t pat_batch_part_bytes(int S, int P, int F) {
    if (S <= 0 || P <= 0 || F < 2) return 0;
    const BbShape sh = bb_shape(S, P, F);
    return sh.groups > 1 ? (size_t)sh.groups * F * P * sizeof(float) : 0;
}

bool pat_batch_eligible(int sig_fmt, int N, int F, const void *sig) {
    if (F < 2) return false;
    const int mult = sig_fmt == PAT_SIG_F16 ? 8 : 4;
    return N % mult == 0 && ((uintptr_t)sig % 16) == 0 && N >= 16;
}

int pat_launch_backproject_batch(pat_ctx *ctx, const void *table, int table_fmt, const void *sig, int sig_fmt,
                                 int sig_is_filtered, const float *frame_scale, const float *w, int S, int P, int N,
                                 int F, double t0, double dt, float *img, hipStream_t st) {
    const BbShape sh = bb_shape(S, P, F);
    float *part = nullptr;
    unsigned int *done = nullptr;
    if (sh.groups > 1) {
        int rc = pat_gather_scratch(ctx, P, F, pat_batch_part_bytes(S, P, F), &part, &done, st);
        if (rc) return rc;
    }
    const dim3 grid(sh.chunks, sh.fgroups, sh.groups);
    const float t0dt = (float)(t0 / dt);
    const uint32_t *tab = static_cast<const uint32_t *>(table);
    const bool filt = sig_is_filtered != 0;
#define PAT_BB(DEC, SF, FI) \
    k_bp_batch<DEC, SF, FI><<<grid, BB_THREADS, 0, st>>>(tab, sig, frame_scale, w, S, P, N, F, sh.spg, sh.groups, d, t0dt, part, img, done)
    if (table_fmt == PAT_TABLE_F32) {
        DelayF32 d;
        const double inv = 1.0 / dt;
        d.inv_hi = (float)inv;
        d.inv_lo = (float)(inv - (double)d.inv_hi);
        d.off = (float)(-t0 / dt);
        d.umax = (float)(N - 1);
        if (sig_fmt == PAT_SIG_F32) { if (filt) PAT_BB(DelayF32, PAT_SIG_F32, true); else PAT_BB(DelayF32, PAT_SIG_F32, false); }
        else { if (filt) PAT_BB(DelayF32, PAT_SIG_F16, true); else PAT_BB(DelayF32, PAT_SIG_F16, false); }
    } else {
        DelayQ16 d;
        if (sig_fmt == PAT_SIG_F32) { if (filt) PAT_BB(DelayQ16, PAT_SIG_F32, true); else PAT_BB(DelayQ16, PAT_SIG_F32, false); }
        else { if (filt) PAT_BB(DelayQ16, PAT_SIG_F16, true); else PAT_BB(DelayQ16, PAT_SIG_F16, false); }
    }
#undef PAT_BB
    PAT_HIP(hipGetLastError());
    return PAT_OK;
}
