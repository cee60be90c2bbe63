// Back projection for frames too small to fill the GPU with LDS windows:
// one pixel per lane, the sensors of a 64-pixel tile split over the waves of
// one workgroup, the partial sums added in LDS in wave order.
//
// The sum itself is the delay-and-sum of Section II (filtered signal b of
// every sensor, read at the pixel's delay with linear interpolation,
// weighted, summed over sensors).  Each lane reads its delay from the table
// (coalesced along pixels) and the four raw samples n-1 .. n+2 around it with
// one vector load; the UBP filter (p - t dp/dt, central differences) is
// evaluated on them for b[n] and b[n+1].  There is no LDS window, so no delay
// can miss one, and no workgroup depends on another: a launch is one pass
// with no partial sums in global memory.
#include "gather_common.h"
#include "pat_internal.h"

using namespace pat_gather;

namespace {

constexpr int PX_WAVE = 64;        // pixels per tile, one per lane
constexpr int PX_U = 4;            // sensors per pipeline step
constexpr int PX_MAX_WAVES = 16;   // waves per workgroup (sensor split)
constexpr int PX_TARGET = 8192;    // waves per launch the split aims for

struct PxShape {
    int tiles, waves, spw;
};

PxShape px_shape(int S, int P, int F) {
    PxShape s;
    s.tiles = (P + PX_WAVE - 1) / PX_WAVE;
    const long per = (long)s.tiles * std::max(F, 1);
    int W = (int)std::min<long>(PX_MAX_WAVES, std::max<long>(1, (PX_TARGET + per - 1) / per));
    W = std::min(W, std::max(S, 1));
    s.spw = (std::max(S, 1) + W - 1) / W;
    s.waves = (std::max(S, 1) + s.spw - 1) / s.spw;
    return s;
}

// x[c .. c+3] of one record, scaled for FP16.  FP32: one 16-byte load at a
// 4-byte-aligned address.  FP16 (N even, record 4-byte aligned): three
// aligned dwords holding halves e .. e+5 with e even and e + 5 <= N - 1, and
// the four wanted halves cut out of them.
template <int SFMT>
__device__ __forceinline__ void load4(const void *__restrict__ sig, long row, int c, int N, float sc, float (&q)[4]) {
    if constexpr (SFMT == PAT_SIG_F32) {
        float4 v;
        __builtin_memcpy(&v, static_cast<const float *>(sig) + row + c, sizeof(v));
        q[0] = v.x; q[1] = v.y; q[2] = v.z; q[3] = v.w;
    } else {
        const int e = min(c & ~1, N - 6);
        const int r = c - e;  // 0, 1 or 2
        uint32_t d[3];
        __builtin_memcpy(d, static_cast<const uint32_t *>(sig) + ((row + e) >> 1), sizeof(d));
        const uint32_t mid0 = __builtin_amdgcn_alignbyte(d[1], d[0], 2);
        const uint32_t mid1 = __builtin_amdgcn_alignbyte(d[2], d[1], 2);
        const uint32_t e0 = r == 0 ? d[0] : (r == 1 ? mid0 : d[1]);
        const uint32_t e1 = r == 0 ? d[1] : (r == 1 ? mid1 : d[2]);
        q[0] = __half2float(__ushort_as_half((unsigned short)(e0 & 0xFFFFu))) * sc;
        q[1] = __half2float(__ushort_as_half((unsigned short)(e0 >> 16))) * sc;
        q[2] = __half2float(__ushort_as_half((unsigned short)(e1 & 0xFFFFu))) * sc;
        q[3] = __half2float(__ushort_as_half((unsigned short)(e1 >> 16))) * sc;
    }
}

template <class Delay, int SFMT, bool FILTERED>
__global__ void __launch_bounds__(PX_WAVE *PX_MAX_WAVES)
    k_bp_px(const uint32_t *__restrict__ tab, const void *__restrict__ sig, const float *__restrict__ scale,
            const float *__restrict__ w, int S, int P, int N, int spw, Delay dec, float t0dt,
            float *__restrict__ img) {
    __shared__ float red[PX_MAX_WAVES][PX_WAVE];
    const int f = blockIdx.y;
    const int lane = threadIdx.x & (PX_WAVE - 1);
    const int wv = threadIdx.x / PX_WAVE;
    const int nw = blockDim.x / PX_WAVE;
    const int p = blockIdx.x * PX_WAVE + lane;
    const int pc = min(p, P - 1);  // lanes past the end read a valid column and add nothing
    const size_t esz = SFMT == PAT_SIG_F16 ? 2 : 4;
    const void *fsig = static_cast<const char *>(sig) + (size_t)f * S * N * esz;
    const float sc = (SFMT == PAT_SIG_F16 && scale) ? scale[f] : 1.0f;
    const int s_begin = wv * spw;
    const int s_end = min(S, s_begin + spw);
    const int nstep = s_end > s_begin ? (s_end - s_begin + PX_U - 1) / PX_U : 0;

    // Step i covers sensors s_begin + i*U + j.  A slot past s_end (or a step
    // past the last) holds the code of a delay that does not contribute; its
    // sample loads read record 0 of this wave's first sensor.  The table is
    // streamed once, so its loads are marked non-temporal to leave the caches
    // to the signals, which every tile re-reads.
    auto delays = [&](int i, uint32_t (&d)[PX_U]) {
#pragma unroll
        for (int j = 0; j < PX_U; ++j) {
            const int s = s_begin + i * PX_U + j;
            d[j] = (i < nstep && s < s_end) ? __builtin_nontemporal_load(tab + (long)s * P + pc) : 0xFFFFFFFFu;
        }
    };
    auto samples = [&](int i, const uint32_t (&d)[PX_U], float (&q)[PX_U][4]) {
#pragma unroll
        for (int j = 0; j < PX_U; ++j) {
            int n = 0;
            float a;
            if (!dec.decode(d[j], N, n, a)) n = 0;
            const int s = min(s_begin + i * PX_U + j, s_end - 1);
            load4<SFMT>(fsig, (long)s * N, min(max(n - 1, 0), N - 4), N, sc, q[j]);
        }
    };

    float acc = 0.0f;
    uint32_t d0[PX_U], d1[PX_U], d2[PX_U];
    float q0[PX_U][4], q1[PX_U][4];
    delays(0, d0);
    delays(1, d1);
    samples(0, d0, q0);
    for (int i = 0; i < nstep; ++i) {
        // in flight while step i is summed: the delays of step i+2 and the
        // samples of step i+1
        delays(i + 2, d2);
        if (i + 1 < nstep) samples(i + 1, d1, q1);
#pragma unroll
        for (int j = 0; j < PX_U; ++j) {
            int n = 0;
            float a = 0.0f;
            const bool ok = dec.decode(d0[j], N, n, a);
            const int s = s_begin + i * PX_U + j;
            const float ws = ok ? (w ? w[min(s, S - 1)] : 1.0f) : 0.0f;
            n = ok ? n : 0;
            a = ok ? a : 0.0f;
            const int sh = (n - 1) - min(max(n - 1, 0), N - 4);  // -1 at n = 0, +1 at n = N-2, else 0
            const float pm = sh == 1 ? q0[j][1] : q0[j][0];
            const float p0 = sh < 0 ? q0[j][0] : (sh == 0 ? q0[j][1] : q0[j][2]);
            const float p1 = sh < 0 ? q0[j][1] : (sh == 0 ? q0[j][2] : q0[j][3]);
            const float p2 = sh < 0 ? q0[j][2] : q0[j][3];
            float b0, b1;
            if constexpr (FILTERED) {
                b0 = p0;
                b1 = p1;
            } else {
                b0 = ubp(pm, p0, p1, n, N, t0dt);
                b1 = ubp(p0, p1, p2, n + 1, N, t0dt);
            }
            acc = fmaf(ws, fmaf(a, b1 - b0, b0), acc);
        }
#pragma unroll
        for (int j = 0; j < PX_U; ++j) {
            d0[j] = d1[j];
            d1[j] = d2[j];
#pragma unroll
            for (int k = 0; k < 4; ++k) q0[j][k] = q1[j][k];
        }
    }

    red[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && p < P) {
        float s = 0.0f;
        for (int k = 0; k < nw; ++k) s += red[k][lane];
        img[(long)f * P + p] = s;
    }
}

template <class Delay, int SFMT>
int launch_px(bool filtered, const PxShape &sh, int F, const uint32_t *tab, const void *sig, const float *scale,
              const float *w, int S, int P, int N, Delay dec, float t0dt, float *img, hipStream_t st) {
    const dim3 grid(sh.tiles, F);
    const dim3 block(PX_WAVE * sh.waves);
    if (filtered)
        k_bp_px<Delay, SFMT, true><<<grid, block, 0, st>>>(tab, sig, scale, w, S, P, N, sh.spw, dec, t0dt, img);
    else
        k_bp_px<Delay, SFMT, false><<<grid, block, 0, st>>>(tab, sig, scale, w, S, P, N, sh.spw, dec, t0dt, img);
    PAT_HIP(hipGetLastError());
    return PAT_OK;
}

}  // namespace

bool pat_px_eligible(int sig_fmt, int N, const void *sig) {
    if (sig_fmt == PAT_SIG_F16) return N >= 6 && N % 2 == 0 && ((uintptr_t)sig % 4) == 0;
    return N >= 4;
}

int pat_launch_backproject_px(const void *table, int table_fmt, const void *sig, int sig_fmt, int sig_is_filtered,
                              const float *frame_scale, const float *w, int S, int P, int N, int F, double t0,
                              double dt, float *img, hipStream_t st) {
    const PxShape sh = px_shape(S, P, F);
    const float t0dt = (float)(t0 / dt);
    const bool filt = sig_is_filtered != 0;
    const uint32_t *tab = static_cast<const uint32_t *>(table);
    if (table_fmt == PAT_TABLE_F32) {
        DelayF32 d;
        const double inv = 1.0 / dt;
        d.inv_hi = (float)inv;
        d.inv_lo = (float)(inv - (double)d.inv_hi);
        d.off = (float)(-t0 / dt);
        d.umax = (float)(N - 1);
        return sig_fmt == PAT_SIG_F32
                   ? launch_px<DelayF32, PAT_SIG_F32>(filt, sh, F, tab, sig, frame_scale, w, S, P, N, d, t0dt, img, st)
                   : launch_px<DelayF32, PAT_SIG_F16>(filt, sh, F, tab, sig, frame_scale, w, S, P, N, d, t0dt, img, st);
    }
    DelayQ16 d;
    return sig_fmt == PAT_SIG_F32
               ? launch_px<DelayQ16, PAT_SIG_F32>(filt, sh, F, tab, sig, frame_scale, w, S, P, N, d, t0dt, img, st)
               : launch_px<DelayQ16, PAT_SIG_F16>(filt, sh, F, tab, sig, frame_scale, w, S, P, N, d, t0dt, img, st);
}
