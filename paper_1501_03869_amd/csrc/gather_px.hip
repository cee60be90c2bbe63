// Back projection for frames too small to fill the GPU with LDS windows:
// 32 pixels per tile, each lane one pixel and one of two sensor slots, the
// sensors of a tile split over the slots of one workgroup and the partial sums
// added in LDS in slot order.
//
// The sum is the delay-and-sum of Section II: the filtered signal b of every
// sensor read at the pixel's delay with linear interpolation, weighted and
// summed over sensors.  Each lane reads its delay from the table (coalesced
// along pixels) and the raw samples n-1 .. n+2 around it with one 16-byte
// load, then evaluates the UBP filter (p - t dp/dt, central differences) for
// b[n] and b[n+1].  There is no LDS window, so no delay can miss one, and no
// workgroup depends on another: a launch is one pass with no partial sums in
// global memory.
//
// Loads go through buffer descriptors whose base is the wave's first record
// (scalar registers) and whose per-lane offset is 32 bits, so an address costs
// one vector instruction; the descriptor's range also bounds every access.
#include <mutex>

#include "gather_common.h"
#include "pat_internal.h"

using namespace pat_gather;

namespace {

constexpr int PX_T = 32;           // pixels per tile
constexpr int PX_U = 4;            // sensors per slot per pipeline step
constexpr int PX_MAX_WAVES = 16;   // waves per workgroup
constexpr int PX_RSRC_W3 = 0x00020000;  // buffer descriptor word 3: raw 32-bit dwords

struct PxShape {
    int tiles, waves, sps;  // sps: sensors per slot (two slots per wave)
};

// Waves per workgroup: as many as keep every workgroup of the launch resident
// at once (blocks_per_cu(W) * CUs >= tiles * F), so that no compute unit runs
// a second round while others idle; at most 16, at least 1.  blocks_per_cu
// comes from the runtime's occupancy calculator for the kernel that runs.
template <class BlocksPerCu>
PxShape px_shape(int S, int P, int F, int cus, BlocksPerCu blocks_per_cu) {
    PxShape s;
    s.tiles = (P + PX_T - 1) / PX_T;
    const long wgs = (long)s.tiles * std::max(F, 1);
    const int S1 = std::max(S, 1);
    int W = 1;
    for (int cand = PX_MAX_WAVES; cand >= 1; --cand) {
        if ((long)blocks_per_cu(cand) * cus >= wgs) { W = cand; break; }
    }
    W = std::min(W, (S1 + 1) / 2);
    W = std::max(W, 1);
    s.sps = (S1 + 2 * W - 1) / (2 * W);
    s.waves = (S1 + 2 * s.sps - 1) / (2 * s.sps);
    return s;
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, PX_RSRC_W3);
}

__device__ __forceinline__ float h2f(uint32_t bits16) {
    return __half2float(__ushort_as_half((unsigned short)bits16));
}

// q[0..3] = x[c .. c+3] of the record at byte offset roff, scaled for FP16.
// FP16 needs N even and c <= N - 4: three dwords from the even half e <= c
// (e + 5 <= N - 1), the wanted halves cut out of them.
template <int SFMT>
__device__ __forceinline__ void load4(__amdgpu_buffer_rsrc_t r, uint32_t roff, int soff, int c, int N, float sc,
                                      float (&q)[4]) {
    if constexpr (SFMT == PAT_SIG_F32) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, roff + 4u * (uint32_t)c, soff, 0);
        q[0] = __uint_as_float(v[0]); q[1] = __uint_as_float(v[1]);
        q[2] = __uint_as_float(v[2]); q[3] = __uint_as_float(v[3]);
    } else {
        const int e = min(c & ~1, N - 6);
        const int k = c - e;  // 0, 1 or 2
        const auto d = __builtin_amdgcn_raw_buffer_load_b96(r, roff + 2u * (uint32_t)e, soff, 0);
        const uint32_t mid0 = __builtin_amdgcn_alignbyte(d[1], d[0], 2);
        const uint32_t mid1 = __builtin_amdgcn_alignbyte(d[2], d[1], 2);
        const uint32_t e0 = k == 0 ? d[0] : (k == 1 ? mid0 : d[1]);
        const uint32_t e1 = k == 0 ? d[1] : (k == 1 ? mid1 : d[2]);
        q[0] = h2f(e0 & 0xFFFFu) * sc; q[1] = h2f(e0 >> 16) * sc;
        q[2] = h2f(e1 & 0xFFFFu) * sc; q[3] = h2f(e1 >> 16) * sc;
    }
}

// b[n], b[n+1] from filtered samples (n <= N - 2 always).
template <int SFMT>
__device__ __forceinline__ void load2(__amdgpu_buffer_rsrc_t r, uint32_t roff, int soff, int n, int N, float sc,
                                      float &b0, float &b1) {
    if constexpr (SFMT == PAT_SIG_F32) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, roff + 4u * (uint32_t)n, soff, 0);
        b0 = __uint_as_float(v[0]);
        b1 = __uint_as_float(v[1]);
    } else {
        const int e = min(n & ~1, N - 4);  // halves e .. e+3 (<= N-1, N even) hold n, n+1
        const int k = n - e;                 // 0, 1 or 2
        const auto d = __builtin_amdgcn_raw_buffer_load_b64(r, roff + 2u * (uint32_t)e, soff, 0);
        const uint32_t pair = k == 0 ? d[0] : (k == 1 ? __builtin_amdgcn_alignbyte(d[1], d[0], 2) : d[1]);
        b0 = h2f(pair & 0xFFFFu) * sc;
        b1 = h2f(pair >> 16) * sc;
    }
}

// One pipeline stage: the delays of U sensors of this lane's slot, decoded,
// and their samples.
struct Stage {
    uint32_t d[PX_U];
    int n[PX_U];
    float a[PX_U], w[PX_U], q[PX_U][4];
};

template <class Delay, int SFMT, bool FILTERED, bool HAS_W>
__global__ void __launch_bounds__(64 * PX_MAX_WAVES)
    k_bp_px(const uint32_t *__restrict__ tab, const void *__restrict__ sig, const float *__restrict__ scale,
            const float *__restrict__ w, int S, int P, int N, int sps, Delay dec, float t0dt,
            float *__restrict__ img) {
    __shared__ float red[2 * PX_MAX_WAVES][PX_T];
    const int f = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform: keeps descriptors scalar
    const int nw = blockDim.x >> 6;
    const int half = lane >> 5;
    const int px = lane & (PX_T - 1);
    const int p = blockIdx.x * PX_T + px;
    const int pc = min(p, P - 1);  // lanes past the end read a valid column and add nothing
    constexpr uint32_t esz = SFMT == PAT_SIG_F16 ? 2 : 4;
    const float sc = (SFMT == PAT_SIG_F16 && scale) ? scale[f] : 1.0f;

    // the wave's two slots: sensors sw .. sw+sps-1 (lanes 0-31) and
    // sw+sps .. sw+2sps-1 (lanes 32-63), both clipped to S
    const int sw = wv * 2 * sps;
    const int nrows = min(2 * sps, S - sw);
    const int s_lo = sw + half * sps;
    const int s_hi = min(S, s_lo + sps);
    const int nstep = (sps + PX_U - 1) / PX_U;
    const __amdgpu_buffer_rsrc_t rt = rsrc(tab + (size_t)sw * P, (uint32_t)nrows * (uint32_t)P * 4u);
    const char *fsig = static_cast<const char *>(sig) + ((size_t)f * S + sw) * N * esz;
    const __amdgpu_buffer_rsrc_t rs = rsrc(fsig, (uint32_t)nrows * (uint32_t)N * esz);
    const uint32_t toff = ((uint32_t)(half * sps) * (uint32_t)P + (uint32_t)pc) * 4u;
    const uint32_t roff = (uint32_t)(half * sps) * (uint32_t)N * esz;

    // Every step issues the same loads, so the waits between the stages are
    // static: a slot position past the slot's end (or a step past the last)
    // re-reads the slot's last record and contributes nothing.
    auto delays = [&](int i, Stage &st) {
#pragma unroll
        for (int j = 0; j < PX_U; ++j) {
            const int k = min(i * PX_U + j, sps - 1);
            st.d[j] = __builtin_amdgcn_raw_buffer_load_b32(rt, toff, k * P * 4, 0);
        }
    };
    // decode the delays of step i and issue its sample loads; returns whether
    // a contributing lane sits at an end of its record (n = 0 or N-2)
    auto samples = [&](int i, Stage &st) -> bool {
        bool end = false;
#pragma unroll
        for (int j = 0; j < PX_U; ++j) {
            const int k = i * PX_U + j;  // sensor within the slot
            int n = 1;
            float a = 0.0f;
            const bool dok = dec.decode(st.d[j], N, n, a);
            const bool ok = dok & (s_lo + k < s_hi);
            float ws = 1.0f;
            if constexpr (HAS_W) {
                const int kk = min(k, sps - 1);
                const float ws0 = w[min(sw + kk, S - 1)];
                const float ws1 = w[min(sw + sps + kk, S - 1)];
                ws = half ? ws1 : ws0;
            }
            st.w[j] = ok ? ws : 0.0f;
            st.n[j] = ok ? n : 1;
            st.a[j] = ok ? a : 0.0f;
            const int soff = min(k, sps - 1) * N * (int)esz;
            if constexpr (FILTERED) {
                load2<SFMT>(rs, roff, soff, st.n[j], N, sc, st.q[j][1], st.q[j][2]);
            } else {
                end |= ok & ((n == 0) | (n == N - 2));
                const int c = min(max(st.n[j] - 1, 0), N - 4);
                load4<SFMT>(rs, roff, soff, c, N, sc, st.q[j]);
            }
        }
        return end;
    };
    float acc = 0.0f;
    auto sum = [&](const Stage &st, bool any_end) {
#pragma unroll
        for (int j = 0; j < PX_U; ++j) {
            const int n = st.n[j];
            float b0, b1;
            if constexpr (FILTERED) {
                b0 = st.q[j][1];
                b1 = st.q[j][2];
            } else if (!any_end) {
                // every contributing lane has 1 <= n <= N-3, so q = p[n-1 .. n+2]
                // and both samples take central differences:
                // b[m] = p[m] - (m + t0/dt) * (p[m+1] - p[m-1]) / 2
                const float k0 = ((float)n + t0dt) * 0.5f;
                b0 = fmaf(-k0, st.q[j][2] - st.q[j][0], st.q[j][1]);
                b1 = fmaf(-(k0 + 0.5f), st.q[j][3] - st.q[j][1], st.q[j][2]);
            } else {  // q = p[c .. c+3] with c = n-1 clipped to [0, N-4]
                const int sh = (n - 1) - min(max(n - 1, 0), N - 4);  // -1 at n = 0, +1 at n = N-2
                const float pm = sh == 1 ? st.q[j][1] : st.q[j][0];
                const float p0 = sh < 0 ? st.q[j][0] : (sh == 0 ? st.q[j][1] : st.q[j][2]);
                const float p1 = sh < 0 ? st.q[j][1] : (sh == 0 ? st.q[j][2] : st.q[j][3]);
                const float p2 = sh < 0 ? st.q[j][2] : st.q[j][3];
                b0 = ubp(pm, p0, p1, n, N, t0dt);
                b1 = ubp(p0, p1, p2, n + 1, N, t0dt);
            }
            acc = fmaf(st.w[j], fmaf(st.a[j], b1 - b0, b0), acc);
        }
    };

    // two stages alternate: while step i is summed from one, the delays of
    // step i+2 and the samples of step i+1 are in flight in the other
    Stage A, B;
    delays(0, A);
    delays(1, B);
    bool endA = samples(0, A), endB = false;
    for (int i = 0; i < nstep; i += 2) {
        endB = samples(i + 1, B);
        delays(i + 2, A);
        sum(A, __any(endA));
        if (i + 1 >= nstep) break;
        endA = samples(i + 2, A);
        delays(i + 3, B);
        sum(B, __any(endB));
    }

    red[wv * 2 + half][px] = acc;
    __syncthreads();
    if (wv == 0 && half == 0 && p < P) {
        float s = 0.0f;
        for (int k = 0; k < 2 * nw; ++k) s += red[k][px];
        img[(long)f * P + p] = s;
    }
}

template <class Delay, int SFMT, bool FILTERED, bool HAS_W>
int launch_one(int S, int P, int F, const uint32_t *tab, const void *sig, const float *scale, const float *w, int N,
               Delay dec, float t0dt, float *img, hipStream_t st) {
    // occupancy per block size, computed once per kernel and device
    static std::mutex mu;
    static int cache_dev = -1, cache_cus = 0, cache_bpc[PX_MAX_WAVES + 1];
    int dev = 0;
    PAT_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    if (cache_dev != dev) {
        PAT_HIP(hipDeviceGetAttribute(&cache_cus, hipDeviceAttributeMultiprocessorCount, dev));
        for (int W = 1; W <= PX_MAX_WAVES; ++W)
            PAT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&cache_bpc[W], k_bp_px<Delay, SFMT, FILTERED, HAS_W>,
                                                                 64 * W, 0));
        cache_dev = dev;
    }
    const PxShape sh = px_shape(S, P, F, cache_cus, [&](int W) { return cache_bpc[W]; });
    const dim3 grid(sh.tiles, F);
    k_bp_px<Delay, SFMT, FILTERED, HAS_W><<<grid, dim3(64 * sh.waves), 0, st>>>(tab, sig, scale, w, S, P, N, sh.sps, dec,
                                                                         t0dt, img);
    PAT_HIP(hipGetLastError());
    return PAT_OK;
}

template <class Delay, int SFMT>
int launch_px(bool filtered, int S, int P, int F, const uint32_t *tab, const void *sig, const float *scale,
              const float *w, int N, Delay dec, float t0dt, float *img, hipStream_t st) {
    if (w)
        return filtered ? launch_one<Delay, SFMT, true, true>(S, P, F, tab, sig, scale, w, N, dec, t0dt, img, st)
                        : launch_one<Delay, SFMT, false, true>(S, P, F, tab, sig, scale, w, N, dec, t0dt, img, st);
    return filtered ? launch_one<Delay, SFMT, true, false>(S, P, F, tab, sig, scale, w, N, dec, t0dt, img, st)
                    : launch_one<Delay, SFMT, false, false>(S, P, F, tab, sig, scale, w, N, dec, t0dt, img, st);
}

}  // namespace

bool pat_px_eligible(int sig_fmt, int S, int P, int N, int F, const void *sig) {
    if (S <= 0 || P <= 0 || F <= 0) return false;
    const size_t esz = sig_fmt == PAT_SIG_F16 ? 2 : 4;
    if (sig_fmt == PAT_SIG_F16 && (N < 6 || N % 2 != 0 || (uintptr_t)sig % 4 != 0)) return false;
    if (sig_fmt == PAT_SIG_F32 && (N < 4 || (uintptr_t)sig % 4 != 0)) return false;
    // 32-bit buffer offsets: the two slots of a wave span at most 2*ceil(S/2)
    // records (the shape with one wave per workgroup)
    const size_t rows = 2 * (((size_t)S + 1) / 2);
    return rows * (size_t)P * 4 < (1ull << 31) && rows * (size_t)N * esz < (1ull << 31);
}

int pat_launch_backproject_px(const void *table, int table_fmt, const void *sig, int sig_fmt, int sig_is_filtered,
                              const float *frame_scale, const float *w, int S, int P, int N, int F, double t0,
                              double dt, float *img, hipStream_t st) {
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
                   ? launch_px<DelayF32, PAT_SIG_F32>(filt, S, P, F, tab, sig, frame_scale, w, N, d, t0dt, img, st)
                   : launch_px<DelayF32, PAT_SIG_F16>(filt, S, P, F, tab, sig, frame_scale, w, N, d, t0dt, img, st);
    }
    DelayQ16 d;
    return sig_fmt == PAT_SIG_F32
               ? launch_px<DelayQ16, PAT_SIG_F32>(filt, S, P, F, tab, sig, frame_scale, w, N, d, t0dt, img, st)
               : launch_px<DelayQ16, PAT_SIG_F16>(filt, S, P, F, tab, sig, frame_scale, w, N, d, t0dt, img, st);
}
