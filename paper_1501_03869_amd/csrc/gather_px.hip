// Back projection for frames too small to fill the GPU with LDS windows, and
// for the frame server: 32 pixels per tile, each lane one pixel and one of two
// sensor slots, the sensors of a tile split over the slots of one workgroup
// and the partial sums added in LDS in slot order.
//
// The sum is the delay-and-sum of Section II: the filtered signal b of every
// sensor read at the pixel's delay with linear interpolation, weighted and
// summed over sensors.  Each lane reads its delay from the table (coalesced
// along pixels) and the raw samples n-1 .. n+2 around it with one vector load,
// then evaluates the UBP filter (p - t dp/dt, central differences) for b[n]
// and b[n+1].  There is no LDS window, so no delay can miss one, and no
// workgroup depends on another: a launch is one pass with no partial sums in
// global memory.
//
// Loads go through buffer descriptors whose base is the wave's first record
// (scalar registers) and whose per-lane offset is 32 bits, so an address costs
// one or two vector instructions; the descriptor's range also bounds every
// access.
#include <mutex>
#include <type_traits>

#include "gather_common.h"
#include "pat_internal.h"

using namespace pat_gather;

namespace {

constexpr int PX_T = 32;           // pixels per tile
constexpr int PX_U = 4;            // sensors per slot per pipeline step
constexpr int PX_MAX_WAVES = 16;   // waves per workgroup
constexpr int PX_MULTI_WAVES = 8;  // waves per workgroup of the multi-frame kernel
constexpr int PX_RSRC_W3 = 0x00020000;  // buffer descriptor word 3: raw 32-bit dwords

struct PxShape {
    int tiles, waves, sps;  // sps: sensors per slot (two slots per wave)
};

int px_sps(int S, int W) {
    const int S1 = std::max(S, 1);
    W = std::max(1, std::min(W, (S1 + 1) / 2));
    const int sps = (S1 + 2 * W - 1) / (2 * W);
    // whole pipeline steps: only a wave's last step can have empty slots,
    // and only in the last wave
    return (sps + PX_U - 1) / PX_U * PX_U;
}

// Waves per workgroup: about per_cu waves per compute unit over the launch
// (enough to cover the load latency, with each wave's pipeline as long as
// that allows), and never more than keep every workgroup resident at once
// (blocks_per_cu(W) * CUs >= tiles * F), so that no compute unit runs a
// second round while others idle; at most 16, at least 1.  blocks_per_cu
// comes from the runtime's occupancy calculator for the kernel that runs.
// Measured with graph-replayed launches at the paper, 3-D head and 512^2
// serving geometries: FP32 samples do best near 12 waves per CU (3 per
// SIMD), FP16 samples, whose steps carry more VALU, near 24; against the
// most resident waves that is 2-17 % faster per launch.
constexpr int PX_WAVES_PER_CU_F32 = 12, PX_WAVES_PER_CU_F16 = 24;
template <class BlocksPerCu>
PxShape px_shape(int S, int P, int F, int cus, long per_cu, BlocksPerCu blocks_per_cu) {
    PxShape s;
    s.tiles = (P + PX_T - 1) / PX_T;
    const long wgs = (long)s.tiles * std::max(F, 1);
    int W = 1;
    for (int cand = PX_MAX_WAVES; cand >= 1; --cand) {
        if ((long)blocks_per_cu(cand) * cus >= wgs) { W = cand; break; }
    }
    const long target = (per_cu * cus + wgs / 2) / wgs;
    W = (int)std::max(1L, std::min<long>(W, target));
    s.sps = px_sps(S, W);
    s.waves = (std::max(S, 1) + 2 * s.sps - 1) / (2 * s.sps);
    return s;
}

// 32-bit offsets: a step's descriptors span 2*U records of the table and of
// the signal, with room for the FP16 alignment residue
bool px_offsets_fit(int P, int N, int sig_fmt) {
    const size_t rows = 2 * (size_t)PX_U;
    const size_t esz = sig_fmt == PAT_SIG_F16 ? 2 : 4;
    return rows * (size_t)P * 4 < (1ull << 31) && (rows * (size_t)N + 8) * esz < (1ull << 31);
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, PX_RSRC_W3);
}

__device__ __forceinline__ float h2f(uint32_t bits16) {
    return __half2float(__ushort_as_half((unsigned short)bits16));
}

// One workgroup's work: tile `tile` of one frame, all S sensors.
struct PxJob {
    const uint32_t *tab;  // [S][P] delays
    const void *sig;      // [S][N] samples of this frame
    const float *w;       // [S] weights (read only when HAS_W)
    float *img;           // [P] output of this frame
    int S, P, N, sps;
    float t0dt, scale;
    // straight-ray delays |x - s| / c instead of a table (conventional back
    // projection): pixel node indices, sensor positions, grid
    const int32_t *pix;
    const float *sxy;     // [S][2] metres (2-D) or [S][3] (3-D)
    int nx, ny;
    float h, x0, y0, z0, inv_c;
};

// One pipeline stage: the delays of U sensors of this lane's slot as loaded
// (d, overwritten by the loads two steps ahead) and as decoded for the sum
// (x: the sample position u for FP32 tables, as bits, or the 16.16 index;
// nf: for FP32 tables the sample index n clamped into the fast range, as a
// float), and their samples.  The fast path's interpolation weight and filter factor follow
// from x and nf when the step is summed, and the general path decodes x
// again; one register per slot less than keeping them.
struct Stage {
    uint32_t d[PX_U], h[PX_U], x[PX_U];  // h: 16-bit tables' tile headers
    float nf[PX_U], q[PX_U][4];
};

// The sensors of wave wv for pixel tile*32 + lane%32: the wave owns sensors
// sw .. sw+2*sps-1 (sw = wv*2*sps, clipped to S); lanes 0-31 take the even
// ones, lanes 32-63 the odd ones.  wv must be wave-uniform (a scalar) and
// sw < S.
// SHDR: 16-bit tables' tile headers by two scalar loads per record pair
// (the table pointer is a read-only kernel argument); else by a vector load
// per lane.
template <class Delay, int SFMT, bool FILTERED, bool HAS_W, int CONSTC = 0, bool SHDR = true>
__device__ __forceinline__ float px_slot_sum(const PxJob &J, const Delay &dec, int tile, int wv) {
    const int S = J.S, P = J.P, N = J.N, sps = J.sps;
    const float t0dt = J.t0dt, sc = J.scale;
    const int lane = threadIdx.x & 63;
    const int half = lane >> 5;
    const int p = tile * PX_T + (lane & (PX_T - 1));
    const int pc = min(p, P - 1);  // lanes past the end read a valid column and add nothing
    const int sw = wv * 2 * sps;
    const int se = min(S, sw + 2 * sps);  // end of this wave's sensors
    // Record of slot j of this half within a step: 2j + half, or 4 half + j
    // for tables with four sensors interleaved per pixel (whose 16-byte load
    // holds the step's four consecutive sensors of one half)
    constexpr int kJR = Delay::kX4 ? 1 : 2;
    const int hr = Delay::kX4 ? 4 * half : half;
    const int nstep = (se - sw + 2 * PX_U - 1) / (2 * PX_U);  // steps of this wave (the last may hold fewer sensors)
    constexpr uint32_t esz = SFMT == PAT_SIG_F16 ? 2 : 4;
    // Step i covers sensors s0 + 2j + half (j < U) with s0 = sw + 2*i*U.  Its
    // descriptors start at record s0 (scalar registers) and end at the last
    // record the step may touch, so per-lane offsets stay below 2*U records
    // however large the table is.  Signal records start on a dword for FP32;
    // for FP16 the base is rounded down to a dword and sample offsets count
    // from there (res = 0 or 1 sample), and the fast path's loads start on the
    // dword holding the first wanted sample.
    const uint32_t toff = ((uint32_t)(half * P) + (uint32_t)pc) * 4u;
    auto step_s0 = [&](int i) { return min(sw + 2 * i * PX_U, se - 1); };
    auto tab_rsrc = [&](int s0) {
        return rsrc(J.tab + (size_t)s0 * P, (uint32_t)min(2 * PX_U, S - s0) * (uint32_t)P * 4u);
    };
    // 16-bit tables: offsets [S][P] and tile headers [S][tiles] (one header
    // per half-wave and sensor, read by all its lanes)
    const int tiles = (P + PX_T - 1) / PX_T;
    const uint16_t *off16 = reinterpret_cast<const uint16_t *>(J.tab);
    const uint32_t *hdr32 =
        reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(J.tab) + pat_r16_hdr_offset(S, P));
    const uint32_t ooff = ((uint32_t)(half * P) + (uint32_t)pc) * 2u;
    const uint32_t hoff = ((uint32_t)(half * tiles) + (uint32_t)tile) * 4u;
    struct SigRsrc {
        __amdgpu_buffer_rsrc_t r;
        uint32_t res;
    };
    auto sig_rsrc = [&](int s0) {
        const uintptr_t a = reinterpret_cast<uintptr_t>(J.sig) + (size_t)s0 * N * esz;
        const uint32_t n = (uint32_t)min(2 * PX_U, S - s0) * (uint32_t)N;
        SigRsrc g;
        g.res = (uint32_t)(a & 3u) / esz;
        g.r = rsrc(reinterpret_cast<const void *>(a & ~(uintptr_t)3), ((g.res + n) * esz + 3u) & ~3u);
        return g;
    };

    // q[0..3] = x[c .. c+3] of record r = 2j + half of the step.  FP16: the
    // three dwords from the one holding c, and the byte shift of c inside the
    // first (0 or 2) in q[3]; the samples are cut out (unscaled) only when
    // they are summed, so nothing waits for the load here.  The third dword
    // may hold no wanted sample: the fast range ends a sample early for FP16
    // so that it still lies in the record.
    auto load4 = [&](const SigRsrc &g, int j, int c, float (&q)[4]) {
        if constexpr (SFMT == PAT_SIG_F32) {
            const auto v = __builtin_amdgcn_raw_buffer_load_b128(g.r, 4u * ((uint32_t)(hr * N) + (uint32_t)c),
                                                                 kJR * j * N * 4, 0);
            q[0] = __uint_as_float(v[0]); q[1] = __uint_as_float(v[1]);
            q[2] = __uint_as_float(v[2]); q[3] = __uint_as_float(v[3]);
        } else {
            const uint32_t h = g.res + (uint32_t)((kJR * j + hr) * N + c);
            const auto v = __builtin_amdgcn_raw_buffer_load_b96(g.r, 2u * (h & ~1u), 0, 0);
            q[0] = __uint_as_float(v[0]);
            q[1] = __uint_as_float(v[1]);
            q[2] = __uint_as_float(v[2]);
            q[3] = __uint_as_float((h & 1u) * 2u);
        }
    };
    // the four samples of a stage slot as floats (FP16: unscaled)
    auto taps = [&](const float (&q)[4], float (&p)[4]) {
        if constexpr (SFMT == PAT_SIG_F32) {
            p[0] = q[0]; p[1] = q[1]; p[2] = q[2]; p[3] = q[3];
        } else {
            const uint32_t d0 = __float_as_uint(q[0]), d1 = __float_as_uint(q[1]), d2 = __float_as_uint(q[2]);
            const uint32_t sh = __float_as_uint(q[3]);
            const uint32_t e0 = __builtin_amdgcn_alignbyte(d1, d0, sh), e1 = __builtin_amdgcn_alignbyte(d2, d1, sh);
            p[0] = h2f(e0 & 0xFFFFu); p[1] = h2f(e0 >> 16);
            p[2] = h2f(e1 & 0xFFFFu); p[3] = h2f(e1 >> 16);
        }
    };
    // b[n], b[n+1] of record 2j + half of the step (filtered input; n <= N-2)
    // into q[1], q[2]; FP16: the two dwords from the one holding n and the
    // byte shift of n in q[3], cut out when summed
    auto load2 = [&](const SigRsrc &g, int j, int n, float (&q)[4]) {
        if constexpr (SFMT == PAT_SIG_F32) {
            const auto v = __builtin_amdgcn_raw_buffer_load_b64(g.r, 4u * ((uint32_t)(hr * N) + (uint32_t)n),
                                                                kJR * j * N * 4, 0);
            q[1] = __uint_as_float(v[0]);
            q[2] = __uint_as_float(v[1]);
        } else {
            const uint32_t h = g.res + (uint32_t)((kJR * j + hr) * N + n);
            const auto v = __builtin_amdgcn_raw_buffer_load_b64(g.r, 2u * (h & ~1u), 0, 0);
            q[1] = __uint_as_float(v[0]);
            q[2] = __uint_as_float(v[1]);
            q[3] = __uint_as_float((h & 1u) * 2u);
        }
    };
    auto pair = [&](const float (&q)[4], float &b0, float &b1) {
        if constexpr (SFMT == PAT_SIG_F32) {
            b0 = q[1];
            b1 = q[2];
        } else {
            const uint32_t e = __builtin_amdgcn_alignbyte(__float_as_uint(q[2]), __float_as_uint(q[1]),
                                                          __float_as_uint(q[3]));
            b0 = h2f(e & 0xFFFFu);
            b1 = h2f(e >> 16);
        }
    };

    // Every step issues the same loads, so the waits between the stages are
    // static: a step past the last re-reads the wave's last records, and a
    // sensor past the wave's end reads zeros (outside the descriptor) and
    // contributes nothing.
    float pxx = 0.0f, pxy = 0.0f, pxz = 0.0f;  // this lane's node position (straight-ray delays)
    if constexpr (CONSTC == 2) {
        const int k = J.pix[pc];
        pxx = J.x0 + (float)(k % J.nx) * J.h;
        pxy = J.y0 + (float)(k / J.nx) * J.h;
    } else if constexpr (CONSTC == 3) {
        const int k = J.pix[pc];
        pxx = J.x0 + (float)(k % J.nx) * J.h;
        pxy = J.y0 + (float)((k / J.nx) % J.ny) * J.h;
        pxz = J.z0 + (float)(k / (J.nx * J.ny)) * J.h;
    }
    auto delays = [&](int i, Stage &st) {
        if constexpr (CONSTC == 2) {
            const int s0 = step_s0(i);
#pragma unroll
            for (int j = 0; j < PX_U; ++j) {
                const int sa = min(s0 + 2 * j, S - 1), sb = min(s0 + 2 * j + 1, S - 1);
                const float sx = half ? J.sxy[2 * sb] : J.sxy[2 * sa];
                const float sy = half ? J.sxy[2 * sb + 1] : J.sxy[2 * sa + 1];
                const float dx = pxx - sx, dy = pxy - sy;
                st.d[j] = __float_as_uint(__builtin_amdgcn_sqrtf(fmaf(dx, dx, dy * dy)) * J.inv_c);
            }
        } else if constexpr (CONSTC == 3) {
            const int s0 = step_s0(i);
#pragma unroll
            for (int j = 0; j < PX_U; ++j) {
                const int sa = min(s0 + 2 * j, S - 1), sb = min(s0 + 2 * j + 1, S - 1);
                const int sr = half ? sb : sa;
                const float dx = pxx - J.sxy[3 * sr], dy = pxy - J.sxy[3 * sr + 1], dz = pxz - J.sxy[3 * sr + 2];
                st.d[j] = __float_as_uint(__builtin_amdgcn_sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz))) * J.inv_c);
            }
        } else if constexpr (Delay::kR16) {
            const int s0 = step_s0(i);
            const uint32_t rows = (uint32_t)min(2 * PX_U, S - s0);
            const __amdgpu_buffer_rsrc_t ro = rsrc(off16 + (size_t)s0 * P, rows * (uint32_t)P * 2u);
            // a tile header is the same for the 32 lanes of a half-wave: two
            // scalar loads per record pair (records past S read the last one,
            // for slots that contribute nothing)
            const __amdgpu_buffer_rsrc_t rh = rsrc(hdr32 + (size_t)s0 * tiles, rows * (uint32_t)tiles * 4u);
#pragma unroll
            for (int j = 0; j < PX_U; ++j) {
                st.d[j] = __builtin_amdgcn_raw_buffer_load_b16(ro, ooff, 2 * j * P * 2, 0);
                if constexpr (SHDR) {
                    const int se0 = min(s0 + 2 * j, S - 1), so0 = min(s0 + 2 * j + 1, S - 1);
                    const uint32_t he = hdr32[(size_t)se0 * tiles + tile], ho = hdr32[(size_t)so0 * tiles + tile];
                    st.h[j] = half ? ho : he;
                } else {
                    st.h[j] = __builtin_amdgcn_raw_buffer_load_b32(rh, hoff, 2 * j * tiles * 4, 0);
                }
            }
        } else if constexpr (Delay::kX4) {
            // quads q0 (this step's first four sensors, half 0) and q0 + 1
            // (half 1): one 16-byte load per lane; a step past the wave's
            // end re-reads the quad of its last sensor
            const int q0 = step_s0(i) >> 2;
            const uint32_t quads = (uint32_t)min(2, ((S + 3) >> 2) - q0);
            const __amdgpu_buffer_rsrc_t rt = rsrc(J.tab + (size_t)q0 * P * 4, quads * (uint32_t)P * 16u);
            const auto v = __builtin_amdgcn_raw_buffer_load_b128(rt, ((uint32_t)(half * P) + (uint32_t)pc) * 16u, 0, 0);
#pragma unroll
            for (int j = 0; j < PX_U; ++j) st.d[j] = v[j];
        } else {
            const __amdgpu_buffer_rsrc_t rt = tab_rsrc(step_s0(i));
#pragma unroll
            for (int j = 0; j < PX_U; ++j) st.d[j] = __builtin_amdgcn_raw_buffer_load_b32(rt, toff, 2 * j * P * 4, 0);
        }
    };
    // Decode the delays of step i and issue its sample loads.  Returns whether
    // a lane of the wave needs the general path for the step: a slot of the step holds
    // no sensor, or a delay lies outside the fast range, where the filter's
    // taps p[n-1 .. n+2] (raw input) or the two samples b[n], b[n+1]
    // (filtered input) are inside the record and the delay contributes.  The
    // sample index is clamped into the fast range for every lane, which makes
    // the first tap n-1 (or n) clipped to [0, N-4] (or [0, N-2]), the start
    // the general path expects, so both paths read the same FP32 loads (FP16:
    // the general path reads its samples again).
    const float t0h = 0.5f * t0dt;
    constexpr int LO = FILTERED ? 0 : 1;
    // FP16 loads start on a dword and read up to two samples past the last
    // tap: the fast range ends one sample earlier so that they stay in the
    // record
    constexpr bool F16 = SFMT == PAT_SIG_F16;
    const int HI = (FILTERED ? N - 1 : N - 2) - (F16 ? 1 : 0);
    // F32 decoding: the offset -t0/dt in a vector register, so the decode's
    // FMA reads only one scalar operand
    Delay dv = dec;
    constexpr bool kF32T = std::is_base_of<DelayF32, Delay>::value;
    if constexpr (kF32T) {
        float offv;
        asm("v_mov_b32 %0, %1" : "=v"(offv) : "s"(dec.off));
        dv.off = offv;
    }
    auto samples = [&](int i, Stage &st) -> bool {
        const SigRsrc g = sig_rsrc(step_s0(i));
        uint64_t slow = sw + 2 * (i + 1) * PX_U <= se ? 0ull : ~0ull;
#pragma unroll
        for (int j = 0; j < PX_U; ++j) {
            int n;
            float a;
            uint32_t dq = st.d[j];
            if constexpr (Delay::kR16) dq = DelayR16::to_q16(st.d[j], st.h[j]);
            slow |= __builtin_amdgcn_ballot_w64(!dv.decode_in(dq, LO, HI, n, a));
            if constexpr (kF32T) {
                st.x[j] = __float_as_uint(dv.u1(__uint_as_float(dq)));
                st.nf[j] = (float)n;
            } else {
                st.x[j] = dq;
            }
            // lo <= n <= hi-1: the first tap n-1 (raw) or n (filtered) is the
            // same clipped start the general path assumes
            if constexpr (FILTERED) {
                load2(g, j, n, st.q[j]);
            } else {
                load4(g, j, n - 1, st.q[j]);
            }
        }
        return slow != 0;  // wave-uniform
    };
    float acc = 0.0f;
    auto sum = [&](const Stage &st, int i, bool general) {
        const int s0 = sw + 2 * i * PX_U;
        if (!general) {
            // every slot holds a sensor and every delay is in the fast range:
            // q = p[n-1 .. n+2] and both samples take central differences,
            // b[m] = p[m] - (m + t0/dt) * (p[m+1] - p[m-1]) / 2
#pragma unroll
            for (int j = 0; j < PX_U; ++j) {
                // in the fast range u is unclamped, so a = u - n
                const float a = kF32T ? __uint_as_float(st.x[j]) - st.nf[j]
                                      : (float)(st.x[j] & 0xFFFFu) * (1.0f / 65536.0f);
                float b0, b1;
                if constexpr (FILTERED) {
                    pair(st.q[j], b0, b1);
                } else {
                    float q[4];
                    taps(st.q[j], q);
                    // 16.16 index: n is its integer part in the fast range
                    const float nf = kF32T ? st.nf[j] : (float)(st.x[j] >> 16);
                    const float k = fmaf(nf, 0.5f, t0h);  // (n + t0/dt) / 2
                    b0 = fmaf(-k, q[2] - q[0], q[1]);
                    b1 = fmaf(-(k + 0.5f), q[3] - q[1], q[2]);
                }
                const float v = fmaf(a, b1 - b0, b0);
                if constexpr (HAS_W) {
                    acc = fmaf(J.w[s0 + kJR * j + hr], v, acc);
                } else {
                    acc += v;
                }
            }
            return;
        }
        // general path: empty slots and non-contributing delays weigh 0; the
        // filter is one-sided at both ends of the record
#pragma unroll
        for (int j = 0; j < PX_U; ++j) {
            int n = 0;
            float a = 0.0f;
            bool dok;  // 0 <= n <= N-2
            if constexpr (kF32T) {
                const float u = __uint_as_float(st.x[j]);
                dok = u >= 0.0f && u <= dv.umax;  // also rejects NaN and inf
                const float uc = dok ? u : 0.0f;
                n = min((int)uc, N - 2);
                a = uc - (float)n;
            } else {
                dok = dv.decode_bf1(st.x[j], N, n, a);
            }
            const int sr = s0 + kJR * j + hr;  // this lane's sensor
            float ws = sr < se ? 1.0f : 0.0f;
            if constexpr (HAS_W) ws *= J.w[min(sr, S - 1)];
            const float w = dok ? ws : 0.0f;
            // FP16 loads were clamped to the shorter fast range: read the
            // samples again at this path's own start (one unaligned load; buffer
            // accesses take any byte address in the unaligned access mode the
            // driver sets on this GPU)
            float qs[4] = {st.q[j][0], st.q[j][1], st.q[j][2], st.q[j][3]};
            if constexpr (F16) {
                const SigRsrc g = sig_rsrc(step_s0(i));
                const uint32_t r = g.res + (uint32_t)((kJR * j + hr) * N);
                if constexpr (FILTERED) {
                    qs[1] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(g.r, 2u * (r + (uint32_t)n), 0, 0));
                    qs[2] = 0.0f;
                    qs[3] = 0.0f;
                } else {
                    const uint32_t c = (uint32_t)min(max(n - 1, 0), N - 4);
                    const auto v = __builtin_amdgcn_raw_buffer_load_b64(g.r, 2u * (r + c), 0, 0);
                    qs[0] = __uint_as_float(v[0]);
                    qs[1] = __uint_as_float(v[1]);
                    qs[2] = 0.0f;
                    qs[3] = 0.0f;
                }
            }
            float b0, b1;
            if constexpr (FILTERED) {
                pair(qs, b0, b1);
            } else {
                float q[4];
                taps(qs, q);
                // q = p[c .. c+3] with c = n-1 clipped to [0, N-4]
                const int sh = (n - 1) - min(max(n - 1, 0), N - 4);  // -1 at n = 0, +1 at n = N-2
                const float pm = sh == 1 ? q[1] : q[0];
                const float p0 = sh < 0 ? q[0] : (sh == 0 ? q[1] : q[2]);
                const float p1 = sh < 0 ? q[1] : (sh == 0 ? q[2] : q[3]);
                const float p2 = sh < 0 ? q[2] : q[3];
                const float k = fmaf((float)n, 0.5f, t0h);
                const float d0 = n == 0 ? 2.0f * (p1 - p0) : p1 - pm;
                const float d1 = n + 1 == N - 1 ? 2.0f * (p1 - p0) : p2 - p0;
                b0 = fmaf(-k, d0, p0);
                b1 = fmaf(-(k + 0.5f), d1, p1);
            }
            acc = fmaf(w, fmaf(a, b1 - b0, b0), acc);
        }
    };

    // Two stages alternate.  Loads are issued in the order they are needed
    // (vector loads complete in order): the delays of step i+2, then the
    // samples of step i+1 (whose delays came two issues earlier), then step i
    // is summed from samples issued one half-iteration before.
    // The scheduling barriers keep the issue order as written.
    Stage A, B;
    delays(0, A);
    delays(1, B);
    __builtin_amdgcn_sched_barrier(0);
    bool genA = samples(0, A), genB = false;
    __builtin_amdgcn_sched_barrier(0);
    for (int i = 0; i < nstep; i += 2) {
        delays(i + 2, A);
        __builtin_amdgcn_sched_barrier(0);
        genB = samples(i + 1, B);
        __builtin_amdgcn_sched_barrier(0);
        sum(A, i, genA);
        if (i + 1 >= nstep) break;
        delays(i + 3, B);
        __builtin_amdgcn_sched_barrier(0);
        genA = samples(i + 2, A);
        __builtin_amdgcn_sched_barrier(0);
        sum(B, i + 1, genB);
    }
    return acc * sc;  // the FP16 frame scale (1 otherwise); filter and interpolation are linear
}

// One tile of one frame: every wave sums its slots, then the slot sums are
// added in slot order.  Waves whose slots start past S add zero.
template <class Delay, int SFMT, bool FILTERED, bool HAS_W, int CONSTC = 0, bool SHDR = true>
__device__ __forceinline__ void px_block(const PxJob &J, const Delay &dec, int tile, int wv, int nw) {
    __shared__ float red[2 * PX_MAX_WAVES][PX_T];
    const int lane = threadIdx.x & 63;
    const int px = lane & (PX_T - 1);
    float acc = 0.0f;
    if (wv * 2 * J.sps < J.S) acc = px_slot_sum<Delay, SFMT, FILTERED, HAS_W, CONSTC, SHDR>(J, dec, tile, wv);
    red[wv * 2 + (lane >> 5)][px] = acc;
    __syncthreads();
    const int p = tile * PX_T + px;
    if (wv == 0 && lane < PX_T && p < J.P) {
        float s = 0.0f;
        for (int k = 0; k < 2 * nw; ++k) s += red[k][px];
        J.img[p] = s;
    }
}

// Straight-ray geometry of the conventional back projection (unused with a
// table).
struct PxGeom {
    const int32_t *pix;
    const float *sxy;
    int nx, ny;
    float h, x0, y0, z0, inv_c;
};

template <class Delay, int SFMT, bool FILTERED, bool HAS_W, int CONSTC, bool SHDR>
__global__ void __launch_bounds__(64 * PX_MAX_WAVES)
    k_bp_px(const uint32_t *__restrict__ tab, const void *__restrict__ sig, const float *__restrict__ scale,
            const float *__restrict__ w, int S, int P, int N, int sps, Delay dec, float t0dt,
            float *__restrict__ img, PxGeom geo) {
    const int f = blockIdx.y;
    constexpr size_t esz = SFMT == PAT_SIG_F16 ? 2 : 4;
    PxJob J;
    J.tab = tab;
    J.sig = static_cast<const char *>(sig) + (size_t)f * S * N * esz;
    J.w = w;
    J.img = img + (size_t)f * P;
    J.S = S; J.P = P; J.N = N; J.sps = sps;
    J.t0dt = t0dt;
    J.scale = (SFMT == PAT_SIG_F16 && scale) ? scale[f] : 1.0f;
    J.pix = geo.pix; J.sxy = geo.sxy; J.nx = geo.nx; J.ny = geo.ny;
    J.h = geo.h; J.x0 = geo.x0; J.y0 = geo.y0; J.z0 = geo.z0; J.inv_c = geo.inv_c;
    // a wave-uniform wave index keeps the descriptors in scalar registers
    const int tile = xcd_tile(blockIdx.x, (P + PX_T - 1) / PX_T);
    if (tile < 0) return;
    px_block<Delay, SFMT, FILTERED, HAS_W, CONSTC, SHDR>(J, dec, tile, __builtin_amdgcn_readfirstlane(threadIdx.x >> 6),
                                                   blockDim.x >> 6);
}

// Frames of different geometries in one launch: workgroup b belongs to the
// last descriptor whose block_begin <= b and computes one tile of that frame;
// the frame's shape depends on its own S, P, N only, so its image does not
// depend on its batch-mates.
template <int TFMT, int SFMT>
__global__ void __launch_bounds__(64 * PX_MULTI_WAVES) k_bp_px_multi(const pat_bp_desc *__restrict__ descs, int nd) {
    const int b = blockIdx.x;
    int lo = 0, hi = nd - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (descs[mid].block_begin <= b) lo = mid; else hi = mid - 1;
    }
    const pat_bp_desc &D = descs[lo];
    PxJob J;
    J.tab = D.tab; J.sig = D.sig; J.w = D.w; J.img = D.img;
    J.S = D.S; J.P = D.P; J.N = D.N; J.sps = D.sps;
    J.t0dt = D.t0dt;
    J.scale = D.scale;
    const int tile = xcd_tile(b - D.block_begin, D.tiles);
    if (tile < 0) return;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if constexpr (TFMT == PAT_TABLE_F32) {
        DelayF32 dec;
        dec.inv_hi = D.inv_hi; dec.inv_lo = D.inv_lo; dec.off = D.off; dec.umax = D.umax;
        if (D.w) px_block<DelayF32, SFMT, false, true>(J, dec, tile, wv, PX_MULTI_WAVES);
        else px_block<DelayF32, SFMT, false, false>(J, dec, tile, wv, PX_MULTI_WAVES);
    } else if constexpr (TFMT == PAT_TABLE_Q16) {
        DelayQ16 dec;
        if (D.w) px_block<DelayQ16, SFMT, false, true>(J, dec, tile, wv, PX_MULTI_WAVES);
        else px_block<DelayQ16, SFMT, false, false>(J, dec, tile, wv, PX_MULTI_WAVES);
    } else {
        DelayR16 dec;
        if (D.w) px_block<DelayR16, SFMT, false, true, 0, false>(J, dec, tile, wv, PX_MULTI_WAVES);
        else px_block<DelayR16, SFMT, false, false, 0, false>(J, dec, tile, wv, PX_MULTI_WAVES);
    }
}

template <class Delay, int SFMT, bool FILTERED, bool HAS_W, int CONSTC = 0, bool SHDR = true>
int launch_one(int S, int P, int F, const uint32_t *tab, const void *sig, const float *scale, const float *w, int N,
               Delay dec, float t0dt, float *img, hipStream_t st, const PxGeom &geo = PxGeom{}) {
    // occupancy per block size, computed once per kernel and device
    static std::mutex mu;
    static int cache_dev = -1, cache_cus = 0, cache_bpc[PX_MAX_WAVES + 1];
    int dev = 0;
    PAT_HIP(hipGetDevice(&dev));
    PxShape sh;
    {
        std::lock_guard<std::mutex> lk(mu);
        if (cache_dev != dev) {
            PAT_HIP(hipDeviceGetAttribute(&cache_cus, hipDeviceAttributeMultiprocessorCount, dev));
            for (int W = 1; W <= PX_MAX_WAVES; ++W)
                PAT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &cache_bpc[W], k_bp_px<Delay, SFMT, FILTERED, HAS_W, CONSTC, SHDR>, 64 * W, 0));
            cache_dev = dev;
        }
        sh = px_shape(S, P, F, cache_cus, SFMT == PAT_SIG_F16 ? PX_WAVES_PER_CU_F16 : PX_WAVES_PER_CU_F32,
                      [&](int W) { return cache_bpc[W]; });
    }

    const dim3 grid(xcd_slots(sh.tiles), F);
    k_bp_px<Delay, SFMT, FILTERED, HAS_W, CONSTC, SHDR><<<grid, dim3(64 * sh.waves), 0, st>>>(
        tab, sig, scale, w, S, P, N, sh.sps, dec, t0dt, img, geo);
    PAT_HIP(hipGetLastError());
    return PAT_OK;
}

template <class Delay, int SFMT>
int launch_px(bool filtered, int S, int P, int F, const uint32_t *tab, const void *sig, const float *scale,
              const float *w, int N, Delay dec, float t0dt, float *img, hipStream_t st) {
    // 16-bit tables: tile headers by scalar loads when the table streams from
    // HBM (the vector-memory path is then the limit); a cached table's short
    // latency-bound pipeline does better with vector loads, which it can wait
    // for one by one
    if constexpr (Delay::kR16) {
        if (pat_r16_bytes(S, P) <= PAT_CACHED_TABLE_BYTES) {
            if (w)
                return filtered ? launch_one<Delay, SFMT, true, true, 0, false>(S, P, F, tab, sig, scale, w, N, dec, t0dt, img, st)
                                : launch_one<Delay, SFMT, false, true, 0, false>(S, P, F, tab, sig, scale, w, N, dec, t0dt, img, st);
            return filtered ? launch_one<Delay, SFMT, true, false, 0, false>(S, P, F, tab, sig, scale, w, N, dec, t0dt, img, st)
                            : launch_one<Delay, SFMT, false, false, 0, false>(S, P, F, tab, sig, scale, w, N, dec, t0dt, img, st);
        }
    }
    if (w)
        return filtered ? launch_one<Delay, SFMT, true, true>(S, P, F, tab, sig, scale, w, N, dec, t0dt, img, st)
                        : launch_one<Delay, SFMT, false, true>(S, P, F, tab, sig, scale, w, N, dec, t0dt, img, st);
    return filtered ? launch_one<Delay, SFMT, true, false>(S, P, F, tab, sig, scale, w, N, dec, t0dt, img, st)
                    : launch_one<Delay, SFMT, false, false>(S, P, F, tab, sig, scale, w, N, dec, t0dt, img, st);
}

template <int SFMT, int DIM>
int launch_px_const(bool filtered, int S, int P, int F, const void *sig, const float *scale, const float *w, int N,
                    DelayF32 dec, float t0dt, float *img, hipStream_t st, const PxGeom &geo) {
    if (w)
        return filtered
                   ? launch_one<DelayF32, SFMT, true, true, DIM>(S, P, F, nullptr, sig, scale, w, N, dec, t0dt, img, st, geo)
                   : launch_one<DelayF32, SFMT, false, true, DIM>(S, P, F, nullptr, sig, scale, w, N, dec, t0dt, img, st, geo);
    return filtered
               ? launch_one<DelayF32, SFMT, true, false, DIM>(S, P, F, nullptr, sig, scale, w, N, dec, t0dt, img, st, geo)
               : launch_one<DelayF32, SFMT, false, false, DIM>(S, P, F, nullptr, sig, scale, w, N, dec, t0dt, img, st, geo);
}

}  // namespace

int pat_launch_backproject_px_const(int nx, double h, double c, const float *d_sxy, int S, const int32_t *d_pix,
                                    int P, const void *sig, int sig_fmt, int sig_is_filtered, const float *frame_scale,
                                    const float *w, int N, int F, double t0, double dt, float *img, int ny,
                                    hipStream_t st, int nz) {
    DelayF32 d;
    const double inv = 1.0 / dt;
    d.inv_hi = (float)inv;
    d.inv_lo = (float)(inv - (double)d.inv_hi);
    d.off = (float)(-t0 / dt);
    d.umax = (float)(N - 1);
    PxGeom g;
    g.pix = d_pix;
    g.sxy = d_sxy;
    g.nx = nx;
    g.ny = ny;
    g.h = (float)h;
    g.x0 = (float)(-0.5 * (nx - 1) * h);
    g.y0 = (float)(-0.5 * (ny - 1) * h);
    g.z0 = (float)(-0.5 * (nz - 1) * h);
    g.inv_c = (float)(1.0 / c);
    const float t0dt = (float)(t0 / dt);
    const bool filt = sig_is_filtered != 0;
    if (nz > 0)
        return sig_fmt == PAT_SIG_F32
                   ? launch_px_const<PAT_SIG_F32, 3>(filt, S, P, F, sig, frame_scale, w, N, d, t0dt, img, st, g)
                   : launch_px_const<PAT_SIG_F16, 3>(filt, S, P, F, sig, frame_scale, w, N, d, t0dt, img, st, g);
    return sig_fmt == PAT_SIG_F32
               ? launch_px_const<PAT_SIG_F32, 2>(filt, S, P, F, sig, frame_scale, w, N, d, t0dt, img, st, g)
               : launch_px_const<PAT_SIG_F16, 2>(filt, S, P, F, sig, frame_scale, w, N, d, t0dt, img, st, g);
}

bool pat_px_eligible(int sig_fmt, int S, int P, int N, int F, const void *sig) {
    if (S <= 0 || P <= 0 || F <= 0 || N < 4) return false;
    if ((uintptr_t)sig % (sig_fmt == PAT_SIG_F16 ? 2 : 4) != 0) return false;
    return px_offsets_fit(P, N, sig_fmt);
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
    if (table_fmt == PAT_TABLE_F32X4) {
        DelayF32X4 d;
        const double inv = 1.0 / dt;
        d.inv_hi = (float)inv;
        d.inv_lo = (float)(inv - (double)d.inv_hi);
        d.off = (float)(-t0 / dt);
        d.umax = (float)(N - 1);
        return sig_fmt == PAT_SIG_F32
                   ? launch_px<DelayF32X4, PAT_SIG_F32>(filt, S, P, F, tab, sig, frame_scale, w, N, d, t0dt, img, st)
                   : launch_px<DelayF32X4, PAT_SIG_F16>(filt, S, P, F, tab, sig, frame_scale, w, N, d, t0dt, img, st);
    }
    if (table_fmt == PAT_TABLE_R16) {
        DelayR16 d;
        return sig_fmt == PAT_SIG_F32
                   ? launch_px<DelayR16, PAT_SIG_F32>(filt, S, P, F, tab, sig, frame_scale, w, N, d, t0dt, img, st)
                   : launch_px<DelayR16, PAT_SIG_F16>(filt, S, P, F, tab, sig, frame_scale, w, N, d, t0dt, img, st);
    }
    DelayQ16 d;
    return sig_fmt == PAT_SIG_F32
               ? launch_px<DelayQ16, PAT_SIG_F32>(filt, S, P, F, tab, sig, frame_scale, w, N, d, t0dt, img, st)
               : launch_px<DelayQ16, PAT_SIG_F16>(filt, S, P, F, tab, sig, frame_scale, w, N, d, t0dt, img, st);
}

bool pat_px_multi_eligible(int sig_fmt, int S, int P, int N) {
    if (S <= 0 || P <= 0 || N < 4) return false;
    return px_offsets_fit(P, N, sig_fmt);
}

int pat_px_frame_shape(pat_bp_desc *d, int S, int P, int N, double t0, double dt) {
    d->S = S;
    d->P = P;
    d->N = N;
    d->sps = px_sps(S, PX_MULTI_WAVES);
    d->tiles = (P + PX_T - 1) / PX_T;  // launch slots: xcd_slots(tiles), a multiple of 8
    d->t0dt = (float)(t0 / dt);
    const double inv = 1.0 / dt;
    d->inv_hi = (float)inv;
    d->inv_lo = (float)(inv - (double)d->inv_hi);
    d->off = (float)(-t0 / dt);
    d->umax = (float)(N - 1);
    d->scale = 1.0f;
    return xcd_slots(d->tiles);
}

int pat_launch_px_multi(const pat_bp_desc *d_descs, int nd, int total_blocks, int table_fmt, int sig_fmt,
                        hipStream_t st) {
    if (nd <= 0 || total_blocks <= 0) return PAT_OK;
    const dim3 grid(total_blocks), block(64 * PX_MULTI_WAVES);
    if (table_fmt == PAT_TABLE_F32) {
        if (sig_fmt == PAT_SIG_F32) k_bp_px_multi<PAT_TABLE_F32, PAT_SIG_F32><<<grid, block, 0, st>>>(d_descs, nd);
        else k_bp_px_multi<PAT_TABLE_F32, PAT_SIG_F16><<<grid, block, 0, st>>>(d_descs, nd);
    } else if (table_fmt == PAT_TABLE_Q16) {
        if (sig_fmt == PAT_SIG_F32) k_bp_px_multi<PAT_TABLE_Q16, PAT_SIG_F32><<<grid, block, 0, st>>>(d_descs, nd);
        else k_bp_px_multi<PAT_TABLE_Q16, PAT_SIG_F16><<<grid, block, 0, st>>>(d_descs, nd);
    } else {
        if (sig_fmt == PAT_SIG_F32) k_bp_px_multi<PAT_TABLE_R16, PAT_SIG_F32><<<grid, block, 0, st>>>(d_descs, nd);
        else k_bp_px_multi<PAT_TABLE_R16, PAT_SIG_F16><<<grid, block, 0, st>>>(d_descs, nd);
    }
    PAT_HIP(hipGetLastError());
    return PAT_OK;
}
