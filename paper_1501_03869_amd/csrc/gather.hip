// Delay-and-sum back projection (Section II-C, Eq. BP):
//   img[f][p] = sum_s w_s * lerp(b_{f,s}, u_{s,p}),  u = (T[s][p] - t0) / dt,
// with b = p - t dp/dt either supplied or computed in the kernel.
//
// Work decomposition (one launch per call):
//  * A workgroup of 256 threads owns a chunk of 1024 consecutive table columns
//    (4 per thread, read as one 16-byte load per sensor: the pixel-major table
//    streams from HBM fully coalesced) and a contiguous group of sensors.
//    Callers order the ROI tile-major (pat_tile_order) so a chunk covers a
//    compact 2-D patch and its delays to one sensor span a short time window.
//  * Sensors are processed 8 at a time.  For each, the workgroup stages a
//    512-sample window of the signal, centred on the delay of the chunk's first
//    pixel, in LDS; when the signal is raw it is filtered there
//    (b = p - t dp/dt, central differences, one-sided ends).  Every gather then
//    reads its two neighbouring samples from LDS.  A delay outside the window
//    (non-compact pixel sets) is served from global memory instead, so any
//    pixel order is correct.
//  * Partial sums of the sensor groups are added by the last workgroup of each
//    chunk to finish, in group order, so results are bitwise reproducible.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <algorithm>
#include <mutex>

#include "gather_common.h"
#include "pat_internal.h"

namespace {

using namespace pat_gather;

constexpr int BP_THREADS = 256;
constexpr int BP_PPT = 4;                          // pixels per thread
constexpr int BP_CHUNK = BP_THREADS * BP_PPT;      // pixels per workgroup
constexpr int BP_SC = 8;                           // sensors staged together
constexpr int BP_W = 512;                          // window samples per sensor
constexpr int BP_RAW = BP_W + 2;                   // raw samples incl. both neighbours
constexpr int BP_NPROBE = 16;                      // window probes per sensor: every 64th pixel
constexpr int BP_MARGIN = 40;                      // window start below the smallest probed delay
// Workgroups the chip holds at once: 256 CUs x 3 (48 KiB of LDS each).
constexpr int BP_RESIDENT = 256 * 3;

struct BpShape {
    int chunks;  // workgroups along pixels
    int groups;  // sensor groups
    int spg;     // sensors per group (a multiple of BP_SC unless one group)
};

// Sensor groups per pixel chunk.  Problems whose pixel chunks fit in one wave
// of resident workgroups split the sensors to fill that wave; larger ones are
// cut into at least four waves (each workgroup keeping >= 4 sensor chunks to
// pipeline) so that the last, partly filled wave costs little.
BpShape bp_shape(int S, int P, int F) {
    BpShape s;
    s.chunks = (P + BP_CHUNK - 1) / BP_CHUNK;
    const long per_group = (long)s.chunks * std::max(F, 1);
    const int S1 = std::max(S, 1);
    const int max_groups = std::max(1, (S1 + BP_SC - 1) / BP_SC);
    long G = BP_RESIDENT / per_group;
    if (G < 1) {
        const long many = (4L * BP_RESIDENT + per_group - 1) / per_group;
        G = std::min<long>(many, std::max(1, S1 / (4 * BP_SC)));
    }
    G = std::max<long>(1, std::min<long>(G, max_groups));
    int spg = (int)((S1 + G - 1) / G);
    spg = ((spg + BP_SC - 1) / BP_SC) * BP_SC;
    s.spg = spg;
    s.groups = (S1 + spg - 1) / spg;
    return s;
}

template <bool VEC4>
__device__ __forceinline__ void load_delays(const uint32_t *__restrict__ tab, long rowoff, int p0, int P,
                                            uint32_t (&v)[BP_PPT]) {
    if constexpr (VEC4) {
        if (p0 < P) {
            const uint4 q = *reinterpret_cast<const uint4 *>(tab + rowoff + p0);
            v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
        } else {
            v[0] = v[1] = v[2] = v[3] = 0xFFFFFFFFu;
        }
    } else {
#pragma unroll
        for (int k = 0; k < BP_PPT; ++k) v[k] = (p0 + k < P) ? tab[rowoff + p0 + k] : 0xFFFFFFFFu;
    }
}

struct BpJob {
    const uint32_t *tab;   // [S][P]
    const void *sig;       // this frame's [S][N]
    const float *w;        // [S] or null
    float *part;           // this frame's [G][P] partial sums (G > 1)
    float *img;            // this frame's [P]
    unsigned int *done;    // this frame's per-chunk completion counters (G > 1)
    int S, P, N, spg, G;
    float t0dt, scale;
    // straight-ray delays instead of a table (conventional back projection)
    const int32_t *pix;    // [P] node indices
    const float *sxy;      // [S][2] sensor positions, metres
    int nx;
    float h, x0, y0, inv_c;
};

// One workgroup's share of one frame: pixel chunk c, sensor group g.
//
// Software pipeline over chunks of BP_SC sensors (i = current chunk):
//   top     - decode the window anchors of chunk i+1 (probe delays loaded one
//             iteration earlier), issue its window loads into registers, its
//             delay loads, and the probe loads of chunk i+2;
//   middle  - gather chunk i from its LDS windows while those loads fly;
//   bottom  - store chunk i+1's raw window, filter it into the other window
//             buffer, barrier.
// So a chunk costs one memory latency overlapped with a chunk of gathers,
// instead of a chain of dependent loads.
template <class Delay, int SFMT, bool FILTERED, bool VEC4, bool CONSTC = false>
__device__ __forceinline__ void bp_block(const BpJob &J, const Delay &dec, int c, int g) {
    const uint32_t *__restrict__ tab = J.tab;
    const void *__restrict__ sig = J.sig;
    const float *__restrict__ w = J.w;
    const int S = J.S, P = J.P, N = J.N, spg = J.spg, G = J.G;
    const float t0dt = J.t0dt;
    constexpr int WLEN = FILTERED ? BP_W : BP_RAW;                 // staged samples per sensor
    constexpr int NR = (WLEN + BP_THREADS - 1) / BP_THREADS;       // staged samples per thread
    __shared__ float bwin[2][BP_SC][BP_W];
    __shared__ float raw[FILTERED ? 1 : BP_SC][FILTERED ? 1 : BP_RAW];
    __shared__ unsigned int is_last;

    const int tid = threadIdx.x;
    const int pbase = c * BP_CHUNK;
    const int p0 = pbase + tid * BP_PPT;  // this thread's first pixel
    const int s_begin = g * spg;
    const int s_end = min(S, s_begin + spg);
    const int nchunk = s_end > s_begin ? (s_end - s_begin + BP_SC - 1) / BP_SC : 0;
    const float sc = J.scale;

    float acc[BP_PPT] = { 0.0f, 0.0f, 0.0f, 0.0f };
    uint32_t cur[BP_SC][BP_PPT], nxt[BP_SC][BP_PPT];
    uint32_t pr_next[BP_SC], pr_next2[BP_SC];
    int an_cur[BP_SC], an_next[BP_SC];
    float rv[BP_SC][NR];

    // delay of the chunk's first pixel to each sensor of chunk i (window probes)
    // straight-ray delay (seconds, as float bits) of node k to sensor s
    auto ray = [&](int s, float px, float py) -> uint32_t {
        const float dx = px - J.sxy[2 * s], dy = py - J.sxy[2 * s + 1];
        return __float_as_uint(__builtin_amdgcn_sqrtf(fmaf(dx, dx, dy * dy)) * J.inv_c);
    };
    float px[BP_PPT], py[BP_PPT], qx[4], qy[4];  // pixel coordinates (conventional BP)
    if constexpr (CONSTC) {
#pragma unroll
        for (int k = 0; k < BP_PPT; ++k) {
            const int kk = J.pix[min(p0 + k, P - 1)];
            px[k] = J.x0 + (float)(kk % J.nx) * J.h;
            py[k] = J.y0 + (float)(kk / J.nx) * J.h;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int kq = J.pix[min(pbase + q * (BP_CHUNK - 1) / 3, P - 1)];
            qx[q] = J.x0 + (float)(kq % J.nx) * J.h;
            qy[q] = J.y0 + (float)(kq / J.nx) * J.h;
        }
    }
    // Window probes of chunk i: per sensor, the smallest of the delays of
    // every 64th pixel of the chunk.  Delays are compared as raw 32-bit
    // patterns (a scalar min): for non-negative float32 seconds and for 16.16
    // indices the order of the patterns is the order of the delays, and the
    // non-contributing codes (NaN, negative, the 16.16 sentinel) sort last.
    auto probe = [&](int i, uint32_t (&pr)[BP_SC]) {
#pragma unroll
        for (int j = 0; j < BP_SC; ++j) {
            const int s = s_begin + i * BP_SC + j;
            uint32_t m = 0xFFFFFFFFu;
            if (i < nchunk && s < s_end) {
                if constexpr (CONSTC) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) m = min(m, ray(s, qx[q], qy[q]));
                } else {
#pragma unroll
                    for (int q = 0; q < BP_NPROBE; ++q)
                        m = min(m, tab[(long)s * P + min(pbase + q * (BP_CHUNK / BP_NPROBE), P - 1)]);
                }
            }
            pr[j] = m;
        }
    };
    auto anchors = [&](const uint32_t (&pr)[BP_SC], int (&an)[BP_SC]) {
#pragma unroll
        for (int j = 0; j < BP_SC; ++j) {
            int n;
            float a;
            an[j] = dec.decode(pr[j], N, n, a) ? n - BP_MARGIN : 0;
        }
    };
    auto delays = [&](int i, uint32_t (&v)[BP_SC][BP_PPT]) {
#pragma unroll
        for (int j = 0; j < BP_SC; ++j) {
            const int s = s_begin + i * BP_SC + j;
            if (s < s_end) {
                if constexpr (CONSTC) {
#pragma unroll
                    for (int k = 0; k < BP_PPT; ++k) v[j][k] = p0 + k < P ? ray(s, px[k], py[k]) : 0xFFFFFFFFu;
                } else {
                    load_delays<VEC4>(tab, (long)s * P, p0, P, v[j]);
                }
            } else {
                v[j][0] = v[j][1] = v[j][2] = v[j][3] = 0xFFFFFFFFu;
            }
        }
    };
    // window samples of chunk i into registers (all loads issued together)
    auto stage_load = [&](int i, const int (&an)[BP_SC]) {
#pragma unroll
        for (int si = 0; si < BP_SC; ++si) {
            const int s = s_begin + i * BP_SC + si;
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const int j = tid + r * BP_THREADS;
                rv[si][r] = 0.0f;
                if (s < s_end && j < WLEN) {
                    const int gi = min(max((FILTERED ? an[si] : an[si] - 1) + j, 0), N - 1);
                    rv[si][r] = load_sig<SFMT>(sig, (long)s * N + gi, sc);
                }
            }
        }
    };
    // registers -> LDS window buffer buf (raw samples are filtered on the way)
    auto stage_store = [&](int i, const int (&an)[BP_SC], int buf) {
        const int ns = min(BP_SC, s_end - (s_begin + i * BP_SC));
        if constexpr (FILTERED) {
#pragma unroll
            for (int si = 0; si < BP_SC; ++si)
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    const int j = tid + r * BP_THREADS;
                    if (si < ns && j < BP_W) bwin[buf][si][j] = rv[si][r];
                }
        } else {
#pragma unroll
            for (int si = 0; si < BP_SC; ++si)
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    const int j = tid + r * BP_THREADS;
                    if (si < ns && j < BP_RAW) raw[si][j] = rv[si][r];
                }
            __syncthreads();
#pragma unroll
            for (int si = 0; si < BP_SC; ++si) {
                if (si >= ns) continue;
#pragma unroll
                for (int r = 0; r < (BP_W + BP_THREADS - 1) / BP_THREADS; ++r) {
                    const int j = tid + r * BP_THREADS;
                    if (j < BP_W) bwin[buf][si][j] = ubp(raw[si][j], raw[si][j + 1], raw[si][j + 2], an[si] + j, N, t0dt);
                }
            }
        }
    };

    if (nchunk > 0) {
        probe(0, pr_next);
        anchors(pr_next, an_cur);
        delays(0, cur);
        stage_load(0, an_cur);
        probe(1, pr_next);
        stage_store(0, an_cur, 0);
        __syncthreads();
    }

    for (int i = 0; i < nchunk; ++i) {
        const int buf = i & 1;
        const bool more = i + 1 < nchunk;
        const int s0 = s_begin + i * BP_SC;
        const int ns = min(BP_SC, s_end - s0);
        if (more) {
            anchors(pr_next, an_next);
            stage_load(i + 1, an_next);
            delays(i + 1, nxt);
            probe(i + 2, pr_next2);
        }
        // gather: branch-free from the windows; a delay outside its window is
        // only noted here and served from global memory below
        bool anyfall = false;
#pragma unroll
        for (int j = 0; j < BP_SC; ++j) {
            if (j < ns) {
                const float ws = w ? w[s0 + j] : 1.0f;
                const auto win = dec.window(an_cur[j]);
                float b0[BP_PPT], b1[BP_PPT], al[BP_PPT], wk[BP_PPT];
#pragma unroll
                for (int k = 0; k < BP_PPT; ++k) {
                    int idx;
                    const bool ok = dec.decode_win(cur[j][k], win, idx, al[k]);
                    const bool inw = (unsigned)idx < (unsigned)(BP_W - 1);
                    wk[k] = (ok && inw) ? ws : 0.0f;
                    anyfall |= !inw;  // a delay that does not contribute decodes to idx 0
                    const int id = inw ? idx : 0;
                    b0[k] = bwin[buf][j][id];
                    b1[k] = bwin[buf][j][id + 1];
                }
#pragma unroll
                for (int k = 0; k < BP_PPT; ++k) acc[k] = fmaf(wk[k], fmaf(al[k], b1[k] - b0[k], b0[k]), acc[k]);
            }
        }
        if (__any(anyfall)) {
            // rare: the delays that missed their window read global memory
#pragma unroll
            for (int j = 0; j < BP_SC; ++j) {
                if (j >= ns) continue;
                const auto win = dec.window(an_cur[j]);
                const float ws = w ? w[s0 + j] : 1.0f;
                const long row = (long)(s0 + j) * N;
#pragma unroll
                for (int k = 0; k < BP_PPT; ++k) {
                    int idx;
                    float al;
                    const bool ok = dec.decode_win(cur[j][k], win, idx, al);
                    int n;
                    float a;
                    if (ok && (unsigned)idx >= (unsigned)(BP_W - 1) && dec.decode(cur[j][k], N, n, a)) {
                        const float b0 = sample_b<SFMT, FILTERED>(sig, row, n, N, sc, t0dt);
                        const float b1 = sample_b<SFMT, FILTERED>(sig, row, n + 1, N, sc, t0dt);
                        acc[k] = fmaf(ws, fmaf(a, b1 - b0, b0), acc[k]);
                    }
                }
            }
        }
        if (more) stage_store(i + 1, an_next, buf ^ 1);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < BP_SC; ++j) {
            an_cur[j] = an_next[j];
            pr_next[j] = pr_next2[j];
#pragma unroll
            for (int k = 0; k < BP_PPT; ++k) cur[j][k] = nxt[j][k];
        }
    }

    float *__restrict__ img = J.img;
    if (G == 1) {
#pragma unroll
        for (int k = 0; k < BP_PPT; ++k)
            if (p0 + k < P) img[p0 + k] = acc[k];
        return;
    }
    float *mine = J.part + (long)g * P;
#pragma unroll
    for (int k = 0; k < BP_PPT; ++k)
        if (p0 + k < P) mine[p0 + k] = acc[k];
    __threadfence();
    __syncthreads();
    if (tid == 0) {
        const unsigned int prev = atomicAdd(&J.done[c], 1u);
        is_last = (prev == (unsigned)(G - 1)) ? 1u : 0u;
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    const float *base = J.part;
#pragma unroll
    for (int k = 0; k < BP_PPT; ++k) {
        const int p = p0 + k;
        if (p >= P) continue;
        float s = 0.0f;
        for (int gg = 0; gg < G; ++gg) s += __builtin_nontemporal_load(base + (long)gg * P + p);
        img[p] = s;
    }
    if (tid == 0) J.done[c] = 0u;  // ready for the next launch
}

template <class Delay, int SFMT, bool FILTERED, bool VEC4>
__global__ void __launch_bounds__(BP_THREADS) k_bp(const uint32_t *__restrict__ tab, const void *__restrict__ sig,
                                                   const float *__restrict__ scale, const float *__restrict__ w,
                                                   int S, int P, int N, int spg, int G, Delay dec, float t0dt,
                                                   float *__restrict__ part, float *__restrict__ img,
                                                   unsigned int *__restrict__ done) {
    const int f = blockIdx.z;
    const size_t esz = SFMT == PAT_SIG_F16 ? 2 : 4;
    BpJob J;
    J.tab = tab;
    J.sig = static_cast<const char *>(sig) + (size_t)f * S * N * esz;
    J.w = w;
    J.part = part ? part + (long)f * G * P : nullptr;
    J.img = img + (long)f * P;
    J.done = done ? done + (long)f * gridDim.x : nullptr;
    J.S = S; J.P = P; J.N = N; J.spg = spg; J.G = G;
    J.t0dt = t0dt;
    J.scale = (SFMT == PAT_SIG_F16 && scale) ? scale[f] : 1.0f;
    bp_block<Delay, SFMT, FILTERED, VEC4>(J, dec, blockIdx.x, blockIdx.y);
}

// Conventional back projection: straight-ray delays |x - s| / c computed per
// gather instead of read from a table (no table traffic; ALU bound).
template <int SFMT, bool FILTERED>
__global__ void __launch_bounds__(BP_THREADS) k_bp_const(const void *__restrict__ sig, const float *__restrict__ scale,
                                                         const float *__restrict__ w, int S, int P, int N, int spg,
                                                         int G, DelayF32 dec, float t0dt, float *__restrict__ part,
                                                         float *__restrict__ img, unsigned int *__restrict__ done,
                                                         const int32_t *__restrict__ pix, const float *__restrict__ sxy,
                                                         int nx, float h, float x0, float y0, float inv_c) {
    const int f = blockIdx.z;
    const size_t esz = SFMT == PAT_SIG_F16 ? 2 : 4;
    BpJob J;
    J.tab = nullptr;
    J.sig = static_cast<const char *>(sig) + (size_t)f * S * N * esz;
    J.w = w;
    J.part = part ? part + (long)f * G * P : nullptr;
    J.img = img + (long)f * P;
    J.done = done ? done + (long)f * gridDim.x : nullptr;
    J.S = S; J.P = P; J.N = N; J.spg = spg; J.G = G;
    J.t0dt = t0dt;
    J.scale = (SFMT == PAT_SIG_F16 && scale) ? scale[f] : 1.0f;
    J.pix = pix; J.sxy = sxy; J.nx = nx; J.h = h; J.x0 = x0; J.y0 = y0; J.inv_c = inv_c;
    bp_block<DelayF32, SFMT, FILTERED, false, true>(J, dec, blockIdx.x, blockIdx.y);
}

template <class Delay, int SFMT>
int launch(bool filtered, bool vec4, dim3 grid, const uint32_t *tab, const void *sig, const float *scale,
           const float *w, int S, int P, int N, int spg, int G, Delay dec, float t0dt, float *part, float *img,
           unsigned int *done, hipStream_t st) {
#define PAT_BP_LAUNCH(FI, V4) \
    k_bp<Delay, SFMT, FI, V4><<<grid, BP_THREADS, 0, st>>>(tab, sig, scale, w, S, P, N, spg, G, dec, t0dt, part, img, done)
    if (filtered) {
        if (vec4) PAT_BP_LAUNCH(true, true); else PAT_BP_LAUNCH(true, false);
    } else {
        if (vec4) PAT_BP_LAUNCH(false, true); else PAT_BP_LAUNCH(false, false);
    }
#undef PAT_BP_LAUNCH
    PAT_HIP(hipGetLastError());
    return PAT_OK;
}

// Zero an image with a kernel rather than a memset node, so that a call with
// no sensors can be captured into a HIP graph like any other.
__global__ void __launch_bounds__(256) k_zero(float *__restrict__ img, long n) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) img[i] = 0.0f;
}

int launch_zero(float *img, long n, hipStream_t st) {
    if (n <= 0) return PAT_OK;
    const long blocks = std::min<long>((n + 255) / 256, 4096);
    k_zero<<<dim3((unsigned)blocks), dim3(256), 0, st>>>(img, n);
    PAT_HIP(hipGetLastError());
    return PAT_OK;
}

}  // namespace

// Gather scratch: the partial sums live in the context's gather buffer; the
// completion counters (at most ceil(P/256) * F for either kernel) live in a
// buffer of their own that is zeroed when it is (re)allocated and that every
// launch leaves at zero, so no call can see another call's partial sums as
// counters whatever the sizes of successive calls.
size_t pat_gather_counter_bytes(int P, int F) {
    return ((((size_t)(P + 255) / 256) * (size_t)F * sizeof(unsigned int) + 255) / 256) * 256;
}

// Fixed device scratch of the allocation-free entry point
// (pat_backproject_noalloc): the completion counters at byte 0, then the
// partial sums.  Each device holds its own copy from module load to process
// end; host code reaches it only through the address hipGetSymbolAddress
// gives on that device.
static __device__ __align__(256) unsigned char scratch[PAT_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_fixed_mu;
void *g_fixed_ptr[kMaxDevices] = {};
}  // namespace

int pat_fixed_scratch_attach(int device, void **out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices)
        return pat_fail(PAT_EINVAL, "device %d beyond the %d the fixed scratch table holds", device, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_fixed_mu);
    if (!g_fixed_ptr[device]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return pat_hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        }
        g_fixed_ptr[device] = p;
    }
    *out = g_fixed_ptr[device];
    return PAT_OK;
}

int pat_gather_scratch(pat_ctx *ctx, int P, int F, size_t part_bytes, float **part, unsigned int **done,
                       hipStream_t st) {
    const size_t cb = pat_gather_counter_bytes(P, F);
    if (ctx->fixed_active) {
        // the device's fixed array: nothing is allocated; the counters are
        // cleared by a kernel on the call's stream (a call may be captured)
        if (!ctx->fixed_scratch) return pat_fail(PAT_EDEVICE, "fixed scratch not attached to this context");
        if (cb > PAT_NOALLOC_SCRATCH_BYTES || part_bytes > PAT_NOALLOC_SCRATCH_BYTES - cb)
            return pat_fail(PAT_EINVAL,
                            "these sizes need %zu bytes of gather scratch (%zu counters + %zu partial sums); the fixed "
                            "scratch holds %zu (use pat_backproject)",
                            cb + part_bytes, cb, part_bytes, (size_t)PAT_NOALLOC_SCRATCH_BYTES);
        unsigned char *base = static_cast<unsigned char *>(ctx->fixed_scratch);
        int rc = launch_zero(reinterpret_cast<float *>(base), (long)(cb / sizeof(float)), st);
        if (rc) return rc;
        *done = reinterpret_cast<unsigned int *>(base);
        *part = reinterpret_cast<float *>(base + cb);
        return PAT_OK;
    }
    if (cb > ctx->gather_done.bytes) {
        int rc = ctx->gather_done.grow(cb);
        if (rc) return rc;
        PAT_HIP(hipMemset(ctx->gather_done.ptr, 0, ctx->gather_done.bytes));
    }
    int rc = ctx->gather_scratch.grow(part_bytes);
    if (rc) return rc;
    *done = static_cast<unsigned int *>(ctx->gather_done.ptr);
    *part = static_cast<float *>(ctx->gather_scratch.ptr);
    return PAT_OK;
}

static size_t single_part_bytes(int S, int P, int F) {
    const BpShape sh = bp_shape(S, P, F);
    return sh.groups > 1 ? (size_t)sh.groups * P * F * sizeof(float) : 0;
}

extern "C" size_t pat_backproject_scratch_bytes(int S, int P, int F) {
    if (S <= 0 || P <= 0 || F <= 0) return 0;
    return std::max(single_part_bytes(S, P, F), pat_batch_part_bytes(S, P, F));
}

int pat_launch_backproject(pat_ctx *ctx, const void *table, int table_fmt, const void *sig, int sig_fmt,
                           int sig_is_filtered, const float *frame_scale, const float *w, int S, int P, int N,
                           int F, double t0, double dt, float *img, hipStream_t st) {
    if (S == 0) {
        return launch_zero(img, (long)P * F, st);
    }
    // Kernel choice.  A table above half the 256 MB Infinity Cache, in any
    // form but the interleaved one, takes the wave-window kernel when it has
    // PAT_WIN_MIN_P columns or, for several frames, enough (group, frame)
    // pairs to fill the GPU (1024^2 workload: 0.62 ms per frame against 0.81
    // for the split-sensor kernel on the interleaved table; 16 frames per
    // launch: 0.22 against 0.64 ms per frame for the batched kernel).
    // Several frames whose table stays in the cache between frames are
    // fastest with the split-sensor kernel, one table read per frame (paper
    // workload, 64 frames: 10 us per frame against 17 for the batched
    // kernel); other large tables are read once per 16 frames by the batched
    // kernel.  A single frame that would split its sensors over workgroups
    // takes the split-sensor kernel; the rest take the windowed kernel.
    const bool px_ok = pat_px_eligible(sig_fmt, S, P, N, F, sig);
    const size_t table_bytes = table_fmt == PAT_TABLE_R16 ? pat_r16_bytes(S, P) : (size_t)S * P * 4;
    if ((pat_win_preferred(P, F, table_bytes) || pat_env_force_win()) &&
        pat_win_eligible(table_fmt, sig_fmt, S, P, N, F, sig))
        return pat_launch_backproject_win(table, table_fmt, sig, sig_fmt, sig_is_filtered, frame_scale, w, S, P, N, F,
                                          t0, dt, img, st);
    if (table_fmt == PAT_TABLE_R16 || table_fmt == PAT_TABLE_F32X4) {
        if (!px_ok || (table_fmt == PAT_TABLE_F32X4 && (size_t)P * 32 >= (1ull << 31)))
            return pat_fail(PAT_EINVAL, "16-bit and interleaved tables need N >= 4, a signal pointer aligned to its "
                                        "sample size and per-step offsets below 2^31 (N=%d P=%d)", N, P);
        return pat_launch_backproject_px(table, table_fmt, sig, sig_fmt, sig_is_filtered, frame_scale, w, S, P, N, F,
                                         t0, dt, img, st);
    }
    if (F >= 2 && pat_batch_eligible(sig_fmt, N, F, sig) && (!px_ok || table_bytes > PAT_CACHED_TABLE_BYTES))
        return pat_launch_backproject_batch(ctx, table, table_fmt, sig, sig_fmt, sig_is_filtered, frame_scale, w, S, P,
                                            N, F, t0, dt, img, st);
    const BpShape sh = bp_shape(S, P, F);
    if (px_ok && (sh.groups > 1 || F >= 2))
        return pat_launch_backproject_px(table, table_fmt, sig, sig_fmt, sig_is_filtered, frame_scale, w, S, P, N, F,
                                         t0, dt, img, st);
    float *part = nullptr;
    unsigned int *done = nullptr;
    if (sh.groups > 1) {
        int rc = pat_gather_scratch(ctx, P, F, single_part_bytes(S, P, F), &part, &done, st);
        if (rc) return rc;
    }
    const dim3 grid(sh.chunks, sh.groups, F);
    const float t0dt = (float)(t0 / dt);
    const bool filt = sig_is_filtered != 0;
    const uint32_t *tab = static_cast<const uint32_t *>(table);
    const bool vec4 = (P % 4 == 0) && ((uintptr_t)table % 16 == 0);
    if (table_fmt == PAT_TABLE_F32) {
        DelayF32 d;
        const double inv = 1.0 / dt;
        d.inv_hi = (float)inv;
        d.inv_lo = (float)(inv - (double)d.inv_hi);
        d.off = (float)(-t0 / dt);
        d.umax = (float)(N - 1);
        return sig_fmt == PAT_SIG_F32
                   ? launch<DelayF32, PAT_SIG_F32>(filt, vec4, grid, tab, sig, frame_scale, w, S, P, N, sh.spg, sh.groups, d, t0dt, part, img, done, st)
                   : launch<DelayF32, PAT_SIG_F16>(filt, vec4, grid, tab, sig, frame_scale, w, S, P, N, sh.spg, sh.groups, d, t0dt, part, img, done, st);
    }
    DelayQ16 d;
    return sig_fmt == PAT_SIG_F32
               ? launch<DelayQ16, PAT_SIG_F32>(filt, vec4, grid, tab, sig, frame_scale, w, S, P, N, sh.spg, sh.groups, d, t0dt, part, img, done, st)
               : launch<DelayQ16, PAT_SIG_F16>(filt, vec4, grid, tab, sig, frame_scale, w, S, P, N, sh.spg, sh.groups, d, t0dt, part, img, done, st);
}


int pat_launch_backproject_const(pat_ctx *ctx, int nx, int ny, double h, double c, const float *d_sxy, int S,
                                 const int32_t *d_pix, int P, const void *sig, int sig_fmt, int sig_is_filtered,
                                 const float *frame_scale, const float *w, int N, int F, double t0, double dt,
                                 float *img, hipStream_t st) {
    if (S == 0) {
        return launch_zero(img, (long)P * F, st);
    }
    const BpShape sh = bp_shape(S, P, F);
    if ((sh.groups > 1 || F >= 2) && pat_px_eligible(sig_fmt, S, P, N, F, sig))
        return pat_launch_backproject_px_const(nx, h, c, d_sxy, S, d_pix, P, sig, sig_fmt, sig_is_filtered,
                                               frame_scale, w, N, F, t0, dt, img, ny, st);
    float *part = nullptr;
    unsigned int *done = nullptr;
    if (sh.groups > 1) {
        int rc = pat_gather_scratch(ctx, P, F, single_part_bytes(S, P, F), &part, &done, st);
        if (rc) return rc;
    }
    DelayF32 d;
    const double inv = 1.0 / dt;
    d.inv_hi = (float)inv;
    d.inv_lo = (float)(inv - (double)d.inv_hi);
    d.off = (float)(-t0 / dt);
    d.umax = (float)(N - 1);
    const dim3 grid(sh.chunks, sh.groups, F);
    const float t0dt = (float)(t0 / dt);
    const float x0 = (float)(-0.5 * (nx - 1) * h), y0 = (float)(-0.5 * (ny - 1) * h);
    const float inv_c = (float)(1.0 / c);
#define PAT_BPC(SF, FI)                                                                                         \
    k_bp_const<SF, FI><<<grid, BP_THREADS, 0, st>>>(sig, frame_scale, w, S, P, N, sh.spg, sh.groups, d, t0dt, \
                                                    part, img, done, d_pix, d_sxy, nx, (float)h, x0, y0, inv_c)
    if (sig_fmt == PAT_SIG_F32) { if (sig_is_filtered) PAT_BPC(PAT_SIG_F32, true); else PAT_BPC(PAT_SIG_F32, false); }
    else { if (sig_is_filtered) PAT_BPC(PAT_SIG_F16, true); else PAT_BPC(PAT_SIG_F16, false); }
#undef PAT_BPC
    PAT_HIP(hipGetLastError());
    return PAT_OK;
}
