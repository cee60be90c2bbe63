// UBP filter b = p - t dp/dt and the 16.16 delay conversion: elementwise,
// HBM-streaming kernels.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "pat_internal.h"

// b[n] = p[n] - t_n D[n], t_n = t0 + n dt, D the central difference inside and
// one-sided at both ends.  Written as p[n] - (n + t0/dt) * 0.5 * (p[n+1] - p[n-1])
// so that dt cancels: the multiplier is an exact small integer when t0 = 0.
//
// One workgroup filters 1024 consecutive samples of one row, 4 per thread, so
// the row and column come from the block index (no division per sample).
// With 16-byte aligned rows (VEC) the 4 samples are one load and one store;
// the two neighbours outside them are separate loads that hit the cache.
template <bool VEC>
__global__ void __launch_bounds__(256) k_filter(const float *__restrict__ p, float *__restrict__ b, int N,
                                                int chunks, float t0_over_dt) {
    const int row = (int)(blockIdx.x / (unsigned)chunks);
    const int n0 = (int)(blockIdx.x - (unsigned)row * chunks) * 1024 + (int)threadIdx.x * 4;
    if (n0 >= N) return;
    const float *x = p + (long)row * N;
    float *y = b + (long)row * N;
    float v[6];  // x[n0-1] ... x[n0+4]
    if (VEC) {
        const float4 c = *reinterpret_cast<const float4 *>(x + n0);
        v[1] = c.x, v[2] = c.y, v[3] = c.z, v[4] = c.w;
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) v[1 + k] = n0 + k < N ? x[n0 + k] : 0.0f;
    }
    v[0] = n0 > 0 ? x[n0 - 1] : 0.0f;
    v[5] = n0 + 4 < N ? x[n0 + 4] : 0.0f;
    float o[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int n = n0 + k;
        float d;
        if (n == 0) d = 2.0f * (v[2] - v[1]);
        else if (n == N - 1) d = 2.0f * (v[k + 1] - v[k]);
        else d = v[k + 2] - v[k];
        const float tn = (float)n + t0_over_dt;
        o[k] = v[k + 1] - tn * (0.5f * d);
    }
    if (VEC) {
        *reinterpret_cast<float4 *>(y + n0) = make_float4(o[0], o[1], o[2], o[3]);
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (n0 + k < N) y[n0 + k] = o[k];
    }
}

int pat_launch_filter(const float *p, long rows, int N, double t0, double dt, float *b, hipStream_t st) {
    const int chunks = (N + 1023) / 1024;
    if (rows * chunks > 0x7FFFFFFFL)
        return pat_fail(PAT_EINVAL, "filter: %ld rows of %d samples exceed one launch", rows, N);
    const bool vec = N % 4 == 0 && ((uintptr_t)p | (uintptr_t)b) % 16 == 0;
    const dim3 grid((unsigned)(rows * chunks)), blk(256);
    const float r = (float)(t0 / dt);
    if (vec) k_filter<true><<<grid, blk, 0, st>>>(p, b, N, chunks, r);
    else k_filter<false><<<grid, blk, 0, st>>>(p, b, N, chunks, r);
    PAT_HIP(hipGetLastError());
    return PAT_OK;
}

// q = rint(u * 65536) with u = (T - t0) / dt in FP64 (division and rounding are
// IEEE round-to-nearest-even on the device), sentinel when out of [0, N-1].
__global__ void __launch_bounds__(256) k_table_to_q16(const float *__restrict__ T, uint32_t *__restrict__ q,
                                                      int64_t n, double t0, double dt, double umax) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double t = (double)T[i];
    const double u = (t - t0) / dt;
    uint32_t r = 0xFFFFFFFFu;
    if (isfinite(t) && u >= 0.0 && u <= umax) r = (uint32_t)rint(u * 65536.0);
    q[i] = r;
}

int pat_launch_table_to_q16(const float *T, int64_t n, double t0, double dt, int N, uint32_t *q, hipStream_t st) {
    const int blk = 256;
    const int64_t grid = (n + blk - 1) / blk;
    k_table_to_q16<<<dim3((unsigned)grid), dim3(blk), 0, st>>>(T, q, n, t0, dt, (double)(N - 1));
    PAT_HIP(hipGetLastError());
    return PAT_OK;
}

// Four sensors interleaved per ROI position: out[q][p][r] = T[4q + r][p],
// NaN (no contribution) for the padding sensors past S.  One thread per
// (quad, position): four coalesced 4-byte reads, one 16-byte write.
__global__ void __launch_bounds__(256) k_table_to_x4(const float *__restrict__ T, float4 *__restrict__ out, int S,
                                                     int P, long n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int q = (int)(i / P);
    const long p = i - (long)q * P;
    float v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int s = 4 * q + r;
        v[r] = s < S ? T[(long)s * P + p] : __builtin_nanf("");
    }
    out[i] = make_float4(v[0], v[1], v[2], v[3]);
}

int pat_launch_table_to_x4(const float *T, int S, int P, float *out, hipStream_t st) {
    const long n = (long)((S + 3) / 4) * P;
    const long blk = 256;
    k_table_to_x4<<<dim3((unsigned)((n + blk - 1) / blk)), dim3((unsigned)blk), 0, st>>>(
        T, reinterpret_cast<float4 *>(out), S, P, n);
    PAT_HIP(hipGetLastError());
    return PAT_OK;
}

// Tile-relative 16-bit delays: 32 lanes per (sensor, 32-entry tile).  The
// tile's smallest and largest valid u come from a butterfly over the 32
// lanes; then b = floor(smallest), k = the largest shift in [0, 16] with
// (largest - b) * 2^k <= 65534, and each valid entry stores
// round-half-even((u - b) * 2^k).  All in FP64 with exact steps (the
// subtraction of b and the scaling by 2^k are exact), so the encoding is
// bit for bit the definition's.
__global__ void __launch_bounds__(256) k_table_to_r16(const float *__restrict__ T, uint16_t *__restrict__ off,
                                                      uint32_t *__restrict__ hdr, int S, int P, int tiles,
                                                      double t0, double dt, double umax) {
    const long pair = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 5;
    const int l = threadIdx.x & 31;
    const bool live = pair < (long)S * tiles;
    const int s = live ? (int)(pair / tiles) : 0, t = live ? (int)(pair % tiles) : 0;
    const long p = (long)t * 32 + l;
    const bool in = live && p < P;
    double u = 0.0;
    bool ok = false;
    if (in) {
        const double tv = (double)T[(long)s * P + p];
        u = (tv - t0) / dt;
        ok = isfinite(tv) && u >= 0.0 && u <= umax;
    }
    double lo = ok ? u : INFINITY, hi = ok ? u : -INFINITY;
    for (int m = 16; m >= 1; m >>= 1) {  // every lane of the wave takes part
        lo = fmin(lo, __shfl_xor(lo, m, 32));
        hi = fmax(hi, __shfl_xor(hi, m, 32));
    }
    if (!in) return;
    const long e = (long)s * P + p;
    if (!(lo <= hi)) {
        if (l == 0) hdr[(long)s * tiles + t] = 0u;
        off[e] = 0xFFFFu;
        return;
    }
    const double b = floor(lo);
    int k = 16;
    while (k > 0 && ldexp(hi - b, k) > 65534.0) --k;
    if (l == 0) hdr[(long)s * tiles + t] = ((uint32_t)b << 16) | (uint32_t)(16 - k);
    off[e] = ok ? (uint16_t)rint(ldexp(u - b, k)) : (uint16_t)0xFFFFu;
}

int pat_launch_table_to_r16(const float *T, int S, int P, double t0, double dt, int N, void *out, hipStream_t st) {
    const int tiles = (P + 31) / 32;
    uint16_t *off = static_cast<uint16_t *>(out);
    uint32_t *hdr = reinterpret_cast<uint32_t *>(static_cast<char *>(out) + pat_r16_hdr_offset(S, P));
    // sensors in chunks of fewer than 2^30 lanes, so the grid stays in range
    const int chunk = (int)std::max<long>(1, std::min<long>(S, (1L << 30) / ((long)tiles * 32)));
    for (int s0 = 0; s0 < S; s0 += chunk) {
        const int n = std::min(chunk, S - s0);
        const long lanes = (long)n * tiles * 32;
        k_table_to_r16<<<dim3((unsigned)((lanes + 255) / 256)), dim3(256), 0, st>>>(
            T + (long)s0 * P, off + (long)s0 * P, hdr + (long)s0 * tiles, n, P, tiles, t0, dt, (double)(N - 1));
        PAT_HIP(hipGetLastError());
    }
    return PAT_OK;
}
