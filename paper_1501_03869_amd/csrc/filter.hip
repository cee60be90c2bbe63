// UBP filter b = p - t dp/dt and the 16.16 delay conversion: elementwise,
// HBM-streaming kernels.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "pat_internal.h"

// b[n] = p[n] - t_n D[n], t_n = t0 + n dt, D the central difference inside and
// one-sided at both ends.  Written as p[n] - (n + t0/dt) * 0.5 * (p[n+1] - p[n-1])
// so that dt cancels: the multiplier is an exact small integer when t0 = 0.
__global__ void __launch_bounds__(256) k_filter(const float *__restrict__ p, float *__restrict__ b, long total,
                                                int N, float t0_over_dt) {
    long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int n = (int)(idx % N);
    const float *x = p + (idx - n);
    float d;
    if (n == 0) d = 2.0f * (x[1] - x[0]);
    else if (n == N - 1) d = 2.0f * (x[N - 1] - x[N - 2]);
    else d = x[n + 1] - x[n - 1];
    const float tn = (float)n + t0_over_dt;
    b[idx] = x[n] - tn * (0.5f * d);
}

int pat_launch_filter(const float *p, long rows, int N, double t0, double dt, float *b, hipStream_t st) {
    const long total = rows * (long)N;
    const int blk = 256;
    const long grid = (total + blk - 1) / blk;
    k_filter<<<dim3((unsigned)grid), dim3(blk), 0, st>>>(p, b, total, N, (float)(t0 / dt));
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
