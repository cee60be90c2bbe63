// UBP filter b = p - t dp/dt and the 16.16 delay conversion: elementwise,
// HBM-streaming kernels.
#include <hip/hip_runtime.h>

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
