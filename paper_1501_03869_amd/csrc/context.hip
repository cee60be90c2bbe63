// Context, error reporting, validation and the small host-side entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "eik_round.h"
#include "pat_internal.h"

static thread_local char g_err[512] = "";

int pat_fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int pat_hip_fail(hipError_t e, const char *what) {
    return pat_fail(e == hipErrorOutOfMemory ? PAT_ENOMEM : PAT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

extern "C" const char *pat_last_error(void) { return g_err; }

extern "C" int pat_version(void) { return 10000; }

size_t pat_env_fault_alloc_bytes() {
    const char *v = std::getenv("PAT_FAULT_ALLOC_BYTES");
    if (!v || !*v) return 0;
    char *end = nullptr;
    const unsigned long long b = std::strtoull(v, &end, 10);
    return (end && *end == 0) ? (size_t)b : 0;
}

long pat_env_round_cap(long builtin_cap) {
    const char *v = std::getenv("PAT_EIK_ROUND_CAP");
    if (!v || !*v) return builtin_cap;
    char *end = nullptr;
    const long r = std::strtol(v, &end, 10);
    return (end && *end == 0 && r >= 1 && r < builtin_cap) ? r : builtin_cap;
}

double pat_env_eik_spin_ms() {
    const char *v = std::getenv("PAT_EIK_SPIN_MS");
    if (!v || !*v) return 50.0;
    char *end = nullptr;
    const double ms = std::strtod(v, &end);
    return (end && *end == 0 && ms >= 0.0 && ms <= 50.0) ? ms : 50.0;
}

bool pat_env_force_win() {
    const char *v = std::getenv("PAT_GATHER_FORCE");
    return v && std::strcmp(v, "win") == 0;
}

int pat_devbuf::grow(size_t need) {
    if (need <= bytes) return PAT_OK;
    release();
    size_t b = std::max(need, (size_t)256);
    if (fault_bytes && b >= fault_bytes)
        return pat_fail(PAT_ENOMEM, "allocation of %zu bytes refused (PAT_FAULT_ALLOC_BYTES=%zu)", b, fault_bytes);
    hipError_t e = hipMalloc(&ptr, b);
    if (e != hipSuccess) {
        ptr = nullptr;
        (void)hipGetLastError();
        return pat_fail(PAT_ENOMEM, "hipMalloc(%zu bytes) failed: %s", b, hipGetErrorString(e));
    }
    bytes = b;
    return PAT_OK;
}

void pat_devbuf::release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

int pat_make_current(pat_ctx *ctx) {
    if (!ctx) return pat_fail(PAT_EINVAL, "null context");
    PAT_HIP(hipSetDevice(ctx->device));
    return PAT_OK;
}

extern "C" int pat_ctx_create(int device, pat_ctx **out) {
    if (!out) return pat_fail(PAT_EINVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    PAT_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return pat_fail(PAT_EINVAL, "device %d out of range [0, %d)", device, n);
    PAT_HIP(hipSetDevice(device));
    pat_ctx *c = new (std::nothrow) pat_ctx();
    if (!c) return pat_fail(PAT_ENOMEM, "host allocation failed");
    c->device = device;
    const size_t fb = pat_env_fault_alloc_bytes();
    for (pat_devbuf *b : { &c->gather_scratch, &c->gather_done, &c->sensors, &c->eik_tq, &c->eik_f, &c->eik_flags,
                           &c->eik_lists, &c->eik_seeds, &c->eik_count })
        b->fault_bytes = fb;
    hipError_t e = hipHostMalloc((void **)&c->eik_count_host, pat_eik::EIK_HOST_WORDS * sizeof(uint32_t),
                                 hipHostMallocDefault);
    if (e != hipSuccess) {
        delete c;
        return pat_hip_fail(e, "hipHostMalloc");
    }
    for (int i = 0; i < pat_eik::EIK_HOST_WORDS; ++i) c->eik_count_host[i] = 0u;
    // the device's fixed scratch array (pat_backproject_noalloc), looked up
    // once per device with this device current
    int rc = pat_fixed_scratch_attach(device, &c->fixed_scratch);
    if (rc) {
        (void)hipHostFree(c->eik_count_host);
        delete c;
        return rc;
    }
    *out = c;
    return PAT_OK;
}

extern "C" int pat_ctx_destroy(pat_ctx *ctx) {
    if (!ctx) return PAT_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    ctx->gather_scratch.release();
    ctx->gather_done.release();
    ctx->sensors.release();
    ctx->eik_tq.release();
    ctx->eik_f.release();
    ctx->eik_flags.release();
    ctx->eik_lists.release();
    ctx->eik_seeds.release();
    ctx->eik_count.release();
    if (ctx->eik_count_host) (void)hipHostFree(ctx->eik_count_host);
    delete ctx;
    return PAT_OK;
}

extern "C" int pat_ctx_reserve(pat_ctx *ctx, int S, int P, int F) {
    int rc = pat_make_current(ctx);
    if (rc) return rc;
    if (S < 0 || P < 0 || F < 0) return pat_fail(PAT_EINVAL, "negative size");
    if (S == 0 || P == 0 || F == 0) return PAT_OK;
    float *part;
    unsigned int *done;
    return pat_gather_scratch(ctx, P, F, pat_backproject_scratch_bytes(S, P, F), &part, &done, nullptr);
}

extern "C" int pat_eikonal_last_stats(pat_ctx *ctx, pat_eikonal_stats *out) {
    if (!ctx || !out) return pat_fail(PAT_EINVAL, "null argument");
    *out = ctx->last_eik;
    return PAT_OK;
}

// Morton (Z-order) index of local tile coordinates: interleaved bits of i and j.
static uint64_t morton2(uint32_t i, uint32_t j) {
    uint64_t r = 0;
    for (int b = 0; b < 16; ++b) {
        r |= (uint64_t)((i >> b) & 1u) << (2 * b);
        r |= (uint64_t)((j >> b) & 1u) << (2 * b + 1);
    }
    return r;
}

extern "C" int pat_tile_order(int nx, int ny, const int32_t *h_pix, int P, int tile_w, int tile_h,
                              int32_t *h_pix_out) {
    if (nx < 1 || ny < 1 || P < 0 || tile_w < 1 || tile_h < 1 || tile_w > 65536 || tile_h > 65536)
        return pat_fail(PAT_EINVAL, "bad sizes nx=%d ny=%d P=%d tile=%dx%d", nx, ny, P, tile_w, tile_h);
    if (P > 0 && (!h_pix || !h_pix_out)) return pat_fail(PAT_EINVAL, "null pixel array");
    if (P > 0 && h_pix == h_pix_out) return pat_fail(PAT_EINVAL, "h_pix_out aliases h_pix");
    const long n = (long)nx * ny;
    const int tx = (nx + tile_w - 1) / tile_w;
    std::vector<std::pair<uint64_t, int32_t>> key((size_t)P);
    for (int p = 0; p < P; ++p) {
        int32_t k = h_pix[p];
        if (k < 0 || k >= n) return pat_fail(PAT_EINVAL, "pixel %d index %d out of range", p, k);
        int i = k % nx, j = k / nx;
        // tile rows run alternately left to right and right to left, so that
        // consecutive tiles are always neighbours
        const int trow = j / tile_h, tcol = (trow & 1) ? tx - 1 - i / tile_w : i / tile_w;
        uint64_t tile = (uint64_t)trow * tx + tcol;
        key[(size_t)p] = { (tile << 32) | morton2((uint32_t)(i % tile_w), (uint32_t)(j % tile_h)), k };
    }
    std::stable_sort(key.begin(), key.end(),
                     [](const std::pair<uint64_t, int32_t> &a, const std::pair<uint64_t, int32_t> &b) {
                         return a.first < b.first;
                     });
    for (int p = 0; p < P; ++p) h_pix_out[p] = key[(size_t)p].second;
    return PAT_OK;
}

// Morton index of local brick coordinates: interleaved bits of i, j and l.
static uint64_t morton3(uint32_t i, uint32_t j, uint32_t l) {
    uint64_t r = 0;
    for (int b = 0; b < 10; ++b) {
        r |= (uint64_t)((i >> b) & 1u) << (3 * b);
        r |= (uint64_t)((j >> b) & 1u) << (3 * b + 1);
        r |= (uint64_t)((l >> b) & 1u) << (3 * b + 2);
    }
    return r;
}

extern "C" int pat_tile_order_3d(int nx, int ny, int nz, const int32_t *h_vox, int P, int tile_w, int tile_h,
                                 int tile_d, int32_t *h_vox_out) {
    if (nx < 1 || ny < 1 || nz < 1 || (long long)nx * ny * nz > (1LL << 31) - 1 || P < 0 || tile_w < 1 ||
        tile_h < 1 || tile_d < 1 || tile_w > 1024 || tile_h > 1024 || tile_d > 1024)
        return pat_fail(PAT_EINVAL, "bad sizes %dx%dx%d P=%d tile=%dx%dx%d", nx, ny, nz, P, tile_w, tile_h, tile_d);
    if (P > 0 && (!h_vox || !h_vox_out)) return pat_fail(PAT_EINVAL, "null voxel array");
    if (P > 0 && h_vox == h_vox_out) return pat_fail(PAT_EINVAL, "h_vox_out aliases h_vox");
    const long n = (long)nx * ny * nz;
    const int tx = (nx + tile_w - 1) / tile_w, ty = (ny + tile_h - 1) / tile_h;
    std::vector<std::pair<uint64_t, int32_t>> key((size_t)P);
    for (int p = 0; p < P; ++p) {
        const int32_t k = h_vox[p];
        if (k < 0 || k >= n) return pat_fail(PAT_EINVAL, "voxel %d index %d out of range", p, k);
        const int i = (int)(k % nx), j = (int)((k / nx) % ny), l = (int)(k / ((long)nx * ny));
        // tiles snake through each layer (rows alternate direction, and so do
        // layers), so that consecutive tiles are always neighbours
        const int tl = l / tile_d;
        int tr = j / tile_h;
        if (tl & 1) tr = ty - 1 - tr;
        const int tc = (tr & 1) ? tx - 1 - i / tile_w : i / tile_w;
        const uint64_t tile = ((uint64_t)tl * ty + tr) * tx + tc;
        key[(size_t)p] = { (tile << 30) | morton3((uint32_t)(i % tile_w), (uint32_t)(j % tile_h),
                                                  (uint32_t)(l % tile_d)), k };
    }
    std::stable_sort(key.begin(), key.end(),
                     [](const std::pair<uint64_t, int32_t> &a, const std::pair<uint64_t, int32_t> &b) {
                         return a.first < b.first;
                     });
    for (int p = 0; p < P; ++p) h_vox_out[p] = key[(size_t)p].second;
    return PAT_OK;
}

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

extern "C" int pat_filter(pat_ctx *ctx, const float *d_p, int rows, int N, double t0, double dt, float *d_b,
                          void *stream) {
    int rc = pat_make_current(ctx);
    if (rc) return rc;
    if (rows < 0 || N < 2) return pat_fail(PAT_EINVAL, "need rows >= 0 and N >= 2 (rows=%d N=%d)", rows, N);
    if (!finite_pos(dt) || !std::isfinite(t0)) return pat_fail(PAT_EINVAL, "need finite t0 and dt > 0");
    if (rows == 0) return PAT_OK;
    if (!d_p || !d_b) return pat_fail(PAT_EINVAL, "null signal pointer");
    if (d_p == d_b) return pat_fail(PAT_EINVAL, "in-place filtering is not supported");
    return pat_launch_filter(d_p, rows, N, t0, dt, d_b, (hipStream_t)stream);
}

extern "C" int pat_table_to_q16(pat_ctx *ctx, const float *d_table, int64_t n, double t0, double dt, int N,
                                uint32_t *d_q, void *stream) {
    int rc = pat_make_current(ctx);
    if (rc) return rc;
    if (n < 0) return pat_fail(PAT_EINVAL, "negative length");
    if (N < 2 || N > 65535) return pat_fail(PAT_EINVAL, "16.16 indices need 2 <= N <= 65535 (N=%d)", N);
    if (!finite_pos(dt) || !std::isfinite(t0)) return pat_fail(PAT_EINVAL, "need finite t0 and dt > 0");
    if (n == 0) return PAT_OK;
    if (!d_table || !d_q) return pat_fail(PAT_EINVAL, "null table pointer");
    return pat_launch_table_to_q16(d_table, n, t0, dt, N, d_q, (hipStream_t)stream);
}

extern "C" int pat_table_to_fixed(pat_ctx *ctx, const float *d_table, int S, int P, double t0, double dt, int N,
                                  uint32_t *d_q, void *stream) {
    if (S < 0 || P < 0) {
        int rc = pat_make_current(ctx);
        return rc ? rc : pat_fail(PAT_EINVAL, "negative size (S=%d P=%d)", S, P);
    }
    return pat_table_to_q16(ctx, d_table, (int64_t)S * P, t0, dt, N, d_q, stream);
}

extern "C" size_t pat_table_r16_bytes(int S, int P) {
    if (S <= 0 || P <= 0) return 0;
    return pat_r16_bytes(S, P);
}

extern "C" size_t pat_table_x4_bytes(int S, int P) {
    if (S <= 0 || P <= 0) return 0;
    return pat_x4_bytes(S, P);
}

extern "C" int pat_table_to_x4(pat_ctx *ctx, const float *d_table, int S, int P, float *d_out, void *stream) {
    int rc = pat_make_current(ctx);
    if (rc) return rc;
    if (S < 0 || P < 0) return pat_fail(PAT_EINVAL, "negative size (S=%d P=%d)", S, P);
    if ((long long)((S + 3) / 4) * P > INT32_MAX) return pat_fail(PAT_EINVAL, "table too large (S=%d P=%d)", S, P);
    if (S == 0 || P == 0) return PAT_OK;
    if (!d_table || !d_out) return pat_fail(PAT_EINVAL, "null table pointer");
    if ((uintptr_t)d_out % 16 != 0) return pat_fail(PAT_EINVAL, "the interleaved table must be 16-byte aligned");
    return pat_launch_table_to_x4(d_table, S, P, d_out, (hipStream_t)stream);
}

extern "C" int pat_table_to_r16(pat_ctx *ctx, const float *d_table, int S, int P, double t0, double dt, int N,
                                void *d_out, void *stream) {
    int rc = pat_make_current(ctx);
    if (rc) return rc;
    if (S < 0 || P < 0) return pat_fail(PAT_EINVAL, "negative size (S=%d P=%d)", S, P);
    if (N < 2 || N > 65535) return pat_fail(PAT_EINVAL, "16-bit tables need 2 <= N <= 65535 (N=%d)", N);
    if (!finite_pos(dt) || !std::isfinite(t0)) return pat_fail(PAT_EINVAL, "need finite t0 and dt > 0");
    if (S == 0 || P == 0) return PAT_OK;
    if (!d_table || !d_out) return pat_fail(PAT_EINVAL, "null table pointer");
    return pat_launch_table_to_r16(d_table, S, P, t0, dt, N, d_out, (hipStream_t)stream);
}

// Checks shared by pat_backproject and pat_backproject_noalloc: PAT_OK to
// launch, 1 when there is nothing to do, else a negative status.
static int backproject_args(pat_ctx *ctx, const void *d_table, int table_fmt, const void *d_sig, int sig_fmt, int S,
                            int P, int N, double t0, double dt, int F, float *d_img) {
    int rc = pat_make_current(ctx);
    if (rc) return rc;
    if (S < 0 || P < 0 || F < 0) return pat_fail(PAT_EINVAL, "negative size (S=%d P=%d F=%d)", S, P, F);
    if (N < 2) return pat_fail(PAT_EINVAL, "need N >= 2 samples (N=%d)", N);
    if (table_fmt != PAT_TABLE_F32 && table_fmt != PAT_TABLE_Q16 && table_fmt != PAT_TABLE_R16 &&
        table_fmt != PAT_TABLE_F32X4)
        return pat_fail(PAT_EINVAL, "unknown table format %d", table_fmt);
    if (sig_fmt != PAT_SIG_F32 && sig_fmt != PAT_SIG_F16) return pat_fail(PAT_EINVAL, "unknown signal format %d", sig_fmt);
    if ((table_fmt == PAT_TABLE_Q16 || table_fmt == PAT_TABLE_R16) && N > 65535)
        return pat_fail(PAT_EINVAL, "16.16 and 16-bit tables need N <= 65535");
    if (table_fmt == PAT_TABLE_F32X4 && d_table && (uintptr_t)d_table % 16 != 0)
        return pat_fail(PAT_EINVAL, "interleaved tables must be 16-byte aligned");
    if (!finite_pos(dt) || !std::isfinite(t0)) return pat_fail(PAT_EINVAL, "need finite t0 and dt > 0");
    if ((long long)S * N > INT32_MAX || (long long)S * P > ((long long)1 << 40))
        return pat_fail(PAT_EINVAL, "sizes too large");
    if (P == 0 || F == 0) return 1;
    if (!d_img) return pat_fail(PAT_EINVAL, "null image pointer");
    if (S > 0 && (!d_table || !d_sig)) return pat_fail(PAT_EINVAL, "null table or signal pointer");
    return PAT_OK;
}

extern "C" int pat_backproject(pat_ctx *ctx, const void *d_table, int table_fmt, const void *d_sig, int sig_fmt,
                               int sig_is_filtered, const float *d_frame_scale, const float *d_w, int S, int P,
                               int N, double t0, double dt, int F, float *d_img, void *stream) {
    int rc = backproject_args(ctx, d_table, table_fmt, d_sig, sig_fmt, S, P, N, t0, dt, F, d_img);
    if (rc) return rc > 0 ? PAT_OK : rc;
    return pat_launch_backproject(ctx, d_table, table_fmt, d_sig, sig_fmt, sig_is_filtered, d_frame_scale, d_w, S, P,
                                  N, F, t0, dt, d_img, (hipStream_t)stream);
}

extern "C" int pat_backproject_noalloc(pat_ctx *ctx, const void *d_table, int table_fmt, const void *d_sig,
                                       int sig_fmt, int sig_is_filtered, const float *d_frame_scale, const float *d_w,
                                       int S, int P, int N, double t0, double dt, int F, float *d_img, void *stream) {
    int rc = backproject_args(ctx, d_table, table_fmt, d_sig, sig_fmt, S, P, N, t0, dt, F, d_img);
    if (rc) return rc > 0 ? PAT_OK : rc;
    // the same kernels as pat_backproject; their scratch comes from the
    // device's fixed array for the duration of this call
    struct Fixed {
        pat_ctx *c;
        explicit Fixed(pat_ctx *x) : c(x) { c->fixed_active = true; }
        ~Fixed() { c->fixed_active = false; }
    } fixed(ctx);
    return pat_launch_backproject(ctx, d_table, table_fmt, d_sig, sig_fmt, sig_is_filtered, d_frame_scale, d_w, S, P,
                                  N, F, t0, dt, d_img, (hipStream_t)stream);
}

extern "C" int pat_backproject_const_3d(pat_ctx *ctx, int nx, int ny, int nz, double h, double c,
                                        const double *h_sensor_xyz, int S, const int32_t *d_vox, int P,
                                        const void *d_sig, int sig_fmt, int sig_is_filtered, const float *d_frame_scale,
                                        const float *d_w, int N, int F, double t0, double dt, float *d_img,
                                        void *stream) {
    int rc = pat_make_current(ctx);
    if (rc) return rc;
    if (nx < 1 || ny < 1 || nz < 1 || (long long)nx * ny * nz > INT32_MAX || !finite_pos(h) || !finite_pos(c))
        return pat_fail(PAT_EINVAL, "need a grid of at most 2^31-1 nodes, h > 0 and c > 0");
    if (S < 0 || P < 0 || F < 0) return pat_fail(PAT_EINVAL, "negative size");
    if (N < 2 || !finite_pos(dt) || !std::isfinite(t0)) return pat_fail(PAT_EINVAL, "need N >= 2, finite t0, dt > 0");
    if (sig_fmt != PAT_SIG_F32 && sig_fmt != PAT_SIG_F16) return pat_fail(PAT_EINVAL, "unknown signal format %d", sig_fmt);
    if ((long long)S * N > INT32_MAX) return pat_fail(PAT_EINVAL, "sizes too large");
    if (P == 0 || F == 0) return PAT_OK;
    if (!d_img || !d_vox || (S > 0 && (!d_sig || !h_sensor_xyz))) return pat_fail(PAT_EINVAL, "null pointer");
    if (S == 0)
        return pat_launch_backproject_const(ctx, nx, ny, h, c, nullptr, 0, d_vox, P, d_sig, sig_fmt, sig_is_filtered,
                                            d_frame_scale, d_w, N, F, t0, dt, d_img, (hipStream_t)stream);
    if (!pat_px_eligible(sig_fmt, S, P, N, F, d_sig))
        return pat_fail(PAT_EINVAL, "3-D straight-ray back projection needs N >= 4, a signal pointer aligned to its "
                                    "sample size and per-step offsets below 2^31 (N=%d)", N);
    std::vector<float> sxyz((size_t)3 * S);
    for (int i = 0; i < 3 * S; ++i) {
        if (!std::isfinite(h_sensor_xyz[i])) return pat_fail(PAT_EINVAL, "non-finite sensor position");
        sxyz[(size_t)i] = (float)h_sensor_xyz[i];
    }
    if ((rc = ctx->sensors.grow(sxyz.size() * sizeof(float)))) return rc;
    PAT_HIP(hipMemcpyAsync(ctx->sensors.ptr, sxyz.data(), sxyz.size() * sizeof(float), hipMemcpyHostToDevice,
                           (hipStream_t)stream));
    return pat_launch_backproject_px_const(nx, h, c, static_cast<const float *>(ctx->sensors.ptr), S, d_vox, P, d_sig,
                                           sig_fmt, sig_is_filtered, d_frame_scale, d_w, N, F, t0, dt, d_img, ny,
                                           (hipStream_t)stream, nz);
}

extern "C" int pat_backproject_const(pat_ctx *ctx, int nx, int ny, double h, double c, const double *h_sensor_xy,
                                     int S, const int32_t *d_pix, int P, const void *d_sig, int sig_fmt,
                                     int sig_is_filtered, const float *d_frame_scale, const float *d_w, int N, int F,
                                     double t0, double dt, float *d_img, void *stream) {
    int rc = pat_make_current(ctx);
    if (rc) return rc;
    if (nx < 1 || ny < 1 || !finite_pos(h) || !finite_pos(c)) return pat_fail(PAT_EINVAL, "need a grid, h > 0 and c > 0");
    if (S < 0 || P < 0 || F < 0) return pat_fail(PAT_EINVAL, "negative size");
    if (N < 2 || !finite_pos(dt) || !std::isfinite(t0)) return pat_fail(PAT_EINVAL, "need N >= 2, finite t0, dt > 0");
    if (sig_fmt != PAT_SIG_F32 && sig_fmt != PAT_SIG_F16) return pat_fail(PAT_EINVAL, "unknown signal format %d", sig_fmt);
    if ((long long)S * N > INT32_MAX) return pat_fail(PAT_EINVAL, "sizes too large");
    if (P == 0 || F == 0) return PAT_OK;
    if (!d_img || !d_pix || (S > 0 && (!d_sig || !h_sensor_xy))) return pat_fail(PAT_EINVAL, "null pointer");
    // stream-ordered copy of the sensor positions (as float32) into context memory
    std::vector<float> sxy((size_t)2 * S);
    for (int i = 0; i < 2 * S; ++i) {
        if (!std::isfinite(h_sensor_xy[i])) return pat_fail(PAT_EINVAL, "non-finite sensor position");
        sxy[(size_t)i] = (float)h_sensor_xy[i];
    }
    if (S > 0) {
        if ((rc = ctx->sensors.grow(sxy.size() * sizeof(float)))) return rc;
        PAT_HIP(hipMemcpyAsync(ctx->sensors.ptr, sxy.data(), sxy.size() * sizeof(float), hipMemcpyHostToDevice,
                               (hipStream_t)stream));
    }
    return pat_launch_backproject_const(ctx, nx, ny, h, c, static_cast<const float *>(ctx->sensors.ptr), S, d_pix, P,
                                        d_sig, sig_fmt, sig_is_filtered, d_frame_scale, d_w, N, F, t0, dt, d_img,
                                        (hipStream_t)stream);
}
