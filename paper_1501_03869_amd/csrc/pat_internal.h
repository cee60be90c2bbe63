// Internal declarations shared by the libpat translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "pat.h"

// Thread-local error message + status helpers.
int pat_fail(int code, const char *fmt, ...);
int pat_hip_fail(hipError_t e, const char *what);

#define PAT_HIP(call)                                   \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return pat_hip_fail(e_, #call); \
    } while (0)

// Failure-injection settings read from the environment (host only).
// PAT_FAULT_ALLOC_BYTES=b, read when a context or server is created: that
// object refuses every device allocation of b bytes or more as if the device
// were out of memory (0 or unset: off).
size_t pat_env_fault_alloc_bytes();
// PAT_EIK_ROUND_CAP=r, read at each table-build call: the relaxation gives up
// with PAT_ENOCONV after r rounds when r is below the built-in cap.
long pat_env_round_cap(long builtin_cap);
// how long the eikonal round loop polls the device's pinned words before it
// synchronises the stream instead: PAT_EIK_SPIN_MS in [0, 50], else 50
double pat_env_eik_spin_ms();
// Test hook: PAT_GATHER_FORCE=win makes pat_backproject take the wave-window
// gather wherever that kernel can run, so tests reach it at sizes the oracle
// checks.
bool pat_env_force_win();

// Growable device buffer owned by a context.
struct pat_devbuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    size_t fault_bytes = 0;  // injected failure threshold (0 = off)
    int grow(size_t need);  // PAT_OK or PAT_ENOMEM; contents are not preserved
    void release();
};

struct pat_ctx {
    int device = 0;
    // gather partial sums
    pat_devbuf gather_scratch;
    // gather completion counters (kept at zero between launches)
    pat_devbuf gather_done;
    // sensor positions (float32) for the straight-ray gather
    pat_devbuf sensors;
    // eikonal working memory
    pat_devbuf eik_tq, eik_f, eik_flags, eik_lists, eik_seeds, eik_count;
    uint32_t *eik_count_host = nullptr;  // pinned words of a relaxation round, laid out in eik_round.h
    pat_eikonal_stats last_eik{};
    // the device's fixed scratch array (pat_backproject_noalloc), and whether
    // the call in progress takes its gather scratch from there
    void *fixed_scratch = nullptr;
    bool fixed_active = false;
};

int pat_make_current(pat_ctx *ctx);

// One frame of a mixed-geometry gather launch (device-visible).  The shape
// fields come from pat_px_frame_shape and depend only on the frame's own
// S, P, N, so a frame's image does not depend on its batch-mates.
struct pat_bp_desc {
    const uint32_t *tab;   // [S][P] delay table of the frame's map
    const void *sig;       // [S][N] raw samples of the frame
    const float *w;        // [S] sensor weights or null
    float *img;            // [P] output
    int S, P, N, sps;      // sps: sensors per slot (two slots per wave)
    int tiles;             // 32-pixel tiles of this frame
    int block_begin;       // first workgroup of this frame in the launch (a multiple of 8)
    float t0dt, scale;                // t0/dt; FP16 frame scale (1 otherwise)
    float inv_hi, inv_lo, off, umax;  // float32-seconds delay decoding
};

// Whether a map of this shape can go through the multi-frame gather.
bool pat_px_multi_eligible(int sig_fmt, int S, int P, int N);
// Fills the shape and decoding fields of d for one frame; returns the number
// of workgroups it needs (a multiple of 8, so that the next frame's
// block_begin stays a multiple of 8).
int pat_px_frame_shape(pat_bp_desc *d, int S, int P, int N, double t0, double dt);
int pat_launch_px_multi(const pat_bp_desc *d_descs, int nd, int total_blocks, int table_fmt, int sig_fmt,
                        hipStream_t st);

// PAT_TABLE_R16 layout: uint16 offsets [S][P] at byte 0, uint32 headers
// [S][ceil(P/32)] from this byte offset.
__host__ __device__ inline size_t pat_r16_hdr_offset(long long S, long long P) { return ((size_t)(2 * S * P) + 255) & ~(size_t)255; }
__host__ __device__ inline size_t pat_r16_bytes(long long S, long long P) { return pat_r16_hdr_offset(S, P) + (size_t)(4 * S * ((P + 31) / 32)); }

// Launchers (stream-ordered; arguments validated by the callers).
int pat_launch_filter(const float *p, long rows, int N, double t0, double dt, float *b, hipStream_t st);
int pat_launch_table_to_q16(const float *T, int64_t n, double t0, double dt, int N, uint32_t *q,
                            hipStream_t st);
int pat_launch_table_to_r16(const float *T, int S, int P, double t0, double dt, int N, void *out, hipStream_t st);
int pat_launch_table_to_x4(const float *T, int S, int P, float *out, hipStream_t st);
// PAT_TABLE_F32X4 layout: float32 [ceil(S/4)][P][4]
__host__ __device__ inline size_t pat_x4_bytes(long long S, long long P) { return (size_t)(16 * ((S + 3) / 4) * P); }
// Gather scratch shared by the single-frame and batched kernels.
size_t pat_gather_counter_bytes(int P, int F);
// Tables up to this size are taken to stay cached between frames (half of
// the 256 MB Infinity Cache, leaving the rest to the frames streaming past).
constexpr size_t PAT_CACHED_TABLE_BYTES = 128ull << 20;
// The Infinity Cache: a larger table streams from HBM on every pass.
constexpr size_t PAT_INFINITY_CACHE_BYTES = 256ull << 20;
// one-pixel-per-lane gather (no LDS windows, no partial sums in global memory)
bool pat_px_eligible(int sig_fmt, int S, int P, int N, int F, const void *sig);
// the same with straight-ray delays |x - s| / c computed per gather (d_sxy: float32 metres)
// nz = 0: 2-D grid, d_sxy [S][2]; nz >= 1: 3-D grid, d_sxy [S][3]
int pat_launch_backproject_px_const(int nx, double h, double c, const float *d_sxy, int S, const int32_t *d_pix,
                                    int P, const void *sig, int sig_fmt, int sig_is_filtered, const float *frame_scale,
                                    const float *w, int N, int F, double t0, double dt, float *img, int ny,
                                    hipStream_t st, int nz = 0);
int pat_launch_backproject_px(const void *table, int table_fmt, const void *sig, int sig_fmt, int sig_is_filtered,
                              const float *frame_scale, const float *w, int S, int P, int N, int F, double t0,
                              double dt, float *img, hipStream_t st);
// wave-window gather: one wave per run of table columns, the signal read
// from a per-wave LDS window (float32, 16.16 or 16-bit tile-relative tables,
// N >= 128).  Single frames take it from PAT_WIN_MIN_P columns (two 256-
// column groups per compute unit): on the 1024^2 workload's first 128K
// columns it took 0.11 ms against 0.13 for the split-sensor kernel, on its
// first 64K 0.059 against 0.054.
constexpr int PAT_WIN_MIN_P = 131072;
bool pat_win_eligible(int table_fmt, int sig_fmt, int S, int P, int N, int F, const void *sig);
// Whether the wave-window kernel is the one to take for a table of this
// size: above PAT_CACHED_TABLE_BYTES, with PAT_WIN_MIN_P columns, or, for
// several frames, at least 8 waves per compute unit of (256-column group,
// frame) pairs.
bool pat_win_preferred(int P, int F, size_t table_bytes);
int pat_launch_backproject_win(const void *table, int table_fmt, const void *sig, int sig_fmt, int sig_is_filtered,
                               const float *frame_scale, const float *w, int S, int P, int N, int F, double t0,
                               double dt, float *img, hipStream_t st);
// Partial sums and zeroed completion counters for one gather launch on st:
// from the context's growable buffers, or, while ctx->fixed_active, from the
// device's fixed array (counters cleared on st; PAT_EINVAL when they do not fit).
int pat_gather_scratch(pat_ctx *ctx, int P, int F, size_t part_bytes, float **part, unsigned int **done,
                       hipStream_t st);
// Device address of the fixed scratch array on `device` (which must be
// current), looked up once per device.
int pat_fixed_scratch_attach(int device, void **out);
size_t pat_batch_part_bytes(int S, int P, int F);
bool pat_batch_eligible(int sig_fmt, int N, int F, const void *sig);
int pat_launch_backproject_batch(pat_ctx *ctx, const void *table, int table_fmt, const void *sig, int sig_fmt,
                                 int sig_is_filtered, const float *frame_scale, const float *w, int S, int P, int N,
                                 int F, double t0, double dt, float *img, hipStream_t st);
int pat_launch_backproject_const(pat_ctx *ctx, int nx, int ny, double h, double c, const float *d_sxy, int S,
                                 const int32_t *d_pix, int P, const void *sig, int sig_fmt, int sig_is_filtered,
                                 const float *frame_scale, const float *w, int N, int F, double t0, double dt,
                                 float *img, hipStream_t st);
int pat_launch_backproject(pat_ctx *ctx, const void *table, int table_fmt, const void *sig, int sig_fmt,
                           int sig_is_filtered, const float *frame_scale, const float *w, int S, int P,
                           int N, int F, double t0, double dt, float *img, hipStream_t st);
