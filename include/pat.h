/*
 * pat.h - C ABI of libpat, fast-marching-based back projection for
 * photoacoustic tomography in heterogeneous media on AMD Instinct MI355X
 * (gfx950).  Method: Wang & Jing, "A fast marching method based back
 * projection algorithm for photoacoustic tomography in heterogeneous media".
 *
 * Three steps form the hot path:
 *   pat_eikonal_tables  per-sensor first-arrival times (Section II-B: the
 *                       eikonal equation solved from each sensor as a point
 *                       source, by ray reversibility), sampled at the
 *                       region-of-interest pixels -> delay table t_{i,j};
 *   pat_filter          b_i(t) = p_i(t) - t dp_i/dt (the bracket of the back
 *                       projection equation, Section II-C);
 *   pat_backproject     P(r_j) = sum_i w_i b_i(t_{i,j}), linear interpolation
 *                       in time (Section II-C, Eq. BP).
 * The tables are built once per geometry and reused for every frame (the
 * paper's offline / online split, Section III).
 *
 * Conventions for every function:
 *   - Return 0 (PAT_OK) or a negative pat_status; nothing throws across the
 *     ABI.  pat_last_error() gives a message for the calling thread's last
 *     failure.
 *   - Arguments named d_* are device pointers (HIP device memory of the
 *     context's device), h_* are host pointers.  The caller owns all of them;
 *     the library never frees caller memory.
 *   - stream is a hipStream_t passed as void* (NULL = the null stream).  Work
 *     is enqueued on it; the caller keeps buffers alive until the stream has
 *     executed the work (hipMemcpyAsync semantics).  Functions that must read
 *     a result back to the host (pat_eikonal_tables) synchronise the stream.
 *   - Inputs are validated before any launch; invalid ones give PAT_EINVAL
 *     and launch nothing.
 *   - Grid convention: node (i, j), i along x, flat index k = j*nx + i, at
 *     x_i = (i - (nx-1)/2) h, y_j = (j - (ny-1)/2) h (grid-centred metres).
 *   - Time convention: sample n of a signal is taken at t_n = t0 + n dt
 *     (the laser pulse fires at t = 0).
 *   - Failure injection, for tests of the error paths (both unset in normal
 *     use; every kernel still runs to completion):
 *       PAT_FAULT_ALLOC_BYTES=b  read by pat_ctx_create and pat_server_create:
 *         that context or server treats every device allocation of b bytes or
 *         more as failed (PAT_ENOMEM, or a failed map build in a server);
 *       PAT_EIK_ROUND_CAP=r  read at each pat_eikonal_tables /
 *         pat_eikonal_tables_3d call: the relaxation stops with PAT_ENOCONV
 *         after r rounds when r is below the built-in cap.
 *   - PAT_EIK_SPIN_MS=t (0 <= t <= 50, default 50), read at each
 *     pat_eikonal_tables / pat_eikonal_tables_3d call: how long the host polls
 *     the device's pinned word between relaxation rounds before it
 *     synchronises the stream instead; 0 synchronises at once.
 */
#ifndef PAT_H
#define PAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pat_status {
    PAT_OK = 0,
    PAT_EINVAL = -1,     /* invalid argument (nothing was launched) */
    PAT_ENOMEM = -2,     /* device or host allocation failed */
    PAT_EDEVICE = -3,    /* a HIP runtime call failed */
    PAT_EBUSY = -4,      /* admission refused (serving API) */
    PAT_ENOTFOUND = -5,  /* unknown map id or ticket (serving API) */
    PAT_ETIMEOUT = -6,   /* wait timed out (serving API) */
    PAT_ENOCONV = -7     /* eikonal iteration exceeded its round cap */
} pat_status;

/* Delay-table formats accepted by pat_backproject. */
enum {
    PAT_TABLE_F32 = 0,   /* float32 seconds; non-finite = no contribution */
    PAT_TABLE_Q16 = 1,   /* uint32 16.16 fractional sample index,
                            0xFFFFFFFF = no contribution */
    PAT_TABLE_R16 = 2,   /* 16-bit offsets from a base per sensor and 32-entry
                            tile (pat_table_to_r16): a 16.16 table in about
                            half the bytes */
    PAT_TABLE_F32X4 = 3  /* float32 seconds with four sensors interleaved per
                            ROI position (pat_table_to_x4): the same entries
                            as PAT_TABLE_F32, read four at a time */
};

/* Signal formats accepted by pat_backproject. */
enum {
    PAT_SIG_F32 = 0,     /* float32 samples */
    PAT_SIG_F16 = 1      /* IEEE binary16 samples, value = half * frame_scale[f] */
};

typedef struct pat_ctx pat_ctx;

/* Message describing the calling thread's most recent failure ("" if none). */
const char *pat_last_error(void);

/* Library version, major*10000 + minor*100 + patch. */
int pat_version(void);

/* Create a context bound to HIP device `device` (it becomes current for the
 * calling thread).  The context owns reusable device scratch (eikonal working
 * maps, gather partial sums).  One context may be used from one host thread
 * at a time. */
int pat_ctx_create(int device, pat_ctx **out);
int pat_ctx_destroy(pat_ctx *ctx);

/* Allocate the context's gather scratch for pat_backproject calls of S
 * sensors, P pixels and F frames now, so that later calls of these sizes
 * allocate nothing (for example inside HIP graph capture).  Synchronous. */
int pat_ctx_reserve(pat_ctx *ctx, int S, int P, int F);

/* Upper bound of the partial-sum scratch pat_backproject may use for these
 * sizes (0 when one workgroup per pixel block covers all sensors); a small
 * zeroed buffer of completion counters comes on top.  Calls that take the
 * split-sensor kernel (N >= 4 and 32-bit offsets suffice; see
 * pat_backproject) use none.  Host-only, no GPU needed. */
size_t pat_backproject_scratch_bytes(int S, int P, int F);

/*
 * Delay tables (Section II-B): for every sensor s, the first-arrival time
 * field of |grad T| = 1/c from s as a point source, discretised by the
 * first-order upwind (Godunov) scheme on the 4-neighbour grid, the discrete
 * solution the fast marching method computes; d_table[s][p] = T_s(pix[p]).
 *
 *   d_speed   float32 [ny][nx] speed of sound (m/s) at the nodes; every value
 *             finite and > 0.
 *   nx, ny    grid size, each >= 2.   h  node spacing (metres), > 0.
 *   h_sensor_xy  float64 [S][2] sensor positions (metres, grid-centred), each
 *             inside the grid's bounding box.
 *   d_pix     int32 [P] region-of-interest node indices k = j*nx + i, each in
 *             [0, nx*ny).  Any order; the table follows it.
 *   d_table   float32 [S][P] output, seconds (pixel-major per sensor).
 *
 * Source seeding: nodes within 2h of the sensor are fixed at the straight-ray
 * time |x_k - s| / c(n*), n* the node nearest the sensor; the rest converge
 * to the upwind fixed point by tile-parallel relaxation in integer fixed
 * point, with an update exact in integers (the first-order root rounded to
 * the nearest unit of lsb_seconds, each node's slowness h/c in whole units),
 * so the same inputs give the same table bit for bit.  The slowest node's
 * slowness is at most 2^23 units, so a medium whose speeds span a ratio rho
 * rounds its fastest nodes' slowness to about 0.5 rho / 2^23 relative or
 * more (1e-5 at rho of about 23 on a 1024^2 grid, where the grid's extent
 * sets the unit).  Synchronises `stream`.  PAT_ENOCONV if the relaxation exceeds its
 * round cap, 100 (tiles_x + tiles_y) + 1000 rounds of 32 x 32 tiles (never
 * expected; PAT_EIK_ROUND_CAP lowers it); the context stays usable.  Between
 * rounds the host waits on a pinned word the device writes (spinning, then
 * synchronising the stream after 50 ms); PAT_EDEVICE if a round reports more
 * active tiles than the maps have (never expected).
 */
int pat_eikonal_tables(pat_ctx *ctx, const float *d_speed, int nx, int ny, double h,
                       const double *h_sensor_xy, int S, const int32_t *d_pix, int P,
                       float *d_table, void *stream);

/*
 * The local update of pat_eikonal_tables and pat_eikonal_tables_3d alone,
 * for checking it against its definition (Section II-B, first-order upwind
 * discretisation).  For entry i, with neighbour minima n_k = d_nbr[i][k]
 * (k < dims; 0xFFFFFFFF = not reached; d_nbr[i][2] unused for dims = 2) and
 * slowness F = d_F[i] in the same units, d_out[i] is the largest T with
 *   sum_k max(2 (T - n_k) - 1, 0)^2 <= 4 F^2,
 * the first-order root rounded to the nearest unit (halves up), held below
 * 0xFFFFFFFF; 0xFFFFFFFF when every neighbour is unreached.  F must be at
 * most 2^23 (entries above give 0).
 *
 *   d_nbr  uint32 [n][3] device, caller-owned.   d_F  uint32 [n] device.
 *   d_out  uint32 [n] device.   dims  2 or 3.
 *
 * Asynchronous on `stream`.  PAT_EINVAL for n < 0, other dims or null
 * buffers with n > 0.
 */
int pat_eikonal_update_eval(const uint32_t *d_nbr, const uint32_t *d_F, int n, int dims, uint32_t *d_out,
                            void *stream);

/*
 * Delay tables with the paper's second-order scheme (Section II-B): the fast
 * marching method itself, with the second-order one-sided difference
 * (3T - 4T1 + T2)/(2h) along an axis where both upwind nodes are accepted and
 * T2 <= T1 (else the first-order difference), the nodes accepted in heap
 * order (smallest trial time first, ties by node index).  Each axis adds
 * c (T - b)^2 to sum = (h/c_node)^2, c = 9/4 and b = (4 T1 - T2)/3 (second
 * order) or c = 1 and b = T1; both axes are used when the root lies at or
 * above both b, else the smaller one-axis root.  Computed in FP64 per map
 * (one map per wave, the marching itself sequential), so the times equal the
 * definition's; rounded once to float32 seconds.  Arguments, seeding and
 * errors as pat_eikonal_tables (grid up to 2^28 nodes); memory
 * about 25 bytes per node per map in flight (maps in chunks of 8 GiB).
 * Synchronises `stream`.  The first 4096 entries of a map's trial set sit in
 * LDS; the environment variable PAT_FMM2_LDS_ENTRIES (0 .. 4096), read at
 * each call, lowers that count, which only moves entries to device memory
 * (used by the tests of that part; the results do not change).
 */
int pat_eikonal_tables_o2(pat_ctx *ctx, const float *d_speed, int nx, int ny, double h,
                          const double *h_sensor_xy, int S, const int32_t *d_pix, int P,
                          float *d_table, void *stream);

/*
 * 3-D delay tables (3-D reconstruction, anticipated in Section IV): the same
 * first-order upwind scheme on a 6-neighbour grid, each node updated from the
 * upwind minima along x, y and z (one-, two- or three-sided root, whichever
 * stays causal).  The delay-and-sum gather is unchanged: a voxel is a "pixel"
 * of pat_backproject.
 *
 *   d_speed   float32 [nz][ny][nx] speed of sound (m/s), finite and > 0.
 *   nx, ny, nz  grid size, each >= 1, at least 2 nodes, at most 2^30 nodes.
 *   h         node spacing (metres), > 0, the same along all axes.
 *   h_sensor_xyz  float64 [S][3] sensor positions (metres, grid-centred:
 *             node (i, j, l) sits at ((i - (nx-1)/2) h, (j - (ny-1)/2) h,
 *             (l - (nz-1)/2) h)), each inside the grid's bounding box.
 *   d_vox     int32 [P] region-of-interest node indices k = (l*ny + j)*nx + i,
 *             each in [0, nx*ny*nz).  Any order; the table follows it.
 *   d_table   float32 [S][P] output, seconds.
 *
 * Seeding as in pat_eikonal_tables (nodes within 2h fixed at the straight-ray
 * time at the nearest node's speed).  Relaxation runs on 8 x 8 x 8 bricks;
 * statistics (pat_eikonal_last_stats) count bricks as tiles.  Synchronises
 * `stream`.  PAT_EINVAL for bad sizes, speeds, sensors or voxel indices;
 * PAT_ENOCONV if the relaxation exceeds its round cap (never expected);
 * PAT_EDEVICE if a round reports more active bricks than the maps have.
 */
int pat_eikonal_tables_3d(pat_ctx *ctx, const float *d_speed, int nx, int ny, int nz, double h,
                          const double *h_sensor_xyz, int S, const int32_t *d_vox, int P,
                          float *d_table, void *stream);

/* Statistics of the calling context's last pat_eikonal_tables or
 * pat_eikonal_tables_3d call. */
typedef struct pat_eikonal_stats {
    int64_t rounds;          /* relaxation rounds, all chunks */
    int64_t tile_visits;     /* tiles (3-D: bricks) processed over all rounds */
    int64_t guard_hits;      /* always 0: the update is exact in integers and has
                                no floating-point fallback */
    int64_t sweeps;          /* in-tile relaxation sweeps over all tile visits; each
                                sweep applies the local update to the tile's
                                32 x 32 nodes (3-D: the brick's 8 x 8 x 8) once */
    double lsb_seconds;      /* fixed-point unit of the working times */
    double seconds;          /* wall time of the call */
} pat_eikonal_stats;
int pat_eikonal_last_stats(pat_ctx *ctx, pat_eikonal_stats *out);

/*
 * Delay table -> 16.16 fixed-point fractional sample index (a storage form of
 * the delays t_{i,j} of Section II-C's back projection sum, not in the paper):
 * u = (T - t0) / dt computed in FP64; d_q[s][p] = round-half-even(u * 65536)
 * when T is finite and 0 <= u <= N-1, else 0xFFFFFFFF (no contribution).
 *
 *   d_table   float32 [S][P] seconds (pat_eikonal_tables).
 *   d_q       uint32 [S][P] output; may not overlap d_table.
 *   t0, dt    sampling of the frames the table will gather (finite t0, dt > 0);
 *             2 <= N <= 65535 samples.
 * Stream-ordered; PAT_EINVAL for negative sizes, bad sampling or null pointers
 * (nothing launched).
 */
int pat_table_to_fixed(pat_ctx *ctx, const float *d_table, int S, int P, double t0, double dt, int N,
                       uint32_t *d_q, void *stream);
/* The same conversion over n consecutive table entries (any [S][P] layout
 * flattened; n = S*P gives pat_table_to_fixed). */
int pat_table_to_q16(pat_ctx *ctx, const float *d_table, int64_t n, double t0, double dt, int N,
                     uint32_t *d_q, void *stream);

/*
 * Delay table -> tile-relative 16-bit form (PAT_TABLE_R16), a compressed
 * 16.16 table for the gather's bandwidth-bound shapes and for resident
 * tables (not in the paper).  The entries of sensor s are cut into tiles of
 * 32 consecutive ROI positions (the last one may be shorter).  With
 * u = (T - t0)/dt in FP64, a delay is valid when T is finite and
 * 0 <= u <= N-1.  For a tile with a valid delay, b = floor(smallest valid u)
 * and k = the largest integer in [0, 16] with (largest valid u - b) * 2^k <=
 * 65534; each valid entry stores off = round-half-even((u - b) * 2^k), each
 * other one 0xFFFF, and the tile's header is (b << 16) | (16 - k).  A tile
 * without valid delays has header 0.  The entry stands for the 16.16 value
 * (b << 16) + (off << (16 - k)), i.e. u' = b + off / 2^k with
 * |u' - u| <= 2^-(k+1) and u' <= N-1; keeping tiles compact (pat_tile_order)
 * keeps k large (11 for compact blocks of the paper geometry, 8 where a run
 * of 32 ROI entries skips nodes outside the ROI).
 *
 *   d_table   float32 [S][P] seconds.  2 <= N <= 65535.
 *   d_out     pat_table_r16_bytes(S, P) bytes: uint16 offsets [S][P] at byte
 *             0, then uint32 headers [S][ceil(P/32)] at byte
 *             2*S*P rounded up to a multiple of 256.
 * Stream-ordered; PAT_EINVAL for bad sizes or parameters.
 */
int pat_table_to_r16(pat_ctx *ctx, const float *d_table, int S, int P, double t0, double dt, int N,
                     void *d_out, void *stream);
/* Bytes of a PAT_TABLE_R16 table of S sensors and P ROI positions.  Host only. */
size_t pat_table_r16_bytes(int S, int P);

/*
 * Delay table -> the same float32 delays (Section II-C's t_{i,j}) with four
 * sensors interleaved per ROI position (PAT_TABLE_F32X4, a layout for the
 * gather, not in the paper): d_out[q][p][r] = d_table[4q + r][p] for
 * q < ceil(S/4), r < 4; entries of padding sensors (4q + r >= S) are NaN and
 * contribute nothing.  The gather then fetches four sensors' delays at a
 * pixel with one 16-byte load instead of four.
 *
 *   d_table   float32 [S][P] seconds.
 *   d_out     pat_table_x4_bytes(S, P) bytes, 16-byte aligned; may not
 *             overlap d_table.  ceil(S/4) * P < 2^31.
 * Stream-ordered; PAT_EINVAL for bad sizes, null or misaligned pointers.
 */
int pat_table_to_x4(pat_ctx *ctx, const float *d_table, int S, int P, float *d_out, void *stream);
/* Bytes of a PAT_TABLE_F32X4 table: 16 ceil(S/4) P.  Host only. */
size_t pat_table_x4_bytes(int S, int P);

/*
 * Host helper: reorder ROI node indices tile-major (tiles of tile_w x tile_h
 * nodes; tile rows alternately left to right and right to left, so that
 * consecutive tiles are neighbours; Z-order (Morton) inside a tile), so that every
 * aligned run of 64, 256 or 1024 pixels of a 32x32-tiled ROI is a compact
 * square or 2:1 patch: the gather's pixel blocks then need short time
 * windows.  Stable for equal keys; h_pix_out may not alias h_pix.  Host only.
 */
int pat_tile_order(int nx, int ny, const int32_t *h_pix, int P, int tile_w, int tile_h,
                   int32_t *h_pix_out);

/*
 * Host helper, the 3-D form of pat_tile_order for voxel indices
 * k = (l*ny + j)*nx + i: tiles of tile_w x tile_h x tile_d voxels (each side
 * <= 1024) snake through each layer of tiles (rows and layers alternate
 * direction); Morton order inside a tile.  With 4 x 4 x 2 tiles every aligned
 * run of 32 voxels of a full tile is one compact brick.  Stable for equal
 * keys; h_vox_out may not alias h_vox.  Host only.
 */
int pat_tile_order_3d(int nx, int ny, int nz, const int32_t *h_vox, int P, int tile_w, int tile_h,
                      int tile_d, int32_t *h_vox_out);

/*
 * UBP filter (Section II-C): b[r][n] = p[r][n] - t_n * D[r][n] with
 * t_n = t0 + n dt and D the central difference (p[n+1]-p[n-1])/(2 dt),
 * one-sided at n = 0 and n = N-1.  rows independent signals of N >= 2 float32
 * samples, row-major.  d_b may equal d_p only if rows == 0.
 */
int pat_filter(pat_ctx *ctx, const float *d_p, int rows, int N, double t0, double dt, float *d_b,
               void *stream);

/*
 * Back projection (Section II-C, Eq. BP):
 *   d_img[f][p] = sum_{s=0}^{S-1} w[s] * lerp(b_f,s, u),  u = (T[s][p] - t0)/dt
 * with linear interpolation between samples floor(u) and floor(u)+1 (the last
 * interval at u = N-1); delays with u < 0, u > N-1 or non-finite contribute 0.
 *
 *   d_table   [S][P], format table_fmt (PAT_TABLE_F32 seconds,
 *             PAT_TABLE_Q16 from pat_table_to_q16 or PAT_TABLE_R16 from
 *             pat_table_to_r16, both with the same t0, dt, N, or
 *             PAT_TABLE_F32X4 from pat_table_to_x4, 16-byte aligned).
 *   d_sig     [F][S][N] signals, format sig_fmt.  If sig_is_filtered is 0 the
 *             signals are raw pressures p and the filter above is applied
 *             inside the kernel; otherwise they are already b.
 *   d_frame_scale  float32 [F] multipliers of PAT_SIG_F16 frames (NULL = 1).
 *   d_w       float32 [S] sensor weights (NULL = all 1).
 *   d_img     float32 [F][P] output.
 * Accumulation is FP32 in a fixed order, so results are bitwise reproducible
 * for fixed inputs and sizes.  Uses context scratch of
 * pat_backproject_scratch_bytes(S, P, F) bytes (allocated on first need, or
 * up front by pat_ctx_reserve).  Kernel choice (results agree to the stated
 * tolerances, not bitwise, across kernels): a table above 128 MiB (half the
 * Infinity Cache) with at least 131072 columns, in any format but
 * PAT_TABLE_F32X4, with N >= 128 and d_sig 4-byte aligned (and N even for
 * FP16), takes one wave per 256 columns reading each sensor's filtered
 * signal from a per-wave window in LDS (no scratch), for any F; else, with
 * F >= 2, a table above 128 MiB, N a multiple of 8 (FP16) or 4 (FP32) and
 * d_sig 16-byte aligned, one launch reads the table once per 16 frames;
 * otherwise, when N >= 4 and d_sig is aligned to its sample size, the
 * sensors of each 32-pixel tile are split inside one workgroup (no scratch)
 * for several frames or for a frame too small to fill the GPU otherwise;
 * the remaining shapes use LDS-windowed workgroups over sensor groups, which
 * add their partial sums in scratch.  PAT_TABLE_R16 and PAT_TABLE_F32X4
 * tables need N >= 4 and an aligned d_sig (else PAT_EINVAL).
 * Sizes: the wave-window kernel takes P < 2^29 and the split-sensor kernel
 * P < 2^26 (32-bit buffer offsets), so PAT_TABLE_F32X4 tables need
 * P < 2^26; larger P in the other forms goes to the kernels with 64-bit
 * offsets.  S, P, N and F are ints, with S*N, P*F and each table row's
 * entries addressable as 64-bit offsets.
 */
int pat_backproject(pat_ctx *ctx, const void *d_table, int table_fmt, const void *d_sig, int sig_fmt,
                    int sig_is_filtered, const float *d_frame_scale, const float *d_w, int S, int P,
                    int N, double t0, double dt, int F, float *d_img, void *stream);

/* Bytes of the fixed device scratch of pat_backproject_noalloc (16 MiB per
 * device, held from the library's load until the process ends). */
#define PAT_NOALLOC_SCRATCH_BYTES (16u << 20)

/*
 * pat_backproject for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, kernels, kernel choice and results (bit for bit) as
 * pat_backproject, but the gather scratch (partial sums and completion
 * counters of the LDS-windowed and batched kernels) comes from a fixed array
 * of PAT_NOALLOC_SCRATCH_BYTES in device memory, one per device, instead of
 * the context's growable buffers: the call makes no hipMalloc, hipFree or
 * other allocating call.  The counters are cleared by a small kernel on
 * `stream` before the gather (no memset node).  PAT_EINVAL, with nothing
 * launched, when the sizes need more scratch than the array holds: at most
 * 4 ceil(P/256) F bytes of counters rounded up to a multiple of 256, plus
 * pat_backproject_scratch_bytes(S, P, F); shapes that take the split-sensor
 * kernel need none.  All calls on one device share that
 * device's array, which keeps the last call's contents: calls that overlap
 * on one device (different streams, contexts or threads) race on it and must
 * be serialised by the caller.
 */
int pat_backproject_noalloc(pat_ctx *ctx, const void *d_table, int table_fmt, const void *d_sig, int sig_fmt,
                            int sig_is_filtered, const float *d_frame_scale, const float *d_w, int S, int P,
                            int N, double t0, double dt, int F, float *d_img, void *stream);

/*
 * Conventional back projection (Section III's comparison reconstruction): the
 * same filtered delay-and-sum as pat_backproject, with the straight-ray delay
 * t = |x_pix[p] - s| / c of a homogeneous medium of speed c computed per
 * gather instead of read from a table.  d_pix are node indices on the grid
 * convention above (used only as coordinates); h_sensor_xy is host float64
 * [S][2] metres (copied stream-ordered into context memory).  Delays are
 * computed in FP32.  Other arguments as pat_backproject; scratch as
 * pat_backproject with the same S, P, F.
 */
int pat_backproject_const(pat_ctx *ctx, int nx, int ny, double h, double c, const double *h_sensor_xy, int S,
                          const int32_t *d_pix, int P, const void *d_sig, int sig_fmt, int sig_is_filtered,
                          const float *d_frame_scale, const float *d_w, int N, int F, double t0, double dt,
                          float *d_img, void *stream);

/*
 * The conventional back projection on a 3-D grid (the 3-D counterpart of
 * pat_backproject_const, for the 3-D reconstruction anticipated in
 * Section IV): straight-ray delays |x_vox[p] - s| / c computed per gather in
 * FP32.  d_vox are node indices k = (l*ny + j)*nx + i on the grid convention
 * of pat_eikonal_tables_3d, each in [0, nx*ny*nz) (used only as
 * coordinates); h_sensor_xyz is host float64 [S][3] metres (copied
 * stream-ordered into context memory).  Runs the split-sensor kernel only:
 * PAT_EINVAL unless N >= 4 and d_sig is aligned to its sample size.  Other
 * arguments as pat_backproject; uses no scratch.
 */
int pat_backproject_const_3d(pat_ctx *ctx, int nx, int ny, int nz, double h, double c, const double *h_sensor_xyz,
                             int S, const int32_t *d_vox, int P, const void *d_sig, int sig_fmt, int sig_is_filtered,
                             const float *d_frame_scale, const float *d_w, int N, int F, double t0, double dt,
                             float *d_img, void *stream);

/* ------------------------------------------------------------------ serving
 *
 * A frame server keeps each speed map's delay table resident in HBM (the
 * paper's table is computed once per geometry offline and reused for every
 * frame, Section III) and gathers incoming frames of any of its maps in
 * mixed-geometry batches: frames that arrive while others are on the GPU join
 * the next batch as slots and memory free up.  Each frame is split across
 * workgroups exactly as a single-frame pat_backproject call of the same sizes
 * would split it, so its image does not depend on its batch-mates.
 */
typedef struct pat_server pat_server;

typedef struct pat_server_config {
    size_t hbm_budget_bytes;  /* device bytes for tables, frames and build working
                                 memory; 0 = 80% of the free memory at creation */
    int table_fmt;            /* PAT_TABLE_F32, PAT_TABLE_Q16 or PAT_TABLE_R16, all maps
                                 (R16: pass the ROI in pat_tile_order order) */
    int max_batch;            /* frames per launch (0 = 64) */
    int max_inflight;         /* batches on the device at once (0 = 2, <= 8) */
    int max_slots;            /* frames submitted and not yet collected by
                                 pat_server_wait (0 = 1024) */
} pat_server_config;

enum { PAT_MAP_BUILDING = 0, PAT_MAP_READY = 1, PAT_MAP_FAILED = 2, PAT_MAP_EVICTED = 3 };

typedef struct pat_stats {
    int64_t frames_submitted, frames_done, frames_refused, batches, builds, evictions;
    double mean_batch_frames;
    double frames_per_s, gathers_per_s;       /* completed frames over the window
                                                 since creation or the last reset */
    double latency_p50_us, latency_p99_us, latency_max_us;  /* submit -> image on host */
    uint64_t bytes_budget, bytes_used, bytes_tables;
    int maps_ready, maps_building, queue_depth, inflight_batches;
} pat_stats;

/* Create a server on ctx's device with an HBM budget (device bytes for
 * tables, frames and build working memory; 0 = 80% of the free memory at
 * creation), float32 resident tables and the defaults of pat_server_config.
 * ctx is not used afterwards; the server owns its streams, threads and a
 * context for table builds.  PAT_EINVAL for a null out, PAT_EDEVICE or
 * PAT_ENOMEM when its streams, events or threads cannot be created. */
int pat_server_create(pat_ctx *ctx, size_t hbm_budget_bytes, pat_server **out);
/* The same with every setting given (cfg may be NULL: all defaults). */
int pat_server_create_ex(pat_ctx *ctx, const pat_server_config *cfg, pat_server **out);
/* Waits for batches on the device, then frees everything. */
int pat_server_destroy(pat_server *s);

/* Register a speed map (host arrays are copied; same conventions as
 * pat_eikonal_tables) with its frames' sampling (t0, dt, N >= 4).  Its table
 * is built asynchronously on the server's build stream; frames may be
 * submitted at once and wait until it is ready.  PAT_EBUSY if its table and
 * build memory cannot fit in the budget even after evicting idle maps;
 * PAT_EINVAL also when an eighth of its table or of a frame exceeds 2 GiB
 * (the gather's 32-bit offsets). */
int pat_server_add_map(pat_server *s, const float *h_speed, int nx, int ny, double h,
                       const double *h_sensor_xy, int S, const int32_t *h_pix, int P,
                       double t0, double dt, int N, int *map_id);
/* The same for a 3-D map (pat_eikonal_tables_3d conventions: speed
 * [nz][ny][nx], sensors [S][3], voxel indices (l*ny + j)*nx + i); its frames
 * are submitted and gathered like any other map's. */
int pat_server_add_map_3d(pat_server *s, const float *h_speed, int nx, int ny, int nz, double h,
                          const double *h_sensor_xyz, int S, const int32_t *h_vox, int P,
                          double t0, double dt, int N, int *map_id);
int pat_server_map_state(pat_server *s, int map_id, int *state);
/* Unregister an idle map (PAT_EBUSY while it has frames or a build). */
int pat_server_remove_map(pat_server *s, int map_id);

/* Submit one raw frame p[S][N] for map_id, host memory, in sig_fmt
 * (PAT_SIG_F32, or PAT_SIG_F16 with value = sample * scale, scale finite and
 * > 0; scale is ignored for float32).  Frames of both formats may be mixed;
 * each launch gathers frames of one format.  The frame is copied to pinned
 * memory before returning.  When all slots are in use: PAT_EBUSY if
 * nonblocking, else wait for a slot.  *ticket identifies the frame.  An
 * evicted map is rebuilt on demand.  PAT_ENOTFOUND for an unknown map,
 * PAT_EINVAL for a bad format or scale, or float32 frames too large for the
 * gather's 32-bit offsets. */
int pat_server_submit(pat_server *s, int map_id, const void *h_frame, int sig_fmt, float scale, int nonblocking,
                      uint64_t *ticket);
/* Wait for a frame and copy its image [P] to h_img (may be NULL); releases the
 * ticket.  timeout_ms < 0 waits forever; PAT_ETIMEOUT keeps the ticket. */
int pat_server_wait(pat_server *s, uint64_t ticket, float *h_img, int timeout_ms);

/* Counters, throughput (frames/s, gathers/s), p50/p99 latency and bytes
 * resident, as of the call. */
int pat_server_stats(pat_server *s, pat_stats *out);
/* Restart the throughput window and the latency record. */
int pat_server_reset_stats(pat_server *s);
/* hold != 0: frames are still admitted and queued but none is launched;
 * hold == 0: launch what is queued (in batches of up to max_batch).  Batches
 * already on the device are not affected.  For callers that collect a burst
 * into shared launches, or pause the device work of a server. */
int pat_server_hold(pat_server *s, int hold);

#ifdef __cplusplus
}
#endif

#endif /* PAT_H */
