// Per-sensor travel-time tables with the paper's second-order scheme
// (Section II-B): fast marching in FP64 with the second-order one-sided
// difference (3T - 4T1 + T2)/(2h) along an axis where both upwind nodes are
// accepted and ordered (T2 <= T1), else the first-order difference.
//
// A second-order update is not monotone in its neighbours, so no parallel
// relaxation is guaranteed to reach the heap-ordered result; the order of
// acceptance is part of the answer.  Each map therefore runs the marching
// itself, in heap order (smallest trial time first, ties by node index),
// on one wave: the wave pops, accepts and updates together, with the map's
// times and states in device memory, its trial set in LDS (spilling to device
// memory), and the maps of a chunk run side by side.
// The arithmetic is the definition's, in FP64 without contraction, so the
// times equal the oracle's.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <vector>

#include "pat_internal.h"

// The definition's arithmetic, operation for operation, on host (seeding)
// and device (marching): no fused multiply-adds.
#pragma clang fp contract(off)

namespace {

constexpr unsigned char ST_FAR = 0, ST_TRIAL = 1, ST_KNOWN = 2;

struct Map2 {
    int nx, ny;
    double h;
    long n;
    long heap_cap;  // entries per map
};

__device__ double godunov1(double a, double b, double fh) {
    const double m = a < b ? a : b;
    if (isinf(m)) return INFINITY;
    const double d = fabs(a - b);
    if (isinf(d) || d >= fh) return m + fh;
    return m + 0.5 * (d + sqrt(2.0 * fh * fh - d * d));
}

// Upwind term along one axis: c = 1, b = T1, or c = 9/4, b = (4 T1 - T2)/3.
template <class State>
__device__ int axis_term(const double *T, const State *st, long m, long step, bool lo, bool hi, bool lo2, bool hi2,
                         double &c, double &b) {
    double t1 = INFINITY;
    int side = 0;
    if (lo && st[m - step] == ST_KNOWN) { t1 = T[m - step]; side = -1; }
    if (hi && st[m + step] == ST_KNOWN && T[m + step] < t1) { t1 = T[m + step]; side = 1; }
    if (side == 0) return 0;
    c = 1.0;
    b = t1;
    const bool ok2 = side < 0 ? lo2 : hi2;
    const long m2 = m + 2 * side * step;
    if (ok2 && st[m2] == ST_KNOWN && T[m2] <= t1) {
        c = 2.25;
        b = (4.0 * t1 - T[m2]) / 3.0;
    }
    return 1;
}

__device__ double update2(int hx, double cx, double bx, int hy, double cy, double by, double fh) {
    if (!hx && !hy) return INFINITY;
    const double ix = cx == 1.0 ? fh : fh / 1.5, iy = cy == 1.0 ? fh : fh / 1.5;
    if (!hy) return bx + ix;
    if (!hx) return by + iy;
    if (cx == 1.0 && cy == 1.0) return godunov1(bx, by, fh);
    const double m = bx < by ? bx : by;
    const double ex = bx - m, ey = by - m;
    const double A = cx + cy, B = cx * ex + cy * ey, C = cx * ex * ex + cy * ey * ey - fh * fh;
    const double disc = B * B - A * C;
    if (disc >= 0.0) {
        const double t = (B + sqrt(disc)) / A;
        if (t >= ex && t >= ey) return m + t;
    }
    const double tx = bx + ix, ty = by + iy;
    return tx < ty ? tx : ty;
}

// The update of node (i, j), stored at m of arrays whose rows are `row`
// apart (the map itself, or a snapshot of a neighbourhood).
template <class State>
__device__ double node_update_at(const double *T, const State *st, long m, long row, int i, int j, const Map2 &g,
                                 double fh) {
    double cx = 0, bx = 0, cy = 0, by = 0;
    const int hx = axis_term(T, st, m, 1, i > 0, i < g.nx - 1, i > 1, i < g.nx - 2, cx, bx);
    const int hy = axis_term(T, st, m, row, j > 0, j < g.ny - 1, j > 1, j < g.ny - 2, cy, by);
    return update2(hx, cx, bx, hy, cy, by, fh);
}

__device__ double node_update(const double *T, const unsigned char *st, const Map2 &g, long m, double fh) {
    return node_update_at(T, st, m, g.nx, (int)(m % g.nx), (int)(m / g.nx), g, fh);
}

// The trial set: one (key, index) pair per trial node, unordered, with each
// node's position in pos.  Every lane of the map's wave takes part: a pop
// scans every 64th entry per lane and finds the smallest with a butterfly
// over the lanes, then moves the last entry into its place; a push appends;
// a smaller time for a node already in the set overwrites its key in place.
// The keys are the nodes' current times and (key, index) is a strict total
// order, so the smallest entry is unique and the nodes come out in the order
// of a lazily deleting binary heap.  The first lcap <= FMM2_LDS_SET entries live
// in the workgroup's LDS, the rest in device memory.  n is the same in every lane;
// lane 0 writes.
constexpr int FMM2_LDS_SET = 4096;

struct TrialSet {
    double *key;  // device memory, entries >= FMM2_LDS_SET
    int *idx;
    double *lkey;  // LDS, entries < lcap
    int *lidx;
    int *pos;  // device memory: position of each trial node
    int n, cap, lcap;
    __device__ void get(int a, double &k, int &i) const {
        if (a < lcap) {
            k = lkey[a];
            i = lidx[a];
        } else {
            k = key[a];
            i = idx[a];
        }
    }
    __device__ void put(int a, double k, int i) {
        if (a < lcap) {
            lkey[a] = k;
            lidx[a] = i;
        } else {
            key[a] = k;
            idx[a] = i;
        }
    }
    __device__ static bool lt(double ka, int ia, double kb, int ib) { return ka < kb || (ka == kb && ia < ib); }
    __device__ bool push(double k, int i, int lane) {
        if (n >= cap) return false;
        if (lane == 0) {
            put(n, k, i);
            pos[i] = n;
        }
        ++n;
        return true;
    }
    __device__ void lower(int p, double k, int i, int lane) {
        if (lane == 0) put(p, k, i);
    }
    // n > 0; every lane returns the smallest entry, and the node moved into
    // its place (mv_i, -1 if none) with its new position mv_p
    __device__ void pop(double &k, int &i, int &mv_i, int &mv_p, int lane) {
        double bk = INFINITY;  // keys are finite
        int bi = 0x7FFFFFFF, bp = -1;
        for (int a = lane; a < n; a += 64) {
            double ka;
            int ia;
            get(a, ka, ia);
            if (lt(ka, ia, bk, bi)) {
                bk = ka;
                bi = ia;
                bp = a;
            }
        }
        for (int off = 32; off >= 1; off >>= 1) {
            const double ok = __shfl_xor(bk, off);
            const int oi = __shfl_xor(bi, off), op = __shfl_xor(bp, off);
            if (lt(ok, oi, bk, bi)) {
                bk = ok;
                bi = oi;
                bp = op;
            }
        }
        k = bk;
        i = bi;
        --n;
        mv_i = -1;
        mv_p = bp;
        if (bp != n) {
            double kl;
            int il;
            get(n, kl, il);
            mv_i = il;
            if (lane == 0) {
                put(bp, kl, il);
                pos[il] = bp;
            }
        }
        if (n >= lcap) __threadfence_block();  // a move in device memory lands before the next scan
    }
};

// One map per wave.  frozen: this map's nf frozen node indices (ascending)
// and their times.  err[m] != 0 reports a full trial set, an exceeded step
// count or a set position out of range (none expected: the set holds n + 64
// entries, each node at most once, and a map takes at most n pops).
__global__ void __launch_bounds__(64) k_fmm2(const float *__restrict__ speed, Map2 g, double *__restrict__ T_all,
                                             unsigned char *__restrict__ st_all, double *__restrict__ hkey_all,
                                             int *__restrict__ hidx_all, int *__restrict__ pos_all,
                                             const int *__restrict__ frozen_idx,
                                             const double *__restrict__ frozen_val, const int *__restrict__ frozen_off,
                                             const int32_t *__restrict__ pix, int P, float *__restrict__ table,
                                             int *__restrict__ err, int lcap) {
    __shared__ double s_hkey[FMM2_LDS_SET];
    __shared__ int s_hidx[FMM2_LDS_SET];
    const int m = blockIdx.x;
    double *T = T_all + (long)m * g.n;
    unsigned char *st = st_all + (long)m * g.n;
    for (long k = threadIdx.x; k < g.n; k += blockDim.x) {
        T[k] = INFINITY;
        st[k] = ST_FAR;
    }
    __syncthreads();
    const int f0 = frozen_off[m], f1 = frozen_off[m + 1];
    for (int q = f0 + (int)threadIdx.x; q < f1; q += blockDim.x) {
        T[frozen_idx[q]] = frozen_val[q];
        st[frozen_idx[q]] = ST_KNOWN;
    }
    __syncthreads();
    TrialSet ts{ hkey_all + (long)m * g.heap_cap, hidx_all + (long)m * g.heap_cap, s_hkey, s_hidx,
                 pos_all + (long)m * g.n, 0, (int)g.heap_cap, lcap };
    const int lane = threadIdx.x;
    const int di[4] = { -1, 1, 0, 0 }, dj[4] = { 0, 0, -1, 1 };
    __shared__ int s_n0, s_bad0;
    if (lane == 0) {
        int bad = 0;
        // initial band: non-frozen neighbours of frozen nodes, valued in index order
        int band[256];
        int nb = 0;
        for (int q = f0; q < f1; ++q) {
            const long k = frozen_idx[q];
            const int i = (int)(k % g.nx), j = (int)(k / g.nx);
            for (int d = 0; d < 4; ++d) {
                const int ii = i + di[d], jj = j + dj[d];
                if (ii < 0 || ii >= g.nx || jj < 0 || jj >= g.ny) continue;
                const long mm = (long)jj * g.nx + ii;
                if (st[mm] != ST_FAR) continue;
                st[mm] = ST_TRIAL;
                if (nb < 256) band[nb++] = (int)mm;
                else bad = 1;
            }
        }
        for (int a = 1; a < nb; ++a)  // insertion sort: at most a few dozen nodes
            for (int b2 = a; b2 > 0 && band[b2 - 1] > band[b2]; --b2) {
                const int t = band[b2]; band[b2] = band[b2 - 1]; band[b2 - 1] = t;
            }
        for (int a = 0; a < nb && !bad; ++a) {
            const long mm = band[a];
            const double fh = (1.0 / (double)speed[mm]) * g.h;
            T[mm] = node_update(T, st, g, mm, fh);
            if (!ts.push(T[mm], (int)mm, 0)) bad = 1;
        }
        s_n0 = ts.n;
        s_bad0 = bad;
    }
    __threadfence_block();
    __syncthreads();
    ts.n = s_n0;
    int bad = s_bad0;  // the same in every lane from here on
    // Marching.  An update reads only accepted nodes, and none is accepted
    // during a pop's four updates, so they all read one snapshot: the 7 x 7
    // neighbourhood of the popped node k (every node the four neighbours'
    // stencils reach) taken after k is accepted.  49 lanes load it and 4
    // more the neighbours' slowness in one round trip, 4 lanes compute the
    // updates, and the wave applies them in neighbour order (lane 0 writes).
    __shared__ double s_T[49], s_t[4], s_fh[4];
    __shared__ int s_S[49], s_ok[4], s_pos[4];
    const int sdx = lane % 7 - 3, sdy = lane / 7 - 3;  // snapshot offset of lanes 0 .. 48
    const long max_steps = 6 * g.n + 64;
    long steps = 0;
    for (;;) {
        if (bad || ts.n == 0) break;
        if (++steps > max_steps) {
            bad = 2;
            break;
        }
        double key;
        int k, mv_i, mv_p;
        ts.pop(key, k, mv_i, mv_p, lane);
        const int i = k % g.nx, j = k / g.nx;
        if (lane < 49) {
            const int ii = i + sdx, jj = j + sdy;
            double tv = INFINITY;
            int sv = ST_FAR;
            if (ii >= 0 && ii < g.nx && jj >= 0 && jj < g.ny) {
                const long q = (long)jj * g.nx + ii;
                tv = T[q];
                sv = st[q];
            }
            s_T[lane] = tv;
            s_S[lane] = sv;
        } else if (lane < 53) {
            const int d = lane - 49, ii = i + di[d], jj = j + dj[d];
            s_fh[d] = (ii >= 0 && ii < g.nx && jj >= 0 && jj < g.ny) ? (1.0 / (double)speed[(long)jj * g.nx + ii]) * g.h
                                                                      : 0.0;
        } else if (lane < 57) {
            // set positions of the neighbours (meaningful for trial ones)
            const int d = lane - 53, ii = i + di[d], jj = j + dj[d];
            s_pos[d] = (ii >= 0 && ii < g.nx && jj >= 0 && jj < g.ny) ? ts.pos[(long)jj * g.nx + ii] : -1;
        }
        __syncthreads();
        if (s_S[24] == ST_KNOWN || key != s_T[24]) {  // a stale entry (none arise: keys are lowered in place)
            __threadfence_block();
            continue;
        }
        if (lane == 0) s_S[24] = ST_KNOWN;
        __syncthreads();
        if (lane < 4) {
            const int d = lane, ii = i + di[d], jj = j + dj[d];
            const int qn = 24 + di[d] + 7 * dj[d];
            const bool ok = ii >= 0 && ii < g.nx && jj >= 0 && jj < g.ny && s_S[qn] != ST_KNOWN;
            s_t[d] = ok ? node_update_at(s_T, s_S, qn, 7, ii, jj, g, s_fh[d]) : 0.0;
            s_ok[d] = ok;
        }
        __syncthreads();
        if (lane == 0) st[k] = ST_KNOWN;
        for (int d = 0; d < 4; ++d) {
            if (!s_ok[d]) continue;
            const int qn = 24 + di[d] + 7 * dj[d];
            const double t = s_t[d];
            if (t < s_T[qn]) {
                const long mm = (long)(j + dj[d]) * g.nx + (i + di[d]);
                if (lane == 0) {
                    T[mm] = t;
                    st[mm] = ST_TRIAL;
                }
                if (s_S[qn] == ST_TRIAL) {
                    // in the set already: its position, unless this pop moved it
                    const int p = (int)mm == mv_i ? mv_p : s_pos[d];
                    if ((unsigned)p >= (unsigned)ts.n) {  // a position outside the set: stop with an error
                        bad = 3;
                        break;
                    }
                    ts.lower(p, t, (int)mm, lane);
                } else if (!ts.push(t, (int)mm, lane)) {
                    bad = 1;
                    break;
                }
            }
        }
        __threadfence_block();  // lane 0's stores land before the next pop and snapshot
        __syncthreads();
    }
    if (lane == 0) err[m] = bad;
    __syncthreads();
    for (int p = threadIdx.x; p < P; p += blockDim.x) table[(long)m * P + p] = (float)T[pix[p]];
}

}  // namespace

extern "C" int pat_eikonal_tables_o2(pat_ctx *ctx, const float *d_speed, int nx, int ny, double h,
                                     const double *h_sensor_xy, int S, const int32_t *d_pix, int P, float *d_table,
                                     void *stream) {
    const auto t_start = std::chrono::steady_clock::now();
    int rc = pat_make_current(ctx);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (nx < 2 || ny < 2) return pat_fail(PAT_EINVAL, "grid must be at least 2x2 (got %dx%d)", nx, ny);
    if ((long long)nx * ny > (1LL << 28)) return pat_fail(PAT_EINVAL, "grid too large");
    if (!(std::isfinite(h) && h > 0.0)) return pat_fail(PAT_EINVAL, "node spacing must be finite and > 0");
    if (S < 0 || P < 0) return pat_fail(PAT_EINVAL, "negative sensor or pixel count");
    if (!d_speed) return pat_fail(PAT_EINVAL, "null speed map");
    if (S > 0 && !h_sensor_xy) return pat_fail(PAT_EINVAL, "null sensor positions");
    if (P > 0 && !d_pix) return pat_fail(PAT_EINVAL, "null pixel list");
    if ((long long)S * P > 0 && !d_table) return pat_fail(PAT_EINVAL, "null table");
    ctx->last_eik = pat_eikonal_stats{};
    const long n = (long)nx * ny;
    std::vector<float> c((size_t)n);
    std::vector<int32_t> pix((size_t)P);
    PAT_HIP(hipMemcpyAsync(c.data(), d_speed, (size_t)n * sizeof(float), hipMemcpyDeviceToHost, st));
    if (P > 0) PAT_HIP(hipMemcpyAsync(pix.data(), d_pix, (size_t)P * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    PAT_HIP(hipStreamSynchronize(st));
    for (long k = 0; k < n; ++k) {
        const double v = c[(size_t)k];
        if (!(std::isfinite(v) && v > 0.0)) return pat_fail(PAT_EINVAL, "speed at node %ld is %g (need finite > 0)", k, v);
    }
    for (int p = 0; p < P; ++p)
        if (pix[(size_t)p] < 0 || pix[(size_t)p] >= n)
            return pat_fail(PAT_EINVAL, "pixel %d index %d outside [0, %ld)", p, pix[(size_t)p], n);
    const double x0 = -0.5 * (nx - 1) * h, y0 = -0.5 * (ny - 1) * h;
    for (int s = 0; s < S; ++s) {
        const double gi = (h_sensor_xy[2 * s] - x0) / h, gj = (h_sensor_xy[2 * s + 1] - y0) / h;
        if (!(gi >= 0.0 && gi <= nx - 1 && gj >= 0.0 && gj <= ny - 1))
            return pat_fail(PAT_EINVAL, "sensor %d lies outside the grid", s);
    }
    if (S == 0 || P == 0) return PAT_OK;

    // per map: times (8 B), states (1 B), set positions (4 B) and a trial set
    // of n + 64 entries (12 B; a node is in it at most once)
    Map2 g;
    g.nx = nx; g.ny = ny; g.h = h; g.n = n; g.heap_cap = n + 64;
    // trial-set entries kept in LDS; PAT_FMM2_LDS_ENTRIES lowers it (tests of
    // the part in device memory)
    int lds_cap = FMM2_LDS_SET;
    if (const char *e = std::getenv("PAT_FMM2_LDS_ENTRIES")) lds_cap = std::max(0, std::min(FMM2_LDS_SET, std::atoi(e)));
    const size_t per_map = (size_t)n * 13 + (size_t)g.heap_cap * 12;
    const int chunk = (int)std::max<long>(1, std::min<long>(S, (long)((8ull << 30) / per_map)));
    if ((rc = ctx->eik_tq.grow((size_t)chunk * per_map))) return rc;
    char *base = static_cast<char *>(ctx->eik_tq.ptr);
    double *T_all = reinterpret_cast<double *>(base);
    double *hkey = T_all + (size_t)chunk * n;
    int *hidx = reinterpret_cast<int *>(hkey + (size_t)chunk * g.heap_cap);
    int *pos_all = hidx + (size_t)chunk * g.heap_cap;
    unsigned char *st_all = reinterpret_cast<unsigned char *>(pos_all + (size_t)chunk * n);

    // seeding, as for the first-order tables: nodes within 2h of the sensor
    // at the straight-ray time with the slowness of the nearest node
    std::vector<int> fidx, foff;
    std::vector<double> fval;
    std::vector<int> errs((size_t)chunk);
    int64_t pops_total = 0;
    for (int s0 = 0; s0 < S; s0 += chunk) {
        const int maps = std::min(chunk, S - s0);
        fidx.clear(); fval.clear(); foff.assign(1, 0);
        for (int m = 0; m < maps; ++m) {
            const double sx = h_sensor_xy[2 * (s0 + m)], sy = h_sensor_xy[2 * (s0 + m) + 1];
            const double gi = (sx - x0) / h, gj = (sy - y0) / h;
            int is = (int)std::floor(gi + 0.5), js = (int)std::floor(gj + 0.5);
            is = std::min(is, nx - 1);
            js = std::min(js, ny - 1);
            const double fs = 1.0 / (double)c[(size_t)((long)js * nx + is)];
            for (int j = js - 3; j <= js + 3; ++j) {
                if (j < 0 || j >= ny) continue;
                for (int i = is - 3; i <= is + 3; ++i) {
                    if (i < 0 || i >= nx) continue;
                    const double dx = (x0 + i * h) - sx, dy = (y0 + j * h) - sy;
                    const double r = std::sqrt(dx * dx + dy * dy);
                    if (r <= 2.0 * h) {
                        fidx.push_back(j * nx + i);
                        fval.push_back(r * fs);
                    }
                }
            }
            foff.push_back((int)fidx.size());
        }
        if ((rc = ctx->eik_seeds.grow(fidx.size() * (sizeof(int) + sizeof(double)) + foff.size() * sizeof(int) + 64)))
            return rc;
        int *d_fidx = static_cast<int *>(ctx->eik_seeds.ptr);
        double *d_fval = reinterpret_cast<double *>(
            (reinterpret_cast<uintptr_t>(d_fidx + fidx.size()) + 7) & ~(uintptr_t)7);
        int *d_foff = reinterpret_cast<int *>(d_fval + fval.size());
        if ((rc = ctx->eik_count.grow((size_t)chunk * sizeof(int)))) return rc;
        int *d_err = static_cast<int *>(ctx->eik_count.ptr);
        PAT_HIP(hipMemcpyAsync(d_fidx, fidx.data(), fidx.size() * sizeof(int), hipMemcpyHostToDevice, st));
        PAT_HIP(hipMemcpyAsync(d_fval, fval.data(), fval.size() * sizeof(double), hipMemcpyHostToDevice, st));
        PAT_HIP(hipMemcpyAsync(d_foff, foff.data(), foff.size() * sizeof(int), hipMemcpyHostToDevice, st));
        k_fmm2<<<dim3(maps), dim3(64), 0, st>>>(d_speed, g, T_all, st_all, hkey, hidx, pos_all, d_fidx, d_fval, d_foff, d_pix,
                                                P, d_table + (long)s0 * P, d_err, lds_cap);
        PAT_HIP(hipGetLastError());
        PAT_HIP(hipMemcpyAsync(errs.data(), d_err, (size_t)maps * sizeof(int), hipMemcpyDeviceToHost, st));
        PAT_HIP(hipStreamSynchronize(st));
        for (int m = 0; m < maps; ++m)
            if (errs[(size_t)m]) return pat_fail(PAT_ENOCONV, "second-order marching of sensor %d stopped (code %d)",
                                                 s0 + m, errs[(size_t)m]);
        pops_total += (int64_t)maps * n;
        ctx->last_eik.rounds += 1;
    }
    ctx->last_eik.tile_visits = pops_total;
    ctx->last_eik.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    return PAT_OK;
}
