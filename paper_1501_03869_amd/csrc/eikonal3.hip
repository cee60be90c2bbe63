// Per-sensor travel-time tables on a 3-D grid: the first-order upwind
// (Godunov) discretisation of |grad T| = 1/c with a 6-neighbour stencil, from
// each sensor as a point source, solved by brick-parallel relaxation to the
// discrete fixed point that fast marching reaches.  This is the 3-D form of
// the method, which the paper anticipates for 3-D reconstruction (Section IV);
// the delay-and-sum gather is the same for 2-D pixels and 3-D voxels.
//
// The scheme follows the 2-D tables: uint32 fixed-point working times,
// values that only decrease, and active-brick lists that repeat until no
// brick changes.  Bricks are 8x8x8 nodes with a one-node halo in LDS.  The
// update is the integer-exact root of eik_update.h over the upwind minima
// a <= b <= c along the three axes, F = round(h / (c lsb)):
//   one-sided   a + F                                      if b - a >= F,
//   two-sided   a + x, x = (d + sqrt(2F^2 - d^2)) / 2       if x <= c - a,
//   three-sided a + ((d + e) + sqrt((d+e)^2 - 3(d^2 + e^2 - F^2))) / 3,
// with d = b - a, e = c - a, rounded to the nearest unit.  It is monotone in
// every neighbour, so the tables do not depend on the brick schedule.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <type_traits>
#include <vector>

#include "eik_update.h"
#include "eik_round.h"
#include "pat_internal.h"

namespace {

constexpr int BS = 8;                   // brick edge (nodes)
constexpr int HB = BS + 2;              // brick edge with halo
constexpr int E3_THREADS = 256;         // 8 x 8 columns x 4 pairs of z nodes
constexpr int NODES_PER_THREAD = BS * BS * BS / E3_THREADS;
constexpr uint32_t TQ_INF = 0xFFFFFFFFu;
constexpr int EX_MAPS = 4;                 // maps per thread in the table extraction
constexpr int SEED_BOX3 = 5;            // frozen nodes lie in a 5^3 box around the nearest node
constexpr int LOCAL_ITER_CAP3 = 6 * BS; // a brick that has not settled re-queues itself

struct EikGrid3 {
    int nx, ny, nz, bx, by, bz, bricks_per_map;
};

__device__ __forceinline__ bool is_frozen3(int gx, int gy, int gz, const int *seed_ijl, const uint32_t *seed_val,
                                           int m, uint32_t &val) {
    const int bx = gx - seed_ijl[3 * m], by = gy - seed_ijl[3 * m + 1], bz = gz - seed_ijl[3 * m + 2];
    if ((unsigned)bx >= (unsigned)SEED_BOX3 || (unsigned)by >= (unsigned)SEED_BOX3 ||
        (unsigned)bz >= (unsigned)SEED_BOX3)
        return false;
    val = seed_val[((m * SEED_BOX3 + bz) * SEED_BOX3 + by) * SEED_BOX3 + bx];
    return val != TQ_INF;
}

// The seed values of the frozen nodes, over maps whose every word the host
// has set to "not reached": one workgroup per map, a thread per node of its
// seed box (a node is frozen where the box holds a value).
__global__ void __launch_bounds__(128) k_eik3_seed(uint32_t *__restrict__ Tq, EikGrid3 g,
                                                   const int *__restrict__ seed_ijl,
                                                   const uint32_t *__restrict__ seed_val) {
    constexpr int B = SEED_BOX3;
    const int m = blockIdx.x, t = threadIdx.x;
    if (t >= B * B * B) return;
    const int gx = seed_ijl[3 * m] + t % B, gy = seed_ijl[3 * m + 1] + (t / B) % B;
    const int gz = seed_ijl[3 * m + 2] + t / (B * B);
    if (gx < 0 || gx >= g.nx || gy < 0 || gy >= g.ny || gz < 0 || gz >= g.nz) return;
    const uint32_t v = seed_val[m * B * B * B + t];
    if (v != TQ_INF) Tq[((long)m * g.nz + gz) * ((long)g.nx * g.ny) + (long)gy * g.nx + gx] = v;
}

__device__ __forceinline__ void activate3(uint32_t brick, uint32_t *flags_next, uint32_t *list_next,
                                          uint32_t *cnt_next) {
    if (atomicExch(&flags_next[brick], 1u) == 0u) {
        const uint32_t pos = atomicAdd(cnt_next, 1u);
        list_next[pos] = brick;
    }
}

__device__ __forceinline__ int hidx(int x, int y, int z) { return (z * HB + y) * HB + x; }

__global__ void __launch_bounds__(E3_THREADS) k_eik3_brick(uint32_t *__restrict__ Tq, const uint32_t *__restrict__ Fmap,
                                                           EikGrid3 g, const int *__restrict__ seed_ijl,
                                                           const uint32_t *__restrict__ seed_val,
                                                           const uint32_t *__restrict__ list_cur,
                                                           uint32_t *__restrict__ flags_cur,
                                                           uint32_t *__restrict__ list_next,
                                                           uint32_t *__restrict__ flags_next,
                                                           uint32_t *__restrict__ counters) {
    __shared__ uint32_t T[HB * HB * HB];
    __shared__ uint32_t side_bits;

    const int tid = threadIdx.x;
    const uint32_t brick = list_cur[blockIdx.x];
    const int m = (int)(brick / g.bricks_per_map);
    const int r = (int)(brick % g.bricks_per_map);
    const int bzi = r / (g.bx * g.by), byi = (r / g.bx) % g.by, bxi = r % g.bx;
    const int gx0 = bxi * BS, gy0 = byi * BS, gz0 = bzi * BS;
    const long nxy = (long)g.nx * g.ny;
    uint32_t *map = Tq + (long)m * nxy * g.nz;
    if (tid == 0) {
        flags_cur[brick] = 0u;
        side_bits = 0u;
    }

    // halo: 6 faces of BS x BS nodes (edges and corners are never read)
    for (int idx = tid; idx < 6 * BS * BS; idx += E3_THREADS) {
        const int face = idx / (BS * BS), o = idx % (BS * BS), u = o % BS, v = o / BS;
        int lx, ly, lz;
        if (face == 0) { lx = -1; ly = u; lz = v; }
        else if (face == 1) { lx = BS; ly = u; lz = v; }
        else if (face == 2) { lx = u; ly = -1; lz = v; }
        else if (face == 3) { lx = u; ly = BS; lz = v; }
        else if (face == 4) { lx = u; ly = v; lz = -1; }
        else { lx = u; ly = v; lz = BS; }
        const int gx = gx0 + lx, gy = gy0 + ly, gz = gz0 + lz;
        const bool in = gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny && gz >= 0 && gz < g.nz;
        T[hidx(lx + 1, ly + 1, lz + 1)] = in ? map[gz * nxy + (long)gy * g.nx + gx] : TQ_INF;
    }

    // this thread's nodes: column (lx, ly), z nodes 2*pair and 2*pair+1
    const int lx = tid % BS, ly = (tid / BS) % BS, pair = tid / (BS * BS);
    const int gx = gx0 + lx, gy = gy0 + ly;
    uint32_t F[NODES_PER_THREAD];
    float F2[NODES_PER_THREAD], F3[NODES_PER_THREAD];  // 2 F^2 and 3 F^2 as floats
    uint32_t own[NODES_PER_THREAD];
    unsigned live = 0;  // bit q: node q is inside the grid and not frozen
    for (int q = 0; q < NODES_PER_THREAD; ++q) {
        const int lz = pair * NODES_PER_THREAD + q;
        const int gz = gz0 + lz;
        const bool in = gx < g.nx && gy < g.ny && gz < g.nz;
        uint32_t v = TQ_INF;
        F[q] = 0u;
        if (in) {
            const long k = gz * nxy + (long)gy * g.nx + gx;
            v = map[k];
            F[q] = Fmap[k];
            uint32_t sv;
            if (!is_frozen3(gx, gy, gz, seed_ijl, seed_val, m, sv)) live |= 1u << q;
        }
        own[q] = v;
        T[hidx(lx + 1, ly + 1, lz + 1)] = v;
        F2[q] = pat_eik::eik_f2(F[q]);
        F3[q] = pat_eik::eik_f3(F[q]);
    }
    __syncthreads();

    unsigned changed = 0;
    // one node (q static, so the per-node registers stay registers)
    auto relax = [&](int q, int &any) {
        if (!(live & (1u << q))) return;
        const int c = hidx(lx + 1, ly + 1, pair * NODES_PER_THREAD + q + 1);
        const uint32_t a = min(T[c - 1], T[c + 1]);
        const uint32_t b = min(T[c - HB], T[c + HB]);
        const uint32_t cz = min(T[c - HB * HB], T[c + HB * HB]);
        const uint32_t nv = pat_eik::godunov3_int(a, b, cz, F[q], F2[q], F3[q]);
        if (nv < own[q]) {
            own[q] = nv;
            T[c] = nv;
            changed |= 1u << q;
            any = 1;
        }
    };
    // sweeps alternate the order of the thread's nodes; false when a sweep
    // changed no node of the brick
    auto sweep = [&](auto rev_c) -> bool {
        int any = 0;
#pragma unroll
        for (int k = 0; k < NODES_PER_THREAD; ++k) relax(decltype(rev_c)::value ? NODES_PER_THREAD - 1 - k : k, any);
        return __syncthreads_or(any) != 0;
    };
    // it ends as the index of the sweep that changed nothing, or the cap
    static_assert(LOCAL_ITER_CAP3 % 2 == 0, "whole sweep pairs");
    int it = 0;
    for (; it < LOCAL_ITER_CAP3; it += 2) {
        if (!sweep(std::false_type{})) break;
        if (!sweep(std::true_type{})) { it += 1; break; }
    }

    unsigned sides = 0;
    for (int q = 0; q < NODES_PER_THREAD; ++q) {
        if (!(changed & (1u << q))) continue;
        const int lz = pair * NODES_PER_THREAD + q;
        map[(gz0 + lz) * nxy + (long)gy * g.nx + gx] = own[q];
        if (lx == 0) sides |= 1u;
        if (lx == BS - 1) sides |= 2u;
        if (ly == 0) sides |= 4u;
        if (ly == BS - 1) sides |= 8u;
        if (lz == 0) sides |= 16u;
        if (lz == BS - 1) sides |= 32u;
    }
    if (it == LOCAL_ITER_CAP3) sides |= 64u;
    if (sides) atomicOr(&side_bits, sides);
    __syncthreads();
    if (tid == 0) {
        atomicAdd(reinterpret_cast<unsigned long long *>(counters + 2),
                  (unsigned long long)min(it + 1, LOCAL_ITER_CAP3));
        const unsigned sb = side_bits;
        uint32_t *cnt_next = counters;
        const uint32_t base = (uint32_t)m * g.bricks_per_map;
        auto id = [&](int x, int y, int z) { return base + (uint32_t)((z * g.by + y) * g.bx + x); };
        if ((sb & 1u) && bxi > 0) activate3(id(bxi - 1, byi, bzi), flags_next, list_next, cnt_next);
        if ((sb & 2u) && bxi + 1 < g.bx) activate3(id(bxi + 1, byi, bzi), flags_next, list_next, cnt_next);
        if ((sb & 4u) && byi > 0) activate3(id(bxi, byi - 1, bzi), flags_next, list_next, cnt_next);
        if ((sb & 8u) && byi + 1 < g.by) activate3(id(bxi, byi + 1, bzi), flags_next, list_next, cnt_next);
        if ((sb & 16u) && bzi > 0) activate3(id(bxi, byi, bzi - 1), flags_next, list_next, cnt_next);
        if ((sb & 32u) && bzi + 1 < g.bz) activate3(id(bxi, byi, bzi + 1), flags_next, list_next, cnt_next);
        if (sb & 64u) activate3(brick, flags_next, list_next, cnt_next);
    }
}

// table[s0 + m][p] = Tq[m][vox[p]] * lsb, rounded once to float32 seconds.
// A thread takes one pixel of EX_MAPS maps (its index read once, the maps'
// loads in flight together); blockIdx.y is the group of EX_MAPS maps within a
// launch that starts at map m0 of the chunk's maps.
__global__ void __launch_bounds__(256) k_eik3_extract(const uint32_t *__restrict__ Tq, long n_nodes,
                                                      const int32_t *__restrict__ vox, int P, int m0, int maps, double lsb,
                                                      float *__restrict__ table) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    const int mb = m0 + (int)blockIdx.y * EX_MAPS;
    const long k = vox[p];
    uint32_t v[EX_MAPS];
#pragma unroll
    for (int j = 0; j < EX_MAPS; ++j)
        if (mb + j < maps) v[j] = Tq[(long)(mb + j) * n_nodes + k];
#pragma unroll
    for (int j = 0; j < EX_MAPS; ++j)
        if (mb + j < maps) table[(long)(mb + j) * P + p] = v[j] == TQ_INF ? INFINITY : (float)((double)v[j] * lsb);
}

}  // namespace

extern "C" int pat_eikonal_tables_3d(pat_ctx *ctx, const float *d_speed, int nx, int ny, int nz, double h,
                                     const double *h_sensor_xyz, int S, const int32_t *d_vox, int P,
                                     float *d_table, void *stream) {
    const auto t_start = std::chrono::steady_clock::now();
    int rc = pat_make_current(ctx);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (nx < 1 || ny < 1 || nz < 1 || (long long)nx * ny * nz < 2)
        return pat_fail(PAT_EINVAL, "grid must have at least 2 nodes (got %dx%dx%d)", nx, ny, nz);
    if ((long long)nx * ny * nz > (1LL << 30)) return pat_fail(PAT_EINVAL, "grid too large");
    if (!(std::isfinite(h) && h > 0.0)) return pat_fail(PAT_EINVAL, "node spacing must be finite and > 0");
    if (S < 0 || P < 0) return pat_fail(PAT_EINVAL, "negative sensor or voxel count");
    if (!d_speed) return pat_fail(PAT_EINVAL, "null speed map");
    if (S > 0 && !h_sensor_xyz) return pat_fail(PAT_EINVAL, "null sensor positions");
    if (P > 0 && !d_vox) return pat_fail(PAT_EINVAL, "null voxel list");
    if ((long long)S * P > 0 && !d_table) return pat_fail(PAT_EINVAL, "null table");
    ctx->last_eik = pat_eikonal_stats{};
    const long nxy = (long)nx * ny, n = nxy * nz;

    std::vector<float> c((size_t)n);
    std::vector<int32_t> vox((size_t)P);
    PAT_HIP(hipMemcpyAsync(c.data(), d_speed, (size_t)n * sizeof(float), hipMemcpyDeviceToHost, st));
    if (P > 0) PAT_HIP(hipMemcpyAsync(vox.data(), d_vox, (size_t)P * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    PAT_HIP(hipStreamSynchronize(st));
    double cmin = INFINITY;
    for (long k = 0; k < n; ++k) {
        const double v = c[(size_t)k];
        if (!(std::isfinite(v) && v > 0.0)) return pat_fail(PAT_EINVAL, "speed at node %ld is %g (need finite > 0)", k, v);
        cmin = std::min(cmin, v);
    }
    for (int p = 0; p < P; ++p)
        if (vox[(size_t)p] < 0 || vox[(size_t)p] >= n)
            return pat_fail(PAT_EINVAL, "voxel %d index %d outside [0, %ld)", p, vox[(size_t)p], n);
    const double x0 = -0.5 * (nx - 1) * h, y0 = -0.5 * (ny - 1) * h, z0 = -0.5 * (nz - 1) * h;
    for (int s = 0; s < S; ++s) {
        const double gi = (h_sensor_xyz[3 * s] - x0) / h, gj = (h_sensor_xyz[3 * s + 1] - y0) / h,
                     gl = (h_sensor_xyz[3 * s + 2] - z0) / h;
        if (!(gi >= 0.0 && gi <= nx - 1 && gj >= 0.0 && gj <= ny - 1 && gl >= 0.0 && gl <= nz - 1))
            return pat_fail(PAT_EINVAL, "sensor %d lies outside the grid", s);
    }
    if (S == 0 || P == 0) return PAT_OK;

    // fixed-point unit: the 6-neighbour Dijkstra bound fits, and F = h/(c lsb) is at most 2^23
    const double tbound = 1.01 * (double)(nx + ny + nz + 3) * h / cmin;
    const double lsb = std::exp2(std::ceil(std::log2(std::max(tbound / 4294967294.0, h / cmin / 8388608.0))));
    ctx->last_eik.lsb_seconds = lsb;
    std::vector<uint32_t> Fh((size_t)n);  // whole units, at most 2^23
    for (long k = 0; k < n; ++k) Fh[(size_t)k] = (uint32_t)std::llround(h / ((double)c[(size_t)k] * lsb));

    EikGrid3 g;
    g.nx = nx; g.ny = ny; g.nz = nz;
    g.bx = (nx + BS - 1) / BS; g.by = (ny + BS - 1) / BS; g.bz = (nz + BS - 1) / BS;
    g.bricks_per_map = g.bx * g.by * g.bz;

    const long budget_maps = std::max<long>(1, (8L << 30) / (n * 4));
    const int chunk = (int)std::min<long>(S, budget_maps);
    const long max_bricks = (long)chunk * g.bricks_per_map;
    if (max_bricks > 0x7FFFFFFFL) return pat_fail(PAT_EINVAL, "too many bricks");

    if ((rc = ctx->eik_tq.grow((size_t)chunk * n * sizeof(uint32_t)))) return rc;
    if ((rc = ctx->eik_f.grow((size_t)n * sizeof(uint32_t)))) return rc;
    if ((rc = ctx->eik_flags.grow((size_t)2 * max_bricks * sizeof(uint32_t)))) return rc;
    if ((rc = ctx->eik_lists.grow((size_t)2 * max_bricks * sizeof(uint32_t)))) return rc;
    if ((rc = ctx->eik_seeds.grow((size_t)chunk * (3 * sizeof(int) + SEED_BOX3 * SEED_BOX3 * SEED_BOX3 * sizeof(uint32_t)))))
        return rc;
    if ((rc = ctx->eik_count.grow(pat_eik::EIK_COUNTERS * sizeof(uint32_t)))) return rc;

    uint32_t *Tq = static_cast<uint32_t *>(ctx->eik_tq.ptr);
    uint32_t *Fd = static_cast<uint32_t *>(ctx->eik_f.ptr);
    uint32_t *flags[2] = { static_cast<uint32_t *>(ctx->eik_flags.ptr),
                           static_cast<uint32_t *>(ctx->eik_flags.ptr) + max_bricks };
    uint32_t *lists[2] = { static_cast<uint32_t *>(ctx->eik_lists.ptr),
                           static_cast<uint32_t *>(ctx->eik_lists.ptr) + max_bricks };
    int *seed_ijl = static_cast<int *>(ctx->eik_seeds.ptr);
    uint32_t *seed_val = reinterpret_cast<uint32_t *>(seed_ijl + 3 * chunk);
    uint32_t *counters = static_cast<uint32_t *>(ctx->eik_count.ptr);  // laid out in eik_round.h
    volatile uint32_t *host_counts = ctx->eik_count_host;
    uint32_t seq = host_counts[4];  // the last round's number, counted on per round
    const double spin_ms = pat_env_eik_spin_ms();

    PAT_HIP(hipMemcpyAsync(Fd, Fh.data(), (size_t)n * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    PAT_HIP(hipMemsetAsync(ctx->eik_flags.ptr, 0, (size_t)2 * max_bricks * sizeof(uint32_t), st));
    // every list entry holds a valid index (0) before its first append
    PAT_HIP(hipMemsetAsync(ctx->eik_lists.ptr, 0, (size_t)2 * max_bricks * sizeof(uint32_t), st));
    PAT_HIP(hipMemsetAsync(counters, 0, pat_eik::EIK_COUNTERS * sizeof(uint32_t), st));

    const long round_cap = pat_env_round_cap(100L * (g.bx + g.by + g.bz) + 1000);
    constexpr int B3 = SEED_BOX3 * SEED_BOX3 * SEED_BOX3;
    std::vector<int> hijl((size_t)3 * chunk);
    std::vector<uint32_t> hval((size_t)chunk * B3);
    std::vector<uint32_t> init_list;
    int64_t rounds = 0, visits = 0;

    for (int s0 = 0; s0 < S; s0 += chunk) {
        const int maps = std::min(chunk, S - s0);
        init_list.clear();
        for (int m = 0; m < maps; ++m) {
            const double sx = h_sensor_xyz[3 * (s0 + m)], sy = h_sensor_xyz[3 * (s0 + m) + 1],
                         sz = h_sensor_xyz[3 * (s0 + m) + 2];
            int is = (int)std::floor((sx - x0) / h + 0.5), js = (int)std::floor((sy - y0) / h + 0.5),
                ls = (int)std::floor((sz - z0) / h + 0.5);
            is = std::min(is, nx - 1);
            js = std::min(js, ny - 1);
            ls = std::min(ls, nz - 1);
            const double cs = (double)c[(size_t)(ls * nxy + (long)js * nx + is)];
            hijl[3 * m] = is - 2;
            hijl[3 * m + 1] = js - 2;
            hijl[3 * m + 2] = ls - 2;
            for (int bl = 0; bl < SEED_BOX3; ++bl)
                for (int bj = 0; bj < SEED_BOX3; ++bj)
                    for (int bi = 0; bi < SEED_BOX3; ++bi) {
                        const int i = is - 2 + bi, j = js - 2 + bj, l = ls - 2 + bl;
                        uint32_t v = TQ_INF;
                        if (i >= 0 && i < nx && j >= 0 && j < ny && l >= 0 && l < nz) {
                            const double dx = (x0 + i * h) - sx, dy = (y0 + j * h) - sy, dz = (z0 + l * h) - sz;
                            const double rr = std::sqrt(dx * dx + dy * dy + dz * dz);
                            if (rr <= 2.0 * h) v = (uint32_t)std::nearbyint(rr / cs / lsb);
                        }
                        hval[(size_t)m * B3 + (bl * SEED_BOX3 + bj) * SEED_BOX3 + bi] = v;
                    }
            // initial bricks: those touching the seed box grown by one node
            const int ia = std::max(0, is - 3) / BS, ib = std::min(nx - 1, is + 3) / BS;
            const int ja = std::max(0, js - 3) / BS, jb = std::min(ny - 1, js + 3) / BS;
            const int la = std::max(0, ls - 3) / BS, lb = std::min(nz - 1, ls + 3) / BS;
            for (int bz = la; bz <= lb; ++bz)
                for (int by = ja; by <= jb; ++by)
                    for (int bx = ia; bx <= ib; ++bx)
                        init_list.push_back((uint32_t)(m * g.bricks_per_map + (bz * g.by + by) * g.bx + bx));
        }
        PAT_HIP(hipMemcpyAsync(seed_ijl, hijl.data(), (size_t)3 * maps * sizeof(int), hipMemcpyHostToDevice, st));
        PAT_HIP(hipMemcpyAsync(seed_val, hval.data(), (size_t)maps * B3 * sizeof(uint32_t), hipMemcpyHostToDevice, st));
        PAT_HIP(hipMemcpyAsync(lists[0], init_list.data(), init_list.size() * sizeof(uint32_t), hipMemcpyHostToDevice, st));
        const long tot = (long)maps * n;
        // every word "not reached" (all ones), then the seed values
        PAT_HIP(hipMemsetAsync(Tq, 0xFF, (size_t)tot * sizeof(uint32_t), st));
        k_eik3_seed<<<dim3((unsigned)maps), 128, 0, st>>>(Tq, g, seed_ijl, seed_val);
        PAT_HIP(hipGetLastError());

        uint32_t cnt = (uint32_t)init_list.size();
        int cur = 0;
        long chunk_rounds = 0;
        while (cnt > 0) {
            if (++chunk_rounds > round_cap)
                return pat_fail(PAT_ENOCONV, "eikonal relaxation did not settle within %ld rounds", round_cap);
            // after the tile kernel, a one-thread kernel writes the next
            // count to the pinned words and clears the device count; the
            // host polls the words' sequence number (eik_round.h)
            k_eik3_brick<<<dim3(cnt), E3_THREADS, 0, st>>>(Tq, Fd, g, seed_ijl, seed_val, lists[cur], flags[cur],
                                                           lists[cur ^ 1], flags[cur ^ 1], counters);
            PAT_HIP(hipGetLastError());
            pat_eik::k_eik_round_end<<<dim3(1), 64, 0, st>>>(counters, ctx->eik_count_host, ++seq);
            PAT_HIP(hipGetLastError());
            PAT_HIP(pat_eik::wait_round(host_counts, seq, st, spin_ms));
            visits += cnt;
            cnt = host_counts[0];
            if (cnt > (uint32_t)max_bricks)
                return pat_fail(PAT_EDEVICE, "eikonal round reported %u active bricks, above the %ld the list holds",
                                cnt, (long)max_bricks);
            cur ^= 1;
        }
        rounds += chunk_rounds;
        for (int m0 = 0; m0 < maps; m0 += 65535 * EX_MAPS) {
            const int groups = (std::min(65535 * EX_MAPS, maps - m0) + EX_MAPS - 1) / EX_MAPS;
            const dim3 grid((unsigned)((P + 255) / 256), (unsigned)groups);
            k_eik3_extract<<<grid, 256, 0, st>>>(Tq, n, d_vox, P, m0, maps, lsb, d_table + (long)s0 * P);
            PAT_HIP(hipGetLastError());
        }
    }
    PAT_HIP(hipStreamSynchronize(st));
    ctx->last_eik.rounds = rounds;
    ctx->last_eik.tile_visits = visits;
    ctx->last_eik.guard_hits = host_counts[1];
    ctx->last_eik.sweeps = (int64_t)host_counts[2] | ((int64_t)host_counts[3] << 32);
    ctx->last_eik.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    return PAT_OK;
}
