// Per-sensor travel-time tables (Section II-B): the first-order upwind
// (Godunov) discretisation of |grad T| = 1/c from each sensor as a point
// source, solved by tile-parallel relaxation to the same discrete fixed point
// that fast marching reaches.
//
// Layout and scheme:
//  * Working times are uint32 fixed point, T = Tq * lsb with lsb a power of two
//    chosen so that the Dijkstra upper bound (nx + ny + 2) h max(1/c) fits below
//    2^32 - 1; 0xFFFFFFFF is "not reached".  Integer adds and mins are exact,
//    so rounding cannot drift systematically along long straight rays, and the
//    minimum is order independent.
//  * Each map is cut into 32x32 tiles.  A workgroup loads one tile plus a
//    one-node halo into LDS and relaxes it in place until no node changes
//    (workgroup OR-reduction), then writes the changed nodes back and
//    activates the neighbour tiles whose shared edge changed.  Rounds repeat
//    until no tile is active.  Values only decrease, and a sweep that changes
//    nothing leaves every node at its update.  Large rounds relax each tile
//    with one wave sweeping anti-diagonals (k_eik_tile_diag), small ones with
//    256 threads sweeping 4-node strips (k_eik_tile).
//  * The update is exact in integers (eik_update.h): with the node's
//    F = round(h / (c lsb)) whole units it is the first-order root
//    T = min(a, b) + F when |a - b| >= F, else
//    min(a, b) + (|a - b| + sqrt(2 F^2 - (a - b)^2)) / 2, rounded to the
//    nearest unit.  It is monotone in both neighbours, so the relaxation ends
//    at the same fixed point whatever the workgroup schedule, and the tables
//    are the same bit for bit from run to run.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "eik_update.h"
#include "eik_round.h"
#include "pat_internal.h"

namespace {

constexpr int TS = 32;                  // tile edge (nodes)
constexpr int HS = TS + 2;              // tile edge with halo
constexpr int EK_THREADS = 256;         // 32 columns x 8 strips of 4 rows
// Rounds with at least this many active tiles (one per SIMD) take the
// one-wave anti-diagonal kernel; smaller rounds, which it cannot fill the GPU
// with, take the strip kernel (4 waves per tile).  Both reach the same fixed
// point.  Thresholds of 0 and 4096 tiles were 1-3 % slower.
constexpr uint32_t EIK_DIAG_MIN_TILES = 1024;
constexpr int ROWS_PER_THREAD = TS * TS / EK_THREADS;
constexpr uint32_t TQ_INF = 0xFFFFFFFFu;
constexpr int EX_MAPS = 4;                 // maps per thread in the table extraction
constexpr int SEED_BOX = 5;             // frozen nodes lie in a 5x5 box around the nearest node
constexpr int LOCAL_ITER_CAP = 6 * TS;  // a tile that has not settled re-queues itself

struct EikGrid {
    int nx, ny, tiles_x, tiles_y, tiles_per_map;
};

__device__ __forceinline__ bool is_frozen(int gx, int gy, const int *seed_ij, const uint32_t *seed_val, int m,
                                          uint32_t &val) {
    const int bx = gx - seed_ij[2 * m], by = gy - seed_ij[2 * m + 1];
    if ((unsigned)bx >= (unsigned)SEED_BOX || (unsigned)by >= (unsigned)SEED_BOX) return false;
    val = seed_val[m * SEED_BOX * SEED_BOX + by * SEED_BOX + bx];
    return val != TQ_INF;
}

// The seed values of the frozen nodes, over maps whose every word the host
// has set to "not reached": one workgroup per map, a thread per node of its
// seed box (a node is frozen where the box holds a value).
__global__ void __launch_bounds__(64) k_eik_seed(uint32_t *__restrict__ Tq, EikGrid g, const int *__restrict__ seed_ij,
                                                 const uint32_t *__restrict__ seed_val) {
    const int m = blockIdx.x, t = threadIdx.x;
    if (t >= SEED_BOX * SEED_BOX) return;
    const int gx = seed_ij[2 * m] + t % SEED_BOX, gy = seed_ij[2 * m + 1] + t / SEED_BOX;
    if (gx < 0 || gx >= g.nx || gy < 0 || gy >= g.ny) return;
    const uint32_t v = seed_val[m * SEED_BOX * SEED_BOX + t];
    if (v != TQ_INF) Tq[(long)m * g.nx * g.ny + (long)gy * g.nx + gx] = v;
}

__device__ __forceinline__ void activate(uint32_t tile, uint32_t *flags_next, uint32_t *list_next, uint32_t *cnt_next) {
    if (atomicExch(&flags_next[tile], 1u) == 0u) {
        const uint32_t pos = atomicAdd(cnt_next, 1u);
        list_next[pos] = tile;
    }
}

__global__ void __launch_bounds__(EK_THREADS) k_eik_tile(uint32_t *__restrict__ Tq, const uint32_t *__restrict__ Fmap,
                                                         EikGrid g, const int *__restrict__ seed_ij,
                                                         const uint32_t *__restrict__ seed_val,
                                                         const uint32_t *__restrict__ list_cur,
                                                         uint32_t *__restrict__ flags_cur,
                                                         uint32_t *__restrict__ list_next,
                                                         uint32_t *__restrict__ flags_next,
                                                         uint32_t *__restrict__ counters) {
    __shared__ uint32_t T[HS * HS];
    __shared__ uint32_t side_bits;

    const int tid = threadIdx.x;
    const uint32_t tile = list_cur[blockIdx.x];
    const int m = (int)(tile / g.tiles_per_map);
    const int r = (int)(tile % g.tiles_per_map);
    const int ty = r / g.tiles_x, tx = r % g.tiles_x;
    const int gx0 = tx * TS, gy0 = ty * TS;
    uint32_t *map = Tq + (long)m * g.nx * g.ny;
    if (tid == 0) {
        flags_cur[tile] = 0u;
        side_bits = 0u;
    }

    // halo: 4 edges of TS nodes each (corners are never read by the 4-point stencil)
    for (int idx = tid; idx < 4 * TS; idx += EK_THREADS) {
        const int side = idx / TS, o = idx % TS;
        int gx, gy, l;
        if (side == 0) { gx = gx0 + o; gy = gy0 - 1; l = o + 1; }
        else if (side == 1) { gx = gx0 + o; gy = gy0 + TS; l = (TS + 1) * HS + o + 1; }
        else if (side == 2) { gx = gx0 - 1; gy = gy0 + o; l = (o + 1) * HS; }
        else { gx = gx0 + TS; gy = gy0 + o; l = (o + 1) * HS + TS + 1; }
        const bool in = gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny;
        T[l] = in ? map[(long)gy * g.nx + gx] : TQ_INF;
    }

    // This thread's nodes in the two sweep layouts: column lx, rows
    // 4*strip .. 4*strip+3 (layout C), and row lx, columns 4*strip ..
    // 4*strip+3 (layout R).  Sweeps alternate C down, R right, C up, R left:
    // information crosses a thread's four nodes within one sweep, along y in
    // layout C and along x in layout R, instead of along y only.
    __shared__ uint32_t Fl[TS * TS];
    const int lx = tid % TS;
    const int strip = tid / TS;
    const int gx = gx0 + lx;
    uint32_t own0[ROWS_PER_THREAD];  // layout C values at the start of the visit
    unsigned live_c = 0, live_r = 0;  // bit q: node q is inside the grid and not frozen
    for (int q = 0; q < ROWS_PER_THREAD; ++q) {
        const int ly = strip * ROWS_PER_THREAD + q;
        const int gy = gy0 + ly;
        const bool in = gx < g.nx && gy < g.ny;
        uint32_t v = TQ_INF;
        uint32_t f = 0u;
        if (in) {
            v = map[(long)gy * g.nx + gx];
            f = Fmap[(long)gy * g.nx + gx];
            uint32_t sv;
            if (!is_frozen(gx, gy, seed_ij, seed_val, m, sv)) live_c |= 1u << q;
        }
        own0[q] = v;
        T[(ly + 1) * HS + lx + 1] = v;
        Fl[ly * TS + lx] = f;
        // layout R: node (4*strip + q, lx)
        const int rx = gx0 + strip * ROWS_PER_THREAD + q, ry = gy0 + lx;
        uint32_t sv;
        if (rx < g.nx && ry < g.ny && !is_frozen(rx, ry, seed_ij, seed_val, m, sv)) live_r |= 1u << q;
    }
    __syncthreads();
    uint32_t Fc[ROWS_PER_THREAD], Fr[ROWS_PER_THREAD];
    float F2c[ROWS_PER_THREAD], F2r[ROWS_PER_THREAD];  // 2 F^2 as floats
    for (int q = 0; q < ROWS_PER_THREAD; ++q) {
        Fc[q] = Fl[(strip * ROWS_PER_THREAD + q) * TS + lx];
        Fr[q] = Fl[lx * TS + strip * ROWS_PER_THREAD + q];
        F2c[q] = pat_eik::eik_f2(Fc[q]);
        F2r[q] = pat_eik::eik_f2(Fr[q]);
    }

    // one node of a sweep (layout and q static, so the per-node registers
    // stay registers and nothing selects between the layouts per node)
    auto relax = [&](auto rows_c, int q, int &any) {
        constexpr bool ROWS = decltype(rows_c)::value;
        if (!((ROWS ? live_r : live_c) & (1u << q))) return;
        const int n = strip * ROWS_PER_THREAD + q;
        const int c = ROWS ? (lx + 1) * HS + n + 1 : (n + 1) * HS + lx + 1;
        const uint32_t a = min(T[c - 1], T[c + 1]);
        const uint32_t b = min(T[c - HS], T[c + HS]);
        const uint32_t nv = pat_eik::godunov2_int(a, b, ROWS ? Fr[q] : Fc[q], ROWS ? F2r[q] : F2c[q]);
        if (nv < T[c]) {
            T[c] = nv;
            any = 1;
        }
    };
    // one sweep; false when it changed no node of the tile
    auto sweep = [&](auto rows_c, auto rev_c) -> bool {
        int any = 0;
#pragma unroll
        for (int k = 0; k < ROWS_PER_THREAD; ++k) relax(rows_c, decltype(rev_c)::value ? ROWS_PER_THREAD - 1 - k : k, any);
        return __syncthreads_or(any) != 0;
    };
    // sweeps cycle through C down, R right, C up, R left; it ends as the
    // index of the sweep that changed nothing, or the cap
    static_assert(LOCAL_ITER_CAP % 4 == 0, "whole sweep cycles");
    using F_ = std::false_type;
    using T_ = std::true_type;
    int it = 0;
    for (; it < LOCAL_ITER_CAP; it += 4) {
        if (!sweep(F_{}, F_{})) break;
        if (!sweep(T_{}, F_{})) { it += 1; break; }
        if (!sweep(F_{}, T_{})) { it += 2; break; }
        if (!sweep(T_{}, T_{})) { it += 3; break; }
    }

    unsigned sides = 0;
    for (int q = 0; q < ROWS_PER_THREAD; ++q) {
        const int ly = strip * ROWS_PER_THREAD + q;
        const uint32_t v = T[(ly + 1) * HS + lx + 1];
        if (v == own0[q]) continue;  // values only decrease: unchanged
        map[(long)(gy0 + ly) * g.nx + gx] = v;
        if (ly == 0) sides |= 1u;
        if (ly == TS - 1) sides |= 2u;
        if (lx == 0) sides |= 4u;
        if (lx == TS - 1) sides |= 8u;
    }
    if (it == LOCAL_ITER_CAP) sides |= 16u;
    if (sides) atomicOr(&side_bits, sides);
    __syncthreads();
    if (tid == 0) {
        atomicAdd(reinterpret_cast<unsigned long long *>(counters + 2), (unsigned long long)min(it + 1, LOCAL_ITER_CAP));
        const unsigned sb = side_bits;
        uint32_t *cnt_next = counters;
        const uint32_t base = (uint32_t)m * g.tiles_per_map;
        if ((sb & 1u) && ty > 0) activate(base + (ty - 1) * g.tiles_x + tx, flags_next, list_next, cnt_next);
        if ((sb & 2u) && ty + 1 < g.tiles_y) activate(base + (ty + 1) * g.tiles_x + tx, flags_next, list_next, cnt_next);
        if ((sb & 4u) && tx > 0) activate(base + ty * g.tiles_x + tx - 1, flags_next, list_next, cnt_next);
        if ((sb & 8u) && tx + 1 < g.tiles_x) activate(base + ty * g.tiles_x + tx + 1, flags_next, list_next, cnt_next);
        if (sb & 16u) activate(tile, flags_next, list_next, cnt_next);
    }
}

// One wave per tile, sweeping anti-diagonals: in each pass the two half-waves
// walk the tile's 63 diagonals in opposite directions (down-right and
// up-left, then down-left and up-right), lane i of a half taking column i
// of its diagonal (the diagonals folded into 32 steps per pass, below), so
// that a front moving with a sweep crosses the tile in at most two passes.  Both halves update the tile at once; the update
// is monotone, so the order in which their writes land changes the work,
// not the result.  Passes repeat until one changes no node.
constexpr int DG_PAIRS = 48;                 // a tile that has not settled re-queues itself
constexpr uint32_t F_DEAD24 = 0xFFFFFFu;     // frozen or outside the grid: never updated (F <= 2^23)

__global__ void __launch_bounds__(64) k_eik_tile_diag(uint32_t *__restrict__ Tq, const uint32_t *__restrict__ Fmap,
                                                      EikGrid g, const int *__restrict__ seed_ij,
                                                      const uint32_t *__restrict__ seed_val,
                                                      const uint32_t *__restrict__ list_cur,
                                                      uint32_t *__restrict__ flags_cur,
                                                      uint32_t *__restrict__ list_next,
                                                      uint32_t *__restrict__ flags_next,
                                                      uint32_t *__restrict__ counters) {
    // F of each node in 24 bits (F <= 2^23), split into a 16-bit and an 8-bit
    // array, F_DEAD24 where not updated: with the tile, 7.7 KB of LDS per
    // wave, so that LDS holds 20 waves per CU
    __shared__ uint32_t T[HS * HS];
    __shared__ uint16_t Flo[TS * TS];
    __shared__ uint8_t Fhi[TS * TS];
    __shared__ uint32_t side_bits;

    const int lane = threadIdx.x;
    const uint32_t tile = list_cur[blockIdx.x];
    const int m = (int)(tile / g.tiles_per_map);
    const int r = (int)(tile % g.tiles_per_map);
    const int ty = r / g.tiles_x, tx = r % g.tiles_x;
    const int gx0 = tx * TS, gy0 = ty * TS;
    uint32_t *map = Tq + (long)m * g.nx * g.ny;
    if (lane == 0) {
        flags_cur[tile] = 0u;
        side_bits = 0u;
    }
    // every global load of the visit is issued before the first is waited
    // for: the halo (two per lane), then the tile's times and slowness (two
    // rows of 32 per load instruction)
    constexpr int HALO_PER_LANE = 4 * TS / 64, NODES_PER_LANE = TS * TS / 64;
    uint32_t hv[HALO_PER_LANE], v[NODES_PER_LANE], f[NODES_PER_LANE];
    int hl[HALO_PER_LANE];
#pragma unroll
    for (int j = 0; j < HALO_PER_LANE; ++j) {
        const int idx = j * 64 + lane, side = idx / TS, o = idx % TS;
        int gx, gy;
        if (side == 0) { gx = gx0 + o; gy = gy0 - 1; hl[j] = o + 1; }
        else if (side == 1) { gx = gx0 + o; gy = gy0 + TS; hl[j] = (TS + 1) * HS + o + 1; }
        else if (side == 2) { gx = gx0 - 1; gy = gy0 + o; hl[j] = (o + 1) * HS; }
        else { gx = gx0 + TS; gy = gy0 + o; hl[j] = (o + 1) * HS + TS + 1; }
        const bool in = gx >= 0 && gx < g.nx && gy >= 0 && gy < g.ny;
        hv[j] = in ? map[(long)gy * g.nx + gx] : TQ_INF;
    }
#pragma unroll
    for (int j = 0; j < NODES_PER_LANE; ++j) {
        const int node = j * 64 + lane, gx = gx0 + node % TS, gy = gy0 + node / TS;
        const bool in = gx < g.nx && gy < g.ny;
        const long k = in ? (long)gy * g.nx + gx : 0;
        v[j] = in ? map[k] : TQ_INF;
        f[j] = in ? Fmap[k] : F_DEAD24;
    }
#pragma unroll
    for (int j = 0; j < HALO_PER_LANE; ++j) T[hl[j]] = hv[j];
    // frozen nodes (the seed box of this sensor) are never updated
    const int sbx = seed_ij[2 * m], sby = seed_ij[2 * m + 1];
#pragma unroll
    for (int j = 0; j < NODES_PER_LANE; ++j) {
        const int node = j * 64 + lane, x = node % TS, y = node / TS;
        const int bx = gx0 + x - sbx, by = gy0 + y - sby;
        uint32_t fj = f[j];
        if ((unsigned)bx < (unsigned)SEED_BOX && (unsigned)by < (unsigned)SEED_BOX &&
            seed_val[m * SEED_BOX * SEED_BOX + by * SEED_BOX + bx] != TQ_INF)
            fj = F_DEAD24;
        T[(y + 1) * HS + x + 1] = v[j];
        Flo[node] = (uint16_t)(fj & 0xFFFFu);
        Fhi[node] = (uint8_t)(fj >> 16);
    }
    __syncthreads();

    const int half = lane >> 5, i = lane & (TS - 1);
    // in the half's sweep frame lane i takes column x' = i; the frame flips x
    // for half 1, and y for half 1 in the first pass and half 0 in the second
    const int xs = half ? TS - 1 - i : i;
    uint32_t mine = 0;  // bit y: this lane lowered node (xs, y)
    // a pass that changes no node ends the visit: every node was evaluated in
    // it against neighbours that held their final values
    int passes = 0;
    bool settled = false;
    for (int pair = 0; pair < DG_PAIRS && !settled; ++pair) {
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
            int any = 0;
            const bool flip_y = (pass == 0) == (half == 1);
            // folded diagonals: in step k lane i takes row y' = k - i of
            // diagonal k while i <= k, else row k + 32 - i of diagonal k + 32,
            // so every lane works in every step; each diagonal follows the one
            // before it within the pass, except diagonal 32, which reads
            // diagonal 31 from the pass before
            const int ymask = flip_y ? TS - 1 : 0;
            for (int k = 0; k < TS; ++k) {
                // (k - i) mod 32, mirrored by ymask (31 - y == y ^ 31)
                const int y = ((k - i) & (TS - 1)) ^ ymask;
                const int c = (y + 1) * HS + xs + 1;
                // every read of the step issued at once, the dead test at the
                // write; a dead node is evaluated with F = 0, which keeps the
                // square root in range and is never written
                const uint32_t f = (uint32_t)Flo[y * TS + xs] | ((uint32_t)Fhi[y * TS + xs] << 16);
                const uint32_t a = min(T[c - 1], T[c + 1]);
                const uint32_t b = min(T[c - HS], T[c + HS]);
                const uint32_t cur = T[c];
                const bool live = f != F_DEAD24;
                const uint32_t fl = live ? f : 0u;
                const uint32_t nv = pat_eik::godunov2_int(a, b, fl, pat_eik::eik_f2(fl));
                if (live && nv < cur) {
                    T[c] = nv;
                    mine |= 1u << y;
                    any = 1;
                }
                // the wave's LDS accesses execute in order, so the next
                // diagonal reads this one's writes
                __builtin_amdgcn_wave_barrier();
            }
            ++passes;
            if (!__syncthreads_or(any)) {
                settled = true;
                break;
            }
        }
    }

    // column c was swept by lane c (half 0) and lane 63 - c (half 1); lane L
    // writes back rows 16 (L / 32) .. +15 of column L % 32
    const int col = lane & (TS - 1);
    const uint32_t cm = (uint32_t)__shfl((int)mine, col) | (uint32_t)__shfl((int)mine, 63 - col);
    unsigned sides = 0;
    for (int q = 0; q < TS / 2; ++q) {
        const int y = (lane >> 5) * (TS / 2) + q;
        if (!((cm >> y) & 1u)) continue;
        map[(long)(gy0 + y) * g.nx + gx0 + col] = T[(y + 1) * HS + col + 1];
        if (y == 0) sides |= 1u;
        if (y == TS - 1) sides |= 2u;
        if (col == 0) sides |= 4u;
        if (col == TS - 1) sides |= 8u;
    }
    if (!settled) sides |= 16u;
    if (sides) atomicOr(&side_bits, sides);
    __syncthreads();
    if (lane == 0) {
        // two directional sweeps per pass
        atomicAdd(reinterpret_cast<unsigned long long *>(counters + 2), (unsigned long long)(2 * passes));
        const unsigned sb = side_bits;
        uint32_t *cnt_next = counters;
        const uint32_t base = (uint32_t)m * g.tiles_per_map;
        if ((sb & 1u) && ty > 0) activate(base + (ty - 1) * g.tiles_x + tx, flags_next, list_next, cnt_next);
        if ((sb & 2u) && ty + 1 < g.tiles_y) activate(base + (ty + 1) * g.tiles_x + tx, flags_next, list_next, cnt_next);
        if ((sb & 4u) && tx > 0) activate(base + ty * g.tiles_x + tx - 1, flags_next, list_next, cnt_next);
        if ((sb & 8u) && tx + 1 < g.tiles_x) activate(base + ty * g.tiles_x + tx + 1, flags_next, list_next, cnt_next);
        if (sb & 16u) activate(tile, flags_next, list_next, cnt_next);
    }
}

// table[s0 + m][p] = Tq[m][pix[p]] * lsb, rounded once to float32 seconds.
// A thread takes one pixel of EX_MAPS maps (its index read once, the maps'
// loads in flight together); blockIdx.y is the group of EX_MAPS maps within a
// launch that starts at map m0 of the chunk's maps.
__global__ void __launch_bounds__(256) k_eik_extract(const uint32_t *__restrict__ Tq, long n_nodes,
                                                     const int32_t *__restrict__ pix, int P, int m0, int maps, double lsb,
                                                     float *__restrict__ table) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    const int mb = m0 + (int)blockIdx.y * EX_MAPS;
    const long k = pix[p];
    uint32_t v[EX_MAPS];
#pragma unroll
    for (int j = 0; j < EX_MAPS; ++j)
        if (mb + j < maps) v[j] = Tq[(long)(mb + j) * n_nodes + k];
#pragma unroll
    for (int j = 0; j < EX_MAPS; ++j)
        if (mb + j < maps) table[(long)(mb + j) * P + p] = v[j] == TQ_INF ? INFINITY : (float)((double)v[j] * lsb);
}

// The local update alone, for checking it against its definition: out[i] =
// the 2-D or 3-D update of neighbour minima nbr[i][0..dims) with slowness
// F[i] units (F above 2^23 gives 0).
__global__ void __launch_bounds__(256) k_eik_update_eval(const uint32_t *__restrict__ nbr,
                                                         const uint32_t *__restrict__ F, int n, int dims,
                                                         uint32_t *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t f = F[i];
    if (f > (1u << 23)) {
        out[i] = 0u;
        return;
    }
    const uint32_t a = nbr[3 * i], b = nbr[3 * i + 1], c = nbr[3 * i + 2];
    out[i] = dims == 2 ? pat_eik::godunov2_int(a, b, f, pat_eik::eik_f2(f))
                       : pat_eik::godunov3_int(a, b, c, f, pat_eik::eik_f2(f), pat_eik::eik_f3(f));
}

}  // namespace

extern "C" int pat_eikonal_update_eval(const uint32_t *d_nbr, const uint32_t *d_F, int n, int dims,
                                       uint32_t *d_out, void *stream) {
    if (n < 0) return pat_fail(PAT_EINVAL, "negative count");
    if (dims != 2 && dims != 3) return pat_fail(PAT_EINVAL, "dims must be 2 or 3 (got %d)", dims);
    if (n == 0) return PAT_OK;
    if (!d_nbr || !d_F || !d_out) return pat_fail(PAT_EINVAL, "null buffer");
    k_eik_update_eval<<<dim3((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(d_nbr, d_F, n, dims, d_out);
    PAT_HIP(hipGetLastError());
    return PAT_OK;
}

extern "C" int pat_eikonal_tables(pat_ctx *ctx, const float *d_speed, int nx, int ny, double h,
                                  const double *h_sensor_xy, int S, const int32_t *d_pix, int P, float *d_table,
                                  void *stream) {
    const auto t_start = std::chrono::steady_clock::now();
    int rc = pat_make_current(ctx);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (nx < 2 || ny < 2) return pat_fail(PAT_EINVAL, "grid must be at least 2x2 (got %dx%d)", nx, ny);
    if ((long long)nx * ny > (1LL << 30)) return pat_fail(PAT_EINVAL, "grid too large");
    if (!(std::isfinite(h) && h > 0.0)) return pat_fail(PAT_EINVAL, "node spacing must be finite and > 0");
    if (S < 0 || P < 0) return pat_fail(PAT_EINVAL, "negative sensor or pixel count");
    if (!d_speed) return pat_fail(PAT_EINVAL, "null speed map");
    if (S > 0 && !h_sensor_xy) return pat_fail(PAT_EINVAL, "null sensor positions");
    if (P > 0 && !d_pix) return pat_fail(PAT_EINVAL, "null pixel list");
    if ((long long)S * P > 0 && !d_table) return pat_fail(PAT_EINVAL, "null table");
    ctx->last_eik = pat_eikonal_stats{};
    const long n = (long)nx * ny;

    // speed map and pixel list to the host for validation and seeding
    std::vector<float> c((size_t)n);
    std::vector<int32_t> pix((size_t)P);
    PAT_HIP(hipMemcpyAsync(c.data(), d_speed, (size_t)n * sizeof(float), hipMemcpyDeviceToHost, st));
    if (P > 0) PAT_HIP(hipMemcpyAsync(pix.data(), d_pix, (size_t)P * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    PAT_HIP(hipStreamSynchronize(st));
    double cmin = INFINITY;
    for (long k = 0; k < n; ++k) {
        const double v = c[(size_t)k];
        if (!(std::isfinite(v) && v > 0.0)) return pat_fail(PAT_EINVAL, "speed at node %ld is %g (need finite > 0)", k, v);
        cmin = std::min(cmin, v);
    }
    for (int p = 0; p < P; ++p)
        if (pix[(size_t)p] < 0 || pix[(size_t)p] >= n)
            return pat_fail(PAT_EINVAL, "pixel %d index %d outside [0, %ld)", p, pix[(size_t)p], n);
    const double x0 = -0.5 * (nx - 1) * h, y0 = -0.5 * (ny - 1) * h;
    for (int s = 0; s < S; ++s) {
        const double gi = (h_sensor_xy[2 * s] - x0) / h, gj = (h_sensor_xy[2 * s + 1] - y0) / h;
        if (!(gi >= 0.0 && gi <= nx - 1 && gj >= 0.0 && gj <= ny - 1))
            return pat_fail(PAT_EINVAL, "sensor %d at (%g, %g) m lies outside the grid", s, h_sensor_xy[2 * s],
                            h_sensor_xy[2 * s + 1]);
    }
    if (S == 0 || P == 0) return PAT_OK;

    // fixed-point unit: the Dijkstra bound fits, and F = h/(c lsb) is at most 2^23
    const double tbound = 1.01 * (double)(nx + ny + 2) * h / cmin;
    const double lsb_range = tbound / 4294967294.0;
    const double lsb_prec = h / cmin / 8388608.0;
    const double lsb = std::exp2(std::ceil(std::log2(std::max(lsb_range, lsb_prec))));
    ctx->last_eik.lsb_seconds = lsb;

    // F in whole units (at most 2^23), the update's integer slowness
    std::vector<uint32_t> Fh((size_t)n);
    for (long k = 0; k < n; ++k) Fh[(size_t)k] = (uint32_t)std::llround(h / ((double)c[(size_t)k] * lsb));

    EikGrid g;
    g.nx = nx;
    g.ny = ny;
    g.tiles_x = (nx + TS - 1) / TS;
    g.tiles_y = (ny + TS - 1) / TS;
    g.tiles_per_map = g.tiles_x * g.tiles_y;

    // sensors per chunk: working maps limited to 8 GiB
    const long budget_maps = std::max<long>(1, (8L << 30) / (n * 4));
    const int chunk = (int)std::min<long>(S, budget_maps);
    const long max_tiles = (long)chunk * g.tiles_per_map;
    if (max_tiles > 0x7FFFFFFFL) return pat_fail(PAT_EINVAL, "too many tiles");

    if ((rc = ctx->eik_tq.grow((size_t)chunk * n * sizeof(uint32_t)))) return rc;
    if ((rc = ctx->eik_f.grow((size_t)n * sizeof(uint32_t)))) return rc;
    if ((rc = ctx->eik_flags.grow((size_t)2 * max_tiles * sizeof(uint32_t)))) return rc;
    if ((rc = ctx->eik_lists.grow((size_t)2 * max_tiles * sizeof(uint32_t)))) return rc;
    if ((rc = ctx->eik_seeds.grow((size_t)chunk * (2 * sizeof(int) + SEED_BOX * SEED_BOX * sizeof(uint32_t))))) return rc;
    if ((rc = ctx->eik_count.grow(pat_eik::EIK_COUNTERS * sizeof(uint32_t)))) return rc;

    uint32_t *Tq = static_cast<uint32_t *>(ctx->eik_tq.ptr);
    uint32_t *Fd = static_cast<uint32_t *>(ctx->eik_f.ptr);
    uint32_t *flags[2] = { static_cast<uint32_t *>(ctx->eik_flags.ptr),
                           static_cast<uint32_t *>(ctx->eik_flags.ptr) + max_tiles };
    uint32_t *lists[2] = { static_cast<uint32_t *>(ctx->eik_lists.ptr),
                           static_cast<uint32_t *>(ctx->eik_lists.ptr) + max_tiles };
    int *seed_ij = static_cast<int *>(ctx->eik_seeds.ptr);
    uint32_t *seed_val = reinterpret_cast<uint32_t *>(seed_ij + 2 * chunk);
    uint32_t *counters = static_cast<uint32_t *>(ctx->eik_count.ptr);  // laid out in eik_round.h
    volatile uint32_t *host_counts = ctx->eik_count_host;
    uint32_t seq = host_counts[4];  // the last round's number, counted on per round
    const double spin_ms = pat_env_eik_spin_ms();

    PAT_HIP(hipMemcpyAsync(Fd, Fh.data(), (size_t)n * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    PAT_HIP(hipMemsetAsync(ctx->eik_flags.ptr, 0, (size_t)2 * max_tiles * sizeof(uint32_t), st));
    // every list entry holds a valid index (0) before its first append
    PAT_HIP(hipMemsetAsync(ctx->eik_lists.ptr, 0, (size_t)2 * max_tiles * sizeof(uint32_t), st));
    PAT_HIP(hipMemsetAsync(counters, 0, pat_eik::EIK_COUNTERS * sizeof(uint32_t), st));

    const long round_cap = pat_env_round_cap(100L * (g.tiles_x + g.tiles_y) + 1000);
    std::vector<int> hij((size_t)2 * chunk);
    std::vector<uint32_t> hval((size_t)chunk * SEED_BOX * SEED_BOX);
    std::vector<uint32_t> init_list;
    int64_t rounds = 0, visits = 0;

    for (int s0 = 0; s0 < S; s0 += chunk) {
        const int maps = std::min(chunk, S - s0);
        init_list.clear();
        for (int m = 0; m < maps; ++m) {
            const double sx = h_sensor_xy[2 * (s0 + m)], sy = h_sensor_xy[2 * (s0 + m) + 1];
            int is = (int)std::floor((sx - x0) / h + 0.5), js = (int)std::floor((sy - y0) / h + 0.5);
            is = std::min(is, nx - 1);
            js = std::min(js, ny - 1);
            const double cs = (double)c[(size_t)js * nx + is];
            hij[2 * m] = is - 2;
            hij[2 * m + 1] = js - 2;
            for (int b = 0; b < SEED_BOX; ++b)
                for (int a = 0; a < SEED_BOX; ++a) {
                    const int i = is - 2 + a, j = js - 2 + b;
                    uint32_t v = TQ_INF;
                    if (i >= 0 && i < nx && j >= 0 && j < ny) {
                        const double dx = (x0 + i * h) - sx, dy = (y0 + j * h) - sy;
                        const double rr = std::sqrt(dx * dx + dy * dy);
                        if (rr <= 2.0 * h) v = (uint32_t)std::nearbyint(rr / cs / lsb);
                    }
                    hval[(size_t)m * SEED_BOX * SEED_BOX + b * SEED_BOX + a] = v;
                }
            // initial tiles: those touching the seed box grown by one node
            const int ta = std::max(0, is - 3) / TS, tb = std::min(nx - 1, is + 3) / TS;
            const int tc = std::max(0, js - 3) / TS, td = std::min(ny - 1, js + 3) / TS;
            for (int ty = tc; ty <= td; ++ty)
                for (int tx = ta; tx <= tb; ++tx) init_list.push_back((uint32_t)(m * g.tiles_per_map + ty * g.tiles_x + tx));
        }
        PAT_HIP(hipMemcpyAsync(seed_ij, hij.data(), (size_t)2 * maps * sizeof(int), hipMemcpyHostToDevice, st));
        PAT_HIP(hipMemcpyAsync(seed_val, hval.data(), (size_t)maps * SEED_BOX * SEED_BOX * sizeof(uint32_t),
                               hipMemcpyHostToDevice, st));
        PAT_HIP(hipMemcpyAsync(lists[0], init_list.data(), init_list.size() * sizeof(uint32_t), hipMemcpyHostToDevice, st));
        // every word "not reached" (all ones), then the seed values
        PAT_HIP(hipMemsetAsync(Tq, 0xFF, (size_t)maps * n * sizeof(uint32_t), st));
        k_eik_seed<<<dim3((unsigned)maps), 64, 0, st>>>(Tq, g, seed_ij, seed_val);
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
            if (cnt >= EIK_DIAG_MIN_TILES)
                k_eik_tile_diag<<<dim3(cnt), 64, 0, st>>>(Tq, Fd, g, seed_ij, seed_val, lists[cur], flags[cur],
                                                          lists[cur ^ 1], flags[cur ^ 1], counters);
            else
                k_eik_tile<<<dim3(cnt), EK_THREADS, 0, st>>>(Tq, Fd, g, seed_ij, seed_val, lists[cur], flags[cur],
                                                             lists[cur ^ 1], flags[cur ^ 1], counters);
            PAT_HIP(hipGetLastError());
            pat_eik::k_eik_round_end<<<dim3(1), 64, 0, st>>>(counters, ctx->eik_count_host, ++seq);
            PAT_HIP(hipGetLastError());
            PAT_HIP(pat_eik::wait_round(host_counts, seq, st, spin_ms));
            visits += cnt;
            cnt = host_counts[0];
            if (cnt > (uint32_t)max_tiles)
                return pat_fail(PAT_EDEVICE, "eikonal round reported %u active tiles, above the %ld the list holds", cnt,
                                (long)max_tiles);
            cur ^= 1;
        }
        rounds += chunk_rounds;
        for (int m0 = 0; m0 < maps; m0 += 65535 * EX_MAPS) {
            const int groups = (std::min(65535 * EX_MAPS, maps - m0) + EX_MAPS - 1) / EX_MAPS;
            const dim3 grid((unsigned)((P + 255) / 256), (unsigned)groups);
            k_eik_extract<<<grid, 256, 0, st>>>(Tq, n, d_pix, P, m0, maps, lsb, d_table + (long)s0 * P);
            PAT_HIP(hipGetLastError());
        }
    }
    PAT_HIP(hipStreamSynchronize(st));
    ctx->last_eik.rounds = rounds;
    ctx->last_eik.tile_visits = visits;
    ctx->last_eik.guard_hits = host_counts[1];
    ctx->last_eik.sweeps = (int64_t)host_counts[2] | ((int64_t)host_counts[3] << 32);
    ctx->last_eik.seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    return PAT_OK;
}
