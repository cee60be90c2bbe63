/*
 * Plain FP64 CPU oracle for fast-marching-based back projection
 * (Wang & Jing, "A fast marching method based back projection algorithm for
 * photoacoustic tomography in heterogeneous media").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It shares
 * no code, header, table or helper with the GPU library.
 *
 * What it computes, in the paper's order:
 *   1. orc_seed + orc_fmm: the first-arrival time T solving |grad T| = 1/c
 *      (Section II-B, the eikonal equation) from a point source, by the fast
 *      marching method: repeatedly accept the trial node with the smallest
 *      arrival time and update its neighbours (Section II-B).  The local
 *      update is the first-order upwind (Godunov) discretisation; the paper's
 *      second-order one-sided difference is not used here.
 *   2. orc_tables: one such map per sensor, the sensor acting as the point
 *      source by reciprocity (Section II-B, last paragraph), sampled at the
 *      region-of-interest pixels -> the delay table t_{i,j}.
 *   3. orc_filter: b_i(t) = p_i(t) - t dp_i/dt, the bracket of the back
 *      projection equation (Section II-C, Eq. BP), on the sample grid.
 *   4. orc_gather: P(r_j) = sum_i w_i b_i(t_{i,j}) with linear interpolation
 *      in time (Section II-C, Eq. BP; weights default to 1 as in the paper).
 *   5. orc_table_to_q16 / orc_gather_q16: the same gather from a delay table
 *      stored as a 16.16 fixed-point fractional sample index.
 *   6. orc_seed3 / orc_fmm3 / orc_tables3: steps 1-2 on a 3-D grid with the
 *      6-neighbour Godunov update (3-D reconstruction, Section IV);
 *      orc_tables_const3: the straight-ray table of the conventional back
 *      projection on the same grid (orc_tables_const is its 2-D form).
 *   8. orc_fmm2 / orc_tables2: steps 1-2 with the paper's second-order
 *      one-sided differences (Section II-B), same heap order.
 *   7. orc_table_to_r16 / orc_r16_to_q16: the 16.16 table of item 5 stored as
 *      16-bit offsets from a base per sensor and tile of 32 ROI positions
 *      (a compressed storage form; not in the paper).
 *
 * Readings where the paper is silent (all FP64):
 *   - nodes carry the speed; missing neighbours beyond the grid edge are +inf;
 *     4-neighbour stencil with isotropic spacing h;
 *   - the source is seeded by freezing every node within r0 of it at the
 *     straight-ray time |x_k - s| / c(n*), n* the node nearest the source;
 *   - derivative by central differences, one-sided at both ends; t_n = t0 + n dt;
 *   - a delay outside [t0, t0 + (N-1) dt] or non-finite contributes zero; at
 *     u = N-1 the last interval is used with weight 1.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <fenv.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_FAR 0
#define ORC_TRIAL 1
#define ORC_KNOWN 2

/* ------------------------------------------------------------------ heap */
typedef struct { double key; int32_t idx; } orc_item;
typedef struct { orc_item *a; long n, cap; } orc_heap;

static int item_less(orc_item x, orc_item y) {
    return x.key < y.key || (x.key == y.key && x.idx < y.idx);
}

static int heap_push(orc_heap *h, double key, int32_t idx) {
    if (h->n == h->cap) {
        long nc = h->cap ? 2 * h->cap : 1024;
        orc_item *na = (orc_item *)realloc(h->a, (size_t)nc * sizeof(orc_item));
        if (!na) return -1;
        h->a = na; h->cap = nc;
    }
    long i = h->n++;
    orc_item it = { key, idx };
    while (i > 0) {
        long p = (i - 1) / 2;
        if (!item_less(it, h->a[p])) break;
        h->a[i] = h->a[p];
        i = p;
    }
    h->a[i] = it;
    return 0;
}

static orc_item heap_pop(orc_heap *h) {
    orc_item top = h->a[0];
    orc_item last = h->a[--h->n];
    long i = 0;
    for (;;) {
        long l = 2 * i + 1, r = l + 1, m = i;
        orc_item mv = last;
        if (l < h->n && item_less(h->a[l], mv)) { m = l; mv = h->a[l]; }
        if (r < h->n && item_less(h->a[r], mv)) { m = r; mv = h->a[r]; }
        if (m == i) break;
        h->a[i] = h->a[m];
        i = m;
    }
    if (h->n > 0) h->a[i] = last;
    return top;
}

/* ------------------------------------------------------------- eikonal */

/* First-order Godunov update of one node from the smallest accepted neighbour
 * along x (a) and along y (b); fh = slowness * h.  Written in the incremental
 * form m + (d + sqrt(2 fh^2 - d^2)) / 2, which equals the textbook root
 * ((a + b) + sqrt(2 fh^2 - (a - b)^2)) / 2 of (T-a)^2 + (T-b)^2 = fh^2. */
static double godunov(double a, double b, double fh) {
    double m = a < b ? a : b;
    if (isinf(m)) return INFINITY;
    double d = fabs(a - b);
    if (isinf(d) || d >= fh) return m + fh;
    return m + 0.5 * (d + sqrt(2.0 * fh * fh - d * d));
}

/* Fast marching over the whole grid.
 * slow[k]  : slowness 1/c at node k (s/m)
 * frozen[k]: nonzero for source nodes whose T[k] is given on entry
 * T[k]     : out (in for frozen nodes), seconds
 * Returns 0, or -1 on allocation failure.  *npop receives the accepted count. */
int orc_fmm(int nx, int ny, double h, const double *slow, const unsigned char *frozen,
            double *T, long *npop) {
    long n = (long)nx * ny;
    unsigned char *state = (unsigned char *)calloc((size_t)n, 1);
    orc_heap hp = { 0, 0, 0 };
    if (!state) return -1;
    for (long k = 0; k < n; ++k) {
        if (frozen[k]) state[k] = ORC_KNOWN;
        else T[k] = INFINITY;
    }
    long pops = 0;
    int rc = 0;
    /* initial trial band: every non-frozen neighbour of a frozen node */
    for (long k = 0; k < n && rc == 0; ++k) {
        if (!frozen[k]) continue;
        int i = (int)(k % nx), j = (int)(k / nx);
        const int di[4] = { -1, 1, 0, 0 }, dj[4] = { 0, 0, -1, 1 };
        for (int q = 0; q < 4; ++q) {
            int ii = i + di[q], jj = j + dj[q];
            if (ii < 0 || ii >= nx || jj < 0 || jj >= ny) continue;
            long m = (long)jj * nx + ii;
            if (state[m] == ORC_KNOWN) continue;
            state[m] = ORC_TRIAL;
        }
    }
    /* compute trial values of the initial band in index order */
    for (long m = 0; m < n && rc == 0; ++m) {
        if (state[m] != ORC_TRIAL) continue;
        int i = (int)(m % nx), j = (int)(m / nx);
        double a = INFINITY, b = INFINITY;
        if (i > 0 && state[m - 1] == ORC_KNOWN) a = fmin(a, T[m - 1]);
        if (i < nx - 1 && state[m + 1] == ORC_KNOWN) a = fmin(a, T[m + 1]);
        if (j > 0 && state[m - nx] == ORC_KNOWN) b = fmin(b, T[m - nx]);
        if (j < ny - 1 && state[m + nx] == ORC_KNOWN) b = fmin(b, T[m + nx]);
        T[m] = godunov(a, b, slow[m] * h);
        if (heap_push(&hp, T[m], (int32_t)m)) rc = -1;
    }
    while (rc == 0 && hp.n > 0) {
        orc_item it = heap_pop(&hp);
        long k = it.idx;
        if (state[k] == ORC_KNOWN || it.key != T[k]) continue; /* stale entry */
        state[k] = ORC_KNOWN;
        ++pops;
        int i = (int)(k % nx), j = (int)(k / nx);
        const int di[4] = { -1, 1, 0, 0 }, dj[4] = { 0, 0, -1, 1 };
        for (int q = 0; q < 4; ++q) {
            int ii = i + di[q], jj = j + dj[q];
            if (ii < 0 || ii >= nx || jj < 0 || jj >= ny) continue;
            long m = (long)jj * nx + ii;
            if (state[m] == ORC_KNOWN) continue;
            double a = INFINITY, b = INFINITY;
            if (ii > 0 && state[m - 1] == ORC_KNOWN) a = fmin(a, T[m - 1]);
            if (ii < nx - 1 && state[m + 1] == ORC_KNOWN) a = fmin(a, T[m + 1]);
            if (jj > 0 && state[m - nx] == ORC_KNOWN) b = fmin(b, T[m - nx]);
            if (jj < ny - 1 && state[m + nx] == ORC_KNOWN) b = fmin(b, T[m + nx]);
            double t = godunov(a, b, slow[m] * h);
            if (t < T[m]) {
                T[m] = t;
                state[m] = ORC_TRIAL;
                if (heap_push(&hp, t, (int32_t)m)) { rc = -1; break; }
            }
        }
    }
    free(hp.a);
    free(state);
    if (npop) *npop = pops;
    return rc;
}

/* ------------------------------------------------- second-order marching */
/*
 * The paper's scheme (Section II-B, after Sethian): the same fast marching,
 * with the one-sided derivative along an axis taken to second order,
 * (3 T - 4 T1 + T2) / (2h), where the two upwind nodes T1 (the smaller
 * accepted neighbour on the axis) and T2 (the node beyond it on the same
 * side) are both accepted and T2 <= T1; otherwise the first-order (T - T1)/h.
 * Each axis then contributes c (T - b)^2 to sum = (f h)^2, with c = 9/4,
 * b = (4 T1 - T2) / 3 (second order) or c = 1, b = T1 (first order).
 */

/* Upwind term of node m along one axis: neighbours at m - st and m + st
 * exist when lo / hi; the nodes two away at m -/+ 2 st exist when lo2 / hi2. */
static int axis_term(const double *T, const unsigned char *state, long m, long st, int lo, int hi, int lo2,
                     int hi2, int order, double *c, double *b) {
    double t1 = INFINITY;
    int side = 0;
    if (lo && state[m - st] == ORC_KNOWN) { t1 = T[m - st]; side = -1; }
    if (hi && state[m + st] == ORC_KNOWN && T[m + st] < t1) { t1 = T[m + st]; side = 1; }
    if (side == 0) return 0;
    *c = 1.0;
    *b = t1;
    if (order == 2) {
        int ok2 = side < 0 ? lo2 : hi2;
        long m2 = m + 2 * side * st;
        if (ok2 && state[m2] == ORC_KNOWN && T[m2] <= t1) {
            *c = 2.25;
            *b = (4.0 * t1 - T[m2]) / 3.0;
        }
    }
    return 1;
}

/* Root of sum over the available axes of c_k (T - b_k)^2 = fh^2: both axes
 * when the root lies at or above both b_k, else the smaller one-axis root
 * b_k + fh / sqrt(c_k).  With first-order terms on both axes this is the
 * first-order update above (computed by it). */
static double update2(int hx, double cx, double bx, int hy, double cy, double by, double fh) {
    if (!hx && !hy) return INFINITY;
    double ix = cx == 1.0 ? fh : fh / 1.5, iy = cy == 1.0 ? fh : fh / 1.5;
    if (!hy) return bx + ix;
    if (!hx) return by + iy;
    if (cx == 1.0 && cy == 1.0) return godunov(bx, by, fh);
    double m = bx < by ? bx : by;
    double ex = bx - m, ey = by - m;
    double A = cx + cy, B = cx * ex + cy * ey, C = cx * ex * ex + cy * ey * ey - fh * fh;
    double disc = B * B - A * C;
    if (disc >= 0.0) {
        double t = (B + sqrt(disc)) / A;
        if (t >= ex && t >= ey) return m + t;
    }
    double tx = bx + ix, ty = by + iy;
    return tx < ty ? tx : ty;
}

static double node_update2(const double *T, const unsigned char *state, int nx, int ny, long m, double fh,
                           int order) {
    int i = (int)(m % nx), j = (int)(m / nx);
    double cx = 0, bx = 0, cy = 0, by = 0;
    int hx = axis_term(T, state, m, 1, i > 0, i < nx - 1, i > 1, i < nx - 2, order, &cx, &bx);
    int hy = axis_term(T, state, m, nx, j > 0, j < ny - 1, j > 1, j < ny - 2, order, &cy, &by);
    return update2(hx, cx, bx, hy, cy, by, fh);
}

/* Fast marching with the update of the given order (1 or 2); otherwise as
 * orc_fmm (same heap order: the smallest trial time first, ties by index;
 * a trial value is replaced when a newly accepted neighbour lowers it).
 * accepted (may be NULL): the node indices in the order they were accepted,
 * one per pop (at most nx*ny entries). */
int orc_fmm2(int nx, int ny, double h, const double *slow, const unsigned char *frozen, double *T, long *npop,
             int order, int32_t *accepted) {
    long n = (long)nx * ny;
    unsigned char *state = (unsigned char *)calloc((size_t)n, 1);
    orc_heap hp = { 0, 0, 0 };
    if (!state) return -1;
    for (long k = 0; k < n; ++k) {
        if (frozen[k]) state[k] = ORC_KNOWN;
        else T[k] = INFINITY;
    }
    long pops = 0;
    int rc = 0;
    for (long k = 0; k < n; ++k) {
        if (!frozen[k]) continue;
        int i = (int)(k % nx), j = (int)(k / nx);
        const int di[4] = { -1, 1, 0, 0 }, dj[4] = { 0, 0, -1, 1 };
        for (int q = 0; q < 4; ++q) {
            int ii = i + di[q], jj = j + dj[q];
            if (ii < 0 || ii >= nx || jj < 0 || jj >= ny) continue;
            long m = (long)jj * nx + ii;
            if (state[m] != ORC_KNOWN) state[m] = ORC_TRIAL;
        }
    }
    for (long m = 0; m < n && rc == 0; ++m) {
        if (state[m] != ORC_TRIAL) continue;
        T[m] = node_update2(T, state, nx, ny, m, slow[m] * h, order);
        if (heap_push(&hp, T[m], (int32_t)m)) rc = -1;
    }
    while (rc == 0 && hp.n > 0) {
        orc_item it = heap_pop(&hp);
        long k = it.idx;
        if (state[k] == ORC_KNOWN || it.key != T[k]) continue; /* stale entry */
        state[k] = ORC_KNOWN;
        if (accepted) accepted[pops] = (int32_t)k;
        ++pops;
        int i = (int)(k % nx), j = (int)(k / nx);
        const int di[4] = { -1, 1, 0, 0 }, dj[4] = { 0, 0, -1, 1 };
        for (int q = 0; q < 4; ++q) {
            int ii = i + di[q], jj = j + dj[q];
            if (ii < 0 || ii >= nx || jj < 0 || jj >= ny) continue;
            long m = (long)jj * nx + ii;
            if (state[m] == ORC_KNOWN) continue;
            double t = node_update2(T, state, nx, ny, m, slow[m] * h, order);
            if (t < T[m]) {
                T[m] = t;
                state[m] = ORC_TRIAL;
                if (heap_push(&hp, t, (int32_t)m)) { rc = -1; break; }
            }
        }
    }
    free(hp.a);
    free(state);
    if (npop) *npop = pops;
    return rc;
}

/* Point-source initial condition: every node within r0 of the source (sx, sy)
 * is frozen at the straight-ray time |x_k - s| * slow(n*), where n* is the node
 * nearest the source.  Coordinates are grid-centred (node i at
 * (i - (nx-1)/2) h).  Returns the number of frozen nodes, or -1 when the
 * source lies outside the grid's bounding box. */
int orc_seed(int nx, int ny, double h, const double *slow, double sx, double sy, double r0,
             unsigned char *frozen, double *T) {
    double x0 = -0.5 * (nx - 1) * h, y0 = -0.5 * (ny - 1) * h;
    double gi = (sx - x0) / h, gj = (sy - y0) / h;
    if (!(gi >= 0.0 && gi <= nx - 1 && gj >= 0.0 && gj <= ny - 1)) return -1;
    int is = (int)floor(gi + 0.5), js = (int)floor(gj + 0.5);
    if (is > nx - 1) is = nx - 1;
    if (js > ny - 1) js = ny - 1;
    double fs = slow[(long)js * nx + is];
    int rad = (int)ceil(r0 / h) + 1;
    int cnt = 0;
    memset(frozen, 0, (size_t)nx * ny);
    for (int j = js - rad; j <= js + rad; ++j) {
        if (j < 0 || j >= ny) continue;
        for (int i = is - rad; i <= is + rad; ++i) {
            if (i < 0 || i >= nx) continue;
            double dx = (x0 + i * h) - sx, dy = (y0 + j * h) - sy;
            double r = sqrt(dx * dx + dy * dy);
            if (r <= r0) {
                long k = (long)j * nx + i;
                frozen[k] = 1;
                T[k] = r * fs;
                ++cnt;
            }
        }
    }
    return cnt;
}

/* Delay table: T[s][p] = first-arrival time from sensor s to ROI node pix[p],
 * one fast-marching solve per sensor, seeded with r0 = 2h.  speed is float32
 * m/s (row-major [ny][nx]); sxy is [S][2] metres.  Returns 0, -1 on bad input
 * (non-positive or non-finite speed, sensor outside the grid, pixel index out
 * of range) or -2 on allocation failure. */
int orc_tables(int nx, int ny, double h, const float *speed, const double *sxy, int S,
               const int32_t *pix, long P, double *table, int nthreads) {
    long n = (long)nx * ny;
    for (long p = 0; p < P; ++p)
        if (pix[p] < 0 || pix[p] >= n) return -1;
    double *slow = (double *)malloc((size_t)n * sizeof(double));
    if (!slow) return -2;
    for (long k = 0; k < n; ++k) {
        double c = (double)speed[k];
        if (!(c > 0.0) || isinf(c)) { free(slow); return -1; }
        slow[k] = 1.0 / c;
    }
    int rc = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
    {
        double *T = (double *)malloc((size_t)n * sizeof(double));
        unsigned char *fr = (unsigned char *)malloc((size_t)n);
        if (!T || !fr) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            rc = -2;
        }
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (int s = 0; s < S; ++s) {
            if (!T || !fr) continue;
            int c = orc_seed(nx, ny, h, slow, sxy[2 * s], sxy[2 * s + 1], 2.0 * h, fr, T);
            if (c < 0) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
                rc = -1;
                continue;
            }
            if (orc_fmm(nx, ny, h, slow, fr, T, 0)) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
                rc = -2;
                continue;
            }
            for (long p = 0; p < P; ++p) table[(long)s * P + p] = T[pix[p]];
        }
        free(T);
        free(fr);
    }
    free(slow);
    return rc;
}

/* orc_tables with the second-order marching of orc_fmm2. */
int orc_tables2(int nx, int ny, double h, const float *speed, const double *sxy, int S,
               const int32_t *pix, long P, double *table, int nthreads) {
    long n = (long)nx * ny;
    for (long p = 0; p < P; ++p)
        if (pix[p] < 0 || pix[p] >= n) return -1;
    double *slow = (double *)malloc((size_t)n * sizeof(double));
    if (!slow) return -2;
    for (long k = 0; k < n; ++k) {
        double c = (double)speed[k];
        if (!(c > 0.0) || isinf(c)) { free(slow); return -1; }
        slow[k] = 1.0 / c;
    }
    int rc = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
    {
        double *T = (double *)malloc((size_t)n * sizeof(double));
        unsigned char *fr = (unsigned char *)malloc((size_t)n);
        if (!T || !fr) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            rc = -2;
        }
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (int s = 0; s < S; ++s) {
            if (!T || !fr) continue;
            int c = orc_seed(nx, ny, h, slow, sxy[2 * s], sxy[2 * s + 1], 2.0 * h, fr, T);
            if (c < 0) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
                rc = -1;
                continue;
            }
            if (orc_fmm2(nx, ny, h, slow, fr, T, 0, 2, 0)) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
                rc = -2;
                continue;
            }
            for (long p = 0; p < P; ++p) table[(long)s * P + p] = T[pix[p]];
        }
        free(T);
        free(fr);
    }
    free(slow);
    return rc;
}

/* Conventional back projection's delays (Section III: the constant-speed
 * comparison): T[s][p] = |x_pix[p] - s| / c, straight rays in a homogeneous
 * medium of speed c.  Returns 0, or -1 on a bad pixel index or c <= 0. */
int orc_tables_const(int nx, int ny, double h, double c, const double *sxy, int S, const int32_t *pix, long P,
                     double *table) {
    long n = (long)nx * ny;
    if (!(c > 0.0)) return -1;
    for (long p = 0; p < P; ++p)
        if (pix[p] < 0 || pix[p] >= n) return -1;
    double x0 = -0.5 * (nx - 1) * h, y0 = -0.5 * (ny - 1) * h;
    for (int s = 0; s < S; ++s) {
        for (long p = 0; p < P; ++p) {
            int i = pix[p] % nx, j = pix[p] / nx;
            double dx = (x0 + i * h) - sxy[2 * s], dy = (y0 + j * h) - sxy[2 * s + 1];
            table[(long)s * P + p] = sqrt(dx * dx + dy * dy) / c;
        }
    }
    return 0;
}

/* ---------------------------------------------------------- 3-D eikonal */

/* Straight-ray delays |x_k - s| / c on a 3-D grid (the conventional back
 * projection's table in 3-D): node k = (l ny + j) nx + i at the grid-centred
 * position of the 3-D convention below; sxyz [S][3]. */
int orc_tables_const3(int nx, int ny, int nz, double h, double c, const double *sxyz, int S, const int32_t *vox,
                      long P, double *table) {
    long n = (long)nx * ny * nz;
    if (!(c > 0.0)) return -1;
    for (long p = 0; p < P; ++p)
        if (vox[p] < 0 || vox[p] >= n) return -1;
    double x0 = -0.5 * (nx - 1) * h, y0 = -0.5 * (ny - 1) * h, z0 = -0.5 * (nz - 1) * h;
    for (int s = 0; s < S; ++s) {
        for (long p = 0; p < P; ++p) {
            int i = vox[p] % nx, j = (vox[p] / nx) % ny, l = vox[p] / (nx * ny);
            double dx = (x0 + i * h) - sxyz[3 * s], dy = (y0 + j * h) - sxyz[3 * s + 1],
                   dz = (z0 + l * h) - sxyz[3 * s + 2];
            table[(long)s * P + p] = sqrt(dx * dx + dy * dy + dz * dz) / c;
        }
    }
    return 0;
}
/*
 * The same method on a 3-D grid, the extension the paper anticipates for 3-D
 * reconstruction (Section IV): node (i, j, l) with index k = (l ny + j) nx + i
 * at ((i - (nx-1)/2) h, (j - (ny-1)/2) h, (l - (nz-1)/2) h), a 6-neighbour
 * stencil, missing neighbours +inf, and the first-order Godunov update with
 * the three upwind minima.  With nz = 1 every z-neighbour is missing and
 * everything below reduces, operation for operation, to the 2-D code above.
 */

/* Godunov update from the smallest accepted neighbours along x, y and z.
 * Sorted a <= b <= c: one-sided a + fh if that is not above b; else the
 * two-sided root of (T-a)^2 + (T-b)^2 = fh^2 if that is not above c; else the
 * three-sided root of (T-a)^2 + (T-b)^2 + (T-c)^2 = fh^2.  Each root is
 * written relative to a (incremental form). */
static double godunov3(double a, double b, double c, double fh) {
    double t;
    if (b < a) { t = a; a = b; b = t; }
    if (c < b) { t = b; b = c; c = t; }
    if (b < a) { t = a; a = b; b = t; }
    if (isinf(a)) return INFINITY;
    double d = b - a;
    if (isinf(d) || d >= fh) return a + fh;
    double x = 0.5 * (d + sqrt(2.0 * fh * fh - d * d));
    double e = c - a;
    if (isinf(e) || x <= e) return a + x;
    double sum = d + e;
    double disc = sum * sum - 3.0 * (d * d + e * e - fh * fh);
    return a + (sum + sqrt(disc)) / 3.0;
}

static void upwind3(int nx, int ny, int nz, long m, const unsigned char *state, const double *T,
                    double *a, double *b, double *c) {
    long nxy = (long)nx * ny;
    int i = (int)(m % nx), j = (int)((m / nx) % ny), l = (int)(m / nxy);
    *a = *b = *c = INFINITY;
    if (i > 0 && state[m - 1] == ORC_KNOWN) *a = fmin(*a, T[m - 1]);
    if (i < nx - 1 && state[m + 1] == ORC_KNOWN) *a = fmin(*a, T[m + 1]);
    if (j > 0 && state[m - nx] == ORC_KNOWN) *b = fmin(*b, T[m - nx]);
    if (j < ny - 1 && state[m + nx] == ORC_KNOWN) *b = fmin(*b, T[m + nx]);
    if (l > 0 && state[m - nxy] == ORC_KNOWN) *c = fmin(*c, T[m - nxy]);
    if (l < nz - 1 && state[m + nxy] == ORC_KNOWN) *c = fmin(*c, T[m + nxy]);
}

/* Fast marching over a 3-D grid; arguments as orc_fmm. */
int orc_fmm3(int nx, int ny, int nz, double h, const double *slow, const unsigned char *frozen, double *T,
             long *npop) {
    long nxy = (long)nx * ny, n = nxy * nz;
    unsigned char *state = (unsigned char *)calloc((size_t)n, 1);
    orc_heap hp = { 0, 0, 0 };
    if (!state) return -1;
    for (long k = 0; k < n; ++k) {
        if (frozen[k]) state[k] = ORC_KNOWN;
        else T[k] = INFINITY;
    }
    const int di[6] = { -1, 1, 0, 0, 0, 0 }, dj[6] = { 0, 0, -1, 1, 0, 0 }, dl[6] = { 0, 0, 0, 0, -1, 1 };
    long pops = 0;
    int rc = 0;
    for (long k = 0; k < n; ++k) {
        if (!frozen[k]) continue;
        int i = (int)(k % nx), j = (int)((k / nx) % ny), l = (int)(k / nxy);
        for (int q = 0; q < 6; ++q) {
            int ii = i + di[q], jj = j + dj[q], ll = l + dl[q];
            if (ii < 0 || ii >= nx || jj < 0 || jj >= ny || ll < 0 || ll >= nz) continue;
            long m = ((long)ll * ny + jj) * nx + ii;
            if (state[m] != ORC_KNOWN) state[m] = ORC_TRIAL;
        }
    }
    for (long m = 0; m < n && rc == 0; ++m) {
        if (state[m] != ORC_TRIAL) continue;
        double a, b, c;
        upwind3(nx, ny, nz, m, state, T, &a, &b, &c);
        T[m] = godunov3(a, b, c, slow[m] * h);
        if (heap_push(&hp, T[m], (int32_t)m)) rc = -1;
    }
    while (rc == 0 && hp.n > 0) {
        orc_item it = heap_pop(&hp);
        long k = it.idx;
        if (state[k] == ORC_KNOWN || it.key != T[k]) continue; /* stale entry */
        state[k] = ORC_KNOWN;
        ++pops;
        int i = (int)(k % nx), j = (int)((k / nx) % ny), l = (int)(k / nxy);
        for (int q = 0; q < 6; ++q) {
            int ii = i + di[q], jj = j + dj[q], ll = l + dl[q];
            if (ii < 0 || ii >= nx || jj < 0 || jj >= ny || ll < 0 || ll >= nz) continue;
            long m = ((long)ll * ny + jj) * nx + ii;
            if (state[m] == ORC_KNOWN) continue;
            double a, b, c;
            upwind3(nx, ny, nz, m, state, T, &a, &b, &c);
            double t = godunov3(a, b, c, slow[m] * h);
            if (t < T[m]) {
                T[m] = t;
                state[m] = ORC_TRIAL;
                if (heap_push(&hp, t, (int32_t)m)) { rc = -1; break; }
            }
        }
    }
    free(hp.a);
    free(state);
    if (npop) *npop = pops;
    return rc;
}

/* Point-source initial condition in 3-D (as orc_seed): nodes within r0 of
 * (sx, sy, sz) frozen at |x_k - s| * slow(n*).  Returns the frozen count, or
 * -1 when the source is outside the grid's bounding box. */
int orc_seed3(int nx, int ny, int nz, double h, const double *slow, double sx, double sy, double sz, double r0,
              unsigned char *frozen, double *T) {
    double x0 = -0.5 * (nx - 1) * h, y0 = -0.5 * (ny - 1) * h, z0 = -0.5 * (nz - 1) * h;
    double gi = (sx - x0) / h, gj = (sy - y0) / h, gl = (sz - z0) / h;
    if (!(gi >= 0.0 && gi <= nx - 1 && gj >= 0.0 && gj <= ny - 1 && gl >= 0.0 && gl <= nz - 1)) return -1;
    int is = (int)floor(gi + 0.5), js = (int)floor(gj + 0.5), ls = (int)floor(gl + 0.5);
    if (is > nx - 1) is = nx - 1;
    if (js > ny - 1) js = ny - 1;
    if (ls > nz - 1) ls = nz - 1;
    double fs = slow[((long)ls * ny + js) * nx + is];
    int rad = (int)ceil(r0 / h) + 1;
    int cnt = 0;
    memset(frozen, 0, (size_t)nx * ny * nz);
    for (int l = ls - rad; l <= ls + rad; ++l) {
        if (l < 0 || l >= nz) continue;
        for (int j = js - rad; j <= js + rad; ++j) {
            if (j < 0 || j >= ny) continue;
            for (int i = is - rad; i <= is + rad; ++i) {
                if (i < 0 || i >= nx) continue;
                double dx = (x0 + i * h) - sx, dy = (y0 + j * h) - sy, dz = (z0 + l * h) - sz;
                double r = sqrt(dx * dx + dy * dy + dz * dz);
                if (r <= r0) {
                    long k = ((long)l * ny + j) * nx + i;
                    frozen[k] = 1;
                    T[k] = r * fs;
                    ++cnt;
                }
            }
        }
    }
    return cnt;
}

/* 3-D delay table (as orc_tables): speed float32 [nz][ny][nx], sensors
 * [S][3] metres, voxel indices pix[P]; returns 0, -1 bad input, -2 memory. */
int orc_tables3(int nx, int ny, int nz, double h, const float *speed, const double *sxyz, int S,
                const int32_t *pix, long P, double *table, int nthreads) {
    long n = (long)nx * ny * nz;
    for (long p = 0; p < P; ++p)
        if (pix[p] < 0 || pix[p] >= n) return -1;
    double *slow = (double *)malloc((size_t)n * sizeof(double));
    if (!slow) return -2;
    for (long k = 0; k < n; ++k) {
        double c = (double)speed[k];
        if (!(c > 0.0) || isinf(c)) { free(slow); return -1; }
        slow[k] = 1.0 / c;
    }
    int rc = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
#endif
    {
        double *T = (double *)malloc((size_t)n * sizeof(double));
        unsigned char *fr = (unsigned char *)malloc((size_t)n);
        if (!T || !fr) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            rc = -2;
        }
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (int s = 0; s < S; ++s) {
            if (!T || !fr) continue;
            int c = orc_seed3(nx, ny, nz, h, slow, sxyz[3 * s], sxyz[3 * s + 1], sxyz[3 * s + 2], 2.0 * h, fr, T);
            if (c < 0) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
                rc = -1;
                continue;
            }
            if (orc_fmm3(nx, ny, nz, h, slow, fr, T, 0)) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
                rc = -2;
                continue;
            }
            for (long p = 0; p < P; ++p) table[(long)s * P + p] = T[pix[p]];
        }
        free(T);
        free(fr);
    }
    free(slow);
    return rc;
}

/* -------------------------------------------------------------- filter */

/* b[r][n] = p[r][n] - t_n * D[r][n], t_n = t0 + n dt, with D the central
 * difference (p[n+1]-p[n-1])/(2 dt) inside and one-sided differences at n = 0
 * and n = N-1.  rows independent signals of N >= 2 samples each. */
void orc_filter(const double *p, long rows, int N, double t0, double dt, double *b) {
    for (long r = 0; r < rows; ++r) {
        const double *x = p + r * N;
        double *y = b + r * N;
        for (int k = 0; k < N; ++k) {
            double D;
            if (k == 0) D = (x[1] - x[0]) / dt;
            else if (k == N - 1) D = (x[N - 1] - x[N - 2]) / dt;
            else D = (x[k + 1] - x[k - 1]) / (2.0 * dt);
            double t = t0 + k * dt;
            y[k] = x[k] - t * D;
        }
    }
}

/* -------------------------------------------------------------- gather */

/* Linear interpolation of b[0..N-1] at fractional sample position u; zero
 * outside [0, N-1]. */
static double lerp_at(const double *b, int N, double u) {
    if (!(u >= 0.0) || !(u <= (double)(N - 1))) return 0.0;
    double fl = floor(u);
    long n = (long)fl;
    if (n > N - 2) n = N - 2;
    double a = u - (double)n;
    return b[n] + a * (b[n + 1] - b[n]);
}

/* img[f][p] = sum_{s=0}^{S-1} w[s] * b[f][s](T[s][p]) for F frames, summed in
 * sensor order.  T in seconds (non-finite = no contribution); w may be NULL
 * (all ones). */
void orc_gather(const double *T, const double *b, const double *w, int S, long P, int N, int F,
                double t0, double dt, double *img, int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (long p = 0; p < P; ++p) {
        for (int f = 0; f < F; ++f) {
            double acc = 0.0;
            for (int s = 0; s < S; ++s) {
                double t = T[(long)s * P + p];
                if (!isfinite(t)) continue;
                double u = (t - t0) / dt;
                double ws = w ? w[s] : 1.0;
                acc += ws * lerp_at(b + ((long)f * S + s) * N, N, u);
            }
            img[(long)f * P + p] = acc;
        }
    }
}

/* 16.16 fixed-point fractional sample index of each delay:
 * u = (T - t0) / dt in FP64; q = round-half-even(u * 65536) when T is finite
 * and 0 <= u <= N-1, otherwise the sentinel 0xFFFFFFFF.  Requires N <= 65535. */
void orc_table_to_q16(const float *T, long n, double t0, double dt, int N, uint32_t *q) {
    int old = fegetround();
    fesetround(FE_TONEAREST);
    for (long k = 0; k < n; ++k) {
        double t = (double)T[k];
        double u = (t - t0) / dt;
        if (!isfinite(t) || !(u >= 0.0) || !(u <= (double)(N - 1))) {
            q[k] = 0xFFFFFFFFu;
            continue;
        }
        q[k] = (uint32_t)nearbyint(u * 65536.0);
    }
    fesetround(old);
}

/* Gather from a 16.16 table: n = q >> 16, alpha = (q & 0xFFFF) / 65536; the
 * sentinel contributes zero; n = N-1 (alpha = 0) is read as the end of the
 * last interval. */
void orc_gather_q16(const uint32_t *q, const double *b, const double *w, int S, long P, int N, int F,
                    double *img, int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (long p = 0; p < P; ++p) {
        for (int f = 0; f < F; ++f) {
            double acc = 0.0;
            for (int s = 0; s < S; ++s) {
                uint32_t v = q[(long)s * P + p];
                if (v == 0xFFFFFFFFu) continue;
                double u = (double)(v >> 16) + (double)(v & 0xFFFFu) / 65536.0;
                double ws = w ? w[s] : 1.0;
                acc += ws * lerp_at(b + ((long)f * S + s) * N, N, u);
            }
            img[(long)f * P + p] = acc;
        }
    }
}

/* Tile-relative 16-bit delays.  The entries of sensor s are cut into tiles of
 * 32 consecutive ROI positions (the last tile may be shorter).  A delay is
 * valid when T is finite and u = (T - t0)/dt lies in [0, N-1].  For a tile with
 * a valid delay: b = floor(smallest valid u), k = the largest integer in
 * [0, 16] with (largest valid u - b) * 2^k <= 65534, every valid entry stores
 * off = round-half-even((u - b) * 2^k) and every other one 0xFFFF, and the
 * header is (b << 16) | (16 - k).  A tile without valid delays has header 0
 * and only 0xFFFF entries.  off <= 65534 always, and the decoded value
 * u' = b + off / 2^k satisfies |u' - u| <= 2^-(k+1) and u' <= N-1.
 * off: [S][P] uint16; hdr: [S][ceil(P/32)] uint32. */
void orc_table_to_r16(const float *T, int S, long P, double t0, double dt, int N, uint16_t *off, uint32_t *hdr) {
    int old = fegetround();
    fesetround(FE_TONEAREST);
    long tiles = (P + 31) / 32;
    for (int s = 0; s < S; ++s) {
        for (long t = 0; t < tiles; ++t) {
            long p0 = t * 32, p1 = p0 + 32 < P ? p0 + 32 : P;
            double lo = INFINITY, hi = -INFINITY;
            double u[32];
            int ok[32];
            for (long p = p0; p < p1; ++p) {
                double tv = (double)T[(long)s * P + p];
                double uu = (tv - t0) / dt;
                int v = isfinite(tv) && uu >= 0.0 && uu <= (double)(N - 1);
                u[p - p0] = uu;
                ok[p - p0] = v;
                if (v) {
                    if (uu < lo) lo = uu;
                    if (uu > hi) hi = uu;
                }
            }
            if (!(lo <= hi)) {  /* no valid delay */
                hdr[(long)s * tiles + t] = 0u;
                for (long p = p0; p < p1; ++p) off[(long)s * P + p] = 0xFFFFu;
                continue;
            }
            double b = floor(lo);
            int k = 16;
            while (k > 0 && ldexp(hi - b, k) > 65534.0) --k;
            hdr[(long)s * tiles + t] = ((uint32_t)b << 16) | (uint32_t)(16 - k);
            for (long p = p0; p < p1; ++p)
                off[(long)s * P + p] = ok[p - p0] ? (uint16_t)nearbyint(ldexp(u[p - p0] - b, k)) : (uint16_t)0xFFFFu;
        }
    }
    fesetround(old);
}

/* The 16.16 value of every entry: (b << 16) + (off << (16 - k)), or the
 * 16.16 sentinel 0xFFFFFFFF for off = 0xFFFF. */
void orc_r16_to_q16(const uint16_t *off, const uint32_t *hdr, int S, long P, uint32_t *q) {
    long tiles = (P + 31) / 32;
    for (int s = 0; s < S; ++s)
        for (long p = 0; p < P; ++p) {
            uint16_t o = off[(long)s * P + p];
            uint32_t h = hdr[(long)s * tiles + p / 32];
            q[(long)s * P + p] = o == 0xFFFFu ? 0xFFFFFFFFu : (h & 0xFFFF0000u) + ((uint32_t)o << (h & 31u));
        }
}

int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
