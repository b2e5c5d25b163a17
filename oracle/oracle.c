/*
 * Plain, slow, obviously-correct CPU oracle for the level-blocked matrix power
 * kernel (MPK).  TEST INFRASTRUCTURE ONLY: nothing in the product path may
 * link, load or call this file.  It shares no code with the GPU library.
 *
 * Contents
 *   orc_spmv_powers      p back-to-back FP64 CSR SpMVs in the stored order
 *                        (the baseline MPK of Sec. 3.1, Fig. 2), which is the
 *                        plain definition of what any MPK computes:
 *                        y_p = A^p x for p = 1..p_m, every y_p kept.
 *   orc_spmv_powers_omp  the same loops with the rows of each SpMV shared
 *                        among OpenMP threads, schedule(static), as the
 *                        paper's baseline runs them (Sec. 3.1, Sec. 6).  A row
 *                        is still summed by one thread in stored order, so the
 *                        result equals orc_spmv_powers bit for bit.
 *   orc_round_values     matrix values rounded to FP32 / BF16 storage, as FP64
 *                        (with orc_spmv_powers: the FP64-arithmetic variant)
 *   orc_spmv_powers_lowp the same with matrix values and inputs rounded to a
 *                        lower precision and the products summed in FP32
 *                        (the mixed-precision variant), written as its
 *                        definition.
 *   orc_bfs_levels       BFS levels of Eq. (3) with the renumbering of
 *                        Sec. 4.1 (levels contiguous, L(i-1) before L(i)).
 *   orc_bfs_distances    unweighted distances from one root inside its
 *                        connected component (used for the root search).
 *   orc_peripheral_root  George-Liu pseudo-peripheral root search.
 *
 * Readings of the paper fixed here (the paper leaves them open):
 *   - The graph of A is the pattern of A + A^T without the diagonal
 *     (Sec. 4 allows non-symmetric A without saying how).
 *   - Inside a level, vertex v is placed by the key (position of the
 *     earliest-numbered vertex of the previous level adjacent to v, original
 *     index of v).  This is Cuthill-McKee discovery order without degree
 *     sorting; the paper only asks that a level be numbered consecutively.
 *   - If a level comes out empty while vertices are left (a disconnected
 *     graph), the smallest unvisited original index forms the next level on
 *     its own and the search continues from it.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

/* ------------------------------------------------------------------ */
/* powers                                                             */
/* ------------------------------------------------------------------ */

/* y has layout [p][n][k]; x has layout [n][k] (row-major). */
int orc_spmv_powers(int64_t n, const int64_t *rowptr, const int32_t *col,
                    const double *val, int32_t k, int32_t p,
                    const double *x, double *y)
{
    if (n < 0 || k < 1 || p < 1) return -1;
    for (int32_t q = 1; q <= p; ++q) {
        const double *in = (q == 1) ? x : y + (int64_t)(q - 2) * n * k;
        double *out = y + (int64_t)(q - 1) * n * k;
        for (int64_t r = 0; r < n; ++r) {
            for (int32_t c = 0; c < k; ++c) {
                double tmp = 0.0;
                for (int64_t j = rowptr[r]; j < rowptr[r + 1]; ++j)
                    tmp += val[j] * in[(int64_t)col[j] * k + c];
                out[r * k + c] = tmp;
            }
        }
    }
    return 0;
}

int orc_spmv_powers_omp(int64_t n, const int64_t *rowptr, const int32_t *col,
                        const double *val, int32_t k, int32_t p,
                        const double *x, double *y, int32_t threads)
{
    if (n < 0 || k < 1 || p < 1 || threads < 1) return -1;
    for (int32_t q = 1; q <= p; ++q) {
        const double *in = (q == 1) ? x : y + (int64_t)(q - 2) * n * k;
        double *out = y + (int64_t)(q - 1) * n * k;
#pragma omp parallel for schedule(static) num_threads(threads)
        for (int64_t r = 0; r < n; ++r) {
            for (int32_t c = 0; c < k; ++c) {
                double tmp = 0.0;
                for (int64_t j = rowptr[r]; j < rowptr[r + 1]; ++j)
                    tmp += val[j] * in[(int64_t)col[j] * k + c];
                out[r * k + c] = tmp;
            }
        }
    }
    return 0;
}

/* Round a double to float with round-to-nearest-even (the C cast does that). */
static float to_f32(double v) { return (float)v; }

/* Round a float to bfloat16 (kept in a float) with round-to-nearest-even.
 * NaN stays NaN. */
static float to_bf16(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) {
        u |= 0x00400000u;
    } else {
        uint32_t lsb = (u >> 16) & 1u;
        u += 0x7fffu + lsb;
    }
    u &= 0xffff0000u;
    memcpy(&f, &u, 4);
    return f;
}

/*
 * Mixed-precision powers.  Matrix values: vdtype 1 = f64 -> f32 (RNE),
 * vdtype 2 = f64 -> f32 -> bf16 (RNE at each step).  Each power:
 *   x_f32 = round_f32(y_{q-1}),  s = sum_j a_j * x_f32[col_j]  (every
 *   product rounded to f32, then added to an f32 running sum that starts at
 *   0, in stored order; no fused multiply-add),  y_q = (double)s.
 */
/* Matrix values as a lower-precision storage holds them, widened back to
 * FP64: vdtype 1 = FP32 (round to nearest even), 2 = BF16 (FP32 first, then
 * the upper 16 bits with round to nearest even).  With these values the
 * FP64-arithmetic variant of the mixed-precision product is the plain
 * definition: p back-to-back FP64 SpMVs (orc_spmv_powers) on them. */
int orc_round_values(int64_t nnz, const double *val, int32_t vdtype, double *out)
{
    if (nnz < 0 || vdtype < 1 || vdtype > 2) return -1;
    for (int64_t j = 0; j < nnz; ++j) {
        float f = to_f32(val[j]);
        out[j] = (double)((vdtype == 2) ? to_bf16(f) : f);
    }
    return 0;
}

int orc_spmv_powers_lowp(int64_t n, const int64_t *rowptr, const int32_t *col,
                         const double *val, int32_t vdtype, int32_t k, int32_t p,
                         const double *x, double *y)
{
    if (n < 0 || k < 1 || p < 1 || vdtype < 1 || vdtype > 2) return -1;
    int64_t nnz = rowptr[n];
    float *a = (float *)malloc(sizeof(float) * (size_t)(nnz > 0 ? nnz : 1));
    float *xin = (float *)malloc(sizeof(float) * (size_t)(n * k > 0 ? n * k : 1));
    if (!a || !xin) { free(a); free(xin); return -2; }
    for (int64_t j = 0; j < nnz; ++j) {
        float f = to_f32(val[j]);
        a[j] = (vdtype == 2) ? to_bf16(f) : f;
    }
    for (int32_t q = 1; q <= p; ++q) {
        const double *in = (q == 1) ? x : y + (int64_t)(q - 2) * n * k;
        double *out = y + (int64_t)(q - 1) * n * k;
        for (int64_t i = 0; i < n * k; ++i) xin[i] = to_f32(in[i]);
        for (int64_t r = 0; r < n; ++r) {
            for (int32_t c = 0; c < k; ++c) {
                float s = 0.0f;
                for (int64_t j = rowptr[r]; j < rowptr[r + 1]; ++j) {
                    volatile float prod = a[j] * xin[(int64_t)col[j] * k + c];
                    s = s + prod;
                }
                out[r * k + c] = (double)s;
            }
        }
    }
    free(a);
    free(xin);
    return 0;
}

/* ------------------------------------------------------------------ */
/* graph of A + A^T                                                   */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t n;
    int64_t *tptr; /* transpose row pointer, n+1 */
    int32_t *tcol; /* transpose columns (= original rows) */
} orc_transpose;

static int build_transpose(int64_t n, const int64_t *rowptr, const int32_t *col,
                           orc_transpose *t)
{
    int64_t nnz = rowptr[n];
    t->n = n;
    t->tptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    t->tcol = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    if (!t->tptr || !t->tcol) return -2;
    for (int64_t j = 0; j < nnz; ++j) t->tptr[col[j] + 1]++;
    for (int64_t i = 0; i < n; ++i) t->tptr[i + 1] += t->tptr[i];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!fill) return -2;
    for (int64_t i = 0; i < n; ++i) fill[i] = t->tptr[i];
    for (int64_t r = 0; r < n; ++r)
        for (int64_t j = rowptr[r]; j < rowptr[r + 1]; ++j)
            t->tcol[fill[col[j]]++] = (int32_t)r;
    free(fill);
    return 0;
}

static void free_transpose(orc_transpose *t)
{
    free(t->tptr);
    free(t->tcol);
}

/* ------------------------------------------------------------------ */
/* BFS distances inside one component                                 */
/* ------------------------------------------------------------------ */

static int64_t bfs_dist(int64_t n, const int64_t *rowptr, const int32_t *col,
                        const orc_transpose *t, int64_t root, int64_t *dist,
                        int64_t *queue)
{
    for (int64_t i = 0; i < n; ++i) dist[i] = -1;
    int64_t head = 0, tail = 0, maxd = 0;
    dist[root] = 0;
    queue[tail++] = root;
    while (head < tail) {
        int64_t u = queue[head++];
        for (int side = 0; side < 2; ++side) {
            const int64_t *ptr = side ? t->tptr : rowptr;
            const int32_t *cc = side ? t->tcol : col;
            for (int64_t j = ptr[u]; j < ptr[u + 1]; ++j) {
                int64_t v = cc[j];
                if (v == u || dist[v] >= 0) continue;
                dist[v] = dist[u] + 1;
                if (dist[v] > maxd) maxd = dist[v];
                queue[tail++] = v;
            }
        }
    }
    return maxd;
}

int orc_bfs_distances(int64_t n, const int64_t *rowptr, const int32_t *col,
                      int64_t root, int64_t *dist)
{
    if (n <= 0 || root < 0 || root >= n) return -1;
    orc_transpose t;
    if (build_transpose(n, rowptr, col, &t)) return -2;
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!queue) { free_transpose(&t); return -2; }
    bfs_dist(n, rowptr, col, &t, root, dist, queue);
    free(queue);
    free_transpose(&t);
    return 0;
}

/* number of distinct neighbours of u in A + A^T, u itself excluded */
static int64_t sym_degree(const int64_t *rowptr, const int32_t *col,
                          const orc_transpose *t, int64_t u, int64_t *mark,
                          int64_t stamp)
{
    int64_t d = 0;
    for (int side = 0; side < 2; ++side) {
        const int64_t *ptr = side ? t->tptr : rowptr;
        const int32_t *cc = side ? t->tcol : col;
        for (int64_t j = ptr[u]; j < ptr[u + 1]; ++j) {
            int64_t v = cc[j];
            if (v == u || mark[v] == stamp) continue;
            mark[v] = stamp;
            ++d;
        }
    }
    return d;
}

/*
 * George-Liu pseudo-peripheral root: start at `start`; BFS; among the
 * vertices at the largest distance pick the one of smallest degree (ties:
 * smallest index); move there if its eccentricity is larger, else stop.
 */
int64_t orc_peripheral_root(int64_t n, const int64_t *rowptr, const int32_t *col,
                            int64_t start)
{
    if (n <= 0 || start < 0 || start >= n) return -1;
    orc_transpose t;
    if (build_transpose(n, rowptr, col, &t)) return -2;
    int64_t *dist = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *mark = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!dist || !queue || !mark) return -2;
    for (int64_t i = 0; i < n; ++i) mark[i] = -1;
    int64_t stamp = 0;
    int64_t r = start;
    int64_t ecc = bfs_dist(n, rowptr, col, &t, r, dist, queue);
    for (;;) {
        int64_t best = -1, bestdeg = 0;
        for (int64_t v = 0; v < n; ++v) {
            if (dist[v] != ecc) continue;
            int64_t d = sym_degree(rowptr, col, &t, v, mark, stamp++);
            if (best < 0 || d < bestdeg) { best = v; bestdeg = d; }
        }
        int64_t e2 = bfs_dist(n, rowptr, col, &t, best, dist, queue);
        if (e2 > ecc) {
            r = best;
            ecc = e2;
        } else {
            break;
        }
    }
    free(dist);
    free(queue);
    free(mark);
    free_transpose(&t);
    return r;
}

/* ------------------------------------------------------------------ */
/* BFS levels and renumbering                                         */
/* ------------------------------------------------------------------ */

typedef struct { int64_t key; int64_t v; } orc_cand;

static int cmp_cand(const void *a, const void *b)
{
    const orc_cand *x = (const orc_cand *)a, *y = (const orc_cand *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->v != y->v) return x->v < y->v ? -1 : 1;
    return 0;
}

/*
 * Levels of Eq. (3) from `root`, computed one level at a time.  Level i+1 is
 * every unvisited neighbour of level i; it is numbered by the key defined in
 * the header.  Outputs: perm[new] = old, level_ptr[0..L] (level i occupies new
 * indices level_ptr[i] .. level_ptr[i+1]-1).  Returns L, or < 0 on error.
 */
int64_t orc_bfs_levels(int64_t n, const int64_t *rowptr, const int32_t *col,
                       int64_t root, int32_t *perm, int64_t *level_ptr)
{
    if (n == 0) { level_ptr[0] = 0; return 0; }
    if (n < 0 || root < 0 || root >= n) return -1;
    orc_transpose t;
    if (build_transpose(n, rowptr, col, &t)) return -2;
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *key = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    orc_cand *cand = (orc_cand *)malloc(sizeof(orc_cand) * (size_t)n);
    if (!pos || !key || !cand) return -2;
    for (int64_t i = 0; i < n; ++i) { pos[i] = -1; key[i] = -1; }

    int64_t assigned = 0, nl = 0, lo = 0, hi = 0, scan = 0;
    level_ptr[0] = 0;
    /* first level: the root */
    perm[0] = (int32_t)root;
    pos[root] = 0;
    assigned = 1;
    lo = 0; hi = 1;
    level_ptr[++nl] = 1;
    while (assigned < n) {
        int64_t m = 0;
        for (int64_t q = lo; q < hi; ++q) {
            int64_t u = perm[q];
            for (int side = 0; side < 2; ++side) {
                const int64_t *ptr = side ? t.tptr : rowptr;
                const int32_t *cc = side ? t.tcol : col;
                for (int64_t j = ptr[u]; j < ptr[u + 1]; ++j) {
                    int64_t v = cc[j];
                    if (pos[v] >= 0) continue;           /* already numbered */
                    if (key[v] < 0) {                    /* first sighting */
                        key[v] = q;
                        cand[m].key = q;
                        cand[m].v = v;
                        ++m;
                    }
                    /* later sightings come from larger q: key stays minimal */
                }
            }
        }
        if (m == 0) {
            /* new component: smallest unvisited original index */
            while (pos[scan] >= 0) ++scan;
            cand[0].key = 0;
            cand[0].v = scan;
            m = 1;
        }
        qsort(cand, (size_t)m, sizeof(orc_cand), cmp_cand);
        lo = assigned;
        for (int64_t i = 0; i < m; ++i) {
            perm[assigned] = (int32_t)cand[i].v;
            pos[cand[i].v] = assigned;
            ++assigned;
        }
        hi = assigned;
        level_ptr[++nl] = assigned;
    }
    free(pos);
    free(key);
    free(cand);
    free_transpose(&t);
    return nl;
}
