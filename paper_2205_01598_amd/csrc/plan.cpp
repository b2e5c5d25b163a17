// Host planner of the level-blocked MPK: CSR validation, the graph of
// A + A^T, BFS levels (Eq. 3) with level-by-level renumbering (Sec. 4.1),
// level groups under Eq. (5) (Sec. 4.3), the diagonal order of the Lp
// diagram (Sec. 4.2, Fig. 6), the renumbered matrix and the device tile
// table with point-to-point dependency ranges (Sec. 4.3).
//
// Everything here runs on the CPU; nothing touches the GPU.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <numeric>
#include <tuple>

#include <omp.h>

#include "mpk_internal.h"

namespace mpk {

namespace {
thread_local std::string g_err;
}

void set_error(const std::string &msg) { g_err = msg; }
mpk_status fail(mpk_status s, const std::string &msg) {
    g_err = msg;
    return s;
}
const char *last_error_cstr() { return g_err.c_str(); }

int32_t bytes_per_nnz(int32_t dtype) {
    switch (dtype) {
        case MPK_F32: return 8;
        case MPK_BF16: return 6;
        default: return 12;
    }
}

// Greedy chunks: a chunk starting at row r takes the most rows, at least
// one and at most max_rows, whose entries fit in max_nnz.  The end row is
// found by a binary search of the row pointers (non-decreasing).
template <typename RP>
static void append_chunks_t(const RP *rowptr, int64_t r0, int64_t r1, int64_t max_nnz, int64_t max_rows,
                            std::vector<int32_t> &out) {
    int64_t r = r0;
    while (r < r1) {
        out.push_back((int32_t)r);
        const int64_t lim = std::min<int64_t>(r1, r + max_rows);
        const int64_t target = (int64_t)rowptr[r] + max_nnz;
        const RP *e = std::upper_bound(rowptr + r + 1, rowptr + lim + 1, target,
                                       [](int64_t t, RP v) { return t < (int64_t)v; });
        r = std::max<int64_t>(r + 1, (e - rowptr) - 1);
    }
}

void append_chunks(const std::vector<int32_t> &rowptr, int64_t r0, int64_t r1, int64_t max_nnz,
                   int64_t max_rows, std::vector<int32_t> &out) {
    append_chunks_t(rowptr.data(), r0, r1, max_nnz, max_rows, out);
}

void append_chunks64(const int64_t *rowptr, int64_t r0, int64_t r1, int64_t max_nnz, int64_t max_rows,
                     std::vector<int32_t> &out) {
    append_chunks_t(rowptr, r0, r1, max_nnz, max_rows, out);
}

// Row boundaries (r0, ..., r1) of the device tiles of rows [r0, r1), one
// level group or refined unit.  A tile of at least one kernel chunk (cnz
// nonzeros) is a run of whole chunks: the rows are cut into chunks as the
// kernel cuts a tile, and the chunks are shared out equally among
// ceil(chunks / m) tiles, m = tile_nnz / cnz rounded; no tile then ends in
// a chunk of a few rows.  Smaller tiles share the nonzeros equally.
static std::vector<int64_t> tile_bounds(const std::vector<int32_t> &rowptr, int64_t r0, int64_t r1,
                                        int64_t tile_nnz, int64_t cnz) {
    std::vector<int64_t> bnd{r0};
    if (tile_nnz >= cnz) {
        std::vector<int32_t> ch;
        append_chunks(rowptr, r0, r1, cnz, kChunkRows, ch);
        const int64_t C = (int64_t)ch.size();
        const int64_t m = std::max<int64_t>((tile_nnz + cnz / 2) / cnz, 1);
        const int64_t nt = std::max<int64_t>(1, (C + m - 1) / m);
        for (int64_t t = 1; t < nt; ++t) bnd.push_back(ch[(size_t)(C * t / nt)]);
    } else {
        // equal-nonzero split into ceil(gnz / tile_nnz) tiles
        const int64_t gnz = rowptr[r1] - rowptr[r0];
        int64_t nt = std::max<int64_t>(1, (gnz + tile_nnz - 1) / tile_nnz);
        nt = std::min<int64_t>(nt, r1 - r0);
        for (int64_t t = 1; t < nt; ++t) {
            const int64_t target = rowptr[r0] + (gnz * t) / nt;
            const int64_t lo = bnd.back() + 1, hi = r1 - (nt - t);
            const int64_t a =
                std::lower_bound(rowptr.begin() + lo, rowptr.begin() + hi + 1, (int32_t)target) - rowptr.begin();
            bnd.push_back(std::min<int64_t>(std::max<int64_t>(a, lo), hi));
        }
    }
    bnd.push_back(r1);
    return bnd;
}

mpk_status validate_csr(const mpk_csr *A) {
    if (!A) return fail(MPK_ERR_ARG, "null matrix");
    if (A->n < 0) return fail(MPK_ERR_CSR, "negative n");
    if (A->n > (int64_t)std::numeric_limits<int32_t>::max() - 1)
        return fail(MPK_ERR_UNSUPPORTED, "n >= 2^31 is not supported");
    if (A->nnz < 0) return fail(MPK_ERR_CSR, "negative nnz");
    if (A->nnz > (int64_t)std::numeric_limits<int32_t>::max())
        return fail(MPK_ERR_UNSUPPORTED, "nnz >= 2^31 is not supported");
    if (!A->rowptr) return fail(MPK_ERR_ARG, "null rowptr");
    if (A->nnz > 0 && (!A->col || !A->val)) return fail(MPK_ERR_ARG, "null col/val");
    if (A->rowptr[0] != 0) return fail(MPK_ERR_CSR, "rowptr[0] != 0");
    for (int64_t i = 0; i < A->n; ++i)
        if (A->rowptr[i + 1] < A->rowptr[i]) return fail(MPK_ERR_CSR, "rowptr not monotone");
    if (A->rowptr[A->n] != A->nnz) return fail(MPK_ERR_CSR, "rowptr[n] != nnz");
    const int64_t n = A->n;
    for (int64_t j = 0; j < A->nnz; ++j)
        if (A->col[j] < 0 || A->col[j] >= n) return fail(MPK_ERR_CSR, "column index out of range");
    return MPK_OK;
}

namespace {

// Undirected graph of A: u ~ v (u != v) iff A_uv or A_vu is stored.
// Neighbour lists are sorted ascending and free of duplicates.
struct Graph {
    std::vector<int64_t> ptr;
    std::vector<int32_t> adj;
    int64_t deg(int64_t u) const { return ptr[u + 1] - ptr[u]; }
};

// Undirected graph of the pattern of A + A^T without the diagonal; every
// adjacency list ascending and free of duplicates.  A pattern that is already
// symmetric (checked by binary search, rows sorted) is taken as is; otherwise
// the transpose is formed and merged with A.
void build_graph(const mpk_csr *A, Graph &g) {
    const int64_t n = A->n;
    const int64_t *rp = A->rowptr;
    const int32_t *ci = A->col;
    bool sorted = true;
#pragma omp parallel for schedule(dynamic, 8192) reduction(&& : sorted)
    for (int64_t u = 0; u < n; ++u) sorted = sorted && std::is_sorted(ci + rp[u], ci + rp[u + 1]);
    bool symmetric = sorted;
    if (sorted) {
#pragma omp parallel for schedule(dynamic, 8192) reduction(&& : symmetric)
        for (int64_t u = 0; u < n; ++u) {
            if (!symmetric) continue;
            for (int64_t j = rp[u]; j < rp[u + 1]; ++j) {
                const int32_t v = ci[j];
                if (v == u) continue;
                if (!std::binary_search(ci + rp[v], ci + rp[v + 1], (int32_t)u)) {
                    symmetric = false;
                    break;
                }
            }
        }
    }
    std::vector<int64_t> len(n, 0);
    g.ptr.assign(n + 1, 0);
    if (symmetric) {
        auto emit = [&](int64_t u, int32_t *o) {
            int64_t m = 0, last = -1;
            for (int64_t j = rp[u]; j < rp[u + 1]; ++j) {
                const int32_t v = ci[j];
                if (v == u || v == last) continue;
                if (o) o[m] = v;
                ++m;
                last = v;
            }
            return m;
        };
#pragma omp parallel for schedule(dynamic, 8192)
        for (int64_t u = 0; u < n; ++u) len[u] = emit(u, nullptr);
        for (int64_t u = 0; u < n; ++u) g.ptr[u + 1] = g.ptr[u] + len[u];
        g.adj.resize(std::max<int64_t>(g.ptr[n], 1));
#pragma omp parallel for schedule(dynamic, 8192)
        for (int64_t u = 0; u < n; ++u) emit(u, g.adj.data() + g.ptr[u]);
        return;
    }
    // transpose by counting sort; each thread owns a range of columns and
    // walks the rows in order, so every transposed row comes out sorted
    std::vector<int64_t> tptr(n + 1, 0);
    std::vector<int32_t> tadj(std::max<int64_t>(A->nnz, 1));
#pragma omp parallel
    {
        const int T = omp_get_num_threads(), t = omp_get_thread_num();
        const int64_t c0 = n * t / T, c1 = n * (t + 1) / T;
        for (int64_t j = 0; j < A->nnz; ++j)
            if (ci[j] >= c0 && ci[j] < c1) tptr[ci[j] + 1]++;
#pragma omp barrier
#pragma omp single
        for (int64_t i = 0; i < n; ++i) tptr[i + 1] += tptr[i];
        std::vector<int64_t> pos(tptr.begin() + c0, tptr.begin() + c1);
        for (int64_t r = 0; r < n; ++r)
            for (int64_t j = rp[r]; j < rp[r + 1]; ++j) {
                const int32_t c = ci[j];
                if (c >= c0 && c < c1) tadj[pos[c - c0]++] = (int32_t)r;
            }
    }
    // merge row u of A (sorted copy where needed) with row u of A^T
    std::vector<int64_t> ub(n + 1, 0);
    for (int64_t u = 0; u < n; ++u) ub[u + 1] = ub[u] + (rp[u + 1] - rp[u]) + (tptr[u + 1] - tptr[u]);
    std::vector<int32_t> tmp(std::max<int64_t>(ub[n], 1));
#pragma omp parallel
    {
        std::vector<int32_t> rb;
#pragma omp for schedule(dynamic, 4096)
        for (int64_t u = 0; u < n; ++u) {
            const int32_t *ra = ci + rp[u];
            int64_t na = rp[u + 1] - rp[u];
            if (!std::is_sorted(ra, ra + na)) {
                rb.assign(ra, ra + na);
                std::sort(rb.begin(), rb.end());
                ra = rb.data();
            }
            const int32_t *rt = tadj.data() + tptr[u];
            int64_t nt = tptr[u + 1] - tptr[u];
            int32_t *o = tmp.data() + ub[u];
            int64_t a = 0, b = 0, m = 0;
            int64_t last = -1;
            while (a < na || b < nt) {
                int32_t v;
                if (b >= nt || (a < na && ra[a] <= rt[b])) v = ra[a++];
                else v = rt[b++];
                if (v == u || v == last) continue;
                o[m++] = v;
                last = v;
            }
            len[u] = m;
        }
    }
    for (int64_t u = 0; u < n; ++u) g.ptr[u + 1] = g.ptr[u] + len[u];
    g.adj.resize(std::max<int64_t>(g.ptr[n], 1));
#pragma omp parallel for schedule(static)
    for (int64_t u = 0; u < n; ++u)
        std::memcpy(g.adj.data() + g.ptr[u], tmp.data() + ub[u], sizeof(int32_t) * len[u]);
}

// Breadth-first levels of one component (Eq. 3) in Cuthill-McKee discovery
// order: each vertex of level i, taken in new order, appends its not yet
// numbered neighbours in ascending original index.  `order` receives the
// component from position `start` on; `owner[v]` must be INT32_MAX for every
// vertex not yet numbered and holds a position below `start` otherwise.
// Level boundaries are appended to `lptr` (the first entry, `start`, is the
// caller's).  Returns the position after the component.
//
// A large frontier is expanded in parallel with the same result as the
// queue: owner[v] = smallest frontier position adjacent to v (atomic
// minimum), then each frontier vertex writes the neighbours it owns, in
// adjacency order, at the prefix sum of the owned counts.
constexpr int64_t kParallelFrontier = 2048;

int64_t bfs_component(const Graph &g, int64_t root, int64_t start, std::vector<int32_t> &order,
                      std::vector<int32_t> &owner, std::vector<int32_t> &lptr, std::vector<int64_t> &cnt) {
    order[start] = (int32_t)root;
    owner[root] = -1;
    int64_t a = start, b = start + 1;
    while (a < b) {
        int64_t tail = b;
        const int64_t F = b - a;
        if (F < kParallelFrontier) {
            for (int64_t f = a; f < b; ++f) {
                const int32_t u = order[f];
                for (int64_t j = g.ptr[u]; j < g.ptr[u + 1]; ++j) {
                    const int32_t v = g.adj[j];
                    if (owner[v] == INT32_MAX) {
                        owner[v] = (int32_t)f;
                        order[tail++] = v;
                    }
                }
            }
        } else {
            if ((int64_t)cnt.size() < F + 1) cnt.resize(F + 1);
            int32_t *own = owner.data();
#pragma omp parallel for schedule(dynamic, 256)
            for (int64_t f = a; f < b; ++f) {
                const int32_t u = order[f];
                for (int64_t j = g.ptr[u]; j < g.ptr[u + 1]; ++j) {
                    int32_t *w = own + g.adj[j];
                    int32_t cur = __atomic_load_n(w, __ATOMIC_RELAXED);
                    while (cur > (int32_t)f &&
                           !__atomic_compare_exchange_n(w, &cur, (int32_t)f, true, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) {
                    }
                }
            }
#pragma omp parallel for schedule(dynamic, 256)
            for (int64_t f = a; f < b; ++f) {
                const int32_t u = order[f];
                int64_t c = 0;
                for (int64_t j = g.ptr[u]; j < g.ptr[u + 1]; ++j) c += owner[g.adj[j]] == (int32_t)f;
                cnt[f - a + 1] = c;
            }
            cnt[0] = 0;
            for (int64_t i = 0; i < F; ++i) cnt[i + 1] += cnt[i];
#pragma omp parallel for schedule(dynamic, 256)
            for (int64_t f = a; f < b; ++f) {
                const int32_t u = order[f];
                int64_t o = b + cnt[f - a];
                for (int64_t j = g.ptr[u]; j < g.ptr[u + 1]; ++j) {
                    const int32_t v = g.adj[j];
                    if (owner[v] == (int32_t)f) order[o++] = v;
                }
            }
            tail = b + cnt[F];
        }
        lptr.push_back((int32_t)b);
        a = b;
        b = tail;
    }
    return a;
}

// Every further component from its smallest unnumbered original index, at
// the next level, after the components already numbered up to `pos`.
void remaining_components(const Graph &g, int64_t n, int64_t pos, std::vector<int32_t> &perm,
                          std::vector<int32_t> &owner, std::vector<int32_t> &level_ptr, std::vector<int64_t> &cnt) {
    int64_t scan = 0;
    while (pos < n) {
        while (owner[scan] != INT32_MAX) ++scan;
        pos = bfs_component(g, scan, pos, perm, owner, level_ptr, cnt);
    }
}

// George-Liu pseudo-peripheral search from `start` (move to the
// smallest-degree vertex, lowest index on ties, of the farthest level while
// that raises the eccentricity), then the levels of the whole graph from
// that root.  The search's sweep from the chosen root is its component's
// levels already (the same expansion from the same state): it is kept, and
// a candidate's sweep that does not raise the eccentricity is dropped.
void peripheral_levels(const Graph &g, int64_t n, int64_t start, int64_t *root_out, std::vector<int32_t> &perm,
                       std::vector<int32_t> &level_ptr) {
    perm.assign(n, 0);
    level_ptr.assign(1, 0);
    *root_out = 0;
    if (n == 0) return;
    std::vector<int32_t> owner(n), order2(n), owner2(n), lptr2;
    std::vector<int64_t> cnt;
    auto sweep = [&](int64_t r, std::vector<int32_t> &order, std::vector<int32_t> &own, std::vector<int32_t> &lp) {
        std::fill(own.begin(), own.end(), INT32_MAX);
        lp.assign(1, 0);
        bfs_component(g, r, 0, order, own, lp, cnt);
        return (int64_t)lp.size() - 2;  // eccentricity = levels - 1
    };
    int64_t r = start;
    int64_t ecc = sweep(r, perm, owner, level_ptr);
    for (;;) {
        int64_t best = -1, bestdeg = 0;
        for (int64_t i = level_ptr[level_ptr.size() - 2]; i < level_ptr.back(); ++i) {
            const int64_t v = perm[i], d = g.deg(v);
            if (best < 0 || d < bestdeg || (d == bestdeg && v < best)) {
                best = v;
                bestdeg = d;
            }
        }
        const int64_t e2 = sweep(best, order2, owner2, lptr2);
        if (e2 <= ecc) break;
        r = best;
        ecc = e2;
        perm.swap(order2);
        owner.swap(owner2);
        level_ptr.swap(lptr2);
    }
    *root_out = r;
    remaining_components(g, n, level_ptr.back(), perm, owner, level_ptr, cnt);
}

// Levels of the whole graph: the root's component first, then each further
// component from its smallest unnumbered original index, at the next level.
void bfs_levels(const Graph &g, int64_t n, int64_t root, std::vector<int32_t> &perm,
                std::vector<int32_t> &level_ptr) {
    perm.assign(n, 0);
    level_ptr.assign(1, 0);
    if (n == 0) return;
    std::vector<int32_t> owner(n, INT32_MAX);
    std::vector<int64_t> cnt;
    const int64_t pos = bfs_component(g, root, 0, perm, owner, level_ptr, cnt);
    remaining_components(g, n, pos, perm, owner, level_ptr, cnt);
}

// ---------------------------------------------------------------------------
// Recursive level refinement (Sec. 4.4)
// ---------------------------------------------------------------------------

// Eq. (5) test for a set of rows: (p+1) * bytes < floor(f*C), bytes = nonzeros
// times b_nz (plus the k vector entries per row with budget_vectors).
struct Eq5 {
    int64_t p, bnz, nrhs;
    bool vectors;
    uint64_t budget;
    bool fits(int64_t nz, int64_t rows) const {
        unsigned __int128 per = (unsigned __int128)nz * (uint64_t)bnz;
        if (vectors) per += (unsigned __int128)rows * 8u * (uint64_t)nrhs;
        return per * (uint64_t)(p + 1) < (unsigned __int128)budget;
    }
};

// Greedy level groups of Eq. (5) over levels [lptr[l], lptr[l+1]) of `rows`.
std::vector<int64_t> eq5_groups(const std::vector<int32_t> &rows, const std::vector<int64_t> &lptr,
                                const int64_t *rowlen, const Eq5 &eq, std::vector<int64_t> &gnz,
                                std::vector<int64_t> &grows) {
    const int64_t L = (int64_t)lptr.size() - 1;
    std::vector<int64_t> lnz(L, 0);
    for (int64_t l = 0; l < L; ++l)
        for (int64_t r = lptr[l]; r < lptr[l + 1]; ++r) lnz[l] += rowlen[rows[r]];
    std::vector<int64_t> gptr{0};
    gnz.clear();
    grows.clear();
    for (int64_t l = 0; l < L;) {
        int64_t nz = lnz[l], nr = lptr[l + 1] - lptr[l], e = l + 1;
        while (e < L && eq.fits(nz + lnz[e], nr + (lptr[e + 1] - lptr[e]))) {
            nz += lnz[e];
            nr += lptr[e + 1] - lptr[e];
            ++e;
        }
        gptr.push_back(e);
        gnz.push_back(nz);
        grows.push_back(nr);
        l = e;
    }
    return gptr;
}

struct Refiner {
    const Graph &g;
    const int64_t *rowlen;
    const std::vector<int32_t> &pos;  // position of every vertex in the stage-0 numbering
    Eq5 eq;
    int stages;
    std::vector<uint8_t> inside, seen;
    std::vector<int32_t> order;       // final numbering, built in order
    std::vector<int32_t> unit_rows, unit_stage;
    std::vector<int64_t> unit_key;

    // Breadth-first levels of the subgraph induced by `region` (listed in the
    // current numbering): root = its first row; every vertex, taken in the
    // new order, appends its unvisited neighbours inside the region in
    // ascending position; an empty frontier restarts at the first unvisited
    // row of the region.
    void sub_levels(const std::vector<int32_t> &region, std::vector<int32_t> &out, std::vector<int64_t> &lptr) {
        for (int32_t v : region) inside[v] = 1;
        out.clear();
        lptr.assign(1, 0);
        size_t scan = 0;
        std::vector<int32_t> nb;
        while (out.size() < region.size()) {
            while (seen[region[scan]]) ++scan;
            size_t a = out.size();
            out.push_back(region[scan]);
            seen[region[scan]] = 1;
            lptr.push_back((int64_t)out.size());
            while (a < out.size()) {
                const size_t b = out.size();
                for (size_t f = a; f < b; ++f) {
                    const int32_t u = out[f];
                    nb.clear();
                    for (int64_t j = g.ptr[u]; j < g.ptr[u + 1]; ++j) {
                        const int32_t v = g.adj[j];
                        if (inside[v] && !seen[v]) nb.push_back(v);
                    }
                    std::sort(nb.begin(), nb.end(), [&](int32_t x, int32_t y) { return pos[x] < pos[y]; });
                    for (int32_t v : nb) {
                        seen[v] = 1;
                        out.push_back(v);
                    }
                }
                if (out.size() > b) lptr.push_back((int64_t)out.size());
                a = b;
            }
        }
        for (int32_t v : region) inside[v] = 0, seen[v] = 0;
    }

    // levels [lptr] of `rows` at stage `stage`, occupying the wavefront key
    // range [key_lo, key_hi): group i gets [key_lo + (key_hi-key_lo) i / G, ...)
    void refine(const std::vector<int32_t> &rows, const std::vector<int64_t> &lptr, int stage, int64_t key_lo,
                int64_t key_hi) {
        std::vector<int64_t> gnz, grows;
        const std::vector<int64_t> gptr = eq5_groups(rows, lptr, rowlen, eq, gnz, grows);
        const int64_t G = (int64_t)gptr.size() - 1;
        auto key_at = [&](int64_t i) {
            return key_lo + (int64_t)(((__int128)(key_hi - key_lo) * i) / std::max<int64_t>(G, 1));
        };
        for (int64_t i = 0; i < G;) {
            if (stage >= stages || eq.fits(gnz[i], grows[i])) {
                for (int64_t r = lptr[gptr[i]]; r < lptr[gptr[i + 1]]; ++r) order.push_back(rows[r]);
                unit_rows.push_back((int32_t)(lptr[gptr[i + 1]] - lptr[gptr[i]]));
                unit_stage.push_back(stage);
                unit_key.push_back(key_at(i));
                ++i;
                continue;
            }
            int64_t j = i;
            while (j < G && !eq.fits(gnz[j], grows[j])) ++j;
            std::vector<int32_t> region(rows.begin() + lptr[gptr[i]], rows.begin() + lptr[gptr[j]]);
            std::vector<int32_t> sub;
            std::vector<int64_t> sub_lptr;
            sub_levels(region, sub, sub_lptr);
            refine(sub, sub_lptr, stage + 1, key_at(i), key_at(j));
            i = j;
        }
    }
};

// Ticket streams.  With S > 1 the tiles of each level group (of each unit of
// a refined plan) are cut into S consecutive slices (slice s = tiles whose
// position in the group falls in [s/S, (s+1)/S)); stream s holds the tickets
// of slice s in the order of hp.work.  A tile of a level reads the neighbour
// levels at about the same relative position, so its dependencies mostly
// stay in its own stream.  Every dependency is an earlier ticket of the
// whole order, and each stream keeps that order, so the earliest unfinished
// ticket is always at the head of its stream and can run.
void split_streams(HostPlan &hp, int S) {
    const int64_t T = (int64_t)hp.tile_group.size();
    const int64_t G = (int64_t)hp.group_tile.size() - 1;
    std::vector<int32_t> tile_stream(T, 0);
    if (S > 1)
        for (int64_t gi = 0; gi < G; ++gi) {
            const int64_t t0 = hp.group_tile[gi], nt = hp.group_tile[gi + 1] - t0;
            for (int64_t t = t0; t < t0 + nt; ++t) tile_stream[t] = (int32_t)(((t - t0) * S) / nt);
        }
    hp.stream_ptr.assign(S + 1, 0);
    for (int32_t w : hp.work) hp.stream_ptr[tile_stream[w >> 6] + 1]++;
    for (int sidx = 0; sidx < S; ++sidx) hp.stream_ptr[sidx + 1] += hp.stream_ptr[sidx];
    hp.work_streams.assign(hp.work.size(), 0);
    std::vector<int32_t> fill(hp.stream_ptr.begin(), hp.stream_ptr.end() - 1);
    for (int32_t w : hp.work) hp.work_streams[fill[tile_stream[w >> 6]]++] = w;
}

constexpr int64_t kKeyUnit = 1 << 24;  // wavefront key of one stage-0 level group
// Dependency ranges of a refined tile with at most this many tiles between
// them are merged (the tiles between are waited for too): a wait polls its
// ranges one after another, each costing a memory round trip, while a
// longer range costs only more flags in the same 64-flag loads.
constexpr int32_t kDepMergeGap = 31;

// Schedule of a refined plan: tiles inside the final groups ("units"),
// per-tile dependency lists (every tile holding a column the tile reads, and
// the tile itself, widened to whole 128-byte lines of an aligned N x k FP64
// slice; ranges less than kDepMergeGap + 2 tiles apart merged), and tickets ordered by a longest-path wavefront number of the
// (unit, power) nodes
//   wf(u, 1) = key(u),  wf(u, q) = max(key(u) + skew*K*(q-1), max_v wf(v, q-1) + 1)
// over the units v holding a dependency of a tile of u, K = kKeyUnit, then
// by power and tile.  Every dependency has a smaller wavefront number (or is
// the node's own earlier power), so the order is topological; for unrefined
// groups (key g*K) it is the order of the diagonal g + skew*q.
mpk_status build_recursive_schedule(HostPlan &hp, int32_t p, const mpk_options &opt) {
    const int64_t n = hp.n;
    int64_t tile_nnz = opt.tile_nnz > 0 ? opt.tile_nnz : 8192;
    const int64_t max_tile_rows = 1 << 14;
    hp.tile_nnz = (int32_t)tile_nnz;
    hp.tile_row.clear();
    hp.tile_group.clear();
    hp.group_tile.clear();
    const int64_t U = (int64_t)hp.unit_ptr.size() - 1;
    for (int64_t u = 0; u < U; ++u) {
        hp.group_tile.push_back((int32_t)hp.tile_group.size());
        const int64_t r0 = hp.unit_ptr[u], r1 = hp.unit_ptr[u + 1];
        const std::vector<int64_t> bnd = tile_bounds(hp.rowptr, r0, r1, tile_nnz, mpk_chunk_nnz(opt.nrhs));
        for (size_t t = 0; t + 1 < bnd.size(); ++t)
            for (int64_t r = bnd[t]; r < bnd[t + 1]; r += max_tile_rows) {
                hp.tile_row.push_back((int32_t)r);
                hp.tile_group.push_back((int32_t)u);
            }
    }
    hp.group_tile.push_back((int32_t)hp.tile_group.size());
    hp.tile_row.push_back((int32_t)n);
    const int64_t T = (int64_t)hp.tile_group.size();
    if (T >= kMaxTiles) return fail(MPK_ERR_UNSUPPORTED, "too many tiles (2^25 or more): raise tile_nnz");

    // dependency lists
    std::vector<int32_t> row_tile(n);
    for (int64_t t = 0; t < T; ++t)
        for (int64_t r = hp.tile_row[t]; r < hp.tile_row[t + 1]; ++r) row_tile[r] = (int32_t)t;
    const int64_t Rl = std::max<int64_t>(1, 128 / (8 * (int64_t)opt.nrhs));
    std::vector<std::vector<int32_t>> ranges(T);
#pragma omp parallel
    {
        std::vector<int32_t> ts;
#pragma omp for schedule(dynamic, 16)
        for (int64_t t = 0; t < T; ++t) {
            ts.clear();
            ts.push_back((int32_t)t);
            for (int64_t j = hp.rowptr[hp.tile_row[t]]; j < hp.rowptr[hp.tile_row[t + 1]]; ++j)
                ts.push_back(row_tile[hp.col[j]]);
            std::sort(ts.begin(), ts.end());
            ts.erase(std::unique(ts.begin(), ts.end()), ts.end());
            std::vector<int32_t> &out = ranges[t];
            for (size_t a = 0; a < ts.size();) {
                size_t b = a;
                while (b + 1 < ts.size() && ts[b + 1] == ts[b] + 1) ++b;
                const int64_t f = hp.tile_row[ts[a]], l = hp.tile_row[ts[b] + 1] - 1;
                const int64_t f2 = f - f % Rl, l2 = std::min<int64_t>(n - 1, l + (Rl - 1 - l % Rl));
                const int32_t lo = row_tile[f2], hi = row_tile[l2];
                if (!out.empty() && lo <= out.back() + 1 + kDepMergeGap)
                    out.back() = std::max(out.back(), hi);
                else {
                    out.push_back(lo);
                    out.push_back(hi);
                }
                a = b + 1;
            }
        }
    }
    hp.dep_ptr.assign(T + 1, 0);
    for (int64_t t = 0; t < T; ++t) hp.dep_ptr[t + 1] = hp.dep_ptr[t] + (int32_t)(ranges[t].size() / 2);
    hp.dep_rng.resize(2 * (size_t)hp.dep_ptr[T]);
    hp.dep_lo.assign(T, 0);
    hp.dep_hi.assign(T, 0);
    for (int64_t t = 0; t < T; ++t) {
        std::copy(ranges[t].begin(), ranges[t].end(), hp.dep_rng.begin() + 2 * (size_t)hp.dep_ptr[t]);
        hp.dep_lo[t] = ranges[t].front();
        hp.dep_hi[t] = ranges[t].back();
    }
    // the three-range tables of unrefined plans: empty here
    hp.dep3.assign(6 * T, 0);
    for (int64_t t = 0; t < T; ++t)
        for (int m = 0; m < 3; ++m) hp.dep3[6 * t + 2 * m] = 1;
    hp.dep3x = hp.dep3;
    hp.line_closed_ok = true;

    // kernel chunks inside every tile
    hp.chunk_row.clear();
    hp.tile_chunk.assign(T + 1, 0);
    const int64_t cnz = mpk_chunk_nnz(opt.nrhs);
    for (int64_t t = 0; t < T; ++t) {
        hp.tile_chunk[t] = (int32_t)hp.chunk_row.size();
        append_chunks(hp.rowptr, hp.tile_row[t], hp.tile_row[t + 1], cnz, kChunkRows, hp.chunk_row);
    }
    hp.tile_chunk[T] = (int32_t)hp.chunk_row.size();
    hp.chunk_row.push_back((int32_t)n);

    // wavefront numbers per (unit, power) node, so the tiles of a node stay
    // contiguous in row order as in the unrefined ticket order
    const int64_t S = (int64_t)opt.skew * kKeyUnit;
    std::vector<int64_t> wf(U), wf_next(U);
    for (int64_t u = 0; u < U; ++u) wf[u] = hp.unit_key[u];
    std::vector<std::tuple<int64_t, int32_t, int32_t>> tk;
    tk.reserve((size_t)T * p);
    for (int64_t t = 0; t < T; ++t) tk.emplace_back(wf[hp.tile_group[t]], 1, (int32_t)t);
    for (int32_t q = 2; q <= p; ++q) {
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t u = 0; u < U; ++u) {
            int64_t w = hp.unit_key[u] + S * (q - 1);
            for (int32_t t = hp.group_tile[u]; t < hp.group_tile[u + 1]; ++t)
                for (int32_t k = hp.dep_ptr[t]; k < hp.dep_ptr[t + 1]; ++k) {
                    const int32_t g0 = hp.tile_group[hp.dep_rng[2 * k]], g1 = hp.tile_group[hp.dep_rng[2 * k + 1]];
                    for (int32_t g = g0; g <= g1; ++g) w = std::max(w, wf[g] + 1);
                }
            wf_next[u] = w;
        }
        wf.swap(wf_next);
        for (int64_t t = 0; t < T; ++t) tk.emplace_back(wf[hp.tile_group[t]], q, (int32_t)t);
    }
    std::sort(tk.begin(), tk.end());
    hp.work.clear();
    hp.work.reserve(tk.size());
    for (const auto &x : tk) hp.work.push_back(std::get<2>(x) * 64 + (std::get<1>(x) - 1));
    split_streams(hp, opt.xcd_streams);
    return MPK_OK;
}

}  // namespace

mpk_status build_schedule(HostPlan &hp, int32_t p, uint64_t cache_bytes, const mpk_options &opt) {
    if (p < 1 || p > MPK_MAX_POWER) return fail(MPK_ERR_ARG, "p must be in [1, 32]");
    if (cache_bytes == 0) return fail(MPK_ERR_ARG, "cache budget must be > 0");
    if (!(opt.safety_factor > 0.0)) return fail(MPK_ERR_ARG, "safety factor must be > 0");
    if (opt.nrhs < 1 || opt.nrhs > MPK_MAX_NRHS) return fail(MPK_ERR_ARG, "nrhs must be in [1, 32]");
    if (opt.val_dtype < MPK_F64 || opt.val_dtype > MPK_BF16) return fail(MPK_ERR_ARG, "bad val_dtype");
    if (opt.reserved0 != 0 || opt.reserved != 0) return fail(MPK_ERR_ARG, "reserved option fields must be 0");
    if (opt.accum_f64 != 0 && opt.accum_f64 != 1) return fail(MPK_ERR_ARG, "accum_f64 must be 0 or 1");
    if (opt.tile_nnz < 0 || opt.workgroups < 0) return fail(MPK_ERR_ARG, "negative launch option");
    if (opt.skew < 1 || opt.skew > MPK_MAX_SKEW) return fail(MPK_ERR_ARG, "skew must be in [1, 32]");
    if (opt.xcd_streams != 1 && opt.xcd_streams != 8) return fail(MPK_ERR_ARG, "xcd_streams must be 1 or 8");
    const int64_t n = hp.n;
    const int64_t L = (int64_t)hp.level_ptr.size() - 1;
    hp.p = p;
    hp.cache_bytes = cache_bytes;
    const int32_t root_mode = hp.opt.root_mode;
    hp.opt = opt;
    hp.opt.root_mode = root_mode;
    try {
        // ---- level groups, Eq. (5) ----------------------------------------------------
        const int64_t bnz = bytes_per_nnz(opt.val_dtype);
        const uint64_t budget = (uint64_t)std::floor(opt.safety_factor * (double)cache_bytes);
        auto group_bytes = [&](int64_t nz, int64_t rows) -> unsigned __int128 {
            unsigned __int128 per = (unsigned __int128)nz * (uint64_t)bnz;
            if (opt.budget_vectors) per += (unsigned __int128)rows * 8u * (uint64_t)opt.nrhs;
            return per * (uint64_t)(p + 1);
        };
        hp.group_ptr.clear();
        hp.group_ptr.push_back(0);
        hp.max_group_nnz = 0;
        hp.violating_groups = 0;
        for (int64_t l = 0; l < L;) {
            int64_t nz = hp.level_nnz[l];
            int64_t rows = hp.level_ptr[l + 1] - hp.level_ptr[l];
            int64_t e = l + 1;
            while (e < L) {
                int64_t nz2 = nz + hp.level_nnz[e];
                int64_t rows2 = rows + (hp.level_ptr[e + 1] - hp.level_ptr[e]);
                if (!(group_bytes(nz2, rows2) < (unsigned __int128)budget)) break;
                nz = nz2;
                rows = rows2;
                ++e;
            }
            if (!(group_bytes(nz, rows) < (unsigned __int128)budget)) hp.violating_groups++;
            hp.max_group_nnz = std::max(hp.max_group_nnz, nz);
            hp.group_ptr.push_back((int32_t)e);
            l = e;
        }
        const int64_t G = (int64_t)hp.group_ptr.size() - 1;

        // ---- Lp diagonal order, Fig. 6 ----------------------------------------------
        hp.schedule.clear();
        hp.schedule.reserve(3 * G * p);
        for (int64_t d = 1; d <= G + p - 1; ++d) {
            int64_t q0 = std::max<int64_t>(1, d - (G - 1)), q1 = std::min<int64_t>(d, p);
            for (int64_t q = q0; q <= q1; ++q) {
                hp.schedule.push_back((int32_t)d);
                hp.schedule.push_back((int32_t)q);
                hp.schedule.push_back((int32_t)(d - q));
            }
        }

        if (hp.recursive) return build_recursive_schedule(hp, p, opt);

        // ---- device tiles --------------------------------------------------------------
        int64_t tile_nnz = opt.tile_nnz;
        if (tile_nnz <= 0) tile_nnz = 8192;
        const int64_t max_tile_rows = 1 << 14;
        hp.tile_nnz = (int32_t)tile_nnz;
        hp.tile_row.clear();
        hp.tile_group.clear();
        hp.group_tile.clear();
        for (int64_t gi = 0; gi < G; ++gi) {
            hp.group_tile.push_back((int32_t)hp.tile_group.size());
            const int64_t r0 = hp.level_ptr[hp.group_ptr[gi]];
            const int64_t r1 = hp.level_ptr[hp.group_ptr[gi + 1]];
            const std::vector<int64_t> bnd = tile_bounds(hp.rowptr, r0, r1, tile_nnz, mpk_chunk_nnz(opt.nrhs));
            for (size_t t = 0; t + 1 < bnd.size(); ++t) {
                for (int64_t r = bnd[t]; r < bnd[t + 1]; r += max_tile_rows) {
                    hp.tile_row.push_back((int32_t)r);
                    hp.tile_group.push_back((int32_t)gi);
                }
            }
        }
        hp.group_tile.push_back((int32_t)hp.tile_group.size());
        hp.tile_row.push_back((int32_t)n);
        const int64_t T = (int64_t)hp.tile_group.size();
        if (T >= kMaxTiles) return fail(MPK_ERR_UNSUPPORTED, "too many tiles (2^25 or more): raise tile_nnz");

        // Point-to-point dependencies of each tile (Sec. 4.3).  By Eq. (4) a
        // tile of group g only reads rows of groups g-1, g and g+1.  For each
        // of the three groups the tile waits for the tiles spanning the
        // smallest and largest column it reads there; in its own group the
        // range also covers the tile itself.  dep_lo/dep_hi is the union.
        hp.dep_lo.assign(T, 0);
        hp.dep_hi.assign(T, 0);
        hp.dep3.assign(6 * T, 0);
        bool bad = false;
        auto tile_of = [&](int64_t row) -> int64_t {
            return std::upper_bound(hp.tile_row.begin(), hp.tile_row.end(), (int32_t)row) - hp.tile_row.begin() - 1;
        };
        // a matrix kept on the device: the column extremes per tile and
        // neighbouring group come from the device (same definition)
        std::vector<int32_t> dev_cols;
        if (hp.dev_col != nullptr) {
            std::vector<int32_t> group_row(G + 1);
            for (int64_t gi = 0; gi <= G; ++gi) group_row[gi] = hp.level_ptr[hp.group_ptr[gi]];
            mpk_status st = device_tile_columns(hp.dev_rowptr, hp.dev_col, hp.tile_row, hp.tile_group, group_row,
                                                dev_cols, &bad);
            if (st != MPK_OK) return st;
        }
#pragma omp parallel for schedule(dynamic, 16) reduction(|| : bad)
        for (int64_t t = 0; t < T; ++t) {
            const int64_t gi = hp.tile_group[t];
            const int64_t r0 = hp.tile_row[t], r1 = hp.tile_row[t + 1];
            int64_t lo[3], hi[3], gstart[3], gend[3];
            for (int m = 0; m < 3; ++m) {
                const int64_t gm = gi - 1 + m;
                lo[m] = std::numeric_limits<int64_t>::max();
                hi[m] = -1;
                gstart[m] = (gm >= 0 && gm < G) ? hp.level_ptr[hp.group_ptr[gm]] : 0;
                gend[m] = (gm >= 0 && gm < G) ? hp.level_ptr[hp.group_ptr[gm + 1]] : 0;
            }
            lo[1] = r0;
            hi[1] = r1 - 1;
            if (!dev_cols.empty()) {
                for (int m = 0; m < 3; ++m)
                    if (dev_cols[6 * t + 2 * m + 1] >= 0) {
                        lo[m] = std::min<int64_t>(lo[m], dev_cols[6 * t + 2 * m]);
                        hi[m] = std::max<int64_t>(hi[m], dev_cols[6 * t + 2 * m + 1]);
                    }
            } else {
                for (int64_t j = hp.rowptr[r0]; j < hp.rowptr[r1]; ++j) {
                    const int64_t c = hp.col[j];
                    int m = -1;
                    for (int mm = 0; mm < 3; ++mm)
                        if (c >= gstart[mm] && c < gend[mm]) m = mm;
                    if (m < 0) {
                        bad = true;
                        continue;
                    }
                    lo[m] = std::min(lo[m], c);
                    hi[m] = std::max(hi[m], c);
                }
            }
            int64_t all_lo = std::numeric_limits<int64_t>::max(), all_hi = -1;
            for (int m = 0; m < 3; ++m) {
                if (hi[m] < 0) {
                    hp.dep3[6 * t + 2 * m] = 1;
                    hp.dep3[6 * t + 2 * m + 1] = 0;
                    continue;
                }
                const int64_t tl = tile_of(lo[m]), th = tile_of(hi[m]);
                hp.dep3[6 * t + 2 * m] = (int32_t)tl;
                hp.dep3[6 * t + 2 * m + 1] = (int32_t)th;
                all_lo = std::min(all_lo, tl);
                all_hi = std::max(all_hi, th);
            }
            hp.dep_lo[t] = (int32_t)all_lo;
            hp.dep_hi[t] = (int32_t)all_hi;
        }
        if (bad) return fail(MPK_ERR_CSR, "internal: tile dependency crosses more than one level group");

        // Line-closed ranges, for runs without the acquire fence: every range
        // widened to whole 128-byte lines of an N x k FP64 vector slice whose
        // rows start on a line boundary (R rows per line), so a tile also
        // waits for every tile that shares a cache line with a row it reads or
        // writes; no line is then read before all its rows are final.  Valid
        // only if every widened dependency (u, q-1) is still an earlier ticket
        // than (t, q): group(u) <= g + skew.
        {
            const int64_t Rl = std::max<int64_t>(1, 128 / (8 * (int64_t)opt.nrhs));
            hp.dep3x.assign(6 * T, 0);
            bool closed_ok = true;
#pragma omp parallel for schedule(static) reduction(&& : closed_ok)
            for (int64_t t = 0; t < T; ++t) {
                for (int m = 0; m < 3; ++m) {
                    const int32_t lo = hp.dep3[6 * t + 2 * m], hi = hp.dep3[6 * t + 2 * m + 1];
                    if (lo > hi) {
                        hp.dep3x[6 * t + 2 * m] = lo;
                        hp.dep3x[6 * t + 2 * m + 1] = hi;
                        continue;
                    }
                    const int64_t f = hp.tile_row[lo], l = hp.tile_row[hi + 1] - 1;
                    const int64_t f2 = f - f % Rl, l2 = std::min<int64_t>(n - 1, l + (Rl - 1 - l % Rl));
                    const int64_t lo2 = tile_of(f2), hi2 = tile_of(l2);
                    hp.dep3x[6 * t + 2 * m] = (int32_t)lo2;
                    hp.dep3x[6 * t + 2 * m + 1] = (int32_t)hi2;
                    closed_ok = closed_ok && hp.tile_group[hi2] <= hp.tile_group[t] + opt.skew;
                }
            }
            hp.line_closed_ok = closed_ok;
        }

        // kernel chunks inside every tile
        hp.chunk_row.clear();
        hp.tile_chunk.assign(T + 1, 0);
        const int64_t cnz = mpk_chunk_nnz(opt.nrhs);
        for (int64_t t = 0; t < T; ++t) {
            hp.tile_chunk[t] = (int32_t)hp.chunk_row.size();
            append_chunks(hp.rowptr, hp.tile_row[t], hp.tile_row[t + 1], cnz, kChunkRows, hp.chunk_row);
        }
        hp.tile_chunk[T] = (int32_t)hp.chunk_row.size();
        hp.chunk_row.push_back((int32_t)n);

        // Tickets: the (group, power) nodes in the order of key g + skew*q,
        // ties by q (skew 1 is exactly the Lp diagonal order of Fig. 6), tiles
        // of a node in row order.  For any skew >= 1 the dependencies of a
        // node, (g-1..g+1, q-1), have a smaller key or, at skew 1, the same
        // key and a smaller q, so every ticket only waits for earlier ones.
        std::vector<std::pair<int64_t, int64_t>> nodes;  // (key * (p+1) + q, g)
        nodes.reserve(G * p);
        for (int64_t gi = 0; gi < G; ++gi)
            for (int64_t q = 1; q <= p; ++q) nodes.push_back({(gi + opt.skew * q) * (p + 1) + q, gi});
        std::sort(nodes.begin(), nodes.end());
        hp.work.clear();
        hp.work.reserve(T * p);
        for (const auto &nd : nodes) {
            const int32_t q = (int32_t)(nd.first % (p + 1)), gi = (int32_t)nd.second;
            for (int32_t t = hp.group_tile[gi]; t < hp.group_tile[gi + 1]; ++t) hp.work.push_back(t * 64 + (q - 1));
        }

        split_streams(hp, opt.xcd_streams);
    } catch (const std::bad_alloc &) {
        return fail(MPK_ERR_OOM, "host allocation failed while planning");
    }
    return MPK_OK;
}

void save_schedule(HostPlan &hp, ScheduleState &s) {
    s.p = hp.p;
    s.cache_bytes = hp.cache_bytes;
    s.opt = hp.opt;
    s.group_ptr = hp.group_ptr;
    s.schedule = hp.schedule;
    s.tile_row = hp.tile_row;
    s.tile_group = hp.tile_group;
    s.dep_lo = hp.dep_lo;
    s.dep_hi = hp.dep_hi;
    s.dep3 = hp.dep3;
    s.dep3x = hp.dep3x;
    s.line_closed_ok = hp.line_closed_ok;
    s.dep_ptr = hp.dep_ptr;
    s.dep_rng = hp.dep_rng;
    s.group_tile = hp.group_tile;
    s.work = hp.work;
    s.stream_ptr = hp.stream_ptr;
    s.work_streams = hp.work_streams;
    s.chunk_row = hp.chunk_row;
    s.tile_chunk = hp.tile_chunk;
    s.max_group_nnz = hp.max_group_nnz;
    s.violating_groups = hp.violating_groups;
    s.tile_nnz = hp.tile_nnz;
}

void restore_schedule(HostPlan &hp, ScheduleState &s) {
    hp.p = s.p;
    hp.cache_bytes = s.cache_bytes;
    hp.opt = s.opt;
    hp.group_ptr.swap(s.group_ptr);
    hp.schedule.swap(s.schedule);
    hp.tile_row.swap(s.tile_row);
    hp.tile_group.swap(s.tile_group);
    hp.dep_lo.swap(s.dep_lo);
    hp.dep_hi.swap(s.dep_hi);
    hp.dep3.swap(s.dep3);
    hp.dep3x.swap(s.dep3x);
    hp.line_closed_ok = s.line_closed_ok;
    hp.dep_ptr.swap(s.dep_ptr);
    hp.dep_rng.swap(s.dep_rng);
    hp.group_tile.swap(s.group_tile);
    hp.work.swap(s.work);
    hp.stream_ptr.swap(s.stream_ptr);
    hp.work_streams.swap(s.work_streams);
    hp.chunk_row.swap(s.chunk_row);
    hp.tile_chunk.swap(s.tile_chunk);
    hp.max_group_nnz = s.max_group_nnz;
    hp.violating_groups = s.violating_groups;
    hp.tile_nnz = s.tile_nnz;
}

void plan_features(const HostPlan &hp, double *f) {
    for (int i = 0; i < MPK_NUM_FEATURES; ++i) f[i] = 0.0;
    const int64_t n = hp.n, nnz = hp.nnz, L = (int64_t)hp.level_ptr.size() - 1;
    if (n <= 0) return;
    double mean = (double)nnz / (double)n, var = 0.0;
    int64_t mx = 0;
    for (int64_t r = 0; r < n; ++r) {
        const int64_t len = hp.rowptr[r + 1] - hp.rowptr[r];
        var += ((double)len - mean) * ((double)len - mean);
        mx = std::max(mx, len);
    }
    f[0] = std::log10((double)n);
    f[1] = std::log10((double)std::max<int64_t>(nnz, 1));
    f[2] = mean;
    f[3] = std::sqrt(var / (double)n);
    f[4] = std::log2((double)mx + 1.0);
    f[5] = std::log10((double)std::max<int64_t>(L, 1));
    f[6] = (double)hp.max_level_rows / (double)n;
    f[7] = std::log2((double)hp.p);
    // level-width histogram: fraction of levels with width/N in
    // [2^-(b+1), 2^-b), b = 0..15 (the last bin takes everything narrower)
    for (int64_t l = 0; l < L; ++l) {
        const double w = (double)(hp.level_ptr[l + 1] - hp.level_ptr[l]) / (double)n;
        int b = (int)std::floor(-std::log2(w));
        b = std::min(std::max(b, 0), 15);
        f[8 + b] += 1.0 / (double)L;
    }
}

namespace {

mpk_status check_create_options(int32_t p, uint64_t cache_bytes, const mpk_options &opt) {
    if (p < 1 || p > MPK_MAX_POWER) return fail(MPK_ERR_ARG, "p must be in [1, 32]");
    if (cache_bytes == 0) return fail(MPK_ERR_ARG, "cache budget must be > 0");
    if (!(opt.safety_factor > 0.0)) return fail(MPK_ERR_ARG, "safety factor must be > 0");
    if (opt.nrhs < 1 || opt.nrhs > MPK_MAX_NRHS) return fail(MPK_ERR_ARG, "nrhs must be in [1, 32]");
    if (opt.val_dtype < MPK_F64 || opt.val_dtype > MPK_BF16) return fail(MPK_ERR_ARG, "bad val_dtype");
    if (opt.root_mode < 0 || opt.root_mode > 1) return fail(MPK_ERR_ARG, "bad root_mode");
    if (opt.reserved0 != 0 || opt.reserved != 0) return fail(MPK_ERR_ARG, "reserved option fields must be 0");
    if (opt.accum_f64 != 0 && opt.accum_f64 != 1) return fail(MPK_ERR_ARG, "accum_f64 must be 0 or 1");
    if (opt.tile_nnz < 0 || opt.workgroups < 0) return fail(MPK_ERR_ARG, "negative launch option");
    if (opt.skew < 1 || opt.skew > MPK_MAX_SKEW) return fail(MPK_ERR_ARG, "skew must be in [1, 32]");
    if (opt.plan_on_device != 0 && opt.plan_on_device != 1) return fail(MPK_ERR_ARG, "plan_on_device must be 0 or 1");
    if (opt.force_acquire != 0 && opt.force_acquire != 1) return fail(MPK_ERR_ARG, "force_acquire must be 0 or 1");
    if (opt.recursion_stages < 0 || opt.recursion_stages > 16)
        return fail(MPK_ERR_ARG, "recursion_stages must be in [0, 16]");
    return MPK_OK;
}

// Nonzeros and widest level from the renumbered row pointers.
void level_counts(HostPlan &hp) {
    const int64_t L = (int64_t)hp.level_ptr.size() - 1;
    hp.level_nnz.assign(L, 0);
    hp.max_level_rows = 0;
    for (int64_t l = 0; l < L; ++l) {
        hp.level_nnz[l] = (int64_t)hp.rowptr[hp.level_ptr[l + 1]] - hp.rowptr[hp.level_ptr[l]];
        hp.max_level_rows = std::max<int64_t>(hp.max_level_rows, hp.level_ptr[l + 1] - hp.level_ptr[l]);
    }
}

}  // namespace

mpk_status build_resident_plan(const mpk_csr *A, int32_t p, uint64_t cache_bytes, const mpk_options &opt,
                               HostPlan &hp, ResidentMatrix *M) {
    auto t0 = std::chrono::steady_clock::now();
    if (!A) return fail(MPK_ERR_ARG, "null matrix");
    if (A->n < 0) return fail(MPK_ERR_CSR, "negative n");
    if (A->n > (int64_t)std::numeric_limits<int32_t>::max() - 1)
        return fail(MPK_ERR_UNSUPPORTED, "n >= 2^31 is not supported");
    if (A->nnz < 0) return fail(MPK_ERR_CSR, "negative nnz");
    if (A->nnz > (int64_t)std::numeric_limits<int32_t>::max())
        return fail(MPK_ERR_UNSUPPORTED, "nnz >= 2^31 is not supported");
    if (!A->rowptr) return fail(MPK_ERR_ARG, "null rowptr");
    if (A->nnz > 0 && (!A->col || !A->val)) return fail(MPK_ERR_ARG, "null col/val");
    mpk_status st = check_create_options(p, cache_bytes, opt);
    if (st != MPK_OK) return st;
    if (opt.recursion_stages != 0)
        return fail(MPK_ERR_UNSUPPORTED, "recursion (Sec. 4.4) refines on the host: plan from host memory");
    hp.n = A->n;
    hp.nnz = A->nnz;
    hp.p = p;
    hp.cache_bytes = cache_bytes;
    hp.opt = opt;
    hp.opt.plan_on_device = 1;
    st = device_plan_resident(A, opt.root_mode, &hp.root, hp.perm, hp.level_ptr, hp.rowptr, M, hp.phase_seconds);
    if (st != MPK_OK) return st;
    hp.dev_rowptr = M->rowptr;
    hp.dev_col = M->col;
    try {
        hp.iperm.resize(hp.n);
        int32_t *ip = hp.iperm.data();
        const int32_t *pm = hp.perm.data();
        const int64_t n = hp.n;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) ip[pm[i]] = (int32_t)i;  // perm is a permutation: distinct targets
        level_counts(hp);
    } catch (const std::bad_alloc &) {
        return fail(MPK_ERR_OOM, "host allocation failed while planning");
    }
    auto ts0 = std::chrono::steady_clock::now();
    st = build_schedule(hp, p, cache_bytes, opt);
    if (st != MPK_OK) return st;
    hp.phase_seconds[3] = std::chrono::duration<double>(std::chrono::steady_clock::now() - ts0).count();
    hp.plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return MPK_OK;
}

mpk_status build_host_plan(const mpk_csr *A, int32_t p, uint64_t cache_bytes,
                           const mpk_options &opt, HostPlan &hp) {
    auto t0 = std::chrono::steady_clock::now();
    mpk_status st = validate_csr(A);
    if (st != MPK_OK) return st;
    if ((st = check_create_options(p, cache_bytes, opt)) != MPK_OK) return st;

    const int64_t n = A->n;
    hp.n = n;
    hp.nnz = A->nnz;
    hp.p = p;
    hp.cache_bytes = cache_bytes;
    hp.opt = opt;

    try {
        // ---- graph, root, levels -------------------------------------------------
        auto now = [] { return std::chrono::steady_clock::now(); };
        auto secs = [](auto a, auto b) { return std::chrono::duration<double>(b - a).count(); };
        auto ta = now();
        // On the GPU: graph, levels and P A P^T for a sorted symmetric pattern;
        // otherwise the host builds the graph (and, on the GPU, only the levels).
        bool on_device = false;
        std::vector<int32_t> perm0;  // stage-0 numbering of a refined plan (its levels)
        if (opt.plan_on_device && opt.recursion_stages == 0) {
            st = device_plan(A, opt.root_mode, &hp.root, hp.perm, hp.level_ptr, hp.rowptr, hp.col, hp.val, &on_device,
                             hp.phase_seconds);
            if (st != MPK_OK) return st;
        }
        if (!on_device) {
            Graph g;
            build_graph(A, g);
            auto tb = now();
            hp.root = 0;
            if (opt.plan_on_device) {
                st = device_bfs_levels(n, g.ptr.data(), g.adj.data(), opt.root_mode, &hp.root, hp.perm, hp.level_ptr);
                if (st != MPK_OK) return st;
            } else {
                if (opt.root_mode == 1)
                    peripheral_levels(g, n, 0, &hp.root, hp.perm, hp.level_ptr);
                else
                    bfs_levels(g, n, hp.root, hp.perm, hp.level_ptr);
            }
            if (opt.recursion_stages > 0 && n > 0) {
                // Sec. 4.4: refine maximal runs of groups that violate Eq. (5)
                std::vector<int64_t> rowlen(n);
                for (int64_t i = 0; i < n; ++i) rowlen[i] = A->rowptr[i + 1] - A->rowptr[i];
                std::vector<int32_t> pos(n);
                for (int64_t i = 0; i < n; ++i) pos[hp.perm[i]] = (int32_t)i;
                Eq5 eq{p, bytes_per_nnz(opt.val_dtype), opt.nrhs, opt.budget_vectors != 0,
                       (uint64_t)std::floor(opt.safety_factor * (double)cache_bytes)};
                std::vector<int64_t> lp64(hp.level_ptr.begin(), hp.level_ptr.end());
                std::vector<int64_t> gnz, grows;
                const int64_t G0 = (int64_t)eq5_groups(hp.perm, lp64, rowlen.data(), eq, gnz, grows).size() - 1;
                Refiner rf{g, rowlen.data(), pos, eq, opt.recursion_stages, std::vector<uint8_t>(n, 0),
                           std::vector<uint8_t>(n, 0), {}, {}, {}, {}};
                rf.order.reserve(n);
                rf.refine(hp.perm, lp64, 0, 0, G0 * kKeyUnit);
                // with no group refined the plan is the unrefined one
                if (std::any_of(rf.unit_stage.begin(), rf.unit_stage.end(), [](int32_t s) { return s > 0; })) {
                    perm0.swap(hp.perm);
                    hp.perm.swap(rf.order);
                    hp.unit_ptr.assign(rf.unit_rows.size() + 1, 0);
                    for (size_t u = 0; u < rf.unit_rows.size(); ++u)
                        hp.unit_ptr[u + 1] = hp.unit_ptr[u] + rf.unit_rows[u];
                    hp.unit_stage = rf.unit_stage;
                    hp.unit_key = rf.unit_key;
                    hp.recursive = true;
                }
            }
            hp.phase_seconds[0] = secs(ta, tb);
            hp.phase_seconds[1] = secs(tb, now());
        }
        hp.iperm.assign(n, 0);
        for (int64_t i = 0; i < n; ++i) hp.iperm[hp.perm[i]] = (int32_t)i;
        const int64_t L = (int64_t)hp.level_ptr.size() - 1;

        // ---- nonzeros per level ------------------------------------------------------
        hp.level_nnz.assign(L, 0);
        hp.max_level_rows = 0;
        for (int64_t l = 0; l < L; ++l) {
            int64_t s = 0;
            for (int64_t r = hp.level_ptr[l]; r < hp.level_ptr[l + 1]; ++r) {
                int64_t o = hp.recursive ? perm0[r] : hp.perm[r];
                s += A->rowptr[o + 1] - A->rowptr[o];
            }
            hp.level_nnz[l] = s;
            hp.max_level_rows = std::max<int64_t>(hp.max_level_rows, hp.level_ptr[l + 1] - hp.level_ptr[l]);
        }

        auto tr0 = std::chrono::steady_clock::now();
        // ---- renumbered matrix P A P^T -------------------------------------------------
        if (!on_device) {
            hp.rowptr.assign(n + 1, 0);
            for (int64_t r = 0; r < n; ++r) {
                int64_t o = hp.perm[r];
                hp.rowptr[r + 1] = hp.rowptr[r] + (int32_t)(A->rowptr[o + 1] - A->rowptr[o]);
            }
            hp.col.resize(A->nnz);
            hp.val.resize(A->nnz);
#pragma omp parallel
            {
                std::vector<std::pair<int32_t, double>> buf;
#pragma omp for schedule(dynamic, 2048)
                for (int64_t r = 0; r < n; ++r) {
                    int64_t o = hp.perm[r];
                    int64_t a = A->rowptr[o], b = A->rowptr[o + 1];
                    buf.resize(b - a);
                    for (int64_t j = a; j < b; ++j) buf[j - a] = {hp.iperm[A->col[j]], A->val[j]};
                    std::stable_sort(buf.begin(), buf.end(),
                                     [](const auto &x, const auto &y) { return x.first < y.first; });
                    int64_t out = hp.rowptr[r];
                    for (size_t t = 0; t < buf.size(); ++t) {
                        hp.col[out + t] = buf[t].first;
                        hp.val[out + t] = buf[t].second;
                    }
                }
            }
            hp.phase_seconds[2] = std::chrono::duration<double>(std::chrono::steady_clock::now() - tr0).count();
        }
    } catch (const std::bad_alloc &) {
        return fail(MPK_ERR_OOM, "host allocation failed while planning");
    }
    auto ts0 = std::chrono::steady_clock::now();
    st = build_schedule(hp, p, cache_bytes, opt);
    if (st != MPK_OK) return st;
    hp.phase_seconds[3] = std::chrono::duration<double>(std::chrono::steady_clock::now() - ts0).count();
    hp.plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return MPK_OK;
}

}  // namespace mpk
