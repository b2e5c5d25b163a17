// Preprocessing on the GPU: graph of the pattern, breadth-first levels (Eq. 3)
// and the renumbered matrix, with the same results as the host planner.
//
// Levels come in the same Cuthill-McKee discovery order as on the host: each
// vertex of level i, taken in new order, numbers its not yet numbered
// neighbours in ascending original index.
//
// One level of the frontier order[a, b) is expanded by these kernels, the
// row-walking ones with a group of 32 lanes per frontier vertex:
//   claim        owner[v] = smallest frontier position adjacent to v (atomic
//                minimum; owner only ever decreases, so a read that is
//                already <= f makes the atomic unnecessary);
//   count_owned  every frontier vertex counts the neighbours it owns;
//   count        a workgroup scan of those counts gives each vertex's offset
//                inside its chunk of 256 frontier positions;
//   scan_blocks  one workgroup scans the chunk totals (the next frontier's
//                size), records the level and writes the next frontier;
//   scatter      every frontier vertex writes the neighbours it owns, in
//                row order, at b + its offset, and marks them seen.
// The frontier bounds live in device memory (Frontier), in two copies that
// alternate from level to level: the kernels of a level read the current
// one and scan_blocks writes the next, so the host enqueues levels in
// batches (1, 2, 4, ... up to 32) and reads the state back once per batch;
// levels enqueued after the component is exhausted do nothing.  An empty frontier with vertices left starts a new component at
// the smallest unnumbered index (a reduction), as a new level.  owner[v] is
// INT32_MAX for an unnumbered vertex and a position below the current
// frontier otherwise; a bitmap of numbered vertices lets the kernels skip
// the owner array for most neighbours.  For a sorted symmetric pattern the
// rows of A are the graph (diagonal and repeated entries skipped).
//
// The George-Liu pseudo-peripheral search runs component-restricted sweeps of
// the same expansion and picks the smallest-degree vertex of the last level
// (lowest index on ties) with a 64-bit atomic minimum of (degree, index).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cstdint>
#include <string>
#include <vector>

#include "mpk_internal.h"

namespace mpk {
namespace {

constexpr int kThreads = 256;

__global__ void fill_i32(int32_t *p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void set_root(int32_t *order, int32_t *owner, uint32_t *seen, int64_t pos, const int32_t *root) {
    const int32_t r = *root;
    order[pos] = r;
    owner[r] = -1;
    seen[r >> 5] |= 1u << (r & 31);
}

// seen[v / 32] bit v % 32: v is numbered (its owner is final).  The bitmap
// (n / 8 bytes) stays in the L2, so the expansion skips the owner array for
// the neighbours numbered in earlier levels, about two thirds of them.
__device__ __forceinline__ bool is_seen(const uint32_t *seen, int32_t v) { return (seen[v >> 5] >> (v & 31)) & 1u; }

// Frontier of the level expansion: order[a, b); next = size of this
// frontier's successor (set with it by scan_blocks); lv = levels recorded in
// the level-end array.
struct Frontier {
    int64_t a, b, next, lv;
};

// The expansion kernels give every frontier vertex a group of kLanes lanes
// (half a wavefront); lane l handles the entries l, l + kLanes, ... of the
// vertex's row, so a level's edges are handled in parallel rather than one
// row per thread.  A row is read as a graph row: the diagonal is skipped by
// the seen bit (the vertex is numbered), a repeated entry (equal to the one
// before it in the sorted row) is skipped explicitly.
constexpr int kLanes = 32;

// lanes of the calling lane's group that have pred set, as a 32-bit mask
__device__ __forceinline__ uint32_t group_ballot(bool pred) {
    const unsigned long long m = __ballot(pred);
    return (uint32_t)(m >> (threadIdx.x & 32));
}

// Grid-stride over (frontier vertex, lane) slots: f = a + slot / kLanes.
#define FOR_FRONTIER_SLOTS(a, b)                                                                          \
    for (int64_t slot = blockIdx.x * (int64_t)kThreads + threadIdx.x; slot < ((b) - (a)) * kLanes;       \
         slot += (int64_t)gridDim.x * kThreads)

__global__ void claim(const int64_t *__restrict__ ptr, const int32_t *__restrict__ adj,
                      const int32_t *__restrict__ order, const Frontier *__restrict__ fr, int32_t *owner,
                      const uint32_t *__restrict__ seen) {
    const int64_t a = fr->a, b = fr->b;
    FOR_FRONTIER_SLOTS(a, b) {
        const int64_t f = a + slot / kLanes;
        const int32_t u = order[f];
        for (int64_t j = ptr[u] + (slot & (kLanes - 1)); j < ptr[u + 1]; j += kLanes) {
            const int32_t v = adj[j];
            if (is_seen(seen, v)) continue;
            // owner only decreases: a plain read, even a stale one, that is
            // already <= f shows the atomic cannot lower it
            if (owner[v] > (int32_t)f) atomicMin(owner + v, (int32_t)f);
        }
    }
}

// per frontier vertex: the number of neighbours it owns, to cnt[f - a]
__global__ void count_owned(const int64_t *__restrict__ ptr, const int32_t *__restrict__ adj,
                            const int32_t *__restrict__ order, const int32_t *__restrict__ owner,
                            const Frontier *__restrict__ fr, int32_t *__restrict__ cnt,
                            const uint32_t *__restrict__ seen) {
    const int64_t a = fr->a, b = fr->b;
    FOR_FRONTIER_SLOTS(a, b) {
        const int64_t f = a + slot / kLanes;
        const int lane = (int)(slot & (kLanes - 1));
        const int32_t u = order[f];
        const int64_t j0 = ptr[u], j1 = ptr[u + 1];
        int32_t k = 0;
        for (int64_t base = j0; base < j1; base += kLanes) {  // uniform in the group
            const int64_t j = base + lane;
            bool own = false;
            if (j < j1) {
                const int32_t v = adj[j];
                own = (j == j0 || adj[j - 1] != v) && !is_seen(seen, v) && owner[v] == (int32_t)f;
            }
            k += __popc(group_ballot(own));
        }
        if (lane == 0) cnt[f - a] = k;
    }
}

// chunks of kThreads frontier positions: exclusive offset of every vertex
// inside its chunk in local[], chunk totals in blocksum[]
__global__ void count(const int32_t *__restrict__ cnt, const Frontier *__restrict__ fr, int32_t *__restrict__ local,
                      int32_t *__restrict__ blocksum) {
    __shared__ int32_t s[kThreads];
    const int64_t a = fr->a, b = fr->b;
    const int64_t nb = (b - a + kThreads - 1) / kThreads;
    for (int64_t c = blockIdx.x; c < nb; c += gridDim.x) {
        const int64_t f = a + c * kThreads + threadIdx.x;
        const int32_t k = f < b ? cnt[f - a] : 0;
        s[threadIdx.x] = k;
        __syncthreads();
        // inclusive Hillis-Steele scan over the chunk
        for (int d = 1; d < kThreads; d <<= 1) {
            const int32_t t = (int)threadIdx.x >= d ? s[threadIdx.x - d] : 0;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        if (f < b) local[f - a] = s[threadIdx.x] - k;
        if (threadIdx.x == kThreads - 1) blocksum[c] = s[kThreads - 1];
        __syncthreads();
    }
}

// one workgroup: exclusive scan of the chunk totals in place; then a
// non-empty frontier fr becomes a level (its end recorded) and the frontier
// after it goes to nx (an empty one is copied: nothing is left to expand)
__global__ void scan_blocks(int32_t *blocksum, const Frontier *fr, Frontier *nx, int32_t *level_end) {
    __shared__ int32_t s[kThreads];
    const int64_t nb = (fr->b - fr->a + kThreads - 1) / kThreads;
    int32_t carry = 0;
    for (int64_t base = 0; base < nb; base += kThreads) {
        const int64_t i = base + threadIdx.x;
        const int32_t v = i < nb ? blocksum[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int d = 1; d < kThreads; d <<= 1) {
            const int32_t t = (int)threadIdx.x >= d ? s[threadIdx.x - d] : 0;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nb) blocksum[i] = carry + s[threadIdx.x] - v;
        const int32_t step = s[kThreads - 1];
        __syncthreads();
        carry += step;
    }
    if (threadIdx.x == 0) {
        const int64_t a = fr->a, b = fr->b, lv = fr->lv;
        if (a >= b) {
            *nx = Frontier{a, b, 0, lv};
        } else {
            level_end[lv] = (int32_t)b;
            *nx = Frontier{b, b + carry, carry, lv + 1};
        }
    }
}

// Each frontier vertex writes the neighbours it owns, in row order, and
// marks them seen: a lane's place is the count of owning lanes before it in
// its group.  Another lane may read a bit (a plain, possibly stale read)
// while it is being set: either value leads it to skip the vertex, which it
// does not own.
__global__ void scatter(const int64_t *__restrict__ ptr, const int32_t *__restrict__ adj,
                        int32_t *__restrict__ order, const int32_t *__restrict__ owner,
                        const Frontier *__restrict__ fr, const int32_t *__restrict__ local,
                        const int32_t *__restrict__ blocksum, uint32_t *seen) {
    const int64_t a = fr->a, b = fr->b;
    FOR_FRONTIER_SLOTS(a, b) {
        const int64_t f = a + slot / kLanes;
        const int lane = (int)(slot & (kLanes - 1));
        const int32_t u = order[f];
        const int64_t j0 = ptr[u], j1 = ptr[u + 1];
        int64_t o = b + blocksum[(f - a) / kThreads] + local[f - a];
        for (int64_t base = j0; base < j1; base += kLanes) {  // uniform in the group
            const int64_t j = base + lane;
            bool own = false;
            int32_t v = 0;
            if (j < j1) {
                v = adj[j];
                own = (j == j0 || adj[j - 1] != v) && !is_seen(seen, v) && owner[v] == (int32_t)f;
            }
            const uint32_t m = group_ballot(own);
            if (own) {
                order[o + __popc(m & ((1u << lane) - 1u))] = v;
                atomicOr(seen + (v >> 5), 1u << (v & 31));
            }
            o += __popc(m);
        }
    }
}

// smallest index v with owner[v] == INT32_MAX (n if none)
__global__ void first_unnumbered(const int32_t *__restrict__ owner, int64_t n, int32_t *out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        if (owner[i] == INT32_MAX) {
            atomicMin(out, (int32_t)i);
            return;  // later indices of this thread are larger
        }
}

// (degree, index) minimum over order[a, b); the degree counts distinct
// neighbours other than the vertex itself, so the rows of a sorted
// symmetric A serve as the graph
__global__ void min_degree(const int64_t *__restrict__ ptr, const int32_t *__restrict__ adj,
                           const int32_t *__restrict__ order, int64_t a, int64_t b, unsigned long long *out) {
    const int64_t f = a + blockIdx.x * (int64_t)kThreads + threadIdx.x;
    if (f >= b) return;
    const int32_t v = order[f];
    int64_t deg = 0;
    int32_t last = -1;
    for (int64_t j = ptr[v]; j < ptr[v + 1]; ++j) {
        const int32_t w = adj[j];
        deg += w != v && w != last;
        last = w;
    }
    const unsigned long long key = ((unsigned long long)deg << 32) | (uint32_t)v;
    atomicMin(out, key);
}

struct DeviceGraph {
    int64_t n = 0;
    int64_t *ptr = nullptr;
    int32_t *adj = nullptr, *owner = nullptr, *order = nullptr, *local = nullptr, *blocksum = nullptr,
            *scalar = nullptr, *level_end = nullptr, *cnt = nullptr;
    uint32_t *seen = nullptr, *bk_seen = nullptr;
    int32_t *bk_order = nullptr, *bk_owner = nullptr;  // the root's sweep while a candidate is tried
    Frontier *front = nullptr;
    unsigned long long *key = nullptr;
    std::vector<void *> allocs;
    ~DeviceGraph() {
        for (void *p : allocs) (void)hipFree(p);
    }
};

#define LV_TRY(expr)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return fail(e_ == hipErrorOutOfMemory ? MPK_ERR_OOM : MPK_ERR_HIP,                         \
                        std::string("device levels: ") + #expr + ": " + hipGetErrorString(e_));        \
    } while (0)

template <typename T>
hipError_t dalloc(DeviceGraph &g, T **p, int64_t count) {
    hipError_t e = hipMalloc((void **)p, sizeof(T) * (size_t)std::max<int64_t>(count, 1));
    if (e == hipSuccess) g.allocs.push_back(*p);
    return e;
}

inline unsigned grid_for(int64_t items) { return (unsigned)((items + kThreads - 1) / kThreads); }

// Expands levels from order[start, start+1) (the root already placed) until
// the component is exhausted; appends level ends to lptr.  Returns the
// position after the component in *end.
mpk_status expand_component(DeviceGraph &g, int64_t start, std::vector<int32_t> &lptr, int64_t *end) {
    Frontier h{start, start + 1, 0, 0};
    int cur = 0;  // which of the two frontier copies is current
    LV_TRY(hipMemcpy(g.front, &h, sizeof(h), hipMemcpyHostToDevice));
    // grids sized for the widest possible frontier, capped; slots beyond the
    // current frontier exit at once
    const unsigned nb = std::max(1u, std::min(grid_for(g.n), 1024u));
    const unsigned ne = std::max(1u, (unsigned)std::min<int64_t>((g.n * kLanes + kThreads - 1) / kThreads, 2048));
    for (int batch = 1;; batch = std::min(2 * batch, 32)) {
        for (int i = 0; i < batch; ++i) {
            const Frontier *fr = g.front + cur;
            hipLaunchKernelGGL(claim, dim3(ne), dim3(kThreads), 0, 0, g.ptr, g.adj, g.order, fr, g.owner, g.seen);
            hipLaunchKernelGGL(count_owned, dim3(ne), dim3(kThreads), 0, 0, g.ptr, g.adj, g.order, g.owner, fr,
                               g.cnt, g.seen);
            hipLaunchKernelGGL(count, dim3(nb), dim3(kThreads), 0, 0, g.cnt, fr, g.local, g.blocksum);
            hipLaunchKernelGGL(scan_blocks, dim3(1), dim3(kThreads), 0, 0, g.blocksum, fr, g.front + (cur ^ 1),
                               g.level_end);
            hipLaunchKernelGGL(scatter, dim3(ne), dim3(kThreads), 0, 0, g.ptr, g.adj, g.order, g.owner, fr, g.local,
                               g.blocksum, g.seen);
            cur ^= 1;
        }
        LV_TRY(hipGetLastError());
        LV_TRY(hipMemcpy(&h, g.front + cur, sizeof(h), hipMemcpyDeviceToHost));
        if (h.b > g.n || h.a > h.b || h.lv > g.n) return fail(MPK_ERR_HIP, "device levels: inconsistent frontier");
        if (h.a == h.b) break;
    }
    if (h.lv > 0) {
        const size_t base = lptr.size();
        lptr.resize(base + (size_t)h.lv);
        LV_TRY(hipMemcpy(lptr.data() + base, g.level_end, sizeof(int32_t) * h.lv, hipMemcpyDeviceToHost));
    }
    *end = h.a;
    return MPK_OK;
}

mpk_status place_root(DeviceGraph &g, int64_t pos, int32_t root) {
    LV_TRY(hipMemcpy(g.scalar, &root, sizeof(int32_t), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(set_root, dim3(1), dim3(1), 0, 0, g.order, g.owner, g.seen, pos, g.scalar);
    LV_TRY(hipGetLastError());
    return MPK_OK;
}

mpk_status reset_owner(DeviceGraph &g) {
    hipLaunchKernelGGL(fill_i32, dim3(1024), dim3(kThreads), 0, 0, g.owner, g.n, (int32_t)INT32_MAX);
    hipLaunchKernelGGL(fill_i32, dim3(256), dim3(kThreads), 0, 0, (int32_t *)g.seen, (g.n + 31) / 32, 0);
    LV_TRY(hipGetLastError());
    return MPK_OK;
}

}  // namespace

namespace {

// work buffers of the level expansion (the graph itself is set by the caller)
mpk_status alloc_bfs(DeviceGraph &g) {
    const int64_t n = g.n;
    LV_TRY(dalloc(g, &g.owner, n));
    LV_TRY(dalloc(g, &g.order, n));
    LV_TRY(dalloc(g, &g.local, n));
    LV_TRY(dalloc(g, &g.blocksum, (n + kThreads - 1) / kThreads));
    LV_TRY(dalloc(g, &g.scalar, 1));
    LV_TRY(dalloc(g, &g.key, 1));
    LV_TRY(dalloc(g, &g.level_end, n + 1));
    LV_TRY(dalloc(g, &g.cnt, n));
    LV_TRY(dalloc(g, &g.seen, (n + 31) / 32));
    LV_TRY(dalloc(g, &g.bk_seen, (n + 31) / 32));
    LV_TRY(dalloc(g, &g.bk_order, n));
    LV_TRY(dalloc(g, &g.bk_owner, n));
    LV_TRY(dalloc(g, &g.front, 2));
    return MPK_OK;
}

// root, levels and the new order (left in g.order) of the graph in g
mpk_status bfs_on_device(DeviceGraph &g, int32_t root_mode, int64_t *root_out, std::vector<int32_t> &level_ptr) {
    const int64_t n = g.n;

    // ---- root: vertex 0, or George-Liu from vertex 0 -------------------------------
    int32_t root = 0;
    std::vector<int32_t> lp_root;  // level ends of the root's component (search sweeps)
    if (root_mode == 1) {
        std::vector<int32_t> lp;
        auto sweep = [&](int32_t r, int64_t *ecc) -> mpk_status {
            mpk_status st;
            if ((st = reset_owner(g)) != MPK_OK) return st;
            if ((st = place_root(g, 0, r)) != MPK_OK) return st;
            lp.assign(1, 0);
            int64_t end = 0;
            if ((st = expand_component(g, 0, lp, &end)) != MPK_OK) return st;
            *ecc = (int64_t)lp.size() - 2;
            return MPK_OK;
        };
        int64_t ecc = 0;
        mpk_status st = sweep(root, &ecc);
        if (st != MPK_OK) return st;
        lp_root = lp;
        for (;;) {
            const unsigned long long init = ~0ull;
            LV_TRY(hipMemcpy(g.key, &init, sizeof(init), hipMemcpyHostToDevice));
            const int64_t a = lp[lp.size() - 2], b = lp.back();
            hipLaunchKernelGGL(min_degree, dim3(grid_for(b - a)), dim3(kThreads), 0, 0, g.ptr, g.adj, g.order, a, b,
                               g.key);
            LV_TRY(hipGetLastError());
            unsigned long long key = 0;
            LV_TRY(hipMemcpy(&key, g.key, sizeof(key), hipMemcpyDeviceToHost));
            const int32_t cand = (int32_t)(key & 0xffffffffu);
            // the root's sweep is kept: a candidate that is no better is
            // undone instead of sweeping from the root once more
            LV_TRY(hipMemcpyAsync(g.bk_order, g.order, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, 0));
            LV_TRY(hipMemcpyAsync(g.bk_owner, g.owner, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, 0));
            LV_TRY(hipMemcpyAsync(g.bk_seen, g.seen, sizeof(uint32_t) * ((n + 31) / 32), hipMemcpyDeviceToDevice,
                                  0));
            int64_t e2 = 0;
            if ((st = sweep(cand, &e2)) != MPK_OK) return st;
            if (e2 > ecc) {
                root = cand;
                ecc = e2;
                lp_root = lp;
            } else {
                LV_TRY(hipMemcpyAsync(g.order, g.bk_order, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, 0));
                LV_TRY(hipMemcpyAsync(g.owner, g.bk_owner, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, 0));
                LV_TRY(hipMemcpyAsync(g.seen, g.bk_seen, sizeof(uint32_t) * ((n + 31) / 32),
                                      hipMemcpyDeviceToDevice, 0));
                break;
            }
        }
    }
    *root_out = root;

    // ---- levels of the whole graph: root's component, then the others --------------
    mpk_status st;
    int64_t pos = 0;
    if (root_mode == 1) {
        // the root's component is numbered already, by the search's sweep
        // from it (the same expansion from the same state)
        level_ptr.insert(level_ptr.end(), lp_root.begin() + 1, lp_root.end());
        pos = lp_root.back();
    } else {
        if ((st = reset_owner(g)) != MPK_OK) return st;
        if ((st = place_root(g, 0, root)) != MPK_OK) return st;
        if ((st = expand_component(g, 0, level_ptr, &pos)) != MPK_OK) return st;
    }
    while (pos < n) {
        const int32_t none = (int32_t)n;
        LV_TRY(hipMemcpy(g.scalar, &none, sizeof(int32_t), hipMemcpyHostToDevice));
        hipLaunchKernelGGL(first_unnumbered, dim3(1024), dim3(kThreads), 0, 0, g.owner, n, g.scalar);
        LV_TRY(hipGetLastError());
        int32_t next_root = 0;
        LV_TRY(hipMemcpy(&next_root, g.scalar, sizeof(int32_t), hipMemcpyDeviceToHost));
        if (next_root < 0 || next_root >= n) return fail(MPK_ERR_HIP, "device levels: lost vertices");
        if ((st = place_root(g, pos, next_root)) != MPK_OK) return st;
        if ((st = expand_component(g, pos, level_ptr, &pos)) != MPK_OK) return st;
    }
    return MPK_OK;
}

}  // namespace

mpk_status device_bfs_levels(int64_t n, const int64_t *ptr, const int32_t *adj, int32_t root_mode, int64_t *root_out,
                             std::vector<int32_t> &perm, std::vector<int32_t> &level_ptr) {
    perm.assign(n, 0);
    level_ptr.assign(1, 0);
    *root_out = 0;
    if (n == 0) return MPK_OK;
    DeviceGraph g;
    g.n = n;
    const int64_t m = ptr[n];
    LV_TRY(dalloc(g, &g.ptr, n + 1));
    LV_TRY(dalloc(g, &g.adj, m));
    mpk_status st = alloc_bfs(g);
    if (st != MPK_OK) return st;
    LV_TRY(hipMemcpy(g.ptr, ptr, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice));
    if (m > 0) LV_TRY(hipMemcpy(g.adj, adj, sizeof(int32_t) * m, hipMemcpyHostToDevice));
    if ((st = bfs_on_device(g, root_mode, root_out, level_ptr)) != MPK_OK) return st;
    LV_TRY(hipMemcpy(perm.data(), g.order, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    return MPK_OK;
}

// ---------------------------------------------------------------------------
// graph and renumbering
// ---------------------------------------------------------------------------

namespace {

constexpr int64_t kSortOnDevice = 256;  // rows up to this length are sorted by one thread
constexpr int kSortInRegisters = 32;    // rows up to this length are sorted in its registers

__global__ void rows_sorted(const int64_t *__restrict__ rp, const int32_t *__restrict__ col, int64_t n, int32_t *ok) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x)
        for (int64_t j = rp[u] + 1; j < rp[u + 1]; ++j)
            if (col[j] < col[j - 1]) {
                atomicMin(ok, 0);
                break;
            }
}

// every stored (u, v), v != u, has a stored (v, u) (rows sorted)
__global__ void pattern_symmetric(const int64_t *__restrict__ rp, const int32_t *__restrict__ col, int64_t n,
                                  int32_t *ok) {
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        for (int64_t j = rp[u]; j < rp[u + 1]; ++j) {
            const int32_t v = col[j];
            if (v == u) continue;
            int64_t lo = rp[v], hi = rp[v + 1];
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (col[mid] < u) lo = mid + 1;
                else hi = mid;
            }
            if (lo == rp[v + 1] || col[lo] != u) {
                atomicMin(ok, 0);
                return;
            }
        }
    }
}

// exclusive scan of n int64 values: out[0..n], out[n] = total
__global__ void scan_local(const int64_t *__restrict__ in, int64_t n, int64_t *__restrict__ out,
                           int64_t *__restrict__ bsum) {
    __shared__ int64_t s[kThreads];
    const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    const int64_t v = i < n ? in[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int d = 1; d < kThreads; d <<= 1) {
        const int64_t t = (int)threadIdx.x >= d ? s[threadIdx.x - d] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    if (i < n) out[i] = s[threadIdx.x] - v;
    if (threadIdx.x == kThreads - 1) bsum[blockIdx.x] = s[kThreads - 1];
}

__global__ void scan_sums(int64_t *bsum, int64_t nb) {  // one workgroup; bsum[nb] = total
    __shared__ int64_t s[kThreads];
    int64_t carry = 0;
    for (int64_t base = 0; base < nb; base += kThreads) {
        const int64_t i = base + threadIdx.x;
        const int64_t v = i < nb ? bsum[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int d = 1; d < kThreads; d <<= 1) {
            const int64_t t = (int)threadIdx.x >= d ? s[threadIdx.x - d] : 0;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nb) bsum[i] = carry + s[threadIdx.x] - v;
        const int64_t step = s[kThreads - 1];
        __syncthreads();
        carry += step;
    }
    if (threadIdx.x == 0) bsum[nb] = carry;
}

__global__ void scan_add(int64_t *__restrict__ out, int64_t n, const int64_t *__restrict__ bsum, int64_t nb) {
    const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    if (i < n) out[i] += bsum[blockIdx.x];
    if (i == 0) out[n] = bsum[nb];
}

__global__ void inverse_perm(const int32_t *__restrict__ perm, int64_t n, int32_t *__restrict__ iperm) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
        iperm[perm[r]] = (int32_t)r;
}

__global__ void new_lengths(const int64_t *__restrict__ rp, const int32_t *__restrict__ perm, int64_t n,
                            int64_t *__restrict__ len) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        const int32_t o = perm[r];
        len[r] = rp[o + 1] - rp[o];
    }
}

// row r of P A P^T: row perm[r] of A with columns mapped through iperm,
// sorted by new column with a stable insertion sort (rows longer than
// kSortOnDevice are listed for the host instead)
__global__ void __launch_bounds__(kThreads)
    renumber_rows(const int64_t *__restrict__ rp, const int32_t *__restrict__ col, const double *__restrict__ val,
                  const int32_t *__restrict__ perm, const int32_t *__restrict__ iperm,
                  const int64_t *__restrict__ nrp, int64_t n, int32_t *__restrict__ ncol,
                  double *__restrict__ nval, int32_t *long_rows, int32_t *n_long) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        const int32_t o = perm[r];
        const int64_t a = rp[o], len = rp[o + 1] - a, base = nrp[r];
        int32_t *c = ncol + base;
        double *v = nval + base;
        if (len <= kSortInRegisters) {
            // short row: sorted in registers by an odd-even transposition
            // network (adjacent swaps of strictly greater keys only, so the
            // order of equal columns is kept); padding keys sort last
            int32_t kc[kSortInRegisters];
            double kv[kSortInRegisters];
#pragma unroll
            for (int j = 0; j < kSortInRegisters; ++j) {
                kc[j] = j < len ? iperm[col[a + j]] : INT32_MAX;
                kv[j] = j < len ? val[a + j] : 0.0;
            }
#pragma unroll
            for (int pass = 0; pass < kSortInRegisters; ++pass)
#pragma unroll
                for (int i = pass & 1; i + 1 < kSortInRegisters; i += 2)
                    if (kc[i] > kc[i + 1]) {
                        const int32_t tc = kc[i];
                        kc[i] = kc[i + 1];
                        kc[i + 1] = tc;
                        const double tv = kv[i];
                        kv[i] = kv[i + 1];
                        kv[i + 1] = tv;
                    }
#pragma unroll
            for (int j = 0; j < kSortInRegisters; ++j)
                if (j < len) {
                    c[j] = kc[j];
                    v[j] = kv[j];
                }
            continue;
        }
        for (int64_t j = 0; j < len; ++j) {
            c[j] = iperm[col[a + j]];
            v[j] = val[a + j];
        }
        if (len > kSortOnDevice) {
            long_rows[atomicAdd(n_long, 1)] = (int32_t)r;
            continue;
        }
        for (int64_t i = 1; i < len; ++i) {
            const int32_t kc = c[i];
            const double kv = v[i];
            int64_t k = i - 1;
            while (k >= 0 && c[k] > kc) {
                c[k + 1] = c[k];
                v[k + 1] = v[k];
                --k;
            }
            c[k + 1] = kc;
            v[k + 1] = kv;
        }
    }
}

mpk_status scan_on_device(DeviceGraph &g, const int64_t *in, int64_t n, int64_t *out) {
    const int64_t nb = std::max<int64_t>(1, (n + kThreads - 1) / kThreads);
    int64_t *bsum = nullptr;
    LV_TRY(dalloc(g, &bsum, nb + 1));
    hipLaunchKernelGGL(scan_local, dim3((unsigned)nb), dim3(kThreads), 0, 0, in, n, out, bsum);
    hipLaunchKernelGGL(scan_sums, dim3(1), dim3(kThreads), 0, 0, bsum, nb);
    hipLaunchKernelGGL(scan_add, dim3((unsigned)nb), dim3(kThreads), 0, 0, out, n, bsum, nb);
    LV_TRY(hipGetLastError());
    return MPK_OK;
}

}  // namespace

mpk_status device_plan(const mpk_csr *A, int32_t root_mode, int64_t *root_out, std::vector<int32_t> &perm,
                       std::vector<int32_t> &level_ptr, std::vector<int32_t> &rowptr, std::vector<int32_t> &col,
                       std::vector<double> &val, bool *handled, double *phase_seconds) {
    *handled = false;
    const int64_t n = A->n, nnz = A->nnz;
    if (n == 0) return MPK_OK;
    auto now = [] { return std::chrono::steady_clock::now(); };
    auto secs = [](auto a, auto b) { return std::chrono::duration<double>(b - a).count(); };
    const auto t0 = now();
    DeviceGraph g;
    g.n = n;
    int64_t *drp = nullptr;
    int32_t *dcol = nullptr, *flag = nullptr;
    LV_TRY(dalloc(g, &drp, n + 1));
    LV_TRY(dalloc(g, &dcol, nnz));
    LV_TRY(dalloc(g, &flag, 1));
    LV_TRY(hipMemcpy(drp, A->rowptr, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice));
    if (nnz > 0) LV_TRY(hipMemcpy(dcol, A->col, sizeof(int32_t) * nnz, hipMemcpyHostToDevice));
    // ---- graph: only for sorted symmetric patterns (else the host builds it) ---------
    const int32_t one = 1;
    LV_TRY(hipMemcpy(flag, &one, sizeof(int32_t), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(rows_sorted, dim3(2048), dim3(kThreads), 0, 0, drp, dcol, n, flag);
    hipLaunchKernelGGL(pattern_symmetric, dim3(2048), dim3(kThreads), 0, 0, drp, dcol, n, flag);
    LV_TRY(hipGetLastError());
    int32_t ok = 0;
    LV_TRY(hipMemcpy(&ok, flag, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (!ok) return MPK_OK;  // not handled: the caller takes the host path
    int64_t *cnt = nullptr;
    LV_TRY(dalloc(g, &cnt, n));
    // the sorted symmetric rows are the graph: the expansion skips the
    // diagonal and repeated entries itself
    g.ptr = drp;
    g.adj = dcol;
    mpk_status st = MPK_OK;
    LV_TRY(hipDeviceSynchronize());
    const auto t1 = now();
    // ---- levels ----------------------------------------------------------------------
    if ((st = alloc_bfs(g)) != MPK_OK) return st;
    level_ptr.assign(1, 0);
    if ((st = bfs_on_device(g, root_mode, root_out, level_ptr)) != MPK_OK) return st;
    LV_TRY(hipDeviceSynchronize());
    const auto t2 = now();
    // ---- renumbered matrix P A P^T ---------------------------------------------------
    double *dval = nullptr, *nval = nullptr;
    int32_t *iperm = nullptr, *ncol = nullptr, *long_rows = nullptr;
    int64_t *nrp = nullptr;
    LV_TRY(dalloc(g, &dval, nnz));
    LV_TRY(dalloc(g, &nval, nnz));
    LV_TRY(dalloc(g, &ncol, nnz));
    LV_TRY(dalloc(g, &iperm, n));
    LV_TRY(dalloc(g, &nrp, n + 1));
    LV_TRY(dalloc(g, &long_rows, n));
    if (nnz > 0) LV_TRY(hipMemcpy(dval, A->val, sizeof(double) * nnz, hipMemcpyHostToDevice));
    const int32_t zero = 0;
    LV_TRY(hipMemcpy(flag, &zero, sizeof(int32_t), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(inverse_perm, dim3(2048), dim3(kThreads), 0, 0, g.order, n, iperm);
    hipLaunchKernelGGL(new_lengths, dim3(2048), dim3(kThreads), 0, 0, drp, g.order, n, cnt);
    LV_TRY(hipGetLastError());
    if ((st = scan_on_device(g, cnt, n, nrp)) != MPK_OK) return st;
    hipLaunchKernelGGL(renumber_rows, dim3(2048), dim3(kThreads), 0, 0, drp, dcol, dval, g.order, iperm, nrp, n, ncol,
                       nval, long_rows, flag);
    LV_TRY(hipGetLastError());
    perm.assign(n, 0);
    std::vector<int64_t> rp64(n + 1);
    rowptr.resize(n + 1);
    col.resize(nnz);
    val.resize(nnz);
    int32_t n_long = 0;
    LV_TRY(hipMemcpy(perm.data(), g.order, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    LV_TRY(hipMemcpy(rp64.data(), nrp, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost));
    if (nnz > 0) {
        LV_TRY(hipMemcpy(col.data(), ncol, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
        LV_TRY(hipMemcpy(val.data(), nval, sizeof(double) * nnz, hipMemcpyDeviceToHost));
    }
    LV_TRY(hipMemcpy(&n_long, flag, sizeof(int32_t), hipMemcpyDeviceToHost));
    for (int64_t i = 0; i <= n; ++i) rowptr[i] = (int32_t)rp64[i];
    if (n_long > 0) {
        std::vector<int32_t> rows(n_long);
        LV_TRY(hipMemcpy(rows.data(), long_rows, sizeof(int32_t) * n_long, hipMemcpyDeviceToHost));
#pragma omp parallel
        {
            std::vector<std::pair<int32_t, double>> buf;
#pragma omp for schedule(dynamic, 1)
            for (int64_t i = 0; i < n_long; ++i) {
                const int64_t a = rowptr[rows[i]], b = rowptr[rows[i] + 1];
                buf.resize(b - a);
                for (int64_t j = a; j < b; ++j) buf[j - a] = {col[j], val[j]};
                std::stable_sort(buf.begin(), buf.end(),
                                 [](const auto &x, const auto &y) { return x.first < y.first; });
                for (int64_t j = a; j < b; ++j) {
                    col[j] = buf[j - a].first;
                    val[j] = buf[j - a].second;
                }
            }
        }
    }
    const auto t3 = now();
    phase_seconds[0] = secs(t0, t1);
    phase_seconds[1] = secs(t1, t2);
    phase_seconds[2] = secs(t2, t3);
    *handled = true;
    return MPK_OK;
}

// ---------------------------------------------------------------------------
// plans from a CSR in device memory: the renumbered matrix stays on the GPU
// ---------------------------------------------------------------------------

namespace {

// The checks of validate_csr and of the pattern, on the device, as flag
// bits: 1 = row pointers (not monotone, outside [0, nnz], rowptr[0] != 0 or
// rowptr[n] != nnz), 2 = a column outside [0, n), 4 = a row not sorted by
// column, 8 = a stored (u, v) without a stored (v, u).  Columns are read only
// in rows whose bounds are valid, so no access leaves the arrays.
// check_rowptr: one thread per row, also the longest row (atomic maximum).
__global__ void check_rowptr(const int64_t *__restrict__ rp, int64_t n, int64_t nnz, int32_t *bad,
                             unsigned long long *longest) {
    if (blockIdx.x == 0 && threadIdx.x == 0 && (rp[0] != 0 || rp[n] != nnz)) atomicOr(bad, 1);
    unsigned long long m = 0;
    for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = rp[u], b = rp[u + 1];
        if (a < 0 || a > b || b > nnz)
            atomicOr(bad, 1);
        else
            m = max(m, (unsigned long long)(b - a));
    }
    if (m) atomicMax(longest, m);
}

// check_pattern: a group of 32 lanes per row, one stored entry per lane.
// Symmetry: every distinct entry (u, v) above the diagonal must have its
// transpose, found by a binary search in row v, and the distinct entries
// above and below the diagonal must be equally many (updown[0], updown[1]);
// the map (u, v) -> (v, u) is then a bijection between the two sets.  The
// repeats of a sorted row are skipped; an unsorted row is reported anyway.
__global__ void __launch_bounds__(kThreads)
    check_pattern(const int64_t *__restrict__ rp, const int32_t *__restrict__ col, int64_t n, int64_t nnz,
                  int32_t *bad, unsigned long long *updown) {
    __shared__ unsigned long long s_up[kThreads], s_down[kThreads];
    int32_t flags = 0;
    unsigned long long up = 0, down = 0;
    for (int64_t slot = blockIdx.x * (int64_t)kThreads + threadIdx.x; slot < n * kLanes;
         slot += (int64_t)gridDim.x * kThreads) {
        const int64_t u = slot / kLanes;
        const int64_t a = rp[u], b = rp[u + 1];
        if (a < 0 || a > b || b > nnz) continue;
        for (int64_t j = a + (slot & (kLanes - 1)); j < b; j += kLanes) {
            const int32_t v = col[j];
            if ((uint32_t)v >= (uint64_t)n) {
                flags |= 2;
                continue;
            }
            if (j > a) {
                const int32_t prev = col[j - 1];
                if (prev > v) flags |= 4;
                if (prev == v) continue;  // a repeat
            }
            if (v < u) {
                ++down;
                continue;
            }
            if (v == u) continue;
            ++up;
            int64_t lo = rp[v], hi = rp[v + 1];
            if (lo < 0 || lo > hi || hi > nnz) continue;  // reported by check_rowptr
            const int64_t end = hi;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (col[mid] < u) lo = mid + 1;
                else hi = mid;
            }
            if (lo == end || col[lo] != u) flags |= 8;
        }
    }
    if (flags) atomicOr(bad, flags);
    s_up[threadIdx.x] = up;
    s_down[threadIdx.x] = down;
    __syncthreads();
    for (int d = kThreads / 2; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) {
            s_up[threadIdx.x] += s_up[threadIdx.x + d];
            s_down[threadIdx.x] += s_down[threadIdx.x + d];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicAdd(updown, s_up[0]);
        atomicAdd(updown + 1, s_down[0]);
    }
}

__global__ void narrow_rowptr(const int64_t *__restrict__ in, int64_t n1, int32_t *__restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n1; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (int32_t)in[i];
}

// Rows longer than kSortOnDevice, one workgroup each: the keys (new column,
// position in the row of A) are sorted in LDS by a bitonic network; the
// positions make every key distinct, so the order is the stable order of
// the host planner.  Values are taken from A at the original positions.
constexpr int kLongRow = (int)kResidentRowMax;
__global__ void __launch_bounds__(kThreads) sort_long_rows(const int32_t *__restrict__ rows,
                                                           const int64_t *__restrict__ nrp,
                                                           const int64_t *__restrict__ rp,
                                                           const double *__restrict__ val,
                                                           const int32_t *__restrict__ perm,
                                                           int32_t *__restrict__ ncol, double *__restrict__ nval) {
    __shared__ unsigned long long key[kLongRow];
    const int32_t r = rows[blockIdx.x];
    const int64_t a = nrp[r], len = nrp[r + 1] - a;  // len <= kLongRow (checked on the host)
    const int64_t a0 = rp[perm[r]];
    int P = 1;
    while (P < len) P <<= 1;
    for (int i = threadIdx.x; i < P; i += kThreads)
        key[i] = i < len ? ((unsigned long long)(uint32_t)ncol[a + i] << 32) | (uint32_t)i : ~0ull;
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < P; i += kThreads) {
                const int l = i ^ j;
                if (l > i) {
                    const unsigned long long x = key[i], y = key[l];
                    if ((x > y) == ((i & k) == 0)) {
                        key[i] = y;
                        key[l] = x;
                    }
                }
            }
            __syncthreads();
        }
    for (int i = threadIdx.x; i < len; i += kThreads) {
        const unsigned long long kk = key[i];
        ncol[a + i] = (int32_t)(kk >> 32);
        nval[a + i] = val[a0 + (uint32_t)kk];
    }
}

// One workgroup per tile (grid stride): per m, the minimum and maximum
// column inside the row range of group g-1+m; bad flag for any other column.
__global__ void __launch_bounds__(kThreads) tile_columns(const int32_t *__restrict__ rowptr,
                                                         const int32_t *__restrict__ col,
                                                         const int32_t *__restrict__ tile_row,
                                                         const int32_t *__restrict__ tile_group,
                                                         const int32_t *__restrict__ group_row, int64_t T,
                                                         int64_t G, int32_t *__restrict__ out, int32_t *bad) {
    __shared__ int32_t red[6][kThreads];
    for (int64_t t = blockIdx.x; t < T; t += gridDim.x) {
        const int64_t g = tile_group[t];
        int32_t gb[3], ge[3], lo[3], hi[3];
        for (int m = 0; m < 3; ++m) {
            const int64_t gm = g - 1 + m;
            gb[m] = (gm >= 0 && gm < G) ? group_row[gm] : 0;
            ge[m] = (gm >= 0 && gm < G) ? group_row[gm + 1] : 0;
            lo[m] = INT32_MAX;
            hi[m] = -1;
        }
        const int64_t j0 = rowptr[tile_row[t]], j1 = rowptr[tile_row[t + 1]];
        bool outside = false;
        for (int64_t j = j0 + threadIdx.x; j < j1; j += kThreads) {
            const int32_t c = col[j];
            int m = -1;
            for (int mm = 0; mm < 3; ++mm)
                if (c >= gb[mm] && c < ge[mm]) m = mm;
            if (m < 0) {
                outside = true;
                continue;
            }
            for (int mm = 0; mm < 3; ++mm)
                if (mm == m) {
                    lo[mm] = min(lo[mm], c);
                    hi[mm] = max(hi[mm], c);
                }
        }
        if (outside) atomicOr(bad, 1);
        for (int m = 0; m < 3; ++m) {
            red[2 * m][threadIdx.x] = lo[m];
            red[2 * m + 1][threadIdx.x] = hi[m];
        }
        __syncthreads();
        for (int d = kThreads / 2; d > 0; d >>= 1) {
            if ((int)threadIdx.x < d)
                for (int m = 0; m < 3; ++m) {
                    red[2 * m][threadIdx.x] = min(red[2 * m][threadIdx.x], red[2 * m][threadIdx.x + d]);
                    red[2 * m + 1][threadIdx.x] = max(red[2 * m + 1][threadIdx.x], red[2 * m + 1][threadIdx.x + d]);
                }
            __syncthreads();
        }
        if (threadIdx.x < 6) out[6 * t + threadIdx.x] = red[threadIdx.x][0];
        __syncthreads();
    }
}

struct ResidentGuard {  // frees the output matrix unless released
    ResidentMatrix *M;
    bool keep = false;
    ~ResidentGuard() {
        if (keep) return;
        (void)hipFree(M->rowptr);
        (void)hipFree(M->col);
        (void)hipFree(M->val);
        *M = ResidentMatrix{};
    }
};

}  // namespace

mpk_status device_plan_resident(const mpk_csr *A, int32_t root_mode, int64_t *root_out,
                                std::vector<int32_t> &perm, std::vector<int32_t> &level_ptr,
                                std::vector<int32_t> &rowptr, ResidentMatrix *M, double *phase_seconds) {
    const int64_t n = A->n, nnz = A->nnz;
    auto now = [] { return std::chrono::steady_clock::now(); };
    auto secs = [](auto a, auto b) { return std::chrono::duration<double>(b - a).count(); };
    const auto t0 = now();
    *M = ResidentMatrix{};
    ResidentGuard guard{M};
    auto mall = [](auto **p, int64_t count) {
        return hipMalloc((void **)p, sizeof(**p) * (size_t)std::max<int64_t>(count, 1));
    };
    LV_TRY(mall(&M->rowptr, n + 1));
    LV_TRY(mall(&M->col, nnz));
    LV_TRY(mall(&M->val, nnz));
    perm.assign(n, 0);
    level_ptr.assign(1, 0);
    rowptr.assign(n + 1, 0);
    *root_out = 0;
    if (n == 0) {
        const int32_t zero = 0;
        LV_TRY(hipMemcpy(M->rowptr, &zero, sizeof(int32_t), hipMemcpyHostToDevice));
        guard.keep = true;
        return MPK_OK;
    }
    const int64_t *drp = A->rowptr;
    const int32_t *dcol = A->col;
    DeviceGraph g;
    g.n = n;
    int32_t *flag = nullptr;
    int64_t *cnt = nullptr;
    unsigned long long *mx = nullptr;  // longest row, entries above and below the diagonal
    LV_TRY(dalloc(g, &flag, 1));
    LV_TRY(dalloc(g, &cnt, n));
    LV_TRY(dalloc(g, &mx, 3));
    // ---- validation (the host planner's checks) and the pattern ----------------------
    const int32_t zero = 0;
    const unsigned long long zero64[3] = {0, 0, 0};
    LV_TRY(hipMemcpy(flag, &zero, sizeof(int32_t), hipMemcpyHostToDevice));
    LV_TRY(hipMemcpy(mx, zero64, sizeof(zero64), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(check_rowptr, dim3(2048), dim3(kThreads), 0, 0, drp, n, nnz, flag, mx);
    hipLaunchKernelGGL(check_pattern, dim3(8192), dim3(kThreads), 0, 0, drp, dcol, n, nnz, flag, mx + 1);
    LV_TRY(hipGetLastError());
    int32_t bad = 0;
    unsigned long long counts[3] = {0, 0, 0};
    LV_TRY(hipMemcpy(&bad, flag, sizeof(int32_t), hipMemcpyDeviceToHost));
    LV_TRY(hipMemcpy(counts, mx, sizeof(counts), hipMemcpyDeviceToHost));
    const unsigned long long longest = counts[0];
    if (counts[1] != counts[2]) bad |= 8;
    if (bad & 1) return fail(MPK_ERR_CSR, "device CSR: row pointers not monotone or not in [0, nnz]");
    if (bad & 2) return fail(MPK_ERR_CSR, "device CSR: column index out of range");
    if ((int64_t)longest > kResidentRowMax)
        return fail(MPK_ERR_UNSUPPORTED, "device CSR: a row holds more than 4096 entries; plan it from host memory");
    if (bad & (4 | 8))
        return fail(MPK_ERR_UNSUPPORTED,
                    "device CSR: rows must be sorted and the pattern symmetric; plan other matrices from host memory");
    // the sorted symmetric rows are the graph
    g.ptr = const_cast<int64_t *>(drp);
    g.adj = const_cast<int32_t *>(dcol);
    mpk_status st = MPK_OK;
    const auto t1 = now();
    // ---- levels ------------------------------------------------------------------------
    if ((st = alloc_bfs(g)) != MPK_OK) return st;
    if ((st = bfs_on_device(g, root_mode, root_out, level_ptr)) != MPK_OK) return st;
    LV_TRY(hipDeviceSynchronize());
    const auto t2 = now();
    // ---- renumbered matrix P A P^T, left on the device -----------------------------------
    int32_t *iperm = nullptr, *long_rows = nullptr;
    int64_t *nrp = nullptr;
    LV_TRY(dalloc(g, &iperm, n));
    LV_TRY(dalloc(g, &nrp, n + 1));
    LV_TRY(dalloc(g, &long_rows, n));
    LV_TRY(hipMemcpy(flag, &zero, sizeof(int32_t), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(inverse_perm, dim3(2048), dim3(kThreads), 0, 0, g.order, n, iperm);
    hipLaunchKernelGGL(new_lengths, dim3(2048), dim3(kThreads), 0, 0, drp, g.order, n, cnt);
    LV_TRY(hipGetLastError());
    if ((st = scan_on_device(g, cnt, n, nrp)) != MPK_OK) return st;
    hipLaunchKernelGGL(renumber_rows, dim3(2048), dim3(kThreads), 0, 0, drp, dcol, A->val, g.order, iperm, nrp, n,
                       M->col, M->val, long_rows, flag);
    LV_TRY(hipGetLastError());
    int32_t n_long = 0;
    LV_TRY(hipMemcpy(&n_long, flag, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (n_long > 0) {
        hipLaunchKernelGGL(sort_long_rows, dim3((unsigned)n_long), dim3(kThreads), 0, 0, long_rows, nrp, drp,
                           A->val, g.order, M->col, M->val);
        LV_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(narrow_rowptr, dim3(2048), dim3(kThreads), 0, 0, nrp, n + 1, M->rowptr);
    LV_TRY(hipGetLastError());
    LV_TRY(hipMemcpy(perm.data(), g.order, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    LV_TRY(hipMemcpy(rowptr.data(), M->rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost));
    const auto t3 = now();
    phase_seconds[0] = secs(t0, t1);
    phase_seconds[1] = secs(t1, t2);
    phase_seconds[2] = secs(t2, t3);
    guard.keep = true;
    return MPK_OK;
}

mpk_status device_tile_columns(const int32_t *d_rowptr, const int32_t *d_col, const std::vector<int32_t> &tile_row,
                               const std::vector<int32_t> &tile_group, const std::vector<int32_t> &group_row,
                               std::vector<int32_t> &out, bool *bad) {
    const int64_t T = (int64_t)tile_group.size(), G = (int64_t)group_row.size() - 1;
    out.assign(6 * (size_t)T, 0);
    *bad = false;
    if (T == 0) return MPK_OK;
    DeviceGraph g;  // owner of the temporary buffers
    int32_t *dtr = nullptr, *dtg = nullptr, *dgr = nullptr, *dout = nullptr, *flag = nullptr;
    LV_TRY(dalloc(g, &dtr, T + 1));
    LV_TRY(dalloc(g, &dtg, T));
    LV_TRY(dalloc(g, &dgr, G + 1));
    LV_TRY(dalloc(g, &dout, 6 * T));
    LV_TRY(dalloc(g, &flag, 1));
    LV_TRY(hipMemcpy(dtr, tile_row.data(), sizeof(int32_t) * (T + 1), hipMemcpyHostToDevice));
    LV_TRY(hipMemcpy(dtg, tile_group.data(), sizeof(int32_t) * T, hipMemcpyHostToDevice));
    LV_TRY(hipMemcpy(dgr, group_row.data(), sizeof(int32_t) * (G + 1), hipMemcpyHostToDevice));
    const int32_t zero = 0;
    LV_TRY(hipMemcpy(flag, &zero, sizeof(int32_t), hipMemcpyHostToDevice));
    const unsigned nb = (unsigned)std::min<int64_t>(T, 8192);
    hipLaunchKernelGGL(tile_columns, dim3(nb), dim3(kThreads), 0, 0, d_rowptr, d_col, dtr, dtg, dgr, T, G, dout,
                       flag);
    LV_TRY(hipGetLastError());
    int32_t f = 0;
    LV_TRY(hipMemcpy(out.data(), dout, sizeof(int32_t) * 6 * T, hipMemcpyDeviceToHost));
    LV_TRY(hipMemcpy(&f, flag, sizeof(int32_t), hipMemcpyDeviceToHost));
    *bad = f != 0;
    return MPK_OK;
}

}  // namespace mpk
