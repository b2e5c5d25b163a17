// Kernels and C-ABI of the MPK library (gfx950).
//
//  * spmv_kernel      one SpMV over all rows (the baseline of Sec. 3.1,
//                     Fig. 2); p launches back to back give the baseline MPK.
//  * mpk_persistent   the level-blocked MPK (Sec. 4.2-4.3): a persistent grid
//                     draws tickets, through striped counters, in the order of
//                     the (level group, power) nodes by g + skew*q (skew 1 =
//                     the Lp diagonals of Fig. 6); a ticket is one device
//                     tile (a row range inside a level group) at one power.
//                     Before computing power q of a tile, one wavefront polls
//                     the "power q-1 done" flags of every tile that holds a
//                     column the tile reads (point-to-point synchronisation,
//                     Sec. 4.3) instead of a barrier; after the tile is
//                     written the workgroup releases its own flag at agent
//                     scope.  Every ticket only waits for earlier tickets, so
//                     the grid needs no co-residency and cannot deadlock; a
//                     bounded spin (watchdog) turns a lost flag into an error.
//  * permute_*        gather/scatter between original and level numbering.
//  * bw_probe         load-only bandwidth probe (the analog of Fig. 1).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "kernels.h"
#include "mpk_internal.h"

namespace mpk {
const char *last_error_cstr();
}

using namespace mpk;

// ----------------------------------------------------------------------------
// plan / handle objects
// ----------------------------------------------------------------------------

struct mpk_plan {
    HostPlan hp;
    bool uploaded = false;
    int device = -1;
    int32_t workgroups = 0;
    int32_t num_cus = 0;
    int32_t last_run_fenced = -1;
    uint64_t device_bytes = 0;
    int32_t *d_rowptr = nullptr, *d_col = nullptr;
    void *d_val = nullptr;
    int32_t *d_tile_row = nullptr, *d_trec = nullptr;
    int32_t *d_perm = nullptr;
    int32_t *d_chunk = nullptr, *d_tile_chunk = nullptr, *d_dep3 = nullptr;  // d_chunk: int4 per chunk
    // the baseline SpMV's own chunks of the whole matrix (spmv_chunk_nnz)
    int32_t *d_chunk_spmv = nullptr;
    int32_t n_chunks_spmv = 0;
    int32_t *d_dep3x = nullptr;
    int32_t *d_dep_ptr = nullptr, *d_dep_rng = nullptr;  // refined plans: per-tile range lists
    uint32_t *d_flags = nullptr, *d_ctrl = nullptr;
    std::vector<void *> allocs;
    // plans made from device memory: P A P^T kept on the GPU (FP64 values)
    // for the plan's lifetime, shared by every upload after a retune
    bool resident = false;
    ResidentMatrix rm;
};

struct mpk_spmv {
    int64_t n = 0, nnz = 0;
    int32_t dtype = MPK_F64, nrhs = 1, acc64 = 0;
    int64_t nchunks = 0;
    int32_t *d_rowptr = nullptr, *d_col = nullptr, *d_chunk = nullptr;
    void *d_val = nullptr;
    std::vector<void *> allocs;
};

namespace {

// control words: [0] epoch of the last run (written by its last workgroup),
// [1] departures, [2] epoch of a timed-out run, [3] ticket
// that timed out, [16..23] arrivals per stream, then one ticket counter per
// (stream, sub-stripe) pair, 256 B apart
constexpr int kMaxStripes = 64;
constexpr int kMaxStreams = 8;
constexpr int kArrivalBase = 16;
// s_waitcnt immediate for gfx9-family: vmcnt(0), expcnt and lgkmcnt left at max
constexpr int kWaitVmcnt0 = 0x0F70;
constexpr int kStripeBase = 64;
constexpr int kStripeStride = 64;
constexpr int kCtrlWords = kStripeBase + kMaxStripes * kStripeStride;

// Device chunk table: (first row, end row, first nonzero, end nonzero) per
// chunk, from the chunk start rows and the row pointers.
std::vector<int32_t> chunk_descriptors(const std::vector<int32_t> &chunk_row, const int32_t *rowptr) {
    const size_t nc = chunk_row.empty() ? 0 : chunk_row.size() - 1;
    std::vector<int32_t> d(4 * nc);
    for (size_t c = 0; c < nc; ++c) {
        d[4 * c + 0] = chunk_row[c];
        d[4 * c + 1] = chunk_row[c + 1];
        d[4 * c + 2] = rowptr[chunk_row[c]];
        d[4 * c + 3] = rowptr[chunk_row[c + 1]];
    }
    return d;
}

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(e_ == hipErrorOutOfMemory ? MPK_ERR_OOM : MPK_ERR_HIP,         \
                        std::string(#expr) + ": " + hipGetErrorString(e_));            \
    } while (0)

template <typename T>
hipError_t dev_alloc(std::vector<void *> &allocs, T **p, size_t count, uint64_t *bytes = nullptr) {
    size_t b = std::max<size_t>(sizeof(T) * count, 256);
    hipError_t e = hipMalloc((void **)p, b);
    if (e == hipSuccess) {
        allocs.push_back((void *)*p);
        if (bytes) *bytes += b;
    }
    return e;
}

void free_all(std::vector<void *> &allocs) {
    for (void *p : allocs) (void)hipFree(p);
    allocs.clear();
}

// f64 -> f32 (round to nearest even, the C conversion) -> bf16 (round to
// nearest even on the upper 16 bits; NaN kept quiet)
uint16_t f32_to_bf16_bits(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x0040u);
    uint32_t rounding = 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)((u + rounding) >> 16);
}

size_t value_bytes(int32_t dtype) { return dtype == MPK_F64 ? 8 : dtype == MPK_F32 ? 4 : 2; }

void convert_values(const double *src, size_t n, int32_t dtype, std::vector<uint8_t> &out) {
    out.resize(std::max<size_t>(n * value_bytes(dtype), 1));
    if (dtype == MPK_F64) {
        std::memcpy(out.data(), src, n * 8);
    } else if (dtype == MPK_F32) {
        float *o = reinterpret_cast<float *>(out.data());
        for (size_t i = 0; i < n; ++i) o[i] = (float)src[i];
    } else {
        uint16_t *o = reinterpret_cast<uint16_t *>(out.data());
        for (size_t i = 0; i < n; ++i) o[i] = f32_to_bf16_bits((float)src[i]);
    }
}

// The same conversions on the device for a matrix that stays there, in
// integer arithmetic so the result does not depend on the device's rounding
// or denormal modes: f64 -> f32 rounds to nearest even (overflow to
// infinity, subnormal results kept, a NaN keeps its sign and upper payload
// bits and becomes quiet, as the host's conversion does), then bf16 as
// f32_to_bf16_bits.
__device__ __forceinline__ uint32_t f64_to_f32_bits(uint64_t u) {
    const uint32_t sign = (uint32_t)(u >> 63) << 31;
    const int32_t ex = (int32_t)((u >> 52) & 0x7ff);
    const uint64_t man = u & ((uint64_t(1) << 52) - 1);
    if (ex == 0x7ff) return man ? sign | 0x7fc00000u | (uint32_t)(man >> 29) : sign | 0x7f800000u;
    const int32_t e = ex - 1023 + 127;
    if (e >= 255) return sign | 0x7f800000u;
    if (e >= 1) {
        uint32_t r = ((uint32_t)e << 23) | (uint32_t)(man >> 29);
        const uint64_t rem = man & ((uint64_t(1) << 29) - 1), half = uint64_t(1) << 28;
        if (rem > half || (rem == half && (r & 1u))) ++r;  // a carry moves into the exponent (or to infinity)
        return sign | r;
    }
    if (ex == 0) return sign;  // FP64 subnormals are far below the FP32 range
    // FP32 subnormal or zero: the value in units of 2^-149 is full * 2^(ex - 926)
    const uint64_t full = (uint64_t(1) << 52) | man;
    const int32_t sh = 926 - ex;  // >= 30 here
    if (sh >= 54) return sign;    // below half the smallest subnormal
    uint32_t r = (uint32_t)(full >> sh);
    const uint64_t rem = full & ((uint64_t(1) << sh) - 1), half = uint64_t(1) << (sh - 1);
    if (rem > half || (rem == half && (r & 1u))) ++r;
    return sign | r;
}

__device__ __forceinline__ uint16_t f32_bits_to_bf16(uint32_t u) {
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x0040u);
    const uint32_t rounding = 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)((u + rounding) >> 16);
}

__global__ void convert_values_kernel(const double *__restrict__ src, int64_t n, int32_t dtype, void *dst) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t f = f64_to_f32_bits((uint64_t)__double_as_longlong(src[i]));
        if (dtype == MPK_F32)
            static_cast<uint32_t *>(dst)[i] = f;
        else
            static_cast<uint16_t *>(dst)[i] = f32_bits_to_bf16(f);
    }
}

// ----------------------------------------------------------------------------
// kernels
// ----------------------------------------------------------------------------

// Rows of chunks [c0, c1), one chunk after another, NP products per thread.
template <typename VT, int K, bool REC, bool COH, int NP>
__device__ __forceinline__ void chunks_body(int c0, int c1, const int4 *__restrict__ chunk,
                                            const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                            const VT *__restrict__ val, const double *__restrict__ x,
                                            double *__restrict__ y, int q, const double *__restrict__ yq2,
                                            const RecArgs &rec) {
    __shared__ ChunkLds<VT, K, NP> lds;
    for (int c = c0; c < c1; ++c)
        chunk_pass<VT, K, REC, COH, NP>(chunk[c], rowptr, col, val, x, y, q, yq2, rec, lds);
}

// Baseline SpMV: one workgroup per chunk (chunks of spmv_chunk_nnz).
template <typename VT, int K, bool REC>
__global__ __launch_bounds__(kBlock) void spmv_kernel(const int4 *__restrict__ chunk,
                                                      const int32_t *__restrict__ rowptr,
                                                      const int32_t *__restrict__ col,
                                                      const VT *__restrict__ val, const double *__restrict__ x,
                                                      double *__restrict__ y, int q,
                                                      const double *__restrict__ yq2, RecArgs rec) {
    constexpr int NP = spmv_products_per_thread(K, std::is_same<typename AccumType<VT>::T, float>::value);
    chunks_body<VT, K, REC, false, NP>(blockIdx.x, blockIdx.x + 1, chunk, rowptr, col, val, x, y, q, yq2, rec);
}

// Bulk-synchronous level-blocked MPK: one launch computes a list of Lp
// nodes (a level group's chunks at one power).  Workgroup b takes chunk
// b - start[s] of segment s.  With one node per launch, or one wavefront of
// independent nodes per launch, the kernel boundary is the barrier between
// dependent nodes (the variants without point-to-point synchronisation,
// Sec. 4.2).
constexpr int kMaxSegments = MPK_MAX_POWER;
struct SegList {
    int32_t n;
    int32_t start[kMaxSegments + 1];  // workgroup offset of each segment
    int32_t c0[kMaxSegments];         // first chunk
    int32_t q[kMaxSegments];          // power
};

template <typename VT, int K>
__global__ __launch_bounds__(kBlock) void segment_kernel(SegList L, const int4 *__restrict__ chunk,
                                                         const int32_t *__restrict__ rowptr,
                                                         const int32_t *__restrict__ col,
                                                         const VT *__restrict__ val, const double *__restrict__ X,
                                                         double *__restrict__ Y, int64_t NK) {
    const int b = blockIdx.x;
    int s = 0;
    while (s + 1 < L.n && L.start[s + 1] <= b) ++s;
    const int c = L.c0[s] + (b - L.start[s]);
    const int q = L.q[s];
    const double *x = q == 1 ? X : Y + (int64_t)(q - 2) * NK;
    double *y = Y + (int64_t)(q - 1) * NK;
    RecArgs none{};
    chunks_body<VT, K, false, false, mpk_products_per_thread(K)>(c, c + 1, chunk, rowptr, col, val, x, y, q, nullptr,
                                                                  none);
}

struct MpkArgs {
    const int4 *chunk;
    const int32_t *tile_chunk;
    const int32_t *rowptr;
    const int32_t *col;
    const void *val;
    const int32_t *tile_row;
    const int32_t *dep3;
    // tickets in stream order, two int4 each: (tile * 64 + q - 1, first
    // chunk, end chunk, 0) and the first chunk's descriptor, so a workgroup
    // reaches the matrix loads of its next ticket after one 32-byte read
    const int4 *trec;
    int32_t n, ntiles, ntickets;
    const double *X;
    double *Y;
    uint32_t *flags;
    uint32_t *ctrl;
    int32_t nstreams;
    int32_t stream_ptr[kMaxStreams + 1];
    int64_t watchdog;
    int32_t acquire;  // 1: agent-scope acquire fence after every dependency wait
    // refined plans: tile t waits for the inclusive tile ranges
    // dep_rng[2k..2k+1], k in [dep_ptr[t], dep_ptr[t+1]), instead of dep3
    const int32_t *dep_ptr;
    const int32_t *dep_rng;
    int32_t dep_lists;
    int32_t p_run;  // powers computed (<= the plan's p); tickets of higher powers are skipped
};

// Element i of a table that no kernel writes while it runs (chunk
// descriptors, dependency ranges), read through the constant address space
// at a uniform index: a scalar load into scalar registers, counted apart
// from the vector loads and stores.  A vector load would complete in order
// behind the loads and write-through stores already issued, so waiting for
// it would also wait for them; and the values are uniform, so the loops and
// branches that use them stay uniform.
typedef __attribute__((address_space(4))) const int32_t const_i32;
__device__ __forceinline__ int4 table4(const int4 *tab, int i) {
    const const_i32 *q = (const const_i32 *)tab + 4 * (int64_t)__builtin_amdgcn_readfirstlane(i);
    return make_int4(q[0], q[1], q[2], q[3]);
}

__device__ __forceinline__ uint32_t ld_agent(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Executed by one full wavefront: polls until the flags f[j] of `total`
// indices j = index(i), i < total, all hold `epoch`, 64 flags per vector
// load.  Returns false if the watchdog expired (and reports the ticket) or
// another workgroup already reported a timeout in this run.
template <typename Index>
__device__ bool poll_flags(const uint32_t *f, int total, Index index, const MpkArgs &a, int ticket,
                           uint32_t epoch) {
    const int lane = threadIdx.x & 63;
    int64_t spins = 0;
    for (int base = 0; base < total; base += 64) {
        const int i = base + lane;
        const int j = i < total ? index(i) : -1;
        for (;;) {
            const bool ok = (j < 0) || (ld_agent(f + j) == epoch);
            if (__all(ok)) break;
            ++spins;
            if (spins > a.watchdog) {
                if (lane == 0) {
                    st_agent(a.ctrl + 3, (uint32_t)ticket);
                    st_agent(a.ctrl + 2, epoch);
                }
                return false;
            }
            if ((spins & 255) == 0 && ld_agent(a.ctrl + 2) == epoch) return false;
            __builtin_amdgcn_s_sleep(1);
        }
    }
    return true;
}

// Waits for the dependencies of `tile` at the previous power (flags f):
// the three tile ranges d[0..1], d[2..3], d[4..5] of dep3 (inclusive,
// lo > hi = empty) or, for refined plans, the tile's range list.
__device__ bool wait_flags(const uint32_t *f, int tile, const MpkArgs &a, int ticket, uint32_t epoch) {
    bool ok;
    if (a.dep_lists) {
        // a list holds few ranges: each is polled on its own
        const int ut = __builtin_amdgcn_readfirstlane(tile);
        const const_i32 *dp = (const const_i32 *)a.dep_ptr, *dr = (const const_i32 *)a.dep_rng;
        const int k0 = dp[ut], k1 = dp[ut + 1];
        ok = true;
        for (int k = k0; k < k1 && ok; ++k) {
            const int lo = dr[2 * (int64_t)k], hi = dr[2 * (int64_t)k + 1];
            ok = poll_flags(f, hi - lo + 1, [=](int i) { return lo + i; }, a, ticket, epoch);
        }
    } else {
        const const_i32 *d = (const const_i32 *)a.dep3 + 6 * (int64_t)__builtin_amdgcn_readfirstlane(tile);
        const int lo0 = d[0], lo1 = d[2], lo2 = d[4];
        const int n0 = max(0, d[1] - lo0 + 1), n1 = max(0, d[3] - lo1 + 1), n2 = max(0, d[5] - lo2 + 1);
        ok = poll_flags(
            f, n0 + n1 + n2,
            [=](int i) { return i < n0 ? lo0 + i : i < n0 + n1 ? lo1 + (i - n0) : lo2 + (i - n0 - n1); }, a,
            ticket, epoch);
    }
    // Without line-closed dependencies a cache may hold a line of y_{q-1}
    // read before all its rows were final: invalidate before reading.
    if (ok && a.acquire) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return ok;
}

__device__ __forceinline__ uint32_t *stripe_counter(const MpkArgs &a, int s) {
    return a.ctrl + kStripeBase + s * kStripeStride;
}

// Before its dependency wait a tile loads its first chunk's row pointers
// and columns, and with FP64 values (k <= 2) the values too; FP32 and BF16
// values are loaded after the wait, together with the gathers, which keeps
// the registers held across the wait low enough for 4 workgroups per CU at
// k = 1 (FP64 holds them all and runs at 3 per CU, the faster of the two for
// each value type).
template <typename VT>
constexpr bool kPreloadValues = std::is_same<VT, double>::value;

template <typename VT, int K, bool REC>
__global__ __launch_bounds__(kBlock, K == 1 && kPreloadValues<VT> ? 3 : 4) void mpk_persistent(MpkArgs a, RecArgs rec) {
    // The tickets form `nstreams` streams (1, or 8 XCD slices); workgroup b
    // serves stream b % nstreams.  Inside a stream the tickets are dealt over
    // S counters: sub-stripe s holds the stream's tickets s, s + S, ...;
    // a workgroup joins sub-stripe (its arrival index in the stream mod S)
    // and takes that sub-stripe's tickets in increasing order, one at a time.
    // Every ticket only waits for earlier tickets of the global order, every
    // stream has at least S workgroups and any S of them cover its
    // sub-stripes, so the smallest unfinished ticket is always held by, or
    // next for, a running workgroup whose earlier tickets are done: the grid
    // needs no co-residency.  The last workgroup to leave resets the counters.
    __shared__ int s_sub, s_ok;
    __shared__ uint32_t s_epoch;
    __shared__ int s_next[2];
    __shared__ int4 s_rec[2][2];  // the current and the next ticket record
    constexpr int NP = mpk_products_per_thread(K);
    __shared__ ChunkLds<VT, K, NP> lds;
    const int nS = a.nstreams;
    const int stream = blockIdx.x % nS;
    const int in_stream = (gridDim.x - stream + nS - 1) / nS;
    const int S = min(kMaxStripes / nS, in_stream);
    const int base = a.stream_ptr[stream];
    const int len = a.stream_ptr[stream + 1] - base;
    const int64_t NK = (int64_t)a.n * K;
    const VT *val = reinterpret_cast<const VT *>(a.val);
    if (threadIdx.x == 0) {
        const uint32_t arrival =
            __hip_atomic_fetch_add(a.ctrl + kArrivalBase + stream, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int sub = (int)(arrival % (uint32_t)S);
        const uint32_t k = __hip_atomic_fetch_add(stripe_counter(a, stream * (kMaxStripes / nS) + sub), 1u,
                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_sub = sub;
        s_next[0] = (int)min<int64_t>((int64_t)sub + (int64_t)k * S, len);
        // The run's epoch: one past the last run's (control word 0, written
        // by the last workgroup of that run, so every workgroup of this run
        // reads the same value); the flags of earlier runs never match it.
        // The launch arguments do not change between runs, so a captured
        // launch can be replayed.
        uint32_t e = ld_agent(a.ctrl) + 1u;
        s_epoch = e == 0u ? 1u : e;
    }
    __syncthreads();
    const uint32_t epoch = s_epoch;
    const int counter = stream * (kMaxStripes / nS) + s_sub;
    const int sub = s_sub;
    // A run of fewer powers than the plan's skips the tickets of the higher
    // powers: nothing waits for them.  Thread 0 moves past them with further
    // counter increments.
    auto next_ticket = [&](int t0, uint32_t &kk) -> int {
        int tn = t0;
        while (tn < len && ((a.trec[2 * (int64_t)(base + tn)].x & 63) + 1) > a.p_run) {
            kk = __hip_atomic_fetch_add(stripe_counter(a, counter), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            tn = (int)min<int64_t>((int64_t)sub + (int64_t)kk * S, len);
        }
        return tn;
    };
    if (threadIdx.x == 0) {
        uint32_t kk = 0;
        int t0 = s_next[0];
        if (a.p_run < MPK_MAX_POWER) t0 = next_ticket(t0, kk);
        if (t0 < len) {
            s_rec[0][0] = a.trec[2 * (int64_t)(base + t0)];
            s_rec[0][1] = a.trec[2 * (int64_t)(base + t0) + 1];
        }
        s_next[0] = t0;
    }
    __syncthreads();
    int t = s_next[0];
    for (int it = 1; t < len; ++it) {
        const int cur = (it - 1) & 1;
        // the ticket is the same for the whole workgroup: kept in scalar
        // registers, so the loops over its chunks are uniform
        const int4 tr = s_rec[cur][0];
        const int4 dl = s_rec[cur][1];
        const int4 d0 = make_int4(__builtin_amdgcn_readfirstlane(dl.x), __builtin_amdgcn_readfirstlane(dl.y),
                                  __builtin_amdgcn_readfirstlane(dl.z), __builtin_amdgcn_readfirstlane(dl.w));
        const int w = __builtin_amdgcn_readfirstlane(tr.x);
        const int tile = w >> 6;
        const int q = (w & 63) + 1;
        const int c0 = __builtin_amdgcn_readfirstlane(tr.y), c1 = __builtin_amdgcn_readfirstlane(tr.z);
        // The first chunk's matrix entries and row pointers do not depend on
        // the flags: they are loaded before the wait, so their latency and
        // the polling overlap.  The barriers around the poll order only LDS
        // (s_ok) and leave those loads in flight.  For k >= 4 the registers
        // held across the wait cost more occupancy than the overlap gains.
        const bool pre = K <= 2 && plain_chunk<K, NP>(d0);
        ChunkRegs<VT, K, NP> g;
        if (pre) chunk_load<VT, K, NP, kPreloadValues<VT>>(d0, a.rowptr, a.col, val, g);
        if (q > 1) {
            if (threadIdx.x == 0) s_ok = 1;
            lds_barrier();
            if (threadIdx.x < 64) {
                const bool ok = wait_flags(a.flags + (int64_t)(q - 2) * a.ntiles, tile, a, base + t, epoch);
                if (!ok && threadIdx.x == 0) s_ok = 0;
            }
            lds_barrier();
            if (!s_ok) break;
        }
        const double *xin = (q == 1) ? a.X : a.Y + (int64_t)(q - 2) * NK;
        double *yout = a.Y + (int64_t)(q - 1) * NK;
        const double *yq2 = (q == 1) ? rec.y_prev : (q == 2 ? a.X : a.Y + (int64_t)(q - 3) * NK);
        if constexpr (K <= 2) {
            if (pre) {
                if constexpr (!kPreloadValues<VT>) chunk_load_vals<VT, K, NP>(d0, val, g);
                chunk_finish<VT, K, REC, true, NP>(d0, g, xin, yout, q, yq2, rec, lds);
            } else {
                chunk_pass<VT, K, REC, true, NP>(d0, a.rowptr, a.col, val, xin, yout, q, yq2, rec, lds);
            }
            // later chunks: each descriptor (a scalar load) is read while the
            // chunk before it runs
            int4 dn = table4(a.chunk, c0 + 1 < c1 ? c0 + 1 : c0);
            for (int c = c0 + 1; c < c1; ++c) {
                const int4 d = dn;
                dn = table4(a.chunk, c + 1 < c1 ? c + 1 : c);
                chunk_pass<VT, K, REC, true, NP>(d, a.rowptr, a.col, val, xin, yout, q, yq2, rec, lds);
            }
        } else {
            chunk_pass<VT, K, REC, true, NP>(d0, a.rowptr, a.col, val, xin, yout, q, yq2, rec, lds);
            // later chunks: each descriptor is read while the chunk before it runs
            int4 dn = table4(a.chunk, c0 + 1 < c1 ? c0 + 1 : c0);
            for (int c = c0 + 1; c < c1; ++c) {
                const int4 d = dn;
                dn = table4(a.chunk, c + 1 < c1 ? c + 1 : c);
                chunk_pass<VT, K, REC, true, NP>(d, a.rowptr, a.col, val, xin, yout, q, yq2, rec, lds);
            }
        }
        // The next ticket is taken only now: a workgroup never holds a ticket
        // it is not working on, so no ticket waits behind an idle one.
        uint32_t kn = 0;
        if (threadIdx.x == 0)
            kn = __hip_atomic_fetch_add(stripe_counter(a, counter), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // Release: the tile's results were written with agent-scope stores;
        // every wavefront waits until its stores have completed (vmcnt = 0)
        // before the workgroup barrier, after which the flag is published.
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
        if (threadIdx.x == 0) {
            int tn = (int)min<int64_t>((int64_t)sub + (int64_t)kn * S, len);
            if (a.p_run < MPK_MAX_POWER) tn = next_ticket(tn, kn);
            if (tn < len) {
                s_rec[cur ^ 1][0] = a.trec[2 * (int64_t)(base + tn)];
                s_rec[cur ^ 1][1] = a.trec[2 * (int64_t)(base + tn) + 1];
            }
            s_next[it & 1] = tn;
        }
        __syncthreads();
        if (threadIdx.x == 0) st_agent(a.flags + (int64_t)(q - 1) * a.ntiles + tile, epoch);
        t = s_next[it & 1];
    }
    if (threadIdx.x == 0) {
        const uint32_t done = __hip_atomic_fetch_add(a.ctrl + 1, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (done == gridDim.x - 1) {
            for (int st = 0; st < kMaxStripes; ++st) st_agent(stripe_counter(a, st), 0u);
            for (int st = 0; st < kMaxStreams; ++st) st_agent(a.ctrl + kArrivalBase + st, 0u);
            st_agent(a.ctrl + 1, 0u);
            st_agent(a.ctrl, epoch);
        }
    }
}

__global__ void permute_gather(const double *__restrict__ in, double *__restrict__ out,
                               const int32_t *__restrict__ perm, int64_t n, int k) {
    const int64_t total = n * k;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / k, c = i - r * k;
        out[i] = in[(int64_t)perm[r] * k + c];
    }
}

__global__ void permute_scatter(const double *__restrict__ in, double *__restrict__ out,
                                const int32_t *__restrict__ perm, int64_t n, int k) {
    const int64_t total = n * k;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i / k, c = i - r * k;
        out[(int64_t)perm[r] * k + c] = in[i];
    }
}

__global__ __launch_bounds__(kBlock) void bw_probe(const double2 *__restrict__ buf, int64_t n2, int reps,
                                                   double *sink) {
    double acc = 0.0;
    for (int rep = 0; rep < reps; ++rep) {
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n2;
             i += (int64_t)gridDim.x * blockDim.x) {
            const double2 v = buf[i];
            acc += v.x + v.y;
        }
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0 && acc == 12345.678) sink[0] = acc;  // keeps the loads alive
}

// The same probe with U independent 16-byte loads per thread in flight and an
// optional split of the buffer into `parts` contiguous parts: workgroup b
// reads part b % parts only, striding over it with the other workgroups of
// that part.  With parts = 8 every XCD re-reads its own part (workgroups
// b, b + 8, ... share an XCD), so a part larger than an XCD's L2 but a buffer
// smaller than the Infinity Cache measures the Infinity Cache read rate.
template <int U>
__global__ __launch_bounds__(kBlock) void bw_probe_ex(const double2 *__restrict__ buf, int64_t n2, int parts, int reps,
                                                      double *sink) {
    const int part = blockIdx.x % parts;
    const int64_t j = blockIdx.x / parts;
    const int64_t cnt = (gridDim.x - part + parts - 1) / parts;
    const double2 *b = buf + (int64_t)part * n2;
    const int64_t step = cnt * kBlock * U;
    double acc = 0.0;
    for (int rep = 0; rep < reps; ++rep) {
        for (int64_t base = j * kBlock * U + threadIdx.x; base < n2; base += step) {
            double2 v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t i = base + (int64_t)u * kBlock;
                v[u] = i < n2 ? b[i] : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) acc += v[u].x + v[u].y;
        }
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0 && acc == 12345.678) sink[0] = acc;
}

// XCD (accelerator complex die) running the calling wavefront: bits [3:0] of
// the XCC_ID hardware register (hwreg 20 on CDNA3/CDNA4).
__device__ __forceinline__ int hw_xcc_id() { return __builtin_amdgcn_s_getreg((3 << 11) | 20) & 15; }

// Records the XCD of every workgroup; each workgroup then sleeps `spin`
// rounds so that later workgroups are placed while earlier ones still hold
// their slots (the situation of a persistent grid).
__global__ __launch_bounds__(kBlock) void xcd_ids_kernel(int32_t *ids, int64_t spin) {
    if (threadIdx.x == 0) ids[blockIdx.x] = hw_xcc_id();
    for (int64_t i = 0; i < spin; ++i) __builtin_amdgcn_s_sleep(16);
}

// Dependency-hop latency: two workgroups (blockIdx 0 and `peer`) pass a
// counter back and forth through two flags, `iters` round trips.  scope 0:
// agent-scope flag stores and loads (written through to the device-coherent
// level, read past the L2); scope 1: workgroup-scope stores and loads (L1
// bypassed, served by the L2 of the XCD; correct only when both workgroups
// share an XCD).  Every poll is bounded by `max_polls`; out[0] = elapsed
// wall-clock ticks of workgroup 0, out[1] = completed round trips.
__global__ void hop_probe_kernel(uint32_t *flags, int peer, int scope, int iters, int64_t max_polls,
                                 uint64_t *out) {
    const int b = blockIdx.x;
    if ((b != 0 && b != peer) || threadIdx.x != 0) return;
    const bool ping = b == 0;
    uint32_t *mine = flags + (ping ? 0 : 32), *theirs = flags + (ping ? 32 : 0);
    auto st = [&](uint32_t *p, uint32_t v) {
        if (scope == 0)
            __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
            __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    auto ld = [&](uint32_t *p) -> uint32_t {
        return scope == 0 ? __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                          : __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    const uint64_t t0 = wall_clock64();
    int done = 0;
    for (int i = 1; i <= iters; ++i) {
        if (ping) st(mine, (uint32_t)i);
        int64_t polls = 0;
        while (ld(theirs) != (uint32_t)i && ++polls < max_polls) {
        }
        if (polls >= max_polls) break;
        if (!ping) st(mine, (uint32_t)i);
        done = i;
    }
    if (ping) {
        out[0] = wall_clock64() - t0;
        out[1] = (uint64_t)done;
    }
}

// ----------------------------------------------------------------------------
// launch dispatch: value type x right-hand sides K x recurrence
// ----------------------------------------------------------------------------

template <typename VT, int K, bool REC>
struct Dispatch {
    static hipError_t spmv(int blocks, hipStream_t s, const int4 *chunks, const int32_t *rp, const int32_t *ci,
                           const void *v, const double *x, double *y, int q, const double *yq2,
                           const RecArgs &rec) {
        hipLaunchKernelGGL((spmv_kernel<VT, K, REC>), dim3(blocks), dim3(kBlock), 0, s, chunks, rp, ci,
                           reinterpret_cast<const VT *>(v), x, y, q, yq2, rec);
        return hipGetLastError();
    }
    static hipError_t seg(int blocks, hipStream_t s, const SegList &L, const int4 *chunks, const int32_t *rp,
                          const int32_t *ci, const void *v, const double *X, double *Y, int64_t NK) {
        if constexpr (REC) {
            return hipErrorInvalidValue;
        } else {
            hipLaunchKernelGGL((segment_kernel<VT, K>), dim3(blocks), dim3(kBlock), 0, s, L, chunks, rp, ci,
                               reinterpret_cast<const VT *>(v), X, Y, NK);
            return hipGetLastError();
        }
    }
    static hipError_t mpk(int blocks, hipStream_t s, const MpkArgs &a, const RecArgs &rec) {
        hipLaunchKernelGGL((mpk_persistent<VT, K, REC>), dim3(blocks), dim3(kBlock), 0, s, a, rec);
        return hipGetLastError();
    }
    static const void *mpk_symbol() { return (const void *)mpk_persistent<VT, K, REC>; }
};

// What is compiled: FP64 for every k in {1,2,4,8,16,32} (recurrence for k <= 2);
// FP32 and BF16 values, with FP32 or FP64 arithmetic, for k in {1, 2} with and
// without the recurrence.
template <typename VT, bool REC>
struct ByK {
    template <typename F>
    static hipError_t call(int K, F &&f) {
        switch (K) {
            case 1: return f(Dispatch<VT, 1, REC>{});
            case 2: return f(Dispatch<VT, 2, REC>{});
        }
        if constexpr (std::is_same<VT, double>::value && !REC) {
            switch (K) {
                case 4: return f(Dispatch<VT, 4, REC>{});
                case 8: return f(Dispatch<VT, 8, REC>{});
                case 16: return f(Dispatch<VT, 16, REC>{});
                case 32: return f(Dispatch<VT, 32, REC>{});
            }
        }
        return hipErrorInvalidValue;
    }
};

// acc64: FP32 / BF16 values with FP64 arithmetic (mpk_options.accum_f64)
template <typename F>
hipError_t dispatch_all(int dtype, int acc64, int K, bool rec, F &&f) {
    switch (dtype) {
        case MPK_F64: return rec ? ByK<double, true>::call(K, f) : ByK<double, false>::call(K, f);
        case MPK_F32:
            if (acc64) return rec ? ByK<f32w_t, true>::call(K, f) : ByK<f32w_t, false>::call(K, f);
            return rec ? ByK<float, true>::call(K, f) : ByK<float, false>::call(K, f);
        case MPK_BF16:
            if (acc64) return rec ? ByK<bf16w_t, true>::call(K, f) : ByK<bf16w_t, false>::call(K, f);
            return rec ? ByK<bf16_t, true>::call(K, f) : ByK<bf16_t, false>::call(K, f);
    }
    return hipErrorInvalidValue;
}

bool supported(int dtype, int K, bool rec) {
    if (K == 1 || K == 2) return true;
    if (K == 4 || K == 8 || K == 16 || K == 32) return dtype == MPK_F64 && !rec;
    return false;
}

mpk_status fill_rec(const mpk_recurrence *r, int p, int K, RecArgs &out) {
    std::memset(&out, 0, sizeof(out));
    for (int i = 0; i < MPK_MAX_POWER; ++i) out.alpha[i] = 1.0;
    if (!r) return MPK_OK;
    if (r->complex_pairs && K != 2) return fail(MPK_ERR_ARG, "complex_pairs needs nrhs == 2");
    for (int i = 0; i < p; ++i) {
        out.alpha[i] = r->alpha ? r->alpha[i] : 1.0;
        out.beta[i] = r->beta ? r->beta[i] : 0.0;
        out.gamma[i] = r->gamma ? r->gamma[i] : 0.0;
        if (r->coef) {
            out.coef_re[i] = r->complex_pairs ? r->coef[2 * i] : r->coef[i];
            out.coef_im[i] = r->complex_pairs ? r->coef[2 * i + 1] : 0.0;
        }
        if (out.gamma[i] != 0.0 && i == 0 && !r->y_prev)
            return fail(MPK_ERR_ARG, "gamma[0] != 0 needs y_prev");
    }
    if (r->acc && !r->coef) return fail(MPK_ERR_ARG, "acc needs coef");
    if (r->coef0 && !r->acc) return fail(MPK_ERR_ARG, "coef0 needs acc");
    out.y_prev = r->y_prev;
    out.acc = r->acc;
    out.complex_pairs = r->complex_pairs;
    if (r->coef0) {
        out.start_acc = 1;
        out.c0_re = r->coef0[0];
        out.c0_im = r->complex_pairs ? r->coef0[1] : 0.0;
    }
    return MPK_OK;
}


}  // namespace

// ----------------------------------------------------------------------------
// C-ABI
// ----------------------------------------------------------------------------

extern "C" {

void mpk_options_default(mpk_options *opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->size = sizeof(mpk_options);
    opt->safety_factor = 0.5;
    opt->root_mode = 0;
    opt->val_dtype = MPK_F64;
    opt->nrhs = 1;
    opt->watchdog_spins = 0;
    opt->skew = 1;
    opt->xcd_streams = 1;
}

const char *mpk_version(void) { return "mpk-gfx950 0.1"; }

const char *mpk_last_error(void) { return last_error_cstr(); }

const char *mpk_status_string(mpk_status s) {
    switch (s) {
        case MPK_OK: return "ok";
        case MPK_ERR_ARG: return "invalid argument";
        case MPK_ERR_CSR: return "malformed CSR matrix";
        case MPK_ERR_OOM: return "out of memory";
        case MPK_ERR_HIP: return "HIP runtime error";
        case MPK_ERR_TIMEOUT: return "device dependency wait timed out";
        case MPK_ERR_UNSUPPORTED: return "unsupported configuration";
        case MPK_ERR_STATE: return "call out of order";
    }
    return "unknown status";
}

mpk_status mpk_plan_create(const mpk_csr *A, int32_t p, uint64_t cache_bytes, const mpk_options *opt,
                           mpk_plan **out) {
    if (!out) return fail(MPK_ERR_ARG, "null output pointer");
    *out = nullptr;
    mpk_options o;
    mpk_options_default(&o);
    if (opt) {
        if (opt->size != sizeof(mpk_options)) return fail(MPK_ERR_ARG, "mpk_options.size mismatch");
        o = *opt;
    }
    if (!supported(o.val_dtype, o.nrhs, false)) return fail(MPK_ERR_UNSUPPORTED, "nrhs/dtype combination");
    mpk_plan *plan = new (std::nothrow) mpk_plan();
    if (!plan) return fail(MPK_ERR_OOM, "host allocation failed");
    mpk_status st = build_host_plan(A, p, cache_bytes, o, plan->hp);
    if (st != MPK_OK) {
        delete plan;
        return st;
    }
    *out = plan;
    return MPK_OK;
}

mpk_status mpk_plan_create_device(const mpk_csr *A, int32_t p, uint64_t cache_bytes, const mpk_options *opt,
                                  mpk_plan **out) {
    if (!out) return fail(MPK_ERR_ARG, "null output pointer");
    *out = nullptr;
    mpk_options o;
    mpk_options_default(&o);
    if (opt) {
        if (opt->size != sizeof(mpk_options)) return fail(MPK_ERR_ARG, "mpk_options.size mismatch");
        o = *opt;
    }
    if (!supported(o.val_dtype, o.nrhs, false)) return fail(MPK_ERR_UNSUPPORTED, "nrhs/dtype combination");
    mpk_plan *plan = new (std::nothrow) mpk_plan();
    if (!plan) return fail(MPK_ERR_OOM, "host allocation failed");
    plan->resident = true;
    mpk_status st = build_resident_plan(A, p, cache_bytes, o, plan->hp, &plan->rm);
    if (st != MPK_OK) {
        mpk_plan_destroy(plan);
        return st;
    }
    *out = plan;
    return MPK_OK;
}

mpk_status mpk_plan_retune(mpk_plan *plan, int32_t p, uint64_t cache_bytes, const mpk_options *opt) {
    if (!plan) return fail(MPK_ERR_ARG, "null plan");
    mpk_options o;
    mpk_options_default(&o);
    if (opt) {
        if (opt->size != sizeof(mpk_options)) return fail(MPK_ERR_ARG, "mpk_options.size mismatch");
        o = *opt;
    }
    if (o.root_mode != plan->hp.opt.root_mode)
        return fail(MPK_ERR_ARG, "retune keeps the BFS levels: root_mode must not change");
    if (plan->hp.recursive || o.recursion_stages != 0)
        return fail(MPK_ERR_UNSUPPORTED, "a refined numbering depends on p and C: create a new plan");
    if (!supported(o.val_dtype, o.nrhs, false)) return fail(MPK_ERR_UNSUPPORTED, "nrhs/dtype combination");
    const bool was_uploaded = plan->uploaded;
    if (was_uploaded) {
        HIP_TRY(hipDeviceSynchronize());
        free_all(plan->allocs);
        plan->uploaded = false;
        plan->device_bytes = 0;
    }
    ScheduleState backup;
    save_schedule(plan->hp, backup);
    mpk_status st = build_schedule(plan->hp, p, cache_bytes, o);
    if (st != MPK_OK) {
        restore_schedule(plan->hp, backup);
        if (was_uploaded) (void)mpk_plan_upload(plan);
        return st;
    }
    if (was_uploaded) return mpk_plan_upload(plan);
    return MPK_OK;
}

mpk_status mpk_plan_query(const mpk_plan *plan, mpk_plan_info *info) {
    if (!plan || !info) return fail(MPK_ERR_ARG, "null argument");
    const HostPlan &h = plan->hp;
    std::memset(info, 0, sizeof(*info));
    info->n = h.n;
    info->nnz = h.nnz;
    info->p = h.p;
    info->nrhs = h.opt.nrhs;
    info->n_levels = (int64_t)h.level_ptr.size() - 1;
    info->n_groups = (int64_t)h.group_ptr.size() - 1;
    info->n_tiles = (int64_t)h.dep_lo.size();
    info->n_tickets = (int64_t)h.work.size();
    info->root = h.root;
    info->max_level_rows = h.max_level_rows;
    info->max_group_nnz = h.max_group_nnz;
    info->violating_groups = h.violating_groups;
    info->device_bytes = plan->device_bytes;
    info->workgroups = plan->workgroups;
    info->n_chunks = (int32_t)std::max<size_t>(1, h.chunk_row.size()) - 1;
    info->tile_nnz = h.tile_nnz;
    info->val_dtype = h.opt.val_dtype;
    info->plan_seconds = h.plan_seconds;
    for (int i = 0; i < 4; ++i) info->phase_seconds[i] = h.phase_seconds[i];
    info->line_closed_deps = h.line_closed_ok ? 1 : 0;
    info->last_run_fenced = plan->last_run_fenced;
    info->recursive = h.recursive ? 1 : 0;
    info->n_units = h.recursive ? (int64_t)h.unit_ptr.size() - 1 : info->n_groups;
    info->n_dep_ranges = h.recursive ? (int64_t)h.dep_rng.size() / 2 : 0;
    info->max_stage = 0;
    for (int32_t st : h.unit_stage) info->max_stage = std::max(info->max_stage, st);
    return MPK_OK;
}

mpk_status mpk_plan_units(const mpk_plan *plan, int32_t *unit_ptr, int32_t *unit_stage, int32_t *dep_ptr,
                          int32_t *dep_rng) {
    if (!plan) return fail(MPK_ERR_ARG, "null plan");
    const HostPlan &h = plan->hp;
    if (!h.recursive) return fail(MPK_ERR_STATE, "the plan has no refined levels (recursion_stages = 0)");
    if (unit_ptr) std::copy(h.unit_ptr.begin(), h.unit_ptr.end(), unit_ptr);
    if (unit_stage) std::copy(h.unit_stage.begin(), h.unit_stage.end(), unit_stage);
    if (dep_ptr) std::copy(h.dep_ptr.begin(), h.dep_ptr.end(), dep_ptr);
    if (dep_rng) std::copy(h.dep_rng.begin(), h.dep_rng.end(), dep_rng);
    return MPK_OK;
}

mpk_status mpk_plan_arrays(const mpk_plan *plan, int32_t *perm, int32_t *level_ptr, int32_t *group_ptr,
                           int32_t *schedule) {
    if (!plan) return fail(MPK_ERR_ARG, "null plan");
    const HostPlan &h = plan->hp;
    if (perm) std::copy(h.perm.begin(), h.perm.end(), perm);
    if (level_ptr) std::copy(h.level_ptr.begin(), h.level_ptr.end(), level_ptr);
    if (group_ptr) std::copy(h.group_ptr.begin(), h.group_ptr.end(), group_ptr);
    if (schedule) std::copy(h.schedule.begin(), h.schedule.end(), schedule);
    return MPK_OK;
}

mpk_status mpk_plan_matrix(const mpk_plan *plan, int64_t *rowptr, int32_t *col, double *val) {
    if (!plan) return fail(MPK_ERR_ARG, "null plan");
    const HostPlan &h = plan->hp;
    if (rowptr)
        for (size_t i = 0; i < h.rowptr.size(); ++i) rowptr[i] = h.rowptr[i];
    if (plan->resident) {
        if (col && h.nnz > 0) HIP_TRY(hipMemcpy(col, plan->rm.col, sizeof(int32_t) * h.nnz, hipMemcpyDeviceToHost));
        if (val && h.nnz > 0) HIP_TRY(hipMemcpy(val, plan->rm.val, sizeof(double) * h.nnz, hipMemcpyDeviceToHost));
        return MPK_OK;
    }
    if (col) std::copy(h.col.begin(), h.col.end(), col);
    if (val) std::copy(h.val.begin(), h.val.end(), val);
    return MPK_OK;
}

mpk_status mpk_plan_tiles(const mpk_plan *plan, int32_t *tile_row, int32_t *dep_lo, int32_t *dep_hi,
                          int32_t *work) {
    if (!plan) return fail(MPK_ERR_ARG, "null plan");
    const HostPlan &h = plan->hp;
    if (tile_row) std::copy(h.tile_row.begin(), h.tile_row.end(), tile_row);
    if (dep_lo) std::copy(h.dep_lo.begin(), h.dep_lo.end(), dep_lo);
    if (dep_hi) std::copy(h.dep_hi.begin(), h.dep_hi.end(), dep_hi);
    if (work) std::copy(h.work.begin(), h.work.end(), work);
    return MPK_OK;
}

mpk_status mpk_plan_tile_deps(const mpk_plan *plan, int32_t *ranges, int32_t line_closed) {
    if (!plan) return fail(MPK_ERR_ARG, "null plan");
    const std::vector<int32_t> &d = line_closed ? plan->hp.dep3x : plan->hp.dep3;
    if (ranges) std::copy(d.begin(), d.end(), ranges);
    return MPK_OK;
}

mpk_status mpk_plan_features(const mpk_plan *plan, double *features) {
    if (!plan || !features) return fail(MPK_ERR_ARG, "null argument");
    plan_features(plan->hp, features);
    return MPK_OK;
}

mpk_status mpk_plan_upload(mpk_plan *plan) {
    if (!plan) return fail(MPK_ERR_ARG, "null plan");
    if (plan->uploaded) return MPK_OK;
    HostPlan &h = plan->hp;
    HIP_TRY(hipGetDevice(&plan->device));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, plan->device));
    plan->num_cus = prop.multiProcessorCount;
    const int64_t T = (int64_t)h.dep_lo.size();
    const int64_t W = (int64_t)h.work.size();
    std::vector<uint8_t> vbuf;
    if (!plan->resident) convert_values(h.val.data(), h.val.size(), h.opt.val_dtype, vbuf);
    uint64_t bytes = 0;
    auto &al = plan->allocs;
    auto cleanup_fail = [&](hipError_t e, const char *what) {
        free_all(al);
        return fail(e == hipErrorOutOfMemory ? MPK_ERR_OOM : MPK_ERR_HIP,
                    std::string(what) + ": " + hipGetErrorString(e));
    };
    hipError_t e;
    if (plan->resident) {
        // the renumbered matrix is already on the device; FP32 / BF16 values
        // are converted there
        bytes += sizeof(int32_t) * (uint64_t)(h.n + 1) + (sizeof(int32_t) + sizeof(double)) * (uint64_t)h.nnz;
        plan->d_rowptr = plan->rm.rowptr;
        plan->d_col = plan->rm.col;
        if (h.opt.val_dtype == MPK_F64) {
            plan->d_val = plan->rm.val;
        } else {
            uint8_t *dv = nullptr;
            if ((e = dev_alloc(al, &dv, (size_t)h.nnz * value_bytes(h.opt.val_dtype), &bytes)) != hipSuccess)
                return cleanup_fail(e, "val");
            plan->d_val = dv;
            if (h.nnz > 0) {
                hipLaunchKernelGGL(convert_values_kernel, dim3(2048), dim3(256), 0, 0, plan->rm.val, h.nnz,
                                   h.opt.val_dtype, dv);
                if ((e = hipGetLastError()) != hipSuccess) return cleanup_fail(e, "value conversion");
            }
        }
    } else {
        if ((e = dev_alloc(al, &plan->d_rowptr, h.n + 1, &bytes)) != hipSuccess) return cleanup_fail(e, "rowptr");
        if ((e = dev_alloc(al, &plan->d_col, h.nnz, &bytes)) != hipSuccess) return cleanup_fail(e, "col");
        uint8_t *dv = nullptr;
        if ((e = dev_alloc(al, &dv, vbuf.size(), &bytes)) != hipSuccess) return cleanup_fail(e, "val");
        plan->d_val = dv;
    }
    if ((e = dev_alloc(al, &plan->d_tile_row, T + 1, &bytes)) != hipSuccess) return cleanup_fail(e, "tiles");
    if ((e = dev_alloc(al, &plan->d_dep3, 6 * T, &bytes)) != hipSuccess) return cleanup_fail(e, "deps");
    if ((e = dev_alloc(al, &plan->d_dep3x, 6 * T, &bytes)) != hipSuccess) return cleanup_fail(e, "deps");
    if ((e = dev_alloc(al, &plan->d_dep_ptr, std::max<size_t>(h.dep_ptr.size(), 1), &bytes)) != hipSuccess)
        return cleanup_fail(e, "deps");
    if ((e = dev_alloc(al, &plan->d_dep_rng, std::max<size_t>(h.dep_rng.size(), 2), &bytes)) != hipSuccess)
        return cleanup_fail(e, "deps");
    if ((e = dev_alloc(al, &plan->d_trec, 8 * W, &bytes)) != hipSuccess) return cleanup_fail(e, "tickets");
    if ((e = dev_alloc(al, &plan->d_flags, W, &bytes)) != hipSuccess) return cleanup_fail(e, "flags");
    if ((e = dev_alloc(al, &plan->d_ctrl, kCtrlWords, &bytes)) != hipSuccess) return cleanup_fail(e, "ctrl");
    if ((e = dev_alloc(al, &plan->d_perm, h.n, &bytes)) != hipSuccess) return cleanup_fail(e, "perm");
    const std::vector<int32_t> desc = chunk_descriptors(h.chunk_row, h.rowptr.data());
    // ticket records in stream order: (ticket, first chunk, end chunk, 0,
    // first chunk's descriptor)
    std::vector<int32_t> trec(8 * (size_t)W);
    for (int64_t i = 0; i < W; ++i) {
        const int32_t w = h.work_streams[i], tile = w >> 6;
        const int32_t c0 = h.tile_chunk[tile], c1 = h.tile_chunk[tile + 1];
        int32_t *r = &trec[8 * (size_t)i];
        r[0] = w;
        r[1] = c0;
        r[2] = c1;
        r[3] = 0;
        for (int m = 0; m < 4; ++m) r[4 + m] = desc[4 * (size_t)c0 + m];
    }
    if ((e = dev_alloc(al, &plan->d_chunk, std::max<size_t>(desc.size(), 4), &bytes)) != hipSuccess)
        return cleanup_fail(e, "chunks");
    if ((e = dev_alloc(al, &plan->d_tile_chunk, h.tile_chunk.size(), &bytes)) != hipSuccess)
        return cleanup_fail(e, "chunks");
    std::vector<int32_t> spmv_rows;
    append_chunks(h.rowptr, 0, h.n, spmv_chunk_nnz(h.opt.nrhs, fp32_products(h.opt.val_dtype, h.opt.accum_f64)),
                  kChunkRows, spmv_rows);
    spmv_rows.push_back((int32_t)h.n);
    const std::vector<int32_t> spmv_desc = chunk_descriptors(spmv_rows, h.rowptr.data());
    plan->n_chunks_spmv = (int32_t)(spmv_rows.size() - 1);
    if ((e = dev_alloc(al, &plan->d_chunk_spmv, std::max<size_t>(spmv_desc.size(), 4), &bytes)) != hipSuccess)
        return cleanup_fail(e, "chunks");
    struct Cp { void *d; const void *s; size_t b; } cps[] = {
        {plan->d_rowptr, h.rowptr.data(), plan->resident ? 0 : sizeof(int32_t) * (h.n + 1)},
        {plan->d_col, h.col.data(), plan->resident ? 0 : sizeof(int32_t) * h.nnz},
        {plan->d_val, vbuf.data(), plan->resident ? 0 : h.nnz * value_bytes(h.opt.val_dtype)},
        {plan->d_tile_row, h.tile_row.data(), sizeof(int32_t) * (T + 1)},
        {plan->d_dep3, h.dep3.data(), sizeof(int32_t) * 6 * T},
        {plan->d_dep3x, h.dep3x.data(), sizeof(int32_t) * 6 * T},
        {plan->d_dep_ptr, h.dep_ptr.data(), sizeof(int32_t) * h.dep_ptr.size()},
        {plan->d_dep_rng, h.dep_rng.data(), sizeof(int32_t) * h.dep_rng.size()},
        {plan->d_trec, trec.data(), sizeof(int32_t) * 8 * W},
        {plan->d_perm, h.perm.data(), sizeof(int32_t) * h.n},
        {plan->d_chunk, desc.data(), sizeof(int32_t) * desc.size()},
        {plan->d_tile_chunk, h.tile_chunk.data(), sizeof(int32_t) * h.tile_chunk.size()},
        {plan->d_chunk_spmv, spmv_desc.data(), sizeof(int32_t) * spmv_desc.size()},
    };
    for (auto &c : cps)
        if (c.b && (e = hipMemcpy(c.d, c.s, c.b, hipMemcpyHostToDevice)) != hipSuccess)
            return cleanup_fail(e, "upload copy");
    if ((e = hipMemset(plan->d_flags, 0, sizeof(uint32_t) * std::max<int64_t>(W, 1))) != hipSuccess)
        return cleanup_fail(e, "flag reset");
    if ((e = hipMemset(plan->d_ctrl, 0, sizeof(uint32_t) * kCtrlWords)) != hipSuccess)
        return cleanup_fail(e, "ctrl reset");
    if ((e = hipDeviceSynchronize()) != hipSuccess) return cleanup_fail(e, "upload sync");
    // grid: all co-resident workgroups unless the caller fixes it
    int occ = 0;
    const void *sym = nullptr;
    (void)dispatch_all(h.opt.val_dtype, h.opt.accum_f64, h.opt.nrhs, false, [&](auto d) {
        sym = decltype(d)::mpk_symbol();
        return hipSuccess;
    });
    if (sym && hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, sym, kBlock, 0) != hipSuccess) occ = 0;
    if (occ <= 0) occ = 2;
    int64_t wg = h.opt.workgroups > 0 ? h.opt.workgroups : (int64_t)occ * plan->num_cus;
    wg = std::max<int64_t>(1, std::min<int64_t>(wg, std::max<int64_t>(W, 1)));
    // every ticket stream needs workgroups of its own
    wg = std::max<int64_t>(wg, (int64_t)h.stream_ptr.size() - 1);
    plan->workgroups = (int32_t)wg;
    plan->device_bytes = bytes;
    plan->uploaded = true;
    return MPK_OK;
}

mpk_status mpk_permute(const mpk_plan *plan, const double *in, double *out, int32_t k, int32_t to_plan,
                       void *stream) {
    if (!plan) return fail(MPK_ERR_ARG, "null plan");
    if (!plan->uploaded) return fail(MPK_ERR_STATE, "plan not uploaded");
    if (k < 1 || k > MPK_MAX_NRHS) return fail(MPK_ERR_ARG, "k out of range");
    if (plan->hp.n == 0) return MPK_OK;
    if (!in || !out) return fail(MPK_ERR_ARG, "null vector");
    if (in == out) return fail(MPK_ERR_ARG, "in and out alias");
    const int64_t total = plan->hp.n * k;
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 65536);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (to_plan)
        hipLaunchKernelGGL(permute_gather, dim3(blocks), dim3(256), 0, s, in, out, plan->d_perm, plan->hp.n, k);
    else
        hipLaunchKernelGGL(permute_scatter, dim3(blocks), dim3(256), 0, s, in, out, plan->d_perm, plan->hp.n, k);
    HIP_TRY(hipGetLastError());
    return MPK_OK;
}

// [a, a + abytes) and [b, b + bbytes) share a byte (null pointers share none)
static bool overlaps(const void *a, uint64_t abytes, const void *b, uint64_t bbytes) {
    const uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
    return a && b && a0 < b0 + bbytes && b0 < a0 + abytes;
}

// Arguments of a run of `powers` powers: the plan is uploaded, the vectors
// are given, and no buffer the run writes (Y: powers x N x k, acc: N x k)
// overlaps another buffer of the run.
static mpk_status check_run_args(mpk_plan *plan, const double *X, double *Y, int32_t powers,
                                 const mpk_recurrence *rec) {
    if (!plan) return fail(MPK_ERR_ARG, "null plan");
    if (!plan->uploaded) return fail(MPK_ERR_STATE, "plan not uploaded (call mpk_plan_upload)");
    if (powers < 1 || powers > plan->hp.p) return fail(MPK_ERR_ARG, "powers must be in [1, plan p]");
    if (plan->hp.n == 0) return MPK_OK;
    if (!X || !Y) return fail(MPK_ERR_ARG, "null vector");
    const uint64_t vb = (uint64_t)plan->hp.n * plan->hp.opt.nrhs * 8, yb = vb * (uint64_t)powers;
    if (overlaps(X, vb, Y, yb)) return fail(MPK_ERR_ARG, "Y overlaps X");
    if (rec) {
        if (overlaps(rec->y_prev, vb, Y, yb)) return fail(MPK_ERR_ARG, "Y overlaps y_prev");
        if (overlaps(rec->acc, vb, Y, yb)) return fail(MPK_ERR_ARG, "Y overlaps acc");
        if (overlaps(rec->acc, vb, X, vb)) return fail(MPK_ERR_ARG, "acc overlaps X");
        if (overlaps(rec->acc, vb, rec->y_prev, vb)) return fail(MPK_ERR_ARG, "acc overlaps y_prev");
    }
    return MPK_OK;
}

mpk_status mpk_run(mpk_plan *plan, const double *X, double *Y, const mpk_recurrence *rec, void *stream) {
    if (!plan) return fail(MPK_ERR_ARG, "null plan");
    return mpk_run_first(plan, plan->hp.p, X, Y, rec, stream);
}

mpk_status mpk_run_first(mpk_plan *plan, int32_t powers, const double *X, double *Y, const mpk_recurrence *rec,
                         void *stream) {
    mpk_status st = check_run_args(plan, X, Y, powers, rec);
    if (st != MPK_OK) return st;
    HostPlan &h = plan->hp;
    if (h.n == 0) return MPK_OK;
    RecArgs ra;
    if ((st = fill_rec(rec, powers, h.opt.nrhs, ra)) != MPK_OK) return st;
    if (!supported(h.opt.val_dtype, h.opt.nrhs, rec != nullptr))
        return fail(MPK_ERR_UNSUPPORTED, "recurrence needs nrhs <= 2");
    MpkArgs a;
    a.chunk = reinterpret_cast<const int4 *>(plan->d_chunk);
    a.tile_chunk = plan->d_tile_chunk;
    a.rowptr = plan->d_rowptr;
    a.col = plan->d_col;
    a.val = plan->d_val;
    a.tile_row = plan->d_tile_row;
    // skip the acquire fence when every line of a power slice belongs to
    // tiles the reader waits for (line-closed ranges, aligned slices)
    const bool closed = h.line_closed_ok && !h.opt.force_acquire && (reinterpret_cast<uintptr_t>(Y) % 128) == 0 &&
                        ((h.n * h.opt.nrhs * 8) % 128) == 0;
    a.acquire = closed ? 0 : 1;
    plan->last_run_fenced = a.acquire;
    a.dep3 = closed ? plan->d_dep3x : plan->d_dep3;
    a.dep_ptr = plan->d_dep_ptr;
    a.dep_rng = plan->d_dep_rng;
    a.dep_lists = h.recursive ? 1 : 0;
    a.trec = reinterpret_cast<const int4 *>(plan->d_trec);
    a.n = (int32_t)h.n;
    a.ntiles = (int32_t)h.dep_lo.size();
    a.ntickets = (int32_t)h.work.size();
    a.nstreams = (int32_t)h.stream_ptr.size() - 1;
    for (int i = 0; i <= kMaxStreams; ++i) a.stream_ptr[i] = h.stream_ptr[std::min<int>(i, a.nstreams)];
    a.X = X;
    a.Y = Y;
    a.flags = plan->d_flags;
    a.ctrl = plan->d_ctrl;
    a.watchdog = h.opt.watchdog_spins > 0 ? h.opt.watchdog_spins : (int64_t)1 << 24;
    // MPK_MAX_POWER marks a full run (no ticket is skipped)
    a.p_run = powers == h.p ? MPK_MAX_POWER : powers;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = dispatch_all(h.opt.val_dtype, h.opt.accum_f64, h.opt.nrhs, rec != nullptr, [&](auto d) {
        return decltype(d)::mpk(plan->workgroups, s, a, ra);
    });
    if (e != hipSuccess) return fail(MPK_ERR_HIP, std::string("mpk launch: ") + hipGetErrorString(e));
    return MPK_OK;
}

mpk_status mpk_run_baseline(mpk_plan *plan, const double *X, double *Y, const mpk_recurrence *rec,
                            void *stream) {
    if (!plan) return fail(MPK_ERR_ARG, "null plan");
    return mpk_run_baseline_first(plan, plan->hp.p, X, Y, rec, stream);
}

mpk_status mpk_run_baseline_first(mpk_plan *plan, int32_t powers, const double *X, double *Y,
                                  const mpk_recurrence *rec, void *stream) {
    mpk_status st = check_run_args(plan, X, Y, powers, rec);
    if (st != MPK_OK) return st;
    HostPlan &h = plan->hp;
    if (h.n == 0) return MPK_OK;
    RecArgs ra;
    if ((st = fill_rec(rec, powers, h.opt.nrhs, ra)) != MPK_OK) return st;
    if (!supported(h.opt.val_dtype, h.opt.nrhs, rec != nullptr))
        return fail(MPK_ERR_UNSUPPORTED, "recurrence needs nrhs <= 2");
    const int K = h.opt.nrhs;
    const int blocks = plan->n_chunks_spmv;
    const int64_t NK = h.n * K;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    for (int q = 1; q <= powers; ++q) {
        const double *x = q == 1 ? X : Y + (int64_t)(q - 2) * NK;
        double *y = Y + (int64_t)(q - 1) * NK;
        const double *yq2 = q == 1 ? ra.y_prev : (q == 2 ? X : Y + (int64_t)(q - 3) * NK);
        hipError_t e = dispatch_all(h.opt.val_dtype, h.opt.accum_f64, K, rec != nullptr, [&](auto d) {
            return decltype(d)::spmv(blocks, s, reinterpret_cast<const int4 *>(plan->d_chunk_spmv), plan->d_rowptr,
                                     plan->d_col, plan->d_val, x, y,
                                     q, yq2, ra);
        });
        if (e != hipSuccess) return fail(MPK_ERR_HIP, std::string("spmv launch: ") + hipGetErrorString(e));
    }
    return MPK_OK;
}

mpk_status mpk_run_sync(mpk_plan *plan, const double *X, double *Y, int32_t granularity, void *stream) {
    if (!plan) return fail(MPK_ERR_ARG, "null plan");
    mpk_status st = check_run_args(plan, X, Y, plan->hp.p, nullptr);
    if (st != MPK_OK) return st;
    if (granularity != MPK_SYNC_NODE && granularity != MPK_SYNC_WAVEFRONT)
        return fail(MPK_ERR_ARG, "granularity must be MPK_SYNC_NODE or MPK_SYNC_WAVEFRONT");
    HostPlan &h = plan->hp;
    if (h.recursive) return fail(MPK_ERR_UNSUPPORTED, "bulk-synchronous runs need an unrefined plan");
    if (h.n == 0) return MPK_OK;
    if (!supported(h.opt.val_dtype, h.opt.nrhs, false)) return fail(MPK_ERR_UNSUPPORTED, "nrhs/dtype combination");
    const int K = h.opt.nrhs;
    const int64_t NK = h.n * K;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int32_t G = (int32_t)h.group_ptr.size() - 1, P = h.p;
    SegList L;
    L.n = 0;
    L.start[0] = 0;
    auto add = [&](int32_t g, int32_t q) {
        const int32_t c0 = h.tile_chunk[h.group_tile[g]], c1 = h.tile_chunk[h.group_tile[g + 1]];
        L.c0[L.n] = c0;
        L.q[L.n] = q;
        L.start[L.n + 1] = L.start[L.n] + (c1 - c0);
        ++L.n;
    };
    auto flush = [&]() -> mpk_status {
        const int blocks = L.n ? L.start[L.n] : 0;
        if (blocks > 0) {
            hipError_t e = dispatch_all(h.opt.val_dtype, h.opt.accum_f64, K, false, [&](auto d) {
                return decltype(d)::seg(blocks, s, L, reinterpret_cast<const int4 *>(plan->d_chunk), plan->d_rowptr,
                                        plan->d_col, plan->d_val, X, Y, NK);
            });
            if (e != hipSuccess) return fail(MPK_ERR_HIP, std::string("segment launch: ") + hipGetErrorString(e));
        }
        L.n = 0;
        return MPK_OK;
    };
    if (granularity == MPK_SYNC_NODE) {
        // the Lp schedule, one node per launch
        const int64_t nodes = (int64_t)h.schedule.size() / 3;
        for (int64_t k = 0; k < nodes; ++k) {
            add(h.schedule[3 * k + 2], h.schedule[3 * k + 1]);
            if ((st = flush()) != MPK_OK) return st;
        }
        return MPK_OK;
    }
    // wavefronts w = g + 2q: node (g, q) needs groups g-1..g+1 at power q-1,
    // whose wavefronts are w-3..w-1, so the nodes of one wavefront are
    // independent and a launch per wavefront respects every dependency
    for (int32_t w = 2; w <= G - 1 + 2 * P; ++w) {
        for (int32_t q = 1; q <= P; ++q) {
            const int32_t g = w - 2 * q;
            if (g >= 0 && g < G) add(g, q);
        }
        if ((st = flush()) != MPK_OK) return st;
    }
    return MPK_OK;
}

mpk_status mpk_plan_status(mpk_plan *plan, void *stream) {
    if (!plan) return fail(MPK_ERR_ARG, "null plan");
    if (!plan->uploaded) return fail(MPK_ERR_STATE, "plan not uploaded");
    HIP_TRY(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)));
    uint32_t ctrl[4];
    HIP_TRY(hipMemcpy(ctrl, plan->d_ctrl, sizeof(ctrl), hipMemcpyDeviceToHost));
    // ctrl[0]: epoch of the last completed run; ctrl[2]: epoch of a run that timed out
    if (ctrl[0] != 0 && ctrl[2] == ctrl[0])
        return fail(MPK_ERR_TIMEOUT, "dependency wait timed out at ticket " + std::to_string(ctrl[3]));
    return MPK_OK;
}

void mpk_plan_destroy(mpk_plan *plan) {
    if (!plan) return;
    free_all(plan->allocs);
    if (plan->resident) {
        (void)hipFree(plan->rm.rowptr);
        (void)hipFree(plan->rm.col);
        (void)hipFree(plan->rm.val);
    }
    delete plan;
}

mpk_status spmv_create(const mpk_csr *A, const mpk_options *opt, mpk_spmv **out) {
    if (!out) return fail(MPK_ERR_ARG, "null output pointer");
    *out = nullptr;
    mpk_options o;
    mpk_options_default(&o);
    if (opt) {
        if (opt->size != sizeof(mpk_options)) return fail(MPK_ERR_ARG, "mpk_options.size mismatch");
        o = *opt;
    }
    mpk_status st = validate_csr(A);
    if (st != MPK_OK) return st;
    if (o.val_dtype < MPK_F64 || o.val_dtype > MPK_BF16) return fail(MPK_ERR_ARG, "bad val_dtype");
    if (o.accum_f64 != 0 && o.accum_f64 != 1) return fail(MPK_ERR_ARG, "accum_f64 must be 0 or 1");
    if (o.reserved0 != 0 || o.reserved != 0) return fail(MPK_ERR_ARG, "reserved option fields must be 0");
    if (o.nrhs < 1 || o.nrhs > MPK_MAX_NRHS || !supported(o.val_dtype, o.nrhs, false))
        return fail(MPK_ERR_UNSUPPORTED, "nrhs/dtype combination");
    mpk_spmv *h = new (std::nothrow) mpk_spmv();
    if (!h) return fail(MPK_ERR_OOM, "host allocation failed");
    h->n = A->n;
    h->nnz = A->nnz;
    h->dtype = o.val_dtype;
    h->acc64 = o.accum_f64;
    h->nrhs = o.nrhs;
    std::vector<int32_t> rp(A->n + 1);
    for (int64_t i = 0; i <= A->n; ++i) rp[i] = (int32_t)A->rowptr[i];
    std::vector<int32_t> chunks;
    append_chunks(rp, 0, A->n, spmv_chunk_nnz(o.nrhs, fp32_products(o.val_dtype, o.accum_f64)), kChunkRows, chunks);
    chunks.push_back((int32_t)A->n);
    h->nchunks = (int64_t)chunks.size() - 1;
    const std::vector<int32_t> desc = chunk_descriptors(chunks, rp.data());
    std::vector<uint8_t> vbuf;
    convert_values(A->val, A->nnz, o.val_dtype, vbuf);
    hipError_t e;
    uint8_t *dv = nullptr;
    if ((e = dev_alloc(h->allocs, &h->d_rowptr, A->n + 1)) != hipSuccess ||
        (e = dev_alloc(h->allocs, &h->d_col, A->nnz)) != hipSuccess ||
        (e = dev_alloc(h->allocs, &dv, vbuf.size())) != hipSuccess ||
        (e = dev_alloc(h->allocs, &h->d_chunk, std::max<size_t>(desc.size(), 4))) != hipSuccess) {
        free_all(h->allocs);
        delete h;
        return fail(e == hipErrorOutOfMemory ? MPK_ERR_OOM : MPK_ERR_HIP, hipGetErrorString(e));
    }
    h->d_val = dv;
    if ((e = hipMemcpy(h->d_rowptr, rp.data(), sizeof(int32_t) * (A->n + 1), hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (A->nnz && (e = hipMemcpy(h->d_col, A->col, sizeof(int32_t) * A->nnz, hipMemcpyHostToDevice)) !=
                       hipSuccess) ||
        (A->nnz && (e = hipMemcpy(h->d_val, vbuf.data(), A->nnz * value_bytes(o.val_dtype),
                                  hipMemcpyHostToDevice)) != hipSuccess) ||
        (!desc.empty() && (e = hipMemcpy(h->d_chunk, desc.data(), sizeof(int32_t) * desc.size(),
                                         hipMemcpyHostToDevice)) != hipSuccess)) {
        free_all(h->allocs);
        delete h;
        return fail(MPK_ERR_HIP, hipGetErrorString(e));
    }
    *out = h;
    return MPK_OK;
}

static mpk_status spmv_launch(mpk_spmv *h, const double *x, double *y, hipStream_t s) {
    RecArgs ra;
    (void)fill_rec(nullptr, 1, h->nrhs, ra);
    hipError_t e = dispatch_all(h->dtype, h->acc64, h->nrhs, false, [&](auto d) {
        return decltype(d)::spmv((int)h->nchunks, s, reinterpret_cast<const int4 *>(h->d_chunk), h->d_rowptr,
                                 h->d_col, h->d_val, x, y, 1,
                                 nullptr, ra);
    });
    if (e != hipSuccess) return fail(MPK_ERR_HIP, std::string("spmv launch: ") + hipGetErrorString(e));
    return MPK_OK;
}

mpk_status spmv_run(mpk_spmv *h, const double *x, double *y, void *stream) {
    if (!h) return fail(MPK_ERR_ARG, "null handle");
    if (h->n == 0) return MPK_OK;
    if (!x || !y) return fail(MPK_ERR_ARG, "null vector");
    if (x == y) return fail(MPK_ERR_ARG, "x and y alias");
    return spmv_launch(h, x, y, reinterpret_cast<hipStream_t>(stream));
}

mpk_status spmv_powers_run(mpk_spmv *h, int32_t p, const double *X, double *Y, void *stream) {
    if (!h) return fail(MPK_ERR_ARG, "null handle");
    if (p < 1 || p > 4096) return fail(MPK_ERR_ARG, "p out of range");
    if (h->n == 0) return MPK_OK;
    if (!X || !Y) return fail(MPK_ERR_ARG, "null vector");
    const int64_t NK = h->n * h->nrhs;
    for (int q = 1; q <= p; ++q) {
        const double *x = q == 1 ? X : Y + (q - 2) * NK;
        mpk_status st = spmv_launch(h, x, Y + (q - 1) * NK, reinterpret_cast<hipStream_t>(stream));
        if (st != MPK_OK) return st;
    }
    return MPK_OK;
}

void spmv_destroy(mpk_spmv *h) {
    if (!h) return;
    free_all(h->allocs);
    delete h;
}

mpk_status mpk_bw_probe(const void *buf, uint64_t bytes, int32_t reps, int32_t workgroups, double *sink,
                        void *stream) {
    if (!buf || !sink) return fail(MPK_ERR_ARG, "null pointer");
    if (bytes % 16 || ((uintptr_t)buf % 16)) return fail(MPK_ERR_ARG, "buffer must be 16-byte aligned");
    if (reps < 1 || workgroups < 1) return fail(MPK_ERR_ARG, "reps and workgroups must be >= 1");
    hipLaunchKernelGGL(bw_probe, dim3(workgroups), dim3(kBlock), 0, reinterpret_cast<hipStream_t>(stream),
                       reinterpret_cast<const double2 *>(buf), (int64_t)(bytes / 16), reps, sink);
    HIP_TRY(hipGetLastError());
    return MPK_OK;
}

mpk_status mpk_bw_probe_ex(const void *buf, uint64_t bytes, int32_t reps, int32_t workgroups,
                           int32_t loads_per_thread, int32_t parts, double *sink, void *stream) {
    if (!buf || !sink) return fail(MPK_ERR_ARG, "null pointer");
    if ((uintptr_t)buf % 16) return fail(MPK_ERR_ARG, "buffer must be 16-byte aligned");
    if (parts != 1 && parts != 8) return fail(MPK_ERR_ARG, "parts must be 1 or 8");
    if (bytes == 0 || bytes % (16u * (uint64_t)parts)) return fail(MPK_ERR_ARG, "bytes must be a multiple of 16*parts");
    if (reps < 1 || workgroups < parts) return fail(MPK_ERR_ARG, "reps >= 1 and workgroups >= parts required");
    const int64_t n2 = (int64_t)(bytes / 16 / (uint64_t)parts);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const double2 *b = reinterpret_cast<const double2 *>(buf);
    switch (loads_per_thread) {
        case 1: hipLaunchKernelGGL(bw_probe_ex<1>, dim3(workgroups), dim3(kBlock), 0, s, b, n2, parts, reps, sink); break;
        case 2: hipLaunchKernelGGL(bw_probe_ex<2>, dim3(workgroups), dim3(kBlock), 0, s, b, n2, parts, reps, sink); break;
        case 4: hipLaunchKernelGGL(bw_probe_ex<4>, dim3(workgroups), dim3(kBlock), 0, s, b, n2, parts, reps, sink); break;
        case 8: hipLaunchKernelGGL(bw_probe_ex<8>, dim3(workgroups), dim3(kBlock), 0, s, b, n2, parts, reps, sink); break;
        default: return fail(MPK_ERR_ARG, "loads_per_thread must be 1, 2, 4 or 8");
    }
    HIP_TRY(hipGetLastError());
    return MPK_OK;
}

mpk_status mpk_xcd_ids(int32_t *ids, int32_t workgroups, int64_t spin, void *stream) {
    if (!ids) return fail(MPK_ERR_ARG, "null pointer");
    if (workgroups < 1 || spin < 0) return fail(MPK_ERR_ARG, "workgroups >= 1 and spin >= 0 required");
    hipLaunchKernelGGL(xcd_ids_kernel, dim3(workgroups), dim3(kBlock), 0, reinterpret_cast<hipStream_t>(stream), ids,
                       spin);
    HIP_TRY(hipGetLastError());
    return MPK_OK;
}

mpk_status mpk_hop_probe(uint32_t *flags, int32_t peer, int32_t scope, int32_t iters, int64_t max_polls,
                         uint64_t *out, int32_t *wall_clock_khz, void *stream) {
    if (!flags || !out) return fail(MPK_ERR_ARG, "null pointer");
    if (wall_clock_khz) {
        int dev = 0;
        HIP_TRY(hipGetDevice(&dev));
        HIP_TRY(hipDeviceGetAttribute(wall_clock_khz, hipDeviceAttributeWallClockRate, dev));
    }
    if (peer < 1 || peer > 255 || (scope != 0 && scope != 1) || iters < 1 || max_polls < 1)
        return fail(MPK_ERR_ARG, "peer in [1, 255], scope 0 or 1, iters >= 1 and max_polls >= 1 required");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIP_TRY(hipMemsetAsync(flags, 0, 64 * sizeof(uint32_t), s));
    hipLaunchKernelGGL(hop_probe_kernel, dim3(peer + 1), dim3(64), 0, s, flags, peer, scope, iters, max_polls, out);
    HIP_TRY(hipGetLastError());
    return MPK_OK;
}

}  // extern "C"
