// Device code of the MPK library for gfx950 (CDNA4, 64-lane wavefronts).
//
// One row kernel serves both the baseline SpMV (Sec. 3.1, Fig. 2) and the
// level-blocked MPK (Sec. 4): chunk_pass computes y = A x on a contiguous
// range of rows (k right-hand sides, row-major N x k vectors), with an
// optional three-term recurrence epilogue (Sec. 7).  The rows are cut into
// chunks of at most chunk_nnz(k, NP) stored nonzeros.  Phase 1: every thread
// forms NP of the chunk's k-column products (nonzero j, column c
// flattened with c fastest), issuing all its val/col loads and then all its
// gathers without waiting in between, and writes them to LDS together with
// the chunk's row pointers.  Phase 2: after a barrier, a thread sums one
// row's products (k = 1) or one column of a row (k >= 2) in stored order,
// reading four products ahead, and applies the epilogue.  A
// chunk is described by (first row, end row, first nonzero, end nonzero).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mpk.h"
#include "mpk_internal.h"

namespace mpk {

constexpr int kBlock = 256;  // threads per workgroup (4 wavefronts)

// bfloat16 values are stored as their upper 16 bits
struct bf16_t {
    uint16_t bits;
};
// The same storage with FP64 arithmetic: values widened to FP64, the input
// vector read as it is, products and row sums in FP64.
struct f32w_t {
    float v;
};
struct bf16w_t {
    uint16_t bits;
};

template <typename VT>
struct AccumType {
    using T = float;  // low-precision values: FP32 accumulation
};
template <>
struct AccumType<double> {
    using T = double;
};
template <>
struct AccumType<f32w_t> {
    using T = double;
};
template <>
struct AccumType<bf16w_t> {
    using T = double;
};

__device__ __forceinline__ double load_value(const double *v, int64_t j) { return v[j]; }
__device__ __forceinline__ float load_value(const float *v, int64_t j) { return v[j]; }
__device__ __forceinline__ float load_value(const bf16_t *v, int64_t j) {
    return __uint_as_float(((uint32_t)v[j].bits) << 16);
}
__device__ __forceinline__ double load_value(const f32w_t *v, int64_t j) { return (double)v[j].v; }
__device__ __forceinline__ double load_value(const bf16w_t *v, int64_t j) {
    return (double)__uint_as_float(((uint32_t)v[j].bits) << 16);
}

// Coefficients of the recurrence epilogue, passed by value in the kernel
// arguments (p <= MPK_MAX_POWER).
struct RecArgs {
    double alpha[MPK_MAX_POWER];
    double beta[MPK_MAX_POWER];
    double gamma[MPK_MAX_POWER];
    double coef_re[MPK_MAX_POWER];
    double coef_im[MPK_MAX_POWER];
    const double *y_prev;  // y_{-1}
    double *acc;           // accumulator or null
    int32_t complex_pairs;
    int32_t start_acc;     // power 1 sets acc = c0 * y_0 + coef_1 * y_1
    double c0_re, c0_im;
};

// Output store.  COH = true (inside the persistent MPK kernel, where other
// workgroups on other XCDs read the result in the same launch): an
// agent-scope relaxed atomic store, which is written through to the
// device-coherent level, so the publishing workgroup only has to wait for its
// stores to complete instead of writing back its whole L2.
// Read of a value other workgroups update in the same launch (the running
// sum of the recurrence): an agent-scope atomic load, coherent whatever the
// caches hold.
template <bool COH>
__device__ __forceinline__ double get(const double *p) {
    if constexpr (COH)
        return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        return *p;
}

template <bool COH>
__device__ __forceinline__ void put(double *p, double v) {
    if constexpr (COH)
        __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        *p = v;
}

static_assert(kBlock == 256, "the chunk lengths of mpk_internal.h assume 256 threads per workgroup");

// nonzeros per chunk for k right-hand sides at NP products per thread:
// kBlock * NP products (NP * 2 KB of LDS in FP64).  The persistent MPK kernel
// and the bulk-synchronous kernels run on the plan's tile chunks with
// NP = mpk_products_per_thread(k), the baseline SpMV on chunks of its own
// with NP = spmv_products_per_thread(k, FP32 products).
__host__ __device__ constexpr int chunk_nnz(int K, int NP) { return kBlock * NP / K; }
template <typename VT, int K, int NP>
struct ChunkLds {
    typename AccumType<VT>::T prod[kBlock * NP];
    int32_t rb[kChunkRows + 1];  // row pointers of the chunk's rows
};

// Barrier for LDS only: each wavefront waits for its own LDS operations, then
// the workgroup meets.  Unlike __syncthreads() it does not wait for
// outstanding global loads, which stay in flight across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Epilogue for one output row, all K columns held by the calling thread.
template <int K, bool REC, bool COH>
__device__ __forceinline__ void store_row(int64_t r, const double *v_in, const double *__restrict__ x,
                                          double *__restrict__ y, int q, const double *__restrict__ yq2,
                                          const RecArgs &rec) {
    double v[K];
#pragma unroll
    for (int c = 0; c < K; ++c) v[c] = v_in[c];
    if constexpr (REC) {
        const double al = rec.alpha[q - 1], be = rec.beta[q - 1], ga = rec.gamma[q - 1];
#pragma unroll
        for (int c = 0; c < K; ++c) {
            v[c] *= al;
            if (be != 0.0) v[c] += be * x[r * K + c];
            if (ga != 0.0) v[c] += ga * yq2[r * K + c];
        }
    }
#pragma unroll
    for (int c = 0; c < K; ++c) put<COH>(y + r * K + c, v[c]);
    if constexpr (REC) {
        if (rec.acc) {
            // the running sum: acc, or c0 * y_0 when power 1 starts it (x is y_0 then)
            const bool start = rec.start_acc && q == 1;
            if (K == 2 && rec.complex_pairs) {
                const double cr = rec.coef_re[q - 1], ci = rec.coef_im[q - 1];
                double a0, a1;
                if (start) {
                    const double x0 = x[r * K + 0], x1 = x[r * K + 1];
                    a0 = rec.c0_re * x0 - rec.c0_im * x1;
                    a1 = rec.c0_re * x1 + rec.c0_im * x0;
                } else {
                    a0 = get<COH>(rec.acc + r * K + 0);
                    a1 = get<COH>(rec.acc + r * K + 1);
                }
                put<COH>(rec.acc + r * K + 0, a0 + (cr * v[0] - ci * v[1]));
                put<COH>(rec.acc + r * K + 1, a1 + (cr * v[1] + ci * v[0]));
            } else {
#pragma unroll
                for (int c = 0; c < K; ++c) {
                    const double a = start ? rec.c0_re * x[r * K + c] : get<COH>(rec.acc + r * K + c);
                    put<COH>(rec.acc + r * K + c, a + rec.coef_re[q - 1] * v[c]);
                }
            }
        }
    }
}

// Epilogue for one output entry (row r, column c) of k = 2 columns, held by
// lane pair (2r', 2r'+1) of a wavefront; the complex accumulator update
// takes the partner column from the other lane of the pair.  Every lane of
// the pair must call it together.  The operands it reads from memory (own
// entry of y_{q-1}, of y_{q-2}, of the running sum) are loaded by
// col2_operands, which a caller may issue early to hide their latency.
struct Col2Ops {
    double xs, yq, acc;
};

template <bool COH>
__device__ __forceinline__ Col2Ops col2_operands(int64_t r, int c, const double *__restrict__ x,
                                                 const double *__restrict__ yq2, int q, const RecArgs &rec) {
    const int64_t i = r * 2 + c;
    const bool start = rec.start_acc && q == 1;
    Col2Ops o;
    o.xs = (rec.beta[q - 1] != 0.0 || (rec.acc && start)) ? x[i] : 0.0;
    o.yq = rec.gamma[q - 1] != 0.0 ? yq2[i] : 0.0;
    o.acc = (rec.acc && !start) ? get<COH>(rec.acc + i) : 0.0;
    return o;
}

template <bool REC, bool COH>
__device__ __forceinline__ void store_col2(int64_t r, int c, double v, const Col2Ops &op, double *__restrict__ y,
                                           int q, const RecArgs &rec) {
    const int64_t i = r * 2 + c;
    if constexpr (REC) {
        const double al = rec.alpha[q - 1], be = rec.beta[q - 1], ga = rec.gamma[q - 1];
        v *= al;
        if (be != 0.0) v += be * op.xs;
        if (ga != 0.0) v += ga * op.yq;
    }
    put<COH>(y + i, v);
    if constexpr (REC) {
        if (rec.acc) {
            const bool start = rec.start_acc && q == 1;
            if (rec.complex_pairs) {
                const double vo = __shfl_xor(v, 1);
                const double cr = rec.coef_re[q - 1], ci = rec.coef_im[q - 1];
                double a;
                if (start) {
                    const double xo = __shfl_xor(op.xs, 1);
                    a = c == 0 ? rec.c0_re * op.xs - rec.c0_im * xo : rec.c0_re * op.xs + rec.c0_im * xo;
                } else {
                    a = op.acc;
                }
                put<COH>(rec.acc + i, a + (c == 0 ? cr * v - ci * vo : cr * v + ci * vo));
            } else {
                const double a = start ? rec.c0_re * op.xs : op.acc;
                put<COH>(rec.acc + i, a + rec.coef_re[q - 1] * v);
            }
        }
    }
}

// Registers of one chunk between its matrix loads and its gathers.
template <typename VT, int K, int NP>
struct ChunkRegs {
    static constexpr int NRB = (kChunkRows + 1 + kBlock - 1) / kBlock;
    int cj[NP];
    typename AccumType<VT>::T a[NP];
    int rbv[NRB];
};

// A chunk of the common kind: at least one and at most chunk_nnz(K, NP)
// stored nonzeros (uniform test).
template <int K, int NP>
__device__ __forceinline__ bool plain_chunk(const int4 d) {
    return d.w > d.z && d.w - d.z <= chunk_nnz(K, NP);
}

// Phase 1, first half, of a plain chunk d = (r0, r1, j0, j1): the row
// pointers rowptr[r0 .. r1] (uniform guards) and the chunk's col entries,
// with its val entries unless VALS is false.  Every load is unconditional
// (slots past the chunk re-read its last entry, whose product phase 2 never
// reads), so they are all in flight together.  Nothing here depends on
// vector data: a caller may issue these loads before it has waited for the
// vector the chunk multiplies.
template <typename VT, int K, int NP, bool VALS = true>
__device__ __forceinline__ void chunk_load(const int4 d, const int32_t *__restrict__ rowptr,
                                           const int32_t *__restrict__ col, const VT *__restrict__ val,
                                           ChunkRegs<VT, K, NP> &g) {
    using AT = typename AccumType<VT>::T;
    const int tid = threadIdx.x;
    const int nr = d.y - d.x;
#pragma unroll
    for (int m = 0; m < ChunkRegs<VT, K, NP>::NRB; ++m)
        if (m * kBlock <= nr) g.rbv[m] = rowptr[d.x + min(tid + m * kBlock, nr)];
#pragma unroll
    for (int m = 0; m < NP; ++m) {
        const int pidx = tid + m * kBlock;
        const int jc = min(d.z + pidx / K, d.w - 1);
        g.cj[m] = col[jc];
        if constexpr (VALS) g.a[m] = (AT)load_value(val, jc);
    }
}

// The values of a plain chunk whose row pointers and columns chunk_load
// (VALS = false) has already loaded.
template <typename VT, int K, int NP>
__device__ __forceinline__ void chunk_load_vals(const int4 d, const VT *__restrict__ val, ChunkRegs<VT, K, NP> &g) {
    using AT = typename AccumType<VT>::T;
    const int tid = threadIdx.x;
#pragma unroll
    for (int m = 0; m < NP; ++m) {
        const int pidx = tid + m * kBlock;
        const int jc = min(d.z + pidx / K, d.w - 1);
        g.a[m] = (AT)load_value(val, jc);
    }
}

// The gathers of a plain chunk (and, for k = 2 with the recurrence, the
// epilogue operands of the calling thread's first output), issued without
// waiting, so a caller may issue the next chunk's matrix loads behind them.
template <typename VT, int K, int NP>
struct ChunkGather {
    typename AccumType<VT>::T xv[NP];
    Col2Ops pre, pre2;  // epilogue operands of outputs tid and tid + kBlock (k = 2, recurrence)
};

template <typename VT, int K, bool REC, bool COH, int NP>
__device__ __forceinline__ void chunk_gather(const int4 d, const ChunkRegs<VT, K, NP> &g, const double *__restrict__ x,
                                             int q, const double *__restrict__ yq2, const RecArgs &rec,
                                             ChunkGather<VT, K, NP> &gx) {
    using AT = typename AccumType<VT>::T;
    const int tid = threadIdx.x;
    const int nr = d.y - d.x;
#pragma unroll
    for (int m = 0; m < NP; ++m) gx.xv[m] = (AT)x[(int64_t)g.cj[m] * K + ((tid + m * kBlock) % K)];
    gx.pre = Col2Ops{};
    gx.pre2 = Col2Ops{};
    if constexpr (K == 2 && REC) {
        // a chunk of 8 products per thread (1024 nonzeros at k = 2) usually
        // has at most 256 rows, i.e. at most two outputs per thread: both
        // have their operands loaded here, so none is loaded after the row
        // sums (with 16 products further outputs load theirs in phase 2)
        if (tid < nr * 2) gx.pre = col2_operands<COH>(d.x + (tid >> 1), tid & 1, x, yq2, q, rec);
        if (tid + kBlock < nr * 2)
            gx.pre2 = col2_operands<COH>(d.x + ((tid + kBlock) >> 1), tid & 1, x, yq2, q, rec);
    }
}

template <typename VT, int K, bool REC, bool COH, int NP>
__device__ __forceinline__ void chunk_reduce(const int4 d, const ChunkRegs<VT, K, NP> &g, const ChunkGather<VT, K, NP> &gx,
                                             const double *__restrict__ x, double *__restrict__ y, int q,
                                             const double *__restrict__ yq2, const RecArgs &rec,
                                             ChunkLds<VT, K, NP> &lds);

// The rest of a plain chunk: gathers of x, products and row pointers to LDS,
// then phase 2 (one thread per row for k = 1, per (row, column) for k >= 2,
// stored order, four products read ahead) and the epilogue.
template <typename VT, int K, bool REC, bool COH, int NP>
__device__ __forceinline__ void chunk_finish(const int4 d, const ChunkRegs<VT, K, NP> &g, const double *__restrict__ x,
                                             double *__restrict__ y, int q, const double *__restrict__ yq2,
                                             const RecArgs &rec, ChunkLds<VT, K, NP> &lds) {
    ChunkGather<VT, K, NP> gx;
    chunk_gather<VT, K, REC, COH, NP>(d, g, x, q, yq2, rec, gx);
    chunk_reduce<VT, K, REC, COH, NP>(d, g, gx, x, y, q, yq2, rec, lds);
}

template <typename VT, int K, bool REC, bool COH, int NP>
__device__ __forceinline__ void chunk_reduce(const int4 d, const ChunkRegs<VT, K, NP> &g, const ChunkGather<VT, K, NP> &gx,
                                             const double *__restrict__ x, double *__restrict__ y, int q,
                                             const double *__restrict__ yq2, const RecArgs &rec,
                                             ChunkLds<VT, K, NP> &lds) {
    using AT = typename AccumType<VT>::T;
    const int tid = threadIdx.x;
    const int r0 = d.x, j0 = d.z;
    const int nr = d.y - d.x;
    const AT *xv = gx.xv;
    const Col2Ops &pre = gx.pre, &pre2 = gx.pre2;
#pragma unroll
    for (int m = 0; m < ChunkRegs<VT, K, NP>::NRB; ++m)
        if (m * kBlock <= nr && tid + m * kBlock <= nr) lds.rb[tid + m * kBlock] = g.rbv[m];
#pragma unroll
    for (int m = 0; m < NP; ++m) lds.prod[tid + m * kBlock] = g.a[m] * xv[m];
    lds_barrier();
    if constexpr (K == 2) {
        // one lane per (row, column): the lanes of a wavefront store and load
        // consecutive entries (a lane per row would leave every store
        // instruction half of each line); stored order per column
        const int nout = nr * 2;
        for (int o = tid; o < nout; o += kBlock) {
            const int r = o >> 1, c = o & 1;
            const int s = lds.rb[r] - j0, e = lds.rb[r + 1] - j0;
            AT sum = (AT)0;
            int i = s;
            for (; i + 4 <= e; i += 4) {
                const AT p0 = lds.prod[i * 2 + c], p1 = lds.prod[(i + 1) * 2 + c];
                const AT p2 = lds.prod[(i + 2) * 2 + c], p3 = lds.prod[(i + 3) * 2 + c];
                sum = sum + p0;
                sum = sum + p1;
                sum = sum + p2;
                sum = sum + p3;
            }
            for (; i < e; ++i) sum = sum + lds.prod[i * 2 + c];
            Col2Ops op{};
            if constexpr (REC)
                op = o == tid ? pre : o == tid + kBlock ? pre2 : col2_operands<COH>(r0 + r, c, x, yq2, q, rec);
            store_col2<REC, COH>(r0 + r, c, (double)sum, op, y, q, rec);
        }
    } else if constexpr (K == 1) {
        for (int r = tid; r < nr; r += kBlock) {
            const int s = lds.rb[r] - j0, e = lds.rb[r + 1] - j0;
            AT sum[K];
#pragma unroll
            for (int c = 0; c < K; ++c) sum[c] = (AT)0;
            int i = s;
            for (; i + 4 <= e; i += 4) {
                AT pr[4][K];
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int c = 0; c < K; ++c) pr[u][c] = lds.prod[(i + u) * K + c];
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int c = 0; c < K; ++c) sum[c] = sum[c] + pr[u][c];
            }
            for (; i < e; ++i) {
#pragma unroll
                for (int c = 0; c < K; ++c) sum[c] = sum[c] + lds.prod[i * K + c];
            }
            double v[K];
#pragma unroll
            for (int c = 0; c < K; ++c) v[c] = (double)sum[c];
            store_row<K, REC, COH>(r0 + r, v, x, y, q, yq2, rec);
        }
    } else {
        const int nout = nr * K;
        for (int o = tid; o < nout; o += kBlock) {
            const int r = o / K, c = o % K;
            const int s = lds.rb[r] - j0, e = lds.rb[r + 1] - j0;
            AT sum = (AT)0;
            int i = s;
            for (; i + 4 <= e; i += 4) {
                const AT p0 = lds.prod[i * K + c], p1 = lds.prod[(i + 1) * K + c];
                const AT p2 = lds.prod[(i + 2) * K + c], p3 = lds.prod[(i + 3) * K + c];
                sum = sum + p0;
                sum = sum + p1;
                sum = sum + p2;
                sum = sum + p3;
            }
            for (; i < e; ++i) sum = sum + lds.prod[i * K + c];
            put<COH>(y + (int64_t)(r0 + r) * K + c, (double)sum);
        }
    }
    lds_barrier();  // LDS is reused by the next chunk
}

// One chunk d = (r0, r1, j0, j1): rows [r0, r1) with stored nonzeros
// [j0, j1), at most chunk_nnz(K, NP) of them and at most kChunkRows rows, or a
// single longer row.
template <typename VT, int K, bool REC, bool COH, int NP>
__device__ __forceinline__ void chunk_pass(const int4 d, const int32_t *__restrict__ rowptr,
                                           const int32_t *__restrict__ col, const VT *__restrict__ val,
                                           const double *__restrict__ x, double *__restrict__ y, int q,
                                           const double *__restrict__ yq2, const RecArgs &rec,
                                           ChunkLds<VT, K, NP> &lds) {
    using AT = typename AccumType<VT>::T;
    static_assert(K == 1 || K == 2 || !REC, "the recurrence epilogue handles k <= 2");
    const int tid = threadIdx.x;
    const int r0 = d.x, r1 = d.y, j0 = d.z, j1 = d.w;
    if (plain_chunk<K, NP>(d)) {
        ChunkRegs<VT, K, NP> g;
        chunk_load<VT, K, NP>(d, rowptr, col, val, g);
        chunk_finish<VT, K, REC, COH, NP>(d, g, x, y, q, yq2, rec, lds);
    } else if (j1 == j0) {  // rows without stored entries: y = 0 (uniform branch)
        for (int r = r0 + tid; r < r1; r += kBlock) {
            double v[K];
#pragma unroll
            for (int c = 0; c < K; ++c) v[c] = 0.0;
            if constexpr (K <= 2) {
                store_row<K, REC, COH>(r, v, x, y, q, yq2, rec);
            } else {
#pragma unroll
                for (int c = 0; c < K; ++c) put<COH>(y + (int64_t)r * K + c, 0.0);
            }
        }
    } else {
        // a single row longer than a chunk: thread (slot, c) accumulates
        // nonzeros slot, slot + S, ... of column c; then a tree over slots
        constexpr int S = kBlock / K;
        const int slot = tid / K, c = tid % K;
        AT part = (AT)0;
        for (int j = j0 + slot; j < j1; j += S)
            part = fma((AT)load_value(val, j), (AT)x[(int64_t)col[j] * K + c], part);
        lds.prod[tid] = part;
        __syncthreads();
        for (int w = S / 2; w > 0; w >>= 1) {
            if (slot < w) lds.prod[tid] += lds.prod[tid + w * K];
            __syncthreads();
        }
        if constexpr (K <= 2) {
            if (tid == 0) {
                double v[K];
#pragma unroll
                for (int cc = 0; cc < K; ++cc) v[cc] = (double)lds.prod[cc];
                store_row<K, REC, COH>(r0, v, x, y, q, yq2, rec);
            }
        } else {
            if (tid < K) put<COH>(y + (int64_t)r0 * K + tid, (double)lds.prod[tid]);
        }
        __syncthreads();
    }
}

}  // namespace mpk
