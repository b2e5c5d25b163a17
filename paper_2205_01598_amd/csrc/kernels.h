// Device code of the MPK library for gfx950 (CDNA4, 64-lane wavefronts).
//
// Two row kernels serve both the baseline SpMV (Sec. 3.1, Fig. 2) and the
// level-blocked MPK (Sec. 4); both compute y = A x on a contiguous range of
// rows, with an optional three-term recurrence epilogue (Sec. 7).
//
//  * chunk_pass (k <= 2 right-hand sides): the rows are cut into chunks of at
//    most chunk_nnz(k) stored nonzeros.  Every thread first loads its share of
//    the chunk's nonzeros (val, col and the gathered x entry, all
//    independent and coalesced, so a wavefront keeps many loads in flight)
//    and writes the products to LDS; after a barrier each thread sums the
//    products of whole rows, in stored order, and applies the epilogue.
//  * rows_pass (k >= 4): G lanes share one row; inside a group K adjacent
//    lanes take the K right-hand sides of one nonzero (row-major N x K
//    vectors), S = G/K slots walk the nonzeros with stride S, and partial
//    sums are combined with cross-lane shuffles.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mpk.h"

namespace mpk {

constexpr int kBlock = 256;  // threads per workgroup (4 wavefronts)

// bfloat16 values are stored as their upper 16 bits
struct bf16_t {
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

__device__ __forceinline__ double load_value(const double *v, int64_t j) { return v[j]; }
__device__ __forceinline__ float load_value(const float *v, int64_t j) { return v[j]; }
__device__ __forceinline__ float load_value(const bf16_t *v, int64_t j) {
    return __uint_as_float(((uint32_t)v[j].bits) << 16);
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
};

// Output store.  COH = true (inside the persistent MPK kernel, where other
// workgroups on other XCDs read the result in the same launch): an
// agent-scope relaxed atomic store, which is written through to the
// device-coherent level, so the publishing workgroup only has to wait for its
// stores to complete instead of writing back its whole L2.
template <bool COH>
__device__ __forceinline__ void put(double *p, double v) {
    if constexpr (COH)
        __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        *p = v;
}

// y[r] = A[r,:] x for rows [r0, r1) (and the epilogue when REC).
//   q      power being computed (1-based), selects the coefficients
//   yq2    y_{q-2} (only read when REC and gamma != 0)
template <typename VT, int K, int G, bool REC, bool COH>
__device__ __forceinline__ void rows_pass(int r0, int r1, const int32_t *__restrict__ rowptr,
                                          const int32_t *__restrict__ col, const VT *__restrict__ val,
                                          const double *__restrict__ x, double *__restrict__ y, int q,
                                          const double *__restrict__ yq2, const RecArgs &rec) {
    using AT = typename AccumType<VT>::T;
    static_assert(G >= K && G <= 64 && (G & (G - 1)) == 0, "bad lane group");
    constexpr int S = G / K;           // nonzero slots per row
    constexpr int RPP = kBlock / G;    // rows per pass of the workgroup
    const int tid = threadIdx.x;
    const int sub = tid / G;
    const int lane = tid % G;
    const int c = lane % K;
    const int slot = lane / K;
    for (int rb = r0; rb < r1; rb += RPP) {
        const int r = rb + sub;
        AT sum = (AT)0;
        if (r < r1) {
            const int s = rowptr[r], e = rowptr[r + 1];
#pragma unroll 4
            for (int j = s + slot; j < e; j += S) {
                const AT a = (AT)load_value(val, j);
                const int cj = col[j];
                const AT xv = (AT)x[(int64_t)cj * K + c];
                sum = fma(a, xv, sum);
            }
        }
#pragma unroll
        for (int off = G / 2; off >= K; off >>= 1) sum += __shfl_xor(sum, off, G);
        if constexpr (!REC) {
            if (slot == 0 && r < r1) put<COH>(y + (int64_t)r * K + c, (double)sum);
        } else {
            const int64_t idx = (int64_t)r * K + c;
            double v = (double)sum;
            if (r < r1) {
                const double al = rec.alpha[q - 1], be = rec.beta[q - 1], ga = rec.gamma[q - 1];
                v = al * v;
                if (be != 0.0) v += be * x[idx];
                if (ga != 0.0) v += ga * yq2[idx];
            }
            if (rec.complex_pairs) {
                // K == 2: lane c = 0 holds the real part, c = 1 the imaginary part
                const double other = __shfl_xor(v, 1, G);
                if (slot == 0 && r < r1) {
                    put<COH>(y + idx, v);
                    if (rec.acc) {
                        const double cr = rec.coef_re[q - 1], ci = rec.coef_im[q - 1];
                        // (cr + i ci)(re + i im): re part cr*re - ci*im, im part cr*im + ci*re
                        const double add = (c == 0) ? (cr * v - ci * other) : (cr * v + ci * other);
                        put<COH>(rec.acc + idx, rec.acc[idx] + add);
                    }
                }
            } else if (slot == 0 && r < r1) {
                put<COH>(y + idx, v);
                if (rec.acc) put<COH>(rec.acc + idx, rec.acc[idx] + rec.coef_re[q - 1] * v);
            }
        }
    }
}

constexpr int kNpt = 8;  // nonzeros per thread and chunk (k = 1)

// nonzeros per chunk for k right-hand sides: the chunk's k-column products
// stay at 16 KB of LDS (FP64), and for k >= 4 the gathered bytes per chunk
// stay constant
__host__ __device__ constexpr int chunk_nnz(int K) {
    return K == 1 ? kBlock * kNpt : K == 2 ? kBlock * kNpt / 2 : 4096 / K;
}
constexpr int kChunkRows = kBlock * kNpt;  // rows per chunk cap (phase 2 loop bound)

template <typename VT, int K>
struct ChunkLds {
    typename AccumType<VT>::T prod[chunk_nnz(K) * K];
};

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
            if (K == 2 && rec.complex_pairs) {
                const double cr = rec.coef_re[q - 1], ci = rec.coef_im[q - 1];
                const double a0 = rec.acc[r * K + 0], a1 = rec.acc[r * K + 1];
                put<COH>(rec.acc + r * K + 0, a0 + (cr * v[0] - ci * v[1]));
                put<COH>(rec.acc + r * K + 1, a1 + (cr * v[1] + ci * v[0]));
            } else {
#pragma unroll
                for (int c = 0; c < K; ++c)
                    put<COH>(rec.acc + r * K + c, rec.acc[r * K + c] + rec.coef_re[q - 1] * v[c]);
            }
        }
    }
}

// One chunk: rows [r0, r1) whose stored nonzeros fit in chunk_nnz(K), or a
// single longer row.
template <typename VT, int K, bool REC, bool COH>
__device__ __forceinline__ void chunk_pass(int r0, int r1, const int32_t *__restrict__ rowptr,
                                           const int32_t *__restrict__ col, const VT *__restrict__ val,
                                           const double *__restrict__ x, double *__restrict__ y, int q,
                                           const double *__restrict__ yq2, const RecArgs &rec,
                                           ChunkLds<VT, K> &lds) {
    using AT = typename AccumType<VT>::T;
    constexpr int NPT = chunk_nnz(K) / kBlock;
    const int tid = threadIdx.x;
    const int j0 = rowptr[r0], j1 = rowptr[r1];
    if (j1 - j0 <= chunk_nnz(K)) {
        if (j1 == j0) {  // rows without stored entries: y = 0 (uniform branch)
            for (int r = r0 + tid; r < r1; r += kBlock) {
                double v[K];
#pragma unroll
                for (int c = 0; c < K; ++c) v[c] = 0.0;
                store_row<K, REC, COH>(r, v, x, y, q, yq2, rec);
            }
            return;
        }
        // phase 1: products of the chunk's nonzeros.  Every load is
        // unconditional (slots past the chunk re-read its last entry, whose
        // product phase 2 never reads), so a thread issues all its val/col
        // loads, then all its gathers, without waiting in between.
        int cj[NPT];
        AT a[NPT];
#pragma unroll
        for (int m = 0; m < NPT; ++m) {
            const int jc = min(j0 + tid + m * kBlock, j1 - 1);
            cj[m] = col[jc];
            a[m] = (AT)load_value(val, jc);
        }
        // row bounds of the thread's first phase-2 row, fetched early
        const int rf = min(r0 + tid, r1);
        const int rs0 = rowptr[rf], re0 = rowptr[min(rf + 1, r1)];
        AT xv[NPT][K];
#pragma unroll
        for (int m = 0; m < NPT; ++m)
#pragma unroll
            for (int c = 0; c < K; ++c) xv[m][c] = (AT)x[(int64_t)cj[m] * K + c];
#pragma unroll
        for (int m = 0; m < NPT; ++m)
#pragma unroll
            for (int c = 0; c < K; ++c) lds.prod[(tid + m * kBlock) * K + c] = a[m] * xv[m][c];
        __syncthreads();
        // phase 2: one thread per row sums its products in stored order
        for (int r = r0 + tid; r < r1; r += kBlock) {
            const int s = (r == rf ? rs0 : rowptr[r]) - j0, e = (r == rf ? re0 : rowptr[r + 1]) - j0;
            AT sum[K];
#pragma unroll
            for (int c = 0; c < K; ++c) sum[c] = (AT)0;
            for (int i = s; i < e; ++i) {
#pragma unroll
                for (int c = 0; c < K; ++c) sum[c] = sum[c] + lds.prod[i * K + c];
            }
            double v[K];
#pragma unroll
            for (int c = 0; c < K; ++c) v[c] = (double)sum[c];
            store_row<K, REC, COH>(r, v, x, y, q, yq2, rec);
        }
        __syncthreads();  // LDS is reused by the next chunk
    } else {
        // a single row longer than a chunk: strided partial sums + tree reduction
        AT part[K];
#pragma unroll
        for (int c = 0; c < K; ++c) part[c] = (AT)0;
        for (int j = j0 + tid; j < j1; j += kBlock) {
            const AT av = (AT)load_value(val, j);
            const int cc = col[j];
#pragma unroll
            for (int c = 0; c < K; ++c) part[c] = fma(av, (AT)x[(int64_t)cc * K + c], part[c]);
        }
#pragma unroll
        for (int c = 0; c < K; ++c) lds.prod[tid * K + c] = part[c];
        __syncthreads();
        for (int w = kBlock / 2; w > 0; w >>= 1) {
            if (tid < w) {
#pragma unroll
                for (int c = 0; c < K; ++c) lds.prod[tid * K + c] += lds.prod[(tid + w) * K + c];
            }
            __syncthreads();
        }
        if (tid == 0) {
            double v[K];
#pragma unroll
            for (int c = 0; c < K; ++c) v[c] = (double)lds.prod[c];
            store_row<K, REC, COH>(r0, v, x, y, q, yq2, rec);
        }
        __syncthreads();
    }
}

}  // namespace mpk
