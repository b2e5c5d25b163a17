// Device code of the MPK library for gfx950 (CDNA4, 64-lane wavefronts).
//
// One building block serves both the baseline SpMV (Sec. 3.1, Fig. 2) and the
// level-blocked MPK (Sec. 4): `rows_pass` computes y = A x (plus an optional
// three-term recurrence epilogue, Sec. 7) on a contiguous range of rows, with
// G lanes cooperating on each row.  Inside one group of G lanes, K adjacent
// lanes share one stored nonzero and handle the K right-hand sides (row-major
// N x K vectors), and S = G/K such slots walk the row's nonzeros with stride
// S, so a wavefront streams the row's val/col entries contiguously; the
// partial sums are combined with cross-lane shuffles.
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

// y[r] = A[r,:] x for rows [r0, r1) (and the epilogue when REC).
//   q      power being computed (1-based), selects the coefficients
//   yq2    y_{q-2} (only read when REC and gamma != 0)
template <typename VT, int K, int G, bool REC>
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
            if (slot == 0 && r < r1) y[(int64_t)r * K + c] = (double)sum;
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
                    y[idx] = v;
                    if (rec.acc) {
                        const double cr = rec.coef_re[q - 1], ci = rec.coef_im[q - 1];
                        // (cr + i ci)(re + i im): re part cr*re - ci*im, im part cr*im + ci*re
                        const double add = (c == 0) ? (cr * v - ci * other) : (cr * v + ci * other);
                        rec.acc[idx] += add;
                    }
                }
            } else if (slot == 0 && r < r1) {
                y[idx] = v;
                if (rec.acc) rec.acc[idx] += rec.coef_re[q - 1] * v;
            }
        }
    }
}

}  // namespace mpk
