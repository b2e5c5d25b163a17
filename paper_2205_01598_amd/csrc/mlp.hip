// Small fully connected network for the learned tuner (FP32, gfx950):
//   z1 = W1 x + b1, a1 = relu(z1); z2 = W2 a1 + b2, a2 = relu(z2); out = w3 . a2 + b3
// with D inputs and H hidden units per layer (H <= 256).  Training minimises
// the mean squared error over a batch with Adam.
//
// Parameter layout (one float array): W1[H][D], b1[H], W2[H][H], b2[H], w3[H], b3.
//
// Kernels
//   mlp_fwd       one workgroup of H threads per sample: thread j forms hidden
//                 unit j of both layers; the output is a workgroup reduction.
//                 z1 and z2 are kept (B x 2H) for the backward pass.
//   mlp_bwd_local per sample: d_out = 2 (out - y) / B, then dz2 = d_out w3 * [z2>0]
//                 and dz1 = (W2^T dz2) * [z1>0], kept (B x 2H).
//   mlp_grads     one thread per parameter sums its gradient over the batch in
//                 sample order (deterministic, no atomics).
//   mlp_adam      one thread per parameter (Kingma & Ba's update with bias
//                 correction).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "mpk_internal.h"

using namespace mpk;

// Scratch of the allocation-free backward pass (mpk_mlp_backward_noalloc):
// the per-sample output gradient and hidden-layer gradients, B * (2H + 1)
// floats, in a fixed device array instead of a caller workspace.  Every GPU
// the library runs on holds its own copy (16 MiB) until the process ends.
constexpr int64_t kMlpScratchFloats = int64_t(1) << 22;
static __device__ __align__(256) float scratch[kMlpScratchFloats];

namespace {

constexpr int kMaxHidden = 256;

struct Layout {
    int64_t w1, b1, w2, b2, w3, b3, total;
};

__host__ __device__ inline Layout layout(int D, int H) {
    Layout L;
    L.w1 = 0;
    L.b1 = L.w1 + (int64_t)H * D;
    L.w2 = L.b1 + H;
    L.b2 = L.w2 + (int64_t)H * H;
    L.w3 = L.b2 + H;
    L.b3 = L.w3 + H;
    L.total = L.b3 + 1;
    return L;
}

__global__ void mlp_fwd(const float *__restrict__ P, int D, int H, const float *__restrict__ X, int B,
                        float *__restrict__ out, float *__restrict__ cache) {
    __shared__ float a1[kMaxHidden];
    __shared__ float red[kMaxHidden];
    const Layout L = layout(D, H);
    const int b = blockIdx.x, j = threadIdx.x;
    if (b >= B) return;
    const float *x = X + (int64_t)b * D;
    float z1 = 0.0f, z2 = 0.0f, a2 = 0.0f;
    if (j < H) {
        z1 = P[L.b1 + j];
        for (int d = 0; d < D; ++d) z1 = fmaf(P[L.w1 + (int64_t)j * D + d], x[d], z1);
        a1[j] = z1 > 0.0f ? z1 : 0.0f;
    }
    __syncthreads();
    if (j < H) {
        z2 = P[L.b2 + j];
        for (int i = 0; i < H; ++i) z2 = fmaf(P[L.w2 + (int64_t)j * H + i], a1[i], z2);
        a2 = z2 > 0.0f ? z2 : 0.0f;
        red[j] = P[L.w3 + j] * a2;
        cache[(int64_t)b * 2 * H + j] = z1;
        cache[(int64_t)b * 2 * H + H + j] = z2;
    }
    __syncthreads();
    if (j == 0) {
        float s = P[L.b3];
        for (int i = 0; i < H; ++i) s += red[i];
        out[b] = s;
    }
}

__global__ void mlp_bwd_local(const float *__restrict__ P, int D, int H, int B, const float *__restrict__ y,
                              const float *__restrict__ out, const float *__restrict__ cache,
                              float *__restrict__ dcache, float *__restrict__ dout) {
    __shared__ float dz2s[kMaxHidden];
    const Layout L = layout(D, H);
    const int b = blockIdx.x, j = threadIdx.x;
    if (b >= B) return;
    const float g = 2.0f * (out[b] - y[b]) / (float)B;
    if (j == 0) dout[b] = g;
    float dz2 = 0.0f;
    if (j < H) {
        const float z2 = cache[(int64_t)b * 2 * H + H + j];
        dz2 = z2 > 0.0f ? g * P[L.w3 + j] : 0.0f;
        dz2s[j] = dz2;
        dcache[(int64_t)b * 2 * H + H + j] = dz2;
    }
    __syncthreads();
    if (j < H) {
        float s = 0.0f;
        for (int i = 0; i < H; ++i) s = fmaf(P[L.w2 + (int64_t)i * H + j], dz2s[i], s);
        const float z1 = cache[(int64_t)b * 2 * H + j];
        dcache[(int64_t)b * 2 * H + j] = z1 > 0.0f ? s : 0.0f;
    }
}

// gradient of one parameter, summed over the batch in sample order
__global__ void mlp_grads(const float *__restrict__ P, int D, int H, int B, const float *__restrict__ X,
                          const float *__restrict__ cache, const float *__restrict__ dcache,
                          const float *__restrict__ dout, float *__restrict__ G) {
    const Layout L = layout(D, H);
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= L.total) return;
    float s = 0.0f;
    if (k < L.b1) {  // W1[j][d]: dz1[j] x[d]
        const int j = (int)(k / D), d = (int)(k % D);
        for (int b = 0; b < B; ++b) s = fmaf(dcache[(int64_t)b * 2 * H + j], X[(int64_t)b * D + d], s);
    } else if (k < L.w2) {  // b1[j]
        const int j = (int)(k - L.b1);
        for (int b = 0; b < B; ++b) s += dcache[(int64_t)b * 2 * H + j];
    } else if (k < L.b2) {  // W2[j][i]: dz2[j] a1[i]
        const int j = (int)((k - L.w2) / H), i = (int)((k - L.w2) % H);
        for (int b = 0; b < B; ++b) {
            const float z1 = cache[(int64_t)b * 2 * H + i];
            if (z1 > 0.0f) s = fmaf(dcache[(int64_t)b * 2 * H + H + j], z1, s);
        }
    } else if (k < L.w3) {  // b2[j]
        const int j = (int)(k - L.b2);
        for (int b = 0; b < B; ++b) s += dcache[(int64_t)b * 2 * H + H + j];
    } else if (k < L.b3) {  // w3[j]: d_out a2[j]
        const int j = (int)(k - L.w3);
        for (int b = 0; b < B; ++b) {
            const float z2 = cache[(int64_t)b * 2 * H + H + j];
            if (z2 > 0.0f) s = fmaf(dout[b], z2, s);
        }
    } else {  // b3
        for (int b = 0; b < B; ++b) s += dout[b];
    }
    G[k] = s;
}

__global__ void mlp_loss(int B, const float *__restrict__ y, const float *__restrict__ out, float *__restrict__ loss) {
    // one workgroup: mean squared error, fixed reduction order
    __shared__ float red[256];
    float s = 0.0f;
    for (int b = threadIdx.x; b < B; b += blockDim.x) {
        const float e = out[b] - y[b];
        s = fmaf(e, e, s);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = red[0] / (float)B;
}

__global__ void mlp_adam(float *__restrict__ P, const float *__restrict__ G, float *__restrict__ M,
                         float *__restrict__ V, int64_t n, float lr, float b1, float b2, float eps, float c1,
                         float c2) {
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float g = G[k];
    const float m = b1 * M[k] + (1.0f - b1) * g;
    const float v = b2 * V[k] + (1.0f - b2) * g * g;
    M[k] = m;
    V[k] = v;
    const float mh = m / c1, vh = v / c2;
    P[k] -= lr * mh / (sqrtf(vh) + eps);
}

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) return fail(MPK_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Device address of `scratch` on each GPU, taken once per device with that
// device current.  In host code the array's name is only a host-side stand-in,
// so kernels and copies use these addresses, never the name.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[kMaxDevices] = {};

mpk_status scratch_of_current_device(float **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(MPK_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(MPK_ERR_UNSUPPORTED, "device ordinal beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(MPK_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<float *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return MPK_OK;
}

mpk_status check_dims(int32_t D, int32_t H, int32_t B) {
    if (D < 1 || D > 4096) return fail(MPK_ERR_ARG, "input width must be in [1, 4096]");
    if (H < 1 || H > kMaxHidden) return fail(MPK_ERR_ARG, "hidden width must be in [1, 256]");
    if (B < 0) return fail(MPK_ERR_ARG, "negative batch");
    return MPK_OK;
}

}  // namespace

extern "C" {

int64_t mpk_mlp_param_count(int32_t D, int32_t H) {
    if (D < 1 || H < 1) return -1;
    return layout(D, H).total;
}

mpk_status mpk_mlp_forward(const float *params, int32_t D, int32_t H, const float *X, int32_t B, float *out,
                           float *cache, void *stream) {
    mpk_status st = check_dims(D, H, B);
    if (st != MPK_OK) return st;
    if (B == 0) return MPK_OK;
    if (!params || !X || !out || !cache) return fail(MPK_ERR_ARG, "null pointer");
    const int threads = ((H + 63) / 64) * 64;
    hipLaunchKernelGGL(mlp_fwd, dim3(B), dim3(threads), 0, reinterpret_cast<hipStream_t>(stream), params, D, H, X,
                       B, out, cache);
    HIP_TRY(hipGetLastError());
    return MPK_OK;
}

mpk_status mpk_mlp_backward(const float *params, int32_t D, int32_t H, const float *X, const float *y, int32_t B,
                            const float *out, const float *cache, float *work, float *grads, float *loss,
                            void *stream) {
    mpk_status st = check_dims(D, H, B);
    if (st != MPK_OK) return st;
    if (B < 1) return fail(MPK_ERR_ARG, "empty batch");
    if (!params || !X || !y || !out || !cache || !work || !grads) return fail(MPK_ERR_ARG, "null pointer");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    float *dcache = work;
    float *dout = work + (int64_t)B * 2 * H;
    const int threads = ((H + 63) / 64) * 64;
    hipLaunchKernelGGL(mlp_bwd_local, dim3(B), dim3(threads), 0, s, params, D, H, B, y, out, cache, dcache, dout);
    const int64_t n = layout(D, H).total;
    hipLaunchKernelGGL(mlp_grads, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, params, D, H, B, X, cache,
                       dcache, dout, grads);
    if (loss) hipLaunchKernelGGL(mlp_loss, dim3(1), dim3(256), 0, s, B, y, out, loss);
    HIP_TRY(hipGetLastError());
    return MPK_OK;
}

mpk_status mpk_mlp_backward_noalloc(const float *params, int32_t D, int32_t H, const float *X, const float *y,
                                    int32_t B, const float *out, const float *cache, float *grads, float *loss,
                                    void *stream) {
    mpk_status st = check_dims(D, H, B);
    if (st != MPK_OK) return st;
    if (B < 1) return fail(MPK_ERR_ARG, "empty batch");
    if ((int64_t)B * (2 * H + 1) > kMlpScratchFloats)
        return fail(MPK_ERR_ARG, "batch too large for the fixed scratch: B * (2H + 1) must be <= 4194304 floats");
    float *work = nullptr;
    if ((st = scratch_of_current_device(&work)) != MPK_OK) return st;
    // every scratch entry the kernels read is written first in the same call,
    // so nothing needs clearing
    return mpk_mlp_backward(params, D, H, X, y, B, out, cache, work, grads, loss, stream);
}

mpk_status mpk_mlp_adam(float *params, const float *grads, float *m, float *v, int64_t n, float lr, float beta1,
                        float beta2, float eps, int32_t step, void *stream) {
    if (!params || !grads || !m || !v) return fail(MPK_ERR_ARG, "null pointer");
    if (n < 0 || step < 1) return fail(MPK_ERR_ARG, "bad size or step");
    if (n == 0) return MPK_OK;
    const float c1 = 1.0f - std::pow(beta1, (float)step), c2 = 1.0f - std::pow(beta2, (float)step);
    hipLaunchKernelGGL(mlp_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), params, grads, m, v, n, lr, beta1, beta2, eps, c1, c2);
    HIP_TRY(hipGetLastError());
    return MPK_OK;
}

}  // extern "C"
