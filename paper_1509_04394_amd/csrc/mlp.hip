// Cost-model network: a 3-layer FP32 perceptron F -> 64 -> 64 -> 1 with ReLU,
// trained on the GPU by the kernels below to predict log kernel time of a fused
// group from its features (the paper's C_i is a predicted execution time,
// Sec. VI, Fig. 5).
//
// Parameter layout (one flat float array, row-major [out][in]):
//   W1[64][F] b1[64] W2[64][64] b2[64] W3[64] b3[1]
// Loss over a batch of N samples: L = (1/N) sum_n (y_n - t_n)^2.
//
// Every reduction runs in a fixed order (per-block partial sums, then a
// second kernel that adds the partials block by block), so gradients are
// deterministic.
#include <hip/hip_runtime.h>

#include <string>

#include "fz_internal.h"

namespace fz {

constexpr int MLP_H = 64;        // hidden width
constexpr int MLP_TILE = 64;     // samples per workgroup
constexpr int MLP_THREADS = 256;
constexpr int MLP_FMAX = 32;     // most features supported

FZ_HD constexpr int mlp_params(int F) { return MLP_H * F + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1; }

struct MlpOffsets {
    int w1, b1, w2, b2, w3, b3;
};
static inline __host__ __device__ MlpOffsets mlp_offsets(int F)
{
    MlpOffsets o;
    o.w1 = 0;
    o.b1 = o.w1 + MLP_H * F;
    o.w2 = o.b1 + MLP_H;
    o.b2 = o.w2 + MLP_H * MLP_H;
    o.w3 = o.b2 + MLP_H;
    o.b3 = o.w3 + MLP_H;
    return o;
}

// Forward for one tile of samples; activations h1, h2 ([tile][64]) stay in LDS
// and are also written out when `save` is given (for the backward pass).
__global__ __launch_bounds__(MLP_THREADS) void k_mlp_forward(const float* __restrict__ prm, int F,
                                                             const float* __restrict__ x, int n, float* __restrict__ y,
                                                             float* __restrict__ h1_out, float* __restrict__ h2_out)
{
    __shared__ float xs[MLP_TILE][MLP_FMAX + 1];
    __shared__ float h1[MLP_TILE][MLP_H + 1];
    __shared__ float h2[MLP_TILE][MLP_H + 1];
    const MlpOffsets o = mlp_offsets(F);
    const int s0 = blockIdx.x * MLP_TILE;
    const int tid = threadIdx.x;
    for (int i = tid; i < MLP_TILE * F; i += MLP_THREADS) {
        const int s = i / F, f = i - s * F;
        xs[s][f] = (s0 + s < n) ? x[(size_t)(s0 + s) * F + f] : 0.0f;
    }
    __syncthreads();
    // layer 1: h1[s][j] = relu(b1[j] + sum_f W1[j][f] x[s][f])
    for (int i = tid; i < MLP_TILE * MLP_H; i += MLP_THREADS) {
        const int s = i / MLP_H, j = i - s * MLP_H;
        float acc = prm[o.b1 + j];
        for (int f = 0; f < F; ++f) acc = __builtin_fmaf(prm[o.w1 + j * F + f], xs[s][f], acc);
        h1[s][j] = acc > 0.0f ? acc : 0.0f;
    }
    __syncthreads();
    for (int i = tid; i < MLP_TILE * MLP_H; i += MLP_THREADS) {
        const int s = i / MLP_H, j = i - s * MLP_H;
        float acc = prm[o.b2 + j];
        for (int k = 0; k < MLP_H; ++k) acc = __builtin_fmaf(prm[o.w2 + j * MLP_H + k], h1[s][k], acc);
        h2[s][j] = acc > 0.0f ? acc : 0.0f;
    }
    __syncthreads();
    if (tid < MLP_TILE && s0 + tid < n) {
        float acc = prm[o.b3];
        for (int k = 0; k < MLP_H; ++k) acc = __builtin_fmaf(prm[o.w3 + k], h2[tid][k], acc);
        y[s0 + tid] = acc;
    }
    if (h1_out) {
        for (int i = tid; i < MLP_TILE * MLP_H; i += MLP_THREADS) {
            const int s = i / MLP_H, j = i - s * MLP_H;
            if (s0 + s < n) {
                h1_out[(size_t)(s0 + s) * MLP_H + j] = h1[s][j];
                h2_out[(size_t)(s0 + s) * MLP_H + j] = h2[s][j];
            }
        }
    }
}

// Backward for one tile: per-block partial gradient (all parameters) into
// part[block][P] and the tile's partial loss into lpart[block].
__global__ __launch_bounds__(MLP_THREADS) void k_mlp_backward(const float* __restrict__ prm, int F,
                                                              const float* __restrict__ x,
                                                              const float* __restrict__ tgt, int n,
                                                              const float* __restrict__ y,
                                                              const float* __restrict__ h1g,
                                                              const float* __restrict__ h2g, float* __restrict__ part,
                                                              float* __restrict__ lpart)
{
    __shared__ float xs[MLP_TILE][MLP_FMAX + 1];
    __shared__ float h1[MLP_TILE][MLP_H + 1];
    __shared__ float d2[MLP_TILE][MLP_H + 1];  // dL/dz2, then reused
    __shared__ float d1[MLP_TILE][MLP_H + 1];  // dL/dz1
    __shared__ float dy[MLP_TILE];
    const MlpOffsets o = mlp_offsets(F);
    const int P = mlp_params(F);
    const int s0 = blockIdx.x * MLP_TILE;
    const int tid = threadIdx.x;
    const float inv_n = 1.0f / (float)n;
    for (int i = tid; i < MLP_TILE * F; i += MLP_THREADS) {
        const int s = i / F, f = i - s * F;
        xs[s][f] = (s0 + s < n) ? x[(size_t)(s0 + s) * F + f] : 0.0f;
    }
    for (int i = tid; i < MLP_TILE * MLP_H; i += MLP_THREADS) {
        const int s = i / MLP_H, j = i - s * MLP_H;
        const bool ok = s0 + s < n;
        h1[s][j] = ok ? h1g[(size_t)(s0 + s) * MLP_H + j] : 0.0f;
        d1[s][j] = ok ? h2g[(size_t)(s0 + s) * MLP_H + j] : 0.0f;  // h2 for now
    }
    if (tid < MLP_TILE) {
        const bool ok = s0 + tid < n;
        const float r = ok ? y[s0 + tid] - tgt[s0 + tid] : 0.0f;
        dy[tid] = 2.0f * r * inv_n;
    }
    __syncthreads();
    float* g = part + (size_t)blockIdx.x * P;
    // layer 3
    if (tid < MLP_H) {
        float acc = 0.0f;
        for (int s = 0; s < MLP_TILE; ++s) acc = __builtin_fmaf(dy[s], d1[s][tid], acc);
        g[o.w3 + tid] = acc;
    }
    if (tid == MLP_H) {
        float acc = 0.0f, l = 0.0f;
        for (int s = 0; s < MLP_TILE; ++s) {
            acc += dy[s];
            if (s0 + s < n) {
                const float r = y[s0 + s] - tgt[s0 + s];
                l = __builtin_fmaf(r, r, l);
            }
        }
        g[o.b3] = acc;
        lpart[blockIdx.x] = l * inv_n;
    }
    // dz2 = dy * w3 masked by h2 > 0
    for (int i = tid; i < MLP_TILE * MLP_H; i += MLP_THREADS) {
        const int s = i / MLP_H, j = i - s * MLP_H;
        d2[s][j] = d1[s][j] > 0.0f ? dy[s] * prm[o.w3 + j] : 0.0f;
    }
    __syncthreads();
    // layer 2 weights: gW2[j][k] = sum_s dz2[s][j] h1[s][k]
    for (int i = tid; i < MLP_H * MLP_H; i += MLP_THREADS) {
        const int j = i / MLP_H, k = i - j * MLP_H;
        float acc = 0.0f;
        for (int s = 0; s < MLP_TILE; ++s) acc = __builtin_fmaf(d2[s][j], h1[s][k], acc);
        g[o.w2 + i] = acc;
    }
    if (tid < MLP_H) {
        float acc = 0.0f;
        for (int s = 0; s < MLP_TILE; ++s) acc += d2[s][tid];
        g[o.b2 + tid] = acc;
    }
    // dz1[s][k] = (sum_j dz2[s][j] W2[j][k]) masked by h1 > 0
    for (int i = tid; i < MLP_TILE * MLP_H; i += MLP_THREADS) {
        const int s = i / MLP_H, k = i - s * MLP_H;
        float acc = 0.0f;
        for (int j = 0; j < MLP_H; ++j) acc = __builtin_fmaf(d2[s][j], prm[o.w2 + j * MLP_H + k], acc);
        d1[s][k] = h1[s][k] > 0.0f ? acc : 0.0f;
    }
    __syncthreads();
    // layer 1 weights: gW1[j][f] = sum_s dz1[s][j] x[s][f]
    for (int i = tid; i < MLP_H * F; i += MLP_THREADS) {
        const int j = i / F, f = i - j * F;
        float acc = 0.0f;
        for (int s = 0; s < MLP_TILE; ++s) acc = __builtin_fmaf(d1[s][j], xs[s][f], acc);
        g[o.w1 + i] = acc;
    }
    if (tid < MLP_H) {
        float acc = 0.0f;
        for (int s = 0; s < MLP_TILE; ++s) acc += d1[s][tid];
        g[o.b1 + tid] = acc;
    }
}

// grad[p] = sum over blocks of part[b][p], blocks in order; loss likewise.
__global__ void k_mlp_reduce(const float* __restrict__ part, const float* __restrict__ lpart, int nblocks, int P,
                             float* __restrict__ grad, float* __restrict__ loss)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < P) {
        float acc = 0.0f;
        for (int b = 0; b < nblocks; ++b) acc += part[(size_t)b * P + p];
        grad[p] = acc;
    }
    if (p == 0 && loss) {
        float l = 0.0f;
        for (int b = 0; b < nblocks; ++b) l += lpart[b];
        *loss = l;
    }
}

__global__ void k_mlp_adam(float* __restrict__ prm, const float* __restrict__ grad, float* __restrict__ m,
                           float* __restrict__ v, int P, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const float g = grad[p];
    const float mm = b1 * m[p] + (1.0f - b1) * g;
    const float vv = b2 * v[p] + (1.0f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const float mh = mm / c1, vh = vv / c2;
    prm[p] -= lr * mh / (__builtin_sqrtf(vh) + eps);
}

static size_t mlp_ws(int F, int n)
{
    const int nb = (n + MLP_TILE - 1) / MLP_TILE;
    const size_t act = (size_t)n * MLP_H * 2 * sizeof(float);
    const size_t yb = (size_t)n * sizeof(float);
    const size_t part = (size_t)nb * mlp_params(F) * sizeof(float) + (size_t)nb * sizeof(float);
    return ((act + 255) & ~(size_t)255) + ((yb + 255) & ~(size_t)255) + part + 256;
}

}  // namespace fz

using namespace fz;

extern "C" {

int32_t fz_mlp_param_count(int32_t n_features) { return (n_features > 0 && n_features <= MLP_FMAX) ? mlp_params(n_features) : -1; }

size_t fz_mlp_workspace_bytes(int32_t n_features, int32_t n)
{
    if (n_features <= 0 || n_features > MLP_FMAX || n <= 0) return 0;
    return mlp_ws(n_features, n);
}

fz_status fz_mlp_forward(const float* d_params, int32_t n_features, const float* d_x, int32_t n, float* d_y,
                         void* stream)
{
    if (!d_params || !d_x || !d_y) return fail(FZ_E_INVALID, "fz_mlp_forward: null pointer");
    if (n_features <= 0 || n_features > MLP_FMAX || n <= 0) return fail(FZ_E_INVALID, "fz_mlp_forward: bad size");
    const int nb = (n + MLP_TILE - 1) / MLP_TILE;
    (void)hipGetLastError();  // drop an error latched by earlier, unrelated runtime calls
    hipLaunchKernelGGL(k_mlp_forward, dim3(nb), dim3(MLP_THREADS), 0, (hipStream_t)stream, d_params, n_features,
                       d_x, n, d_y, nullptr, nullptr);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FZ_OK : fail(FZ_E_HIP, std::string("mlp forward: ") + hipGetErrorString(e));
}

fz_status fz_mlp_loss_grad(const float* d_params, int32_t n_features, const float* d_x, const float* d_target,
                           int32_t n, float* d_grad, float* d_loss, void* d_ws, size_t ws_bytes, void* stream)
{
    if (!d_params || !d_x || !d_target || !d_grad) return fail(FZ_E_INVALID, "fz_mlp_loss_grad: null pointer");
    if (n_features <= 0 || n_features > MLP_FMAX || n <= 0) return fail(FZ_E_INVALID, "fz_mlp_loss_grad: bad size");
    if (!d_ws || ws_bytes < mlp_ws(n_features, n))
        return fail(FZ_E_WORKSPACE, "fz_mlp_loss_grad: workspace needs " + std::to_string(mlp_ws(n_features, n)));
    hipStream_t s = (hipStream_t)stream;
    (void)hipGetLastError();  // drop an error latched by earlier, unrelated runtime calls
    const int nb = (n + MLP_TILE - 1) / MLP_TILE;
    const int P = mlp_params(n_features);
    char* w = (char*)d_ws;
    float* h1 = (float*)w;
    float* h2 = h1 + (size_t)n * MLP_H;
    w += ((size_t)n * MLP_H * 2 * sizeof(float) + 255) & ~(size_t)255;
    float* y = (float*)w;
    w += ((size_t)n * sizeof(float) + 255) & ~(size_t)255;
    float* part = (float*)w;
    float* lpart = part + (size_t)nb * P;
    hipLaunchKernelGGL(k_mlp_forward, dim3(nb), dim3(MLP_THREADS), 0, s, d_params, n_features, d_x, n, y, h1, h2);
    hipLaunchKernelGGL(k_mlp_backward, dim3(nb), dim3(MLP_THREADS), 0, s, d_params, n_features, d_x, d_target, n, y,
                       h1, h2, part, lpart);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((P + 255) / 256), dim3(256), 0, s, part, lpart, nb, P, d_grad, d_loss);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FZ_OK : fail(FZ_E_HIP, std::string("mlp loss/grad: ") + hipGetErrorString(e));
}

fz_status fz_mlp_adam_step(float* d_params, const float* d_grad, float* d_m, float* d_v, int32_t n_params,
                           int32_t step, float lr, float beta1, float beta2, float eps, void* stream)
{
    if (!d_params || !d_grad || !d_m || !d_v) return fail(FZ_E_INVALID, "fz_mlp_adam_step: null pointer");
    if (n_params <= 0 || step < 1) return fail(FZ_E_INVALID, "fz_mlp_adam_step: bad size or step");
    const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
    (void)hipGetLastError();  // drop an error latched by earlier, unrelated runtime calls
    hipLaunchKernelGGL(k_mlp_adam, dim3((n_params + 255) / 256), dim3(256), 0, (hipStream_t)stream, d_params, d_grad,
                       d_m, d_v, n_params, lr, beta1, beta2, eps, c1, c2);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FZ_OK : fail(FZ_E_HIP, std::string("mlp adam: ") + hipGetErrorString(e));
}

}  // extern "C"
