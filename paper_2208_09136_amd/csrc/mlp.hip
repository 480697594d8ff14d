// mlp.hip -- the threshold-bracket network: a 66 -> 128 -> 128 -> 20
// perceptron with GELU hidden layers, its forward and backward passes, the
// mean-squared-error loss and Adam, as plain FP32 HIP kernels.
//
// The network maps the distance sketch of a series to the offsets
// t_r = (bits(eps_r) - scale) / 2^23 of its exact thresholds; it only
// narrows the key window in which exact selection looks (an extension of the
// method, not part of the paper).  Its arithmetic never decides a result:
// every threshold is still an exact order statistic.
//
// Parameter vector (float32, MLP_PARAMS entries):
//   W1 [IN][H], b1 [H], W2 [H][H], b2 [H], W3 [H][OUT], b3 [OUT]
// with W[i][o] at i * O + o.  The layers are small (at most 128 x 128), so
// one thread per output element with a sequential dot product keeps every
// kernel simple; they are latency-bound, not a dense contraction worth the
// matrix cores.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mlp.h"

namespace rqa {

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

// d gelu / dz = Phi(z) + z phi(z)
__device__ __forceinline__ float gelu_grad(float z)
{
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// Z = X W + b, A = gelu(Z) (act) or Z; thread per (b, o).
__global__ void k_dense(const float* __restrict__ X, int B, int I, const float* __restrict__ W,
                        const float* __restrict__ bias, int O, float* __restrict__ Z, float* __restrict__ A, int act)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * O) return;
    const int b = idx / O, o = idx % O;
    float z = bias[o];
    const float* x = X + (size_t)b * I;
    for (int i = 0; i < I; ++i) z = fmaf(x[i], W[(size_t)i * O + o], z);
    if (Z) Z[idx] = z;
    A[idx] = act ? gelu(z) : z;
}

// dY = 2 (Y - T) / (B O); per-block partial sums of (Y - T)^2 / (B O).
__global__ void k_mse(const float* __restrict__ Y, const float* __restrict__ T, int n, float* __restrict__ dY,
                      float* __restrict__ partial)
{
    __shared__ float red[256];
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    float e = 0.f;
    if (idx < n) {
        const float d = Y[idx] - T[idx];
        dY[idx] = 2.0f * d / (float)n;
        e = d * d / (float)n;
    }
    red[threadIdx.x] = e;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// dZprev[b][i] = (sum_o dZ[b][o] W[i][o]) * gelu'(Zprev[b][i]); thread per (b, i).
__global__ void k_dense_bwd_x(const float* __restrict__ dZ, int B, int O, const float* __restrict__ W, int I,
                              const float* __restrict__ Zprev, float* __restrict__ dZprev)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= B * I) return;
    const int b = idx / I, i = idx % I;
    float g = 0.f;
    const float* dz = dZ + (size_t)b * O;
    const float* w = W + (size_t)i * O;
    for (int o = 0; o < O; ++o) g = fmaf(dz[o], w[o], g);
    dZprev[idx] = g * gelu_grad(Zprev[idx]);
}

// dW[i][o] = sum_b Aprev[b][i] dZ[b][o] (i < I), db[o] = sum_b dZ[b][o] (row I);
// thread per (i, o).
__global__ void k_dense_bwd_w(const float* __restrict__ Aprev, int B, int I, const float* __restrict__ dZ, int O,
                              float* __restrict__ dW, float* __restrict__ db)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (I + 1) * O) return;
    const int i = idx / O, o = idx % O;
    float g = 0.f;
    if (i < I) {
        for (int b = 0; b < B; ++b) g = fmaf(Aprev[(size_t)b * I + i], dZ[(size_t)b * O + o], g);
        dW[(size_t)i * O + o] = g;
    } else {
        for (int b = 0; b < B; ++b) g += dZ[(size_t)b * O + o];
        db[o] = g;
    }
}

// Adam (Kingma and Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// theta -= lr * (m / c1) / (sqrt(v / c2) + eps) with c1 = 1 - b1^t, c2 = 1 - b2^t.
__global__ void k_adam(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

static inline unsigned blocks(long n, int t) { return (unsigned)((n + t - 1) / t); }

hipError_t mlp_forward(hipStream_t st, const float* params, const float* X, int B, MlpActs& a, float* Y)
{
    const MlpOffsets o;
    hipLaunchKernelGGL(k_dense, dim3(blocks((long)B * MLP_H, 256)), dim3(256), 0, st, X, B, MLP_IN,
                       params + o.W1, params + o.b1, MLP_H, a.Z1, a.A1, 1);
    hipLaunchKernelGGL(k_dense, dim3(blocks((long)B * MLP_H, 256)), dim3(256), 0, st, a.A1, B, MLP_H,
                       params + o.W2, params + o.b2, MLP_H, a.Z2, a.A2, 1);
    hipLaunchKernelGGL(k_dense, dim3(blocks((long)B * MLP_OUT, 256)), dim3(256), 0, st, a.A2, B, MLP_H,
                       params + o.W3, params + o.b3, MLP_OUT, (float*)nullptr, Y, 0);
    return hipGetLastError();
}

hipError_t mlp_backward(hipStream_t st, const float* params, const float* X, const float* T, int B, MlpActs& a,
                        float* grad, float* loss_partial, int* n_partial)
{
    const MlpOffsets o;
    const int n = B * MLP_OUT;
    *n_partial = (int)blocks(n, 256);
    hipLaunchKernelGGL(k_mse, dim3(*n_partial), dim3(256), 0, st, a.Y, T, n, a.dY, loss_partial);
    // layer 3
    hipLaunchKernelGGL(k_dense_bwd_w, dim3(blocks((long)(MLP_H + 1) * MLP_OUT, 256)), dim3(256), 0, st, a.A2, B,
                       MLP_H, a.dY, MLP_OUT, grad + o.W3, grad + o.b3);
    hipLaunchKernelGGL(k_dense_bwd_x, dim3(blocks((long)B * MLP_H, 256)), dim3(256), 0, st, a.dY, B, MLP_OUT,
                       params + o.W3, MLP_H, a.Z2, a.dZ2);
    // layer 2
    hipLaunchKernelGGL(k_dense_bwd_w, dim3(blocks((long)(MLP_H + 1) * MLP_H, 256)), dim3(256), 0, st, a.A1, B,
                       MLP_H, a.dZ2, MLP_H, grad + o.W2, grad + o.b2);
    hipLaunchKernelGGL(k_dense_bwd_x, dim3(blocks((long)B * MLP_H, 256)), dim3(256), 0, st, a.dZ2, B, MLP_H,
                       params + o.W2, MLP_H, a.Z1, a.dZ1);
    // layer 1
    hipLaunchKernelGGL(k_dense_bwd_w, dim3(blocks((long)(MLP_IN + 1) * MLP_H, 256)), dim3(256), 0, st, X, B,
                       MLP_IN, a.dZ1, MLP_H, grad + o.W1, grad + o.b1);
    return hipGetLastError();
}

hipError_t mlp_adam(hipStream_t st, float* params, const float* grad, float* m, float* v, float lr, float b1,
                    float b2, float eps, float c1, float c2)
{
    hipLaunchKernelGGL(k_adam, dim3(blocks(MLP_PARAMS, 256)), dim3(256), 0, st, params, grad, m, v, MLP_PARAMS, lr, b1,
                       b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace rqa
