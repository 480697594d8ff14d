// mlp.h -- layout of the threshold-bracket network and its kernel launchers
// (mlp.hip).  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>

namespace rqa {

constexpr int MLP_IN = 66;    // sketch features
constexpr int MLP_H = 128;    // hidden width (two GELU layers)
constexpr int MLP_OUT = 20;   // one offset per target recurrence rate
constexpr int MLP_PARAMS = MLP_IN * MLP_H + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H * MLP_OUT + MLP_OUT;  // 27668

struct MlpOffsets {
    int W1 = 0;
    int b1 = W1 + MLP_IN * MLP_H;
    int W2 = b1 + MLP_H;
    int b2 = W2 + MLP_H * MLP_H;
    int W3 = b2 + MLP_H;
    int b3 = W3 + MLP_H * MLP_OUT;
};

// Activations of one batch (device buffers of B rows).
struct MlpActs {
    float *Z1, *A1, *Z2, *A2, *Y;  // pre-activations, activations, output
    float *dY, *dZ2, *dZ1;         // gradients w.r.t. output and pre-activations
};

hipError_t mlp_forward(hipStream_t st, const float* params, const float* X, int B, MlpActs& a, float* Y);
hipError_t mlp_backward(hipStream_t st, const float* params, const float* X, const float* T, int B, MlpActs& a,
                        float* grad, float* loss_partial, int* n_partial);
hipError_t mlp_adam(hipStream_t st, float* params, const float* grad, float* m, float* v, float lr, float b1,
                    float b2, float eps, float c1, float c2);

}  // namespace rqa
