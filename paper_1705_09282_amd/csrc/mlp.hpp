// Learned-damping perceptron (see mlp.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace dfmg {

// outputs 0 .. MLP_ETA-1: damping logits; MLP_ETA .. MLP_OUT-1: smoothing
// steps per level; both finest level first
constexpr int MLP_IN = 4, MLP_H = 32, MLP_OUT = 10, MLP_ETA = 5;
constexpr int MLP_NPARAM = MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_OUT * MLP_H + MLP_OUT;  // 1546

// Z (n x 10) = outputs of the samples X (n x 4).
void launch_mlp_forward(int n, const float *W, const float *X, float *Z, hipStream_t s);
// G = gradient of scale * sum M (Z - Y)^2 and *loss its value; work holds
// n * MLP_NPARAM floats, lw n floats.  Fixed summation order.
void launch_mlp_grad(int n, const float *W, const float *X, const float *Y, const float *Mk, float scale,
                     float *work, float *lw, float *G, float *loss, hipStream_t s);
// The same gradient with the per-sample rows in the library's static device
// scratch (at most MLP_SCRATCH_SAMPLES samples): scr = mlp_scratch(device).
constexpr int MLP_SCRATCH_SAMPLES = 512;
float *mlp_scratch(int device, hipError_t *err);
void launch_mlp_grad_scratch(int n, const float *W, const float *X, const float *Y, const float *Mk, float scale,
                             float *scr, float *G, float *loss, hipStream_t s);
void launch_mlp_adam(float *W, float *m, float *v, const float *G, int t, float lr, hipStream_t s);
// eta[p * L + l] for l = 1 .. L-1 from the features of problem p.
// Host evaluation of one sample (FP64 arithmetic on the FP32 weights).
void mlp_forward_host(const float *W, const float *x, double *z);
void launch_mlp_damping(int np, const float *W, const float *feat, int L, double *eta, hipStream_t s);

}  // namespace dfmg
