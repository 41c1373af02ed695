// Rank predictor: a 16-64-64-1 tanh MLP in FP32 (device kernels in kernels_mlp.hip, host
// drivers in mlp.cpp).  Parameter vector layout (floats):
//   mu[16], sd[16]            input normalisation (x - mu) / sd, fixed, not trained
//   W1[64][16], b1[64]        first layer (row-major: W1[o * 16 + i])
//   W2[64][64], b2[64]        second layer
//   W3[64], b3                output: log of the predicted rank
#pragma once
#include "internal.h"

namespace qps {

constexpr int MLP_IN = 16;
constexpr int MLP_H = 64;
constexpr int MLP_OFF_MU = 0;
constexpr int MLP_OFF_SD = MLP_OFF_MU + MLP_IN;
constexpr int MLP_OFF_W1 = MLP_OFF_SD + MLP_IN;
constexpr int MLP_OFF_B1 = MLP_OFF_W1 + MLP_H * MLP_IN;
constexpr int MLP_OFF_W2 = MLP_OFF_B1 + MLP_H;
constexpr int MLP_OFF_B2 = MLP_OFF_W2 + MLP_H * MLP_H;
constexpr int MLP_OFF_W3 = MLP_OFF_B2 + MLP_H;
constexpr int MLP_OFF_B3 = MLP_OFF_W3 + MLP_H;
constexpr int MLP_NPARAM = MLP_OFF_B3 + 1;

// y[b] = model(x[b]) for b < n (x: n x 16 row-major); device pointers, on stream s
hipError_t mlp_forward(const float* params, const float* x, int64_t n, float* y, hipStream_t s);

// Pinball loss at quantile tau of the predictions against targets t, summed over the samples
// (loss = sum_b max(tau r_b, (tau - 1) r_b), r_b = t_b - y_b), and its gradient with respect to
// every parameter (grad[i] = 0 for mu, sd).  Device pointers; work grows as needed.
hipError_t mlp_grad(DevBuf& work, const float* params, const float* x, const float* t, int64_t n, float tau, float* grad,
                    float* loss, hipStream_t s);

// Adam on the mean pinball loss: `steps` full-batch steps with learning rate lr (beta1 0.9, beta2 0.999,
// eps 1e-8); params updated in place (mu, sd untouched).  loss_hist[steps] receives the mean loss
// before each step (device pointer, nullable).
hipError_t mlp_train(DevBuf& work, float* params, const float* x, const float* t, int64_t n, float tau, int steps, float lr,
                     float* loss_hist, hipStream_t s);

}  // namespace qps
