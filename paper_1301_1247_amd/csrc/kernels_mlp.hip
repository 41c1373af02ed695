// Device kernels of the rank-predictor MLP (mlp.h): forward pass, per-sample backward pass of
// the pinball loss, deterministic reductions over the samples for the parameter gradients, and
// the Adam update.  One thread per sample; the parameters sit in LDS (5345 floats).
#include "mlp.h"

namespace qps {
namespace {

constexpr int NT = 256;

__device__ inline void load_params(const float* __restrict__ params, float* sp) {
  for (int i = threadIdx.x; i < MLP_NPARAM; i += NT) sp[i] = params[i];
  __syncthreads();
}

// y = W3 tanh(W2 tanh(W1 xn + b1) + b2) + b3 with xn = (x - mu) / sd.  Optionally stores xn, h1, h2.
__global__ __launch_bounds__(NT) void k_mlp_fwd(const float* __restrict__ params, const float* __restrict__ x, int64_t n,
                                                float* __restrict__ y, float* __restrict__ XN, float* __restrict__ H1,
                                                float* __restrict__ H2) {
  __shared__ float sp[MLP_NPARAM];
  load_params(params, sp);
  const int64_t b = blockIdx.x * (int64_t)NT + threadIdx.x;
  if (b >= n) return;
  float xn[MLP_IN];
#pragma unroll
  for (int i = 0; i < MLP_IN; ++i) {
    xn[i] = (x[b * MLP_IN + i] - sp[MLP_OFF_MU + i]) / sp[MLP_OFF_SD + i];
    if (XN) XN[b * MLP_IN + i] = xn[i];
  }
  float h1[MLP_H];
#pragma unroll
  for (int o = 0; o < MLP_H; ++o) {
    float a = sp[MLP_OFF_B1 + o];
#pragma unroll
    for (int i = 0; i < MLP_IN; ++i) a = fmaf(sp[MLP_OFF_W1 + o * MLP_IN + i], xn[i], a);
    h1[o] = tanhf(a);
    if (H1) H1[b * MLP_H + o] = h1[o];
  }
  float out = sp[MLP_OFF_B3];
  for (int o = 0; o < MLP_H; ++o) {
    float a = sp[MLP_OFF_B2 + o];
#pragma unroll
    for (int j = 0; j < MLP_H; ++j) a = fmaf(sp[MLP_OFF_W2 + o * MLP_H + j], h1[j], a);
    const float h2 = tanhf(a);
    if (H2) H2[b * MLP_H + o] = h2;
    out = fmaf(sp[MLP_OFF_W3 + o], h2, out);
  }
  y[b] = out;
}

// Backward pass of the pinball loss for one sample: dy = dL/dy, D2 = dL/d(pre-activation 2),
// D1 = dL/d(pre-activation 1); lossv = the sample's loss.
__global__ __launch_bounds__(NT) void k_mlp_bwd(const float* __restrict__ params, int64_t n, const float* __restrict__ t,
                                                float tau, const float* __restrict__ y, const float* __restrict__ H1,
                                                const float* __restrict__ H2, float* __restrict__ dY, float* __restrict__ D1,
                                                float* __restrict__ D2, float* __restrict__ lossv) {
  __shared__ float sp[MLP_NPARAM];
  load_params(params, sp);
  const int64_t b = blockIdx.x * (int64_t)NT + threadIdx.x;
  if (b >= n) return;
  const float r = t[b] - y[b];
  const float dy = r > 0.f ? -tau : 1.f - tau;
  lossv[b] = r > 0.f ? tau * r : (tau - 1.f) * r;
  dY[b] = dy;
  float d2[MLP_H];
#pragma unroll
  for (int o = 0; o < MLP_H; ++o) {
    const float h2 = H2[b * MLP_H + o];
    d2[o] = dy * sp[MLP_OFF_W3 + o] * (1.f - h2 * h2);
    D2[b * MLP_H + o] = d2[o];
  }
  for (int j = 0; j < MLP_H; ++j) {
    float a = 0.f;
#pragma unroll
    for (int o = 0; o < MLP_H; ++o) a = fmaf(sp[MLP_OFF_W2 + o * MLP_H + j], d2[o], a);
    const float h1 = H1[b * MLP_H + j];
    D1[b * MLP_H + j] = a * (1.f - h1 * h1);
  }
}

// out[p * ldo + q] = sum_b A[b * P + p] * (Bm ? Bm[b * Q + q] : 1), q < Q <= 64; one workgroup per p,
// fixed summation order (deterministic).
__global__ __launch_bounds__(NT) void k_outer(const float* __restrict__ A, int P, const float* __restrict__ Bm, int Q, int64_t n,
                                              float* __restrict__ out, int ldo) {
  __shared__ float part[NT][MLP_H + 1];
  const int p = blockIdx.x;
  float acc[MLP_H];
#pragma unroll
  for (int q = 0; q < MLP_H; ++q) acc[q] = 0.f;
  for (int64_t b = threadIdx.x; b < n; b += NT) {
    const float a = A[b * P + p];
#pragma unroll
    for (int q = 0; q < MLP_H; ++q)
      if (q < Q) acc[q] = fmaf(a, Bm ? Bm[b * Q + q] : 1.f, acc[q]);
  }
#pragma unroll
  for (int q = 0; q < MLP_H; ++q)
    if (q < Q) part[threadIdx.x][q] = acc[q];
  __syncthreads();
  if (threadIdx.x < Q) {
    float s = 0.f;
    for (int r = 0; r < NT; ++r) s += part[r][threadIdx.x];
    out[(size_t)p * ldo + threadIdx.x] = s;
  }
}

__global__ void k_zero(float* __restrict__ p, int n) {
  for (int i = blockIdx.x * NT + threadIdx.x; i < n; i += gridDim.x * NT) p[i] = 0.f;
}

// Adam on the mean loss (gradient scaled by inv_n) for parameters [MLP_OFF_W1, MLP_NPARAM)
__global__ __launch_bounds__(NT) void k_adam(float* __restrict__ params, const float* __restrict__ grad, float* __restrict__ m,
                                             float* __restrict__ v, float inv_n, float lr, float bc1, float bc2,
                                             const float* __restrict__ loss, float* __restrict__ loss_hist) {
  const int i = MLP_OFF_W1 + blockIdx.x * NT + threadIdx.x;
  if (loss_hist && blockIdx.x == 0 && threadIdx.x == 0) *loss_hist = loss[0] * inv_n;
  if (i >= MLP_NPARAM) return;
  const float g = grad[i] * inv_n;
  const float mi = 0.9f * m[i] + 0.1f * g;
  const float vi = 0.999f * v[i] + 0.001f * g * g;
  m[i] = mi;
  v[i] = vi;
  params[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + 1e-8f);
}

inline int blocks_for(int64_t n) { return (int)std::max<int64_t>(1, (n + NT - 1) / NT); }

}  // namespace

hipError_t mlp_forward(const float* params, const float* x, int64_t n, float* y, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_fwd, dim3(blocks_for(n)), dim3(NT), 0, s, params, x, n, y, nullptr, nullptr, nullptr);
  return hipGetLastError();
}

namespace {
struct MlpWork {
  float *XN, *H1, *H2, *Y, *dY, *D1, *D2, *lv, *loss;
};
hipError_t mlp_work(DevBuf& work, int64_t n, MlpWork* w) {
  const size_t per = (size_t)n * (MLP_IN + 4 * MLP_H + 3) + 64;
  hipError_t e = work.reserve(sizeof(float) * per);
  if (e != hipSuccess) return e;
  float* p = work.as<float>();
  w->XN = p; p += (size_t)n * MLP_IN;
  w->H1 = p; p += (size_t)n * MLP_H;
  w->H2 = p; p += (size_t)n * MLP_H;
  w->D1 = p; p += (size_t)n * MLP_H;
  w->D2 = p; p += (size_t)n * MLP_H;
  w->Y = p; p += n;
  w->dY = p; p += n;
  w->lv = p; p += n;
  w->loss = p;
  return hipSuccess;
}
hipError_t grad_steps(const MlpWork& w, const float* params, const float* x, const float* t, int64_t n, float tau, float* grad,
                      hipStream_t s) {
  const int nb = blocks_for(n);
  hipLaunchKernelGGL(k_mlp_fwd, dim3(nb), dim3(NT), 0, s, params, x, n, w.Y, w.XN, w.H1, w.H2);
  hipLaunchKernelGGL(k_mlp_bwd, dim3(nb), dim3(NT), 0, s, params, n, t, tau, w.Y, w.H1, w.H2, w.dY, w.D1, w.D2, w.lv);
  hipLaunchKernelGGL(k_zero, dim3(1), dim3(NT), 0, s, grad, MLP_OFF_W1);
  hipLaunchKernelGGL(k_outer, dim3(MLP_H), dim3(NT), 0, s, w.D1, MLP_H, w.XN, MLP_IN, n, grad + MLP_OFF_W1, MLP_IN);
  hipLaunchKernelGGL(k_outer, dim3(MLP_H), dim3(NT), 0, s, w.D1, MLP_H, (const float*)nullptr, 1, n, grad + MLP_OFF_B1, 1);
  hipLaunchKernelGGL(k_outer, dim3(MLP_H), dim3(NT), 0, s, w.D2, MLP_H, w.H1, MLP_H, n, grad + MLP_OFF_W2, MLP_H);
  hipLaunchKernelGGL(k_outer, dim3(MLP_H), dim3(NT), 0, s, w.D2, MLP_H, (const float*)nullptr, 1, n, grad + MLP_OFF_B2, 1);
  hipLaunchKernelGGL(k_outer, dim3(1), dim3(NT), 0, s, w.dY, 1, w.H2, MLP_H, n, grad + MLP_OFF_W3, MLP_H);
  hipLaunchKernelGGL(k_outer, dim3(1), dim3(NT), 0, s, w.dY, 1, (const float*)nullptr, 1, n, grad + MLP_OFF_B3, 1);
  hipLaunchKernelGGL(k_outer, dim3(1), dim3(NT), 0, s, w.lv, 1, (const float*)nullptr, 1, n, w.loss, 1);
  return hipGetLastError();
}
}  // namespace

hipError_t mlp_grad(DevBuf& work, const float* params, const float* x, const float* t, int64_t n, float tau, float* grad,
                    float* loss, hipStream_t s) {
  MlpWork w;
  hipError_t e = mlp_work(work, n, &w);
  if (e != hipSuccess) return e;
  e = grad_steps(w, params, x, t, n, tau, grad, s);
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(loss, w.loss, sizeof(float), hipMemcpyDeviceToDevice, s);
}

hipError_t mlp_train(DevBuf& work, float* params, const float* x, const float* t, int64_t n, float tau, int steps, float lr,
                     float* loss_hist, hipStream_t s) {
  MlpWork w;
  hipError_t e = mlp_work(work, n, &w);
  if (e != hipSuccess) return e;
  DevBuf opt;
  e = opt.reserve(sizeof(float) * 3 * MLP_NPARAM);
  if (e != hipSuccess) return e;
  float* grad = opt.as<float>();
  float* m = grad + MLP_NPARAM;
  float* v = m + MLP_NPARAM;
  hipLaunchKernelGGL(k_zero, dim3(8), dim3(NT), 0, s, m, 2 * MLP_NPARAM);
  const int nupd = MLP_NPARAM - MLP_OFF_W1;
  float bc1 = 1.f, bc2 = 1.f;
  for (int it = 0; it < steps; ++it) {
    e = grad_steps(w, params, x, t, n, tau, grad, s);
    if (e != hipSuccess) return e;
    bc1 *= 0.9f;
    bc2 *= 0.999f;
    hipLaunchKernelGGL(k_adam, dim3((nupd + NT - 1) / NT), dim3(NT), 0, s, params, grad, m, v, 1.f / (float)n, lr, 1.f - bc1,
                       1.f - bc2, w.loss, loss_hist ? loss_hist + it : nullptr);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

}  // namespace qps
