// mlp.hip - FP32 kernels of the learned schedule cost model: a perceptron
// 7 -> 64 -> 64 -> 1 with ReLU hidden layers, mean squared error, Adam.
//
// Parameters are one flat array: W1[64][7], b1[64], W2[64][64], b2[64], W3[64], b3
// (4673 floats, 18.3 KiB), staged into LDS by every forward/backward workgroup.
// One thread handles one row (sample) in the forward and per-row backward
// kernels; weight gradients are reductions over rows, one thread per parameter
// with a fixed summation order (deterministic).  The network is tiny next to
// the timings it replaces, so plain FP32 VALU is used throughout.
#include "../../include/moma.h"
#include "common.hpp"

namespace moma {

constexpr int kIn = MOMA_COSTMODEL_FEATURES, kH = 64;
constexpr int kOffB1 = kH * kIn, kOffW2 = kOffB1 + kH, kOffB2 = kOffW2 + kH * kH, kOffW3 = kOffB2 + kH,
              kOffB3 = kOffW3 + kH, kNParam = kOffB3 + 1;

__device__ __forceinline__ void stage_params(float* sp, const float* __restrict__ p) {
  for (int i = threadIdx.x; i < kNParam; i += blockDim.x) sp[i] = p[i];
  __syncthreads();
}

// forward for rows [0, rows): y[r], and optionally the hidden activations
__global__ __launch_bounds__(256) void mlp_forward_kernel(const float* __restrict__ params,
                                                          const float* __restrict__ x, unsigned rows,
                                                          float* __restrict__ y, float* __restrict__ h1o,
                                                          float* __restrict__ h2o) {
  __shared__ float sp[kNParam];
  stage_params(sp, params);
  unsigned r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  float xi[kIn], h1[kH];
#pragma unroll
  for (int i = 0; i < kIn; i++) xi[i] = x[(size_t)r * kIn + i];
#pragma unroll
  for (int o = 0; o < kH; o++) {
    float s = sp[kOffB1 + o];
#pragma unroll
    for (int i = 0; i < kIn; i++) s = fmaf(sp[o * kIn + i], xi[i], s);
    h1[o] = s > 0.f ? s : 0.f;
    if (h1o) h1o[(size_t)r * kH + o] = h1[o];
  }
  float out = sp[kOffB3];
  for (int o = 0; o < kH; o++) {
    float s = sp[kOffB2 + o];
#pragma unroll
    for (int i = 0; i < kH; i++) s = fmaf(sp[kOffW2 + o * kH + i], h1[i], s);
    float h = s > 0.f ? s : 0.f;
    if (h2o) h2o[(size_t)r * kH + o] = h;
    out = fmaf(sp[kOffW3 + o], h, out);
  }
  y[r] = out;
}

// per-row backward: dy = 2 (y - t) / rows, d2 = relu'(h2) * dy * W3, d1 = relu'(h1) * W2^T d2;
// also (y - t)^2 per row for the loss
__global__ __launch_bounds__(256) void mlp_backrow_kernel(const float* __restrict__ params,
                                                          const float* __restrict__ y, const float* __restrict__ t,
                                                          const float* __restrict__ h1, const float* __restrict__ h2,
                                                          unsigned rows, float* __restrict__ dy,
                                                          float* __restrict__ d1, float* __restrict__ d2,
                                                          float* __restrict__ sq) {
  __shared__ float sp[kNParam];
  stage_params(sp, params);
  unsigned r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  float e = y[r] - t[r];
  float g = 2.f * e / (float)rows;
  dy[r] = g;
  sq[r] = e * e;
  float dd2[kH];
#pragma unroll
  for (int o = 0; o < kH; o++) {
    dd2[o] = h2[(size_t)r * kH + o] > 0.f ? g * sp[kOffW3 + o] : 0.f;
    d2[(size_t)r * kH + o] = dd2[o];
  }
  for (int i = 0; i < kH; i++) {
    float s = 0.f;
#pragma unroll
    for (int o = 0; o < kH; o++) s = fmaf(sp[kOffW2 + o * kH + i], dd2[o], s);
    d1[(size_t)r * kH + i] = h1[(size_t)r * kH + i] > 0.f ? s : 0.f;
  }
}

// gradient of every parameter: a fixed-order sum over rows
__global__ __launch_bounds__(256) void mlp_wgrad_kernel(const float* __restrict__ x, const float* __restrict__ h1,
                                                        const float* __restrict__ h2, const float* __restrict__ dy,
                                                        const float* __restrict__ d1, const float* __restrict__ d2,
                                                        const float* __restrict__ sq, unsigned rows,
                                                        float* __restrict__ grad, float* __restrict__ loss) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kNParam) return;
  float s = 0.f;
  if (p == kNParam) {  // one extra thread sums the loss
    for (unsigned r = 0; r < rows; r++) s += sq[r];
    *loss = s / (float)rows;
    return;
  }
  if (p < kOffB1) {
    int o = p / kIn, i = p % kIn;
    for (unsigned r = 0; r < rows; r++) s = fmaf(d1[(size_t)r * kH + o], x[(size_t)r * kIn + i], s);
  } else if (p < kOffW2) {
    int o = p - kOffB1;
    for (unsigned r = 0; r < rows; r++) s += d1[(size_t)r * kH + o];
  } else if (p < kOffB2) {
    int o = (p - kOffW2) / kH, i = (p - kOffW2) % kH;
    for (unsigned r = 0; r < rows; r++) s = fmaf(d2[(size_t)r * kH + o], h1[(size_t)r * kH + i], s);
  } else if (p < kOffW3) {
    int o = p - kOffB2;
    for (unsigned r = 0; r < rows; r++) s += d2[(size_t)r * kH + o];
  } else if (p < kOffB3) {
    int i = p - kOffW3;
    for (unsigned r = 0; r < rows; r++) s = fmaf(dy[r], h2[(size_t)r * kH + i], s);
  } else {
    for (unsigned r = 0; r < rows; r++) s += dy[r];
  }
  grad[p] = s;
}

// Adam with bias correction (Kingma and Ba, ICLR 2015); c1 = 1 - beta1^t, c2 = 1 - beta2^t
__global__ __launch_bounds__(256) void mlp_adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                                       float* __restrict__ m, float* __restrict__ v, float lr,
                                                       float b1, float b2, float eps, float c1, float c2) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kNParam) return;
  float gi = g[i];
  float mi = b1 * m[i] + (1.f - b1) * gi;
  float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

int mlp_nparams() { return kNParam; }

int launch_mlp_forward(const float* params, const float* x, unsigned rows, float* y, float* h1, float* h2,
                       hipStream_t s) {
  if (rows == 0) return 0;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((rows + 255) / 256), dim3(256), 0, s, params, x, rows, y, h1, h2);
  return (int)hipGetLastError();
}

// ws: 4 * rows * 64 + 3 * rows floats of workspace (h1, h2, d1, d2, y, dy, sq)
int launch_mlp_grad(const float* params, const float* x, const float* t, unsigned rows, float* grad, float* loss,
                    float* ws, hipStream_t s) {
  if (rows == 0) return (int)hipErrorInvalidValue;
  float *h1 = ws, *h2 = h1 + (size_t)rows * kH, *d1 = h2 + (size_t)rows * kH, *d2 = d1 + (size_t)rows * kH,
        *y = d2 + (size_t)rows * kH, *dy = y + rows, *sq = dy + rows;
  unsigned b = (rows + 255) / 256;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3(b), dim3(256), 0, s, params, x, rows, y, h1, h2);
  hipLaunchKernelGGL(mlp_backrow_kernel, dim3(b), dim3(256), 0, s, params, y, t, h1, h2, rows, dy, d1, d2, sq);
  hipLaunchKernelGGL(mlp_wgrad_kernel, dim3((kNParam + 1 + 255) / 256), dim3(256), 0, s, x, h1, h2, dy, d1, d2, sq,
                     rows, grad, loss);
  return (int)hipGetLastError();
}

size_t mlp_grad_workspace_floats(unsigned rows) { return (size_t)rows * kH * 4 + (size_t)rows * 3; }

int launch_mlp_adam(float* p, const float* g, float* m, float* v, unsigned step, float lr, float b1, float b2,
                    float eps, hipStream_t s) {
  float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((kNParam + 255) / 256), dim3(256), 0, s, p, g, m, v, lr, b1, b2, eps, c1,
                     c2);
  return (int)hipGetLastError();
}

}  // namespace moma
