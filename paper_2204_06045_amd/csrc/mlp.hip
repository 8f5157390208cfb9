// Learned cost model: a 16-64-64-4 multilayer perceptron predicting the log
// launch time of a group under each kernel variant, trained on timings the
// autotuner measures.  Forward, backward and Adam are hand-written FP32
// kernels; every reduction runs in a fixed order, so results are
// deterministic.
//
// Parameter layout (floats): W1[16][64], b1[64], W2[64][64], b2[64],
// W3[64][4], b3[4], row-major with the input index first.
#include <hip/hip_runtime.h>

#include "mlp.hpp"

namespace qtn {
namespace {

// out_z[i][j] = b[j] + sum_k in[i][k] W[k][j];  out_h = max(out_z, 0) if relu.
__global__ void k_mlp_layer(const float *__restrict__ in, const float *__restrict__ W,
                            const float *__restrict__ b, float *__restrict__ out_z,
                            float *__restrict__ out_h, int n, int K, int J, int relu) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * J) return;
  const int i = e / J, j = e % J;
  float a = b[j];
  for (int k = 0; k < K; k++) a = fmaf(in[i * K + k], W[k * J + j], a);
  out_z[e] = a;
  if (out_h) out_h[e] = relu ? fmaxf(a, 0.0f) : a;
}

// Mean squared error over measured entries: loss and dL/dy.  One block.
__global__ void k_mlp_loss(const float *__restrict__ y, const float *__restrict__ t,
                           const float *__restrict__ m, int count, float *__restrict__ dy,
                           float *__restrict__ loss) {
  __shared__ float s_m[256], s_l[256];
  float pm = 0.0f;
  for (int q = threadIdx.x; q < count; q += blockDim.x) pm += m[q];
  s_m[threadIdx.x] = pm;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s_m[threadIdx.x] += s_m[threadIdx.x + w];
    __syncthreads();
  }
  const float msum = fmaxf(s_m[0], 1.0f);
  float pl = 0.0f;
  for (int q = threadIdx.x; q < count; q += blockDim.x) {
    const float e = y[q] - t[q];
    pl += m[q] * e * e;
    dy[q] = 2.0f * m[q] * e / msum;
  }
  s_l[threadIdx.x] = pl;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s_l[threadIdx.x] += s_l[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = s_l[0] / msum;
}

// d_in[i][k] = [z_in[i][k] > 0] * sum_j d_out[i][j] W[k][j]
__global__ void k_mlp_back(const float *__restrict__ d_out, const float *__restrict__ W,
                           const float *__restrict__ z_in, float *__restrict__ d_in, int n,
                           int K, int J) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * K) return;
  const int i = e / K, k = e % K;
  float a = 0.0f;
  for (int j = 0; j < J; j++) a = fmaf(d_out[i * J + j], W[k * J + j], a);
  d_in[e] = z_in[e] > 0.0f ? a : 0.0f;
}

// gW[k][j] = sum_i in[i][k] d_out[i][j] for k < K; row K is the bias.
__global__ void k_mlp_wgrad(const float *__restrict__ in, const float *__restrict__ d_out,
                            float *__restrict__ gW, float *__restrict__ gb, int n, int K,
                            int J) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (K + 1) * J) return;
  const int k = e / J, j = e % J;
  float a = 0.0f;
  if (k < K) {
    for (int i = 0; i < n; i++) a = fmaf(in[i * K + k], d_out[i * J + j], a);
    gW[k * J + j] = a;
  } else {
    for (int i = 0; i < n; i++) a += d_out[i * J + j];
    gb[j] = a;
  }
}

__global__ void k_mlp_adam(float *__restrict__ p, const float *__restrict__ g,
                           float *__restrict__ m1, float *__restrict__ m2, int np, float lr,
                           float b1, float b2, float eps, float c1, float c2) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= np) return;
  const float gq = g[q];
  const float a = b1 * m1[q] + (1.0f - b1) * gq;
  const float b = b2 * m2[q] + (1.0f - b2) * gq * gq;
  m1[q] = a;
  m2[q] = b;
  p[q] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

inline int blocks_for(int n) { return (n + 255) / 256; }

}  // namespace

MlpBuffers mlp_buffers(void *ws, int64_t n) {
  MlpBuffers b;
  float *f = (float *)ws;
  auto take = [&](int64_t count) {
    float *p = f;
    f += (count + 63) / 64 * 64;
    return p;
  };
  b.params = take(kMlpParams);
  b.grad = take(kMlpParams);
  b.m1 = take(kMlpParams);
  b.m2 = take(kMlpParams);
  b.x = take(n * kMlpIn);
  b.t = take(n * kMlpOut);
  b.m = take(n * kMlpOut);
  b.z1 = take(n * kMlpHidden);
  b.h1 = take(n * kMlpHidden);
  b.z2 = take(n * kMlpHidden);
  b.h2 = take(n * kMlpHidden);
  b.y = take(n * kMlpOut);
  b.dy = take(n * kMlpOut);
  b.d2 = take(n * kMlpHidden);
  b.d1 = take(n * kMlpHidden);
  b.loss = take(64);
  b.bytes = (size_t)((char *)f - (char *)ws);
  return b;
}

hipError_t mlp_forward(const MlpBuffers &b, int n, hipStream_t s) {
  const float *w1 = b.params, *b1 = w1 + kMlpIn * kMlpHidden, *w2 = b1 + kMlpHidden;
  const float *b2 = w2 + kMlpHidden * kMlpHidden, *w3 = b2 + kMlpHidden;
  const float *b3 = w3 + kMlpHidden * kMlpOut;
  hipLaunchKernelGGL(k_mlp_layer, dim3(blocks_for(n * kMlpHidden)), dim3(256), 0, s, b.x, w1, b1,
                     b.z1, b.h1, n, kMlpIn, kMlpHidden, 1);
  hipLaunchKernelGGL(k_mlp_layer, dim3(blocks_for(n * kMlpHidden)), dim3(256), 0, s, b.h1, w2,
                     b2, b.z2, b.h2, n, kMlpHidden, kMlpHidden, 1);
  hipLaunchKernelGGL(k_mlp_layer, dim3(blocks_for(n * kMlpOut)), dim3(256), 0, s, b.h2, w3, b3,
                     b.y, (float *)nullptr, n, kMlpHidden, kMlpOut, 0);
  return hipGetLastError();
}

hipError_t mlp_loss_grad(const MlpBuffers &b, int n, hipStream_t s) {
  hipError_t e = mlp_forward(b, n, s);
  if (e != hipSuccess) return e;
  const float *w1 = b.params, *b1 = w1 + kMlpIn * kMlpHidden, *w2 = b1 + kMlpHidden;
  const float *b2 = w2 + kMlpHidden * kMlpHidden, *w3 = b2 + kMlpHidden;
  (void)b1;
  (void)b2;
  float *gw1 = b.grad, *gb1 = gw1 + kMlpIn * kMlpHidden, *gw2 = gb1 + kMlpHidden;
  float *gb2 = gw2 + kMlpHidden * kMlpHidden, *gw3 = gb2 + kMlpHidden;
  float *gb3 = gw3 + kMlpHidden * kMlpOut;
  hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(256), 0, s, b.y, b.t, b.m, n * kMlpOut, b.dy,
                     b.loss);
  hipLaunchKernelGGL(k_mlp_wgrad, dim3(blocks_for((kMlpHidden + 1) * kMlpOut)), dim3(256), 0, s,
                     b.h2, b.dy, gw3, gb3, n, kMlpHidden, kMlpOut);
  hipLaunchKernelGGL(k_mlp_back, dim3(blocks_for(n * kMlpHidden)), dim3(256), 0, s, b.dy, w3,
                     b.z2, b.d2, n, kMlpHidden, kMlpOut);
  hipLaunchKernelGGL(k_mlp_wgrad, dim3(blocks_for((kMlpHidden + 1) * kMlpHidden)), dim3(256), 0,
                     s, b.h1, b.d2, gw2, gb2, n, kMlpHidden, kMlpHidden);
  hipLaunchKernelGGL(k_mlp_back, dim3(blocks_for(n * kMlpHidden)), dim3(256), 0, s, b.d2, w2,
                     b.z1, b.d1, n, kMlpHidden, kMlpHidden);
  hipLaunchKernelGGL(k_mlp_wgrad, dim3(blocks_for((kMlpIn + 1) * kMlpHidden)), dim3(256), 0, s,
                     b.x, b.d1, gw1, gb1, n, kMlpIn, kMlpHidden);
  return hipGetLastError();
}

hipError_t mlp_adam(const MlpBuffers &b, int step, float lr, hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_mlp_adam, dim3(blocks_for(kMlpParams)), dim3(256), 0, s, b.params, b.grad,
                     b.m1, b.m2, kMlpParams, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace qtn
