// Cost-model network kernels (mlp.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace qtn {

constexpr int kMlpIn = 16, kMlpHidden = 64, kMlpOut = 4;
constexpr int kMlpParams = kMlpIn * kMlpHidden + kMlpHidden + kMlpHidden * kMlpHidden +
                           kMlpHidden + kMlpHidden * kMlpOut + kMlpOut;

// Device buffers carved from one workspace for a batch of n samples.
struct MlpBuffers {
  float *params, *grad, *m1, *m2;  // parameters, gradient, Adam moments
  float *x, *t, *m;                // inputs [n][16], targets and mask [n][3]
  float *z1, *h1, *z2, *h2;        // pre/post activations [n][64]
  float *y, *dy, *d2, *d1;         // outputs [n][3] and back-propagated errors
  float *loss;
  size_t bytes;
};

// Layout for n samples starting at ws (ws == nullptr: sizes only).
MlpBuffers mlp_buffers(void *ws, int64_t n);

hipError_t mlp_forward(const MlpBuffers &b, int n, hipStream_t s);
// Forward, loss (masked mean squared error) and the full gradient.
hipError_t mlp_loss_grad(const MlpBuffers &b, int n, hipStream_t s);
// One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) at step >= 1.
hipError_t mlp_adam(const MlpBuffers &b, int step, float lr, hipStream_t s);

}  // namespace qtn
