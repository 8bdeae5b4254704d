// Selector network (internal to libspx).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace spx {

constexpr int kMlpIn = 40, kMlpHid = 64, kMlpOut = 24;
constexpr int kMlpParams = kMlpHid * kMlpIn + kMlpHid + kMlpHid * kMlpHid + kMlpHid + kMlpOut * kMlpHid + kMlpOut;

size_t mlp_workspace_floats(int B);
hipError_t mlp_forward(const float *theta, const float *X, int B, float *logits, float *ws, hipStream_t s);
hipError_t mlp_loss_grad(const float *theta, const float *X, const int32_t *labels, int B, float *loss, float *grad,
                         float *ws, hipStream_t s);
// Device address of this GPU's workspace for batches of up to
// mlp_noalloc_max_batch() samples (a file-scope device array; no allocation).
hipError_t mlp_noalloc_scratch(float **out);
int mlp_noalloc_max_batch();
hipError_t mlp_adam(float *theta, const float *grad, float *m, float *v, int t, float lr, float b1, float b2,
                    float eps, hipStream_t s);

}  // namespace spx
