// Cost-model network kernels (see qs_mlp.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace qs {

constexpr int kMlpHidden = 64;

size_t mlp_num_params(int f, int h);
hipError_t launch_mlp_forward(const float *params, int f, int h, const float *x, int64_t n, float *y,
                              hipStream_t st);
hipError_t launch_mlp_grad(const float *params, int f, int h, const float *x, const float *t, int64_t n,
                           float *grad, float *loss, hipStream_t st);
hipError_t launch_mlp_train(float *params, float *mom, float *vel, int f, int h, const float *x, const float *t,
                            const int *idx, int batch, int steps, int step0, float lr, float *loss,
                            hipStream_t st);

}  // namespace qs
