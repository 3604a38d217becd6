// Kernels of the selector's multilayer perceptron (FP32): forward, backward, masked MSE, Adam.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ffc {

int64_t mlp_param_count(int in, int h, int out);
hipError_t mlp_forward(int in, int h, int out, int64_t batch, const float* params, const float* x, float* act,
                       float* y, hipStream_t s);
hipError_t mlp_backward(int in, int h, int out, int64_t batch, const float* params, const float* x, const float* act,
                        const float* dy, float* grad, float* work, hipStream_t s);
hipError_t mlp_mse(int64_t n, const float* y, const float* t, const float* m, float* dy, float* loss, hipStream_t s);
hipError_t adam_step(int64_t n, float* p, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                     float wd, int step, hipStream_t s);

}  // namespace ffc
