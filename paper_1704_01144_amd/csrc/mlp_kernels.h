// Launchers of the learned-guess kernels (defined in mlp.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "mlp.h"

namespace tafv {

// FP32 parameter vector th[1313] -> device network (BF16 fragments)
hipError_t mlp_pack(hipStream_t s, const float* th, MlpDev* w);
// y[n] for inputs x[n][6]
hipError_t mlp_forward(hipStream_t s, int n, const float* x, const MlpDev* w, float* y);
// gradient of the mean squared error over `count` rows: batch row i maps to
// data row (a (first + i) + b) mod n; gpart: [ceil(count/64)][1313] scratch,
// lpart: [ceil(count/64)] scratch; loss_acc += sum of squared errors * loss_scale
hipError_t mlp_gradient(hipStream_t s, unsigned long long a, unsigned long long b,
                        unsigned long long n, long long first, long long count, const float* x,
                        const float* t, const MlpDev* w, float* gpart, float* lpart, float* grad,
                        float* loss_acc, float loss_scale);
// one Adam step (step >= 1) with beta = (0.9, 0.999), eps = 1e-8
hipError_t mlp_adam(hipStream_t s, float* th, float* m, float* v, const float* grad, float lr,
                    int step);
hipError_t mlp_fill(hipStream_t s, float* p, float v, int n);

}  // namespace tafv
