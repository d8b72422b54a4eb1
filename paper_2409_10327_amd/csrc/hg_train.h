// Host-side launch interface of the multi-tensor Adam step (hg_train.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace hg {
constexpr int kAdamMax = 16;  // tensors per launch
// kernel argument: per tensor the arrays, size, weight decay and shadow kind
// (0 none, 1 FP16, 2 BF16); block0 is filled by launch_adam_multi
struct AdamMultiK {
    float *param[kAdamMax], *grad[kAdamMax], *m[kAdamMax], *v[kAdamMax];
    void *shadow[kAdamMax];
    int64_t n[kAdamMax];
    float wd[kAdamMax];
    int32_t kind[kAdamMax];
    uint32_t block0[kAdamMax + 1];
    int32_t count, zero_grad;
    float lr, b1, b2, eps, inv_bc1, inv_sqrt_bc2;
};
hipError_t launch_adam_multi(AdamMultiK &a, hipStream_t s);
}  // namespace hg
