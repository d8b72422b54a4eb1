// hg_train.hip -- L2 distillation loss and Adam.
#include <hip/hip_bf16.h>

#include "hg_launch.h"
#include "hg_train.h"

namespace hg {

__global__ void k_zero1(float *p) { *p = 0.0f; }

// Per-sample squared errors; the gradient is elementwise (deterministic),
// the scalar loss is a wave reduction followed by one atomic per wave.
// One atomic add per block into the loss (a grid of at most kLossBlocks
// blocks, each striding over the samples): adds on one address serialise,
// about 13 ns each, so one per wave cost 55 us at 2^18 samples.
constexpr unsigned kLossBlocks = 512;
__global__ __launch_bounds__(256) void k_l2_loss(const float *__restrict__ rgb, const float *__restrict__ vis,
                                                 const float *__restrict__ dep, const float *__restrict__ tgt,
                                                 int64_t n, float inv_n, float *loss, float *g_rgb, float *g_vis,
                                                 float *g_dep) {
    __shared__ float part[4];
    float l = 0.0f;
    const float s = 2.0f * inv_n;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const float *t = tgt + 5 * p;
        const float e0 = rgb[3 * p] - t[0], e1 = rgb[3 * p + 1] - t[1], e2 = rgb[3 * p + 2] - t[2];
        const float ev = vis[p] - t[3], ed = dep[p] - t[4];
        l += e0 * e0 + e1 * e1 + e2 * e2 + ev * ev + ed * ed;
        g_rgb[3 * p] = s * e0;
        g_rgb[3 * p + 1] = s * e1;
        g_rgb[3 * p + 2] = s * e2;
        g_vis[p] = s * ev;
        g_dep[p] = s * ed;
    }
    for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = l;
    __syncthreads();
    if (threadIdx.x == 0) unsafeAtomicAdd(loss, (part[0] + part[1] + part[2] + part[3]) * inv_n);
}

hipError_t launch_l2_loss(const float *rgb, const float *vis, const float *dep, const float *tgt, int64_t n,
                          float *loss, float *g_rgb, float *g_vis, float *g_dep, hipStream_t s) {
    hipLaunchKernelGGL(k_zero1, dim3(1), dim3(1), 0, s, loss);
    if (n > 0) {
        const int64_t want = (n + 255) / 256;
        const unsigned blocks = (unsigned)(want < (int64_t)kLossBlocks ? want : (int64_t)kLossBlocks);
        hipLaunchKernelGGL(k_l2_loss, dim3(blocks), dim3(256), 0, s, rgb, vis, dep, tgt, n, 1.0f / (float)n, loss,
                           g_rgb, g_vis, g_dep);
    }
    return hipGetLastError();
}

// Adam with bias correction (bc1 = 1 - b1^t, bc2 = 1 - b2^t computed on the
// host in double); weight decay added to the gradient.  Four parameters per
// lane with 16-byte accesses; the tail is handled element by element.
// The update of parameters i0 .. i0 + 3 (fewer at the tail), shared by the
// single-tensor and the multi-tensor kernels.
template <int KIND>  // 0: no shadow, 1: FP16 shadow, 2: BF16 shadow
__device__ __forceinline__ void adam_update(float *__restrict__ param, const float *__restrict__ grad,
                                            float *__restrict__ m, float *__restrict__ v, int64_t n, int64_t i0,
                                            float lr, float b1, float b2, float eps, float wd, float inv_bc1,
                                            float inv_sqrt_bc2, void *__restrict__ shadow) {
    const int cnt = (int)((n - i0) < 4 ? (n - i0) : 4);
    float pp[4], gg[4], mm[4], vv[4];
    if (cnt == 4) {
        const float4 a = *reinterpret_cast<const float4 *>(param + i0);
        const float4 b = *reinterpret_cast<const float4 *>(grad + i0);
        const float4 c = *reinterpret_cast<const float4 *>(m + i0);
        const float4 d = *reinterpret_cast<const float4 *>(v + i0);
        pp[0] = a.x; pp[1] = a.y; pp[2] = a.z; pp[3] = a.w;
        gg[0] = b.x; gg[1] = b.y; gg[2] = b.z; gg[3] = b.w;
        mm[0] = c.x; mm[1] = c.y; mm[2] = c.z; mm[3] = c.w;
        vv[0] = d.x; vv[1] = d.y; vv[2] = d.z; vv[3] = d.w;
    } else {
        for (int k = 0; k < cnt; ++k) {
            pp[k] = param[i0 + k]; gg[k] = grad[i0 + k]; mm[k] = m[i0 + k]; vv[k] = v[i0 + k];
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float g = gg[k] + wd * pp[k];
        mm[k] = b1 * mm[k] + (1.0f - b1) * g;
        vv[k] = b2 * vv[k] + (1.0f - b2) * g * g;
        const float den = sqrtf(vv[k]) * inv_sqrt_bc2 + eps;
        pp[k] = pp[k] - lr * (mm[k] * inv_bc1) / den;
    }
    if (cnt == 4) {
        *reinterpret_cast<float4 *>(param + i0) = make_float4(pp[0], pp[1], pp[2], pp[3]);
        *reinterpret_cast<float4 *>(m + i0) = make_float4(mm[0], mm[1], mm[2], mm[3]);
        *reinterpret_cast<float4 *>(v + i0) = make_float4(vv[0], vv[1], vv[2], vv[3]);
    } else {
        for (int k = 0; k < cnt; ++k) {
            param[i0 + k] = pp[k]; m[i0 + k] = mm[k]; v[i0 + k] = vv[k];
        }
    }
    if (KIND == 1) {
        __half *sh = static_cast<__half *>(shadow);
        for (int k = 0; k < cnt; ++k) sh[i0 + k] = __float2half_rn(pp[k]);
    } else if (KIND == 2) {
        __hip_bfloat16 *sh = static_cast<__hip_bfloat16 *>(shadow);
        for (int k = 0; k < cnt; ++k) sh[i0 + k] = __float2bfloat16(pp[k]);
    }
}

template <int KIND>
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ param, const float *__restrict__ grad,
                                              float *__restrict__ m, float *__restrict__ v, int64_t n, float lr,
                                              float b1, float b2, float eps, float wd, float inv_bc1,
                                              float inv_sqrt_bc2, void *__restrict__ shadow) {
    const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (i0 >= n) return;
    adam_update<KIND>(param, grad, m, v, n, i0, lr, b1, b2, eps, wd, inv_bc1, inv_sqrt_bc2, shadow);
}

// Several tensors in one launch: tensor t owns blocks block0[t] ..
// block0[t + 1] - 1 (the block's tensor is wave-uniform); with zero_grad each
// lane clears the gradients it has read.
__global__ __launch_bounds__(256) void k_adam_multi(const AdamMultiK a) {
    int t = 0;
    for (int k = 1; k < a.count; ++k) t = blockIdx.x >= a.block0[k] ? k : t;
    const int64_t n = a.n[t];
    const int64_t i0 = ((int64_t)(blockIdx.x - a.block0[t]) * blockDim.x + threadIdx.x) * 4;
    if (i0 >= n) return;
    float *const g = a.grad[t];
    if (a.kind[t] == 1)
        adam_update<1>(a.param[t], g, a.m[t], a.v[t], n, i0, a.lr, a.b1, a.b2, a.eps, a.wd[t], a.inv_bc1,
                       a.inv_sqrt_bc2, a.shadow[t]);
    else if (a.kind[t] == 2)
        adam_update<2>(a.param[t], g, a.m[t], a.v[t], n, i0, a.lr, a.b1, a.b2, a.eps, a.wd[t], a.inv_bc1,
                       a.inv_sqrt_bc2, a.shadow[t]);
    else
        adam_update<0>(a.param[t], g, a.m[t], a.v[t], n, i0, a.lr, a.b1, a.b2, a.eps, a.wd[t], a.inv_bc1,
                       a.inv_sqrt_bc2, a.shadow[t]);
    if (a.zero_grad) {
        if (n - i0 >= 4) {
            *reinterpret_cast<float4 *>(g + i0) = make_float4(0.f, 0.f, 0.f, 0.f);
        } else {
            for (int64_t k = i0; k < n; ++k) g[k] = 0.0f;
        }
    }
}

hipError_t launch_adam_multi(AdamMultiK &a, hipStream_t s) {
    uint32_t b = 0;
    for (int t = 0; t < a.count; ++t) {
        a.block0[t] = b;
        b += (uint32_t)(((a.n[t] + 3) / 4 + 255) / 256);
    }
    a.block0[a.count] = b;
    if (b == 0) return hipSuccess;
    hipLaunchKernelGGL(k_adam_multi, dim3(b), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_adam(float *param, const float *grad, float *m, float *v, int64_t n, float lr, float b1,
                       float b2, float eps, float wd, float bc1, float bc2, void *shadow, int shadow_kind,
                       hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)(((n + 3) / 4 + 255) / 256);
    const float inv_bc1 = 1.0f / bc1, inv_sqrt_bc2 = 1.0f / sqrtf(bc2);
    if (shadow_kind == 1)
        hipLaunchKernelGGL(k_adam<1>, dim3(blocks), dim3(256), 0, s, param, grad, m, v, n, lr, b1, b2, eps, wd,
                           inv_bc1, inv_sqrt_bc2, shadow);
    else if (shadow_kind == 2)
        hipLaunchKernelGGL(k_adam<2>, dim3(blocks), dim3(256), 0, s, param, grad, m, v, n, lr, b1, b2, eps, wd,
                           inv_bc1, inv_sqrt_bc2, shadow);
    else
        hipLaunchKernelGGL(k_adam<0>, dim3(blocks), dim3(256), 0, s, param, grad, m, v, n, lr, b1, b2, eps, wd,
                           inv_bc1, inv_sqrt_bc2, shadow);
    return hipGetLastError();
}

}  // namespace hg
