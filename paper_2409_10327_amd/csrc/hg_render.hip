// hg_render.hip -- the multi-resolution hash encoding as kernels of its own
// (the renderer's encodes run inside the matrix-core kernel).
//
// encode:        f = H(x) per (point, level) pair.
// encode_index:  the corner indices and trilinear weights of every (point,
//                level), for tests and for the gather-replay ceiling.
#include "hg_device.h"
#include "hg_launch.h"

namespace hg {

// --------------------------------------------------------------------------
// Encode: one lane per (point, level).  Consecutive lanes take consecutive
// levels of one point, so the 8-byte feature writes of a wave are contiguous.
// --------------------------------------------------------------------------
template <typename TT>
__global__ __launch_bounds__(256) void k_encode(const GridK g, const float *__restrict__ pos, int64_t n,
                                                float *__restrict__ feat) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p = g.L == 16 ? (t >> 4) : t / g.L;
    const int l = (int)(t - p * g.L);
    if (p >= n) return;
    float u[3];
    bool in[3];
    pos_to_u(g, pos[3 * p], pos[3 * p + 1], pos[3 * p + 2], u, in);
    uint32_t c[3];
    float w[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) cell_of(u[d], g.resf[l], g.nm1f[l], c[d], w[d]);
    uint32_t ix[8];
    corner_idx(g, l, c, ix);
    const void *lvl = TabLoad<TT>::level(g.table, l, g.log2T);
    float2 e[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) e[k] = TabLoad<TT>::ld(lvl, ix[k]);
    const float wx0 = 1.0f - w[0], wy0 = 1.0f - w[1], wz0 = 1.0f - w[2];
    float f0 = 0.0f, f1 = 0.0f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const float wt = ((k & 1) ? w[0] : wx0) * (((k >> 1) & 1) ? w[1] : wy0) * (((k >> 2) & 1) ? w[2] : wz0);
        f0 = fmaf(wt, e[k].x, f0);
        f1 = fmaf(wt, e[k].y, f1);
    }
    reinterpret_cast<float2 *>(feat)[t] = make_float2(f0, f1);
}

hipError_t launch_encode(const GridK &g, bool f16, const float *pos, int64_t n, float *feat, hipStream_t s) {
    const int64_t threads = n * g.L;
    const unsigned blocks = (unsigned)((threads + 255) / 256);
    if (f16)
        hipLaunchKernelGGL(k_encode<__half>, dim3(blocks), dim3(256), 0, s, g, pos, n, feat);
    else
        hipLaunchKernelGGL(k_encode<float>, dim3(blocks), dim3(256), 0, s, g, pos, n, feat);
    return hipGetLastError();
}

// Index stage only: corner indices and in-cell weights per (point, level).
__global__ __launch_bounds__(256) void k_encode_index(const GridK g, const float *__restrict__ pos, int64_t n,
                                                      uint32_t *__restrict__ idx, float *__restrict__ wout) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p = g.L == 16 ? (t >> 4) : t / g.L;
    const int l = (int)(t - p * g.L);
    if (p >= n) return;
    float u[3];
    bool in[3];
    pos_to_u(g, pos[3 * p], pos[3 * p + 1], pos[3 * p + 2], u, in);
    uint32_t c[3];
    float w[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) cell_of(u[d], g.resf[l], g.nm1f[l], c[d], w[d]);
    uint32_t ix[8];
    corner_idx(g, l, c, ix);
#pragma unroll
    for (int k = 0; k < 8; ++k) idx[t * 8 + k] = ix[k];
    if (wout) {
#pragma unroll
        for (int d = 0; d < 3; ++d) wout[t * 3 + d] = w[d];
    }
}

hipError_t launch_encode_index(const GridK &g, const float *pos, int64_t n, uint32_t *idx, float *w, hipStream_t s) {
    const int64_t threads = n * g.L;
    const unsigned blocks = (unsigned)((threads + 255) / 256);
    hipLaunchKernelGGL(k_encode_index, dim3(blocks), dim3(256), 0, s, g, pos, n, idx, w);
    return hipGetLastError();
}

}  // namespace hg
