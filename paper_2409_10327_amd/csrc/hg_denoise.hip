// hg_denoise.hip -- spatial variance-guided a-trous filter (SVGF without its
// temporal parts), applied to the Monte Carlo frame (paper Sec. 4.1; depth
// gradient by finite differences of the depth map, supplementary "Rendering
// Details").
//
// Workspace (floats per pixel): two colour+luminance buffers (4 each), two
// variance buffers, depth gradient (2).  One thread per pixel; taps are read
// through L1/L2 (neighbouring pixels share them).
#include <mutex>

#include "hg_launch.h"

namespace hg {

constexpr int kDnBlock = 16;
constexpr int kDnFloatsPerPixel = 12;

// Workspace of hg_denoise_noalloc: one copy per GPU (the runtime places it
// when the code object is loaded on a device; it is held until the process
// ends), sized for HG_DENOISE_NOALLOC_MAX_PIXELS pixels = 48 MiB.  Host code
// never passes this name to a kernel (on the host it is only a stand-in for
// the symbol): it passes the device address that denoise_scratch() obtains.
static __device__ __align__(256) float scratch[(size_t)HG_DENOISE_NOALLOC_MAX_PIXELS * kDnFloatsPerPixel];

__device__ __forceinline__ float luminance(float r, float g, float b) {
    return 0.2126f * r + 0.7152f * g + 0.0722f * b;
}

// colour + luminance, forward-difference depth gradient, 7x7 luminance
// moments (taps inside the image only)
__global__ __launch_bounds__(kDnBlock * kDnBlock) void k_dn_init(const float *__restrict__ rgb,
                                                                  const float *__restrict__ depth, int H, int W,
                                                                  float4 *__restrict__ col, float *__restrict__ var,
                                                                  float2 *__restrict__ grad) {
    const int x = blockIdx.x * kDnBlock + threadIdx.x;
    const int y = blockIdx.y * kDnBlock + threadIdx.y;
    if (x >= W || y >= H) return;
    const size_t p = (size_t)y * W + x;
    const float r = rgb[3 * p], g = rgb[3 * p + 1], b = rgb[3 * p + 2];
    col[p] = make_float4(r, g, b, luminance(r, g, b));
    const float z = depth[p];
    // forward differences, backward at the last column/row, zero along an
    // axis that is one pixel long
    const float gx = x + 1 < W ? depth[p + 1] - z : (x > 0 ? z - depth[p - 1] : 0.0f);
    const float gy = y + 1 < H ? depth[p + W] - z : (y > 0 ? z - depth[p - W] : 0.0f);
    grad[p] = make_float2(gx, gy);
    float s1 = 0.f, s2 = 0.f;
    int cnt = 0;
    for (int dy = -3; dy <= 3; ++dy) {
        const int yy = y + dy;
        if (yy < 0 || yy >= H) continue;
        for (int dx = -3; dx <= 3; ++dx) {
            const int xx = x + dx;
            if (xx < 0 || xx >= W) continue;
            const size_t q = (size_t)yy * W + xx;
            const float l = luminance(rgb[3 * q], rgb[3 * q + 1], rgb[3 * q + 2]);
            s1 += l;
            s2 += l * l;
            ++cnt;
        }
    }
    const float m = s1 / (float)cnt;
    var[p] = fmaxf(s2 / (float)cnt - m * m, 0.0f);
}

// one a-trous iteration with step `step`; writes colour (and luminance) and
// the propagated variance; `out_rgb` (if set) receives the colour as [P][3]
__global__ __launch_bounds__(kDnBlock * kDnBlock) void k_dn_atrous(
    const float4 *__restrict__ col, const float *__restrict__ var, const float2 *__restrict__ grad,
    const float *__restrict__ depth, const float *__restrict__ nrm, int H, int W, int step, float sz, float sn,
    float sl, float4 *__restrict__ col_out, float *__restrict__ var_out, float *__restrict__ out_rgb) {
    const int x = blockIdx.x * kDnBlock + threadIdx.x;
    const int y = blockIdx.y * kDnBlock + threadIdx.y;
    if (x >= W || y >= H) return;
    const size_t p = (size_t)y * W + x;
    // 3x3 binomial blur of the variance (edges clamped)
    float g3 = 0.f;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            const int xx = min(max(x + dx, 0), W - 1), yy = min(max(y + dy, 0), H - 1);
            g3 += (dx ? 0.25f : 0.5f) * (dy ? 0.25f : 0.5f) * var[(size_t)yy * W + xx];
        }
    const float4 cp = col[p];
    const float zp = depth[p];
    const float2 gp = grad[p];
    const float npx = nrm[3 * p], npy = nrm[3 * p + 1], npz = nrm[3 * p + 2];
    const float lden = sl * sqrtf(fmaxf(g3, 0.0f)) + 1e-10f;
    const float h[5] = {1.0f / 16, 1.0f / 4, 3.0f / 8, 1.0f / 4, 1.0f / 16};
    float ws = 0.f, ar = 0.f, ag = 0.f, ab = 0.f, av = 0.f;
#pragma unroll
    for (int j = -2; j <= 2; ++j) {
        const int yy = y + j * step;
        if (yy < 0 || yy >= H) continue;
#pragma unroll
        for (int i = -2; i <= 2; ++i) {
            const int xx = x + i * step;
            if (xx < 0 || xx >= W) continue;
            const size_t q = (size_t)yy * W + xx;
            const float4 cq = col[q];
            const float wz = __expf(-fabsf(zp - depth[q]) /
                                    (sz * fabsf(gp.x * (float)(i * step) + gp.y * (float)(j * step)) + 1e-6f));
            const float nd = npx * nrm[3 * q] + npy * nrm[3 * q + 1] + npz * nrm[3 * q + 2];
            // nd^sn as exp2(sn log2 nd) by the hardware log2 / exp2
            const float wn = nd > 0.0f ? __builtin_amdgcn_exp2f(sn * __builtin_amdgcn_logf(nd))
                                       : (sn == 0.0f ? 1.0f : 0.0f);
            const float wl = __expf(-fabsf(cp.w - cq.w) / lden);
            const float w = h[i + 2] * h[j + 2] * wz * wn * wl;
            ws += w;
            ar = fmaf(w, cq.x, ar);
            ag = fmaf(w, cq.y, ag);
            ab = fmaf(w, cq.z, ab);
            av = fmaf(w * w, var[q], av);
        }
    }
    const float inv = 1.0f / ws;
    const float r = ar * inv, g = ag * inv, b = ab * inv;
    col_out[p] = make_float4(r, g, b, luminance(r, g, b));
    var_out[p] = av * inv * inv;
    if (out_rgb) {
        out_rgb[3 * p] = r;
        out_rgb[3 * p + 1] = g;
        out_rgb[3 * p + 2] = b;
    }
}

__global__ void k_dn_copy(const float *__restrict__ src, float *__restrict__ dst, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

size_t denoise_workspace_floats(int H, int W) { return (size_t)H * W * kDnFloatsPerPixel; }

namespace {
constexpr int kMaxScratchDev = 64;
std::mutex g_scratch_mu;
std::atomic<float *> g_scratch_ptr[kMaxScratchDev];
}  // namespace

// Device address of `scratch` on the device that `s` belongs to (the current
// device for the null stream).  Resolved once per device with that device
// current, then read from the per-device cache.
hipError_t denoise_scratch(hipStream_t s, float **ptr, size_t *floats) {
    int dev = 0;
    hipError_t e = s ? hipStreamGetDevice(s, &dev) : hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxScratchDev) return hipErrorInvalidDevice;
    float *p = g_scratch_ptr[dev].load(std::memory_order_acquire);
    if (p == nullptr) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        p = g_scratch_ptr[dev].load(std::memory_order_relaxed);
        if (p == nullptr) {
            int cur = 0;
            if ((e = hipGetDevice(&cur)) != hipSuccess) return e;
            if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
            void *q = nullptr;
            e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
            if (cur != dev) {
                const hipError_t back = hipSetDevice(cur);
                if (e == hipSuccess) e = back;
            }
            if (e != hipSuccess) return e;
            if (q == nullptr) return hipErrorInvalidSymbol;
            p = static_cast<float *>(q);
            g_scratch_ptr[dev].store(p, std::memory_order_release);
        }
    }
    *ptr = p;
    *floats = sizeof(scratch) / sizeof(float);
    return hipSuccess;
}

hipError_t launch_denoise(const float *rgb, const float *depth, const float *nrm, int H, int W, int iters, float sz,
                          float sn, float sl, float *out, float *work, hipStream_t s) {
    const size_t P = (size_t)H * W;
    float4 *ca = reinterpret_cast<float4 *>(work);
    float4 *cb = ca + P;
    float *va = reinterpret_cast<float *>(cb + P);
    float *vb = va + P;
    float2 *grad = reinterpret_cast<float2 *>(vb + P);
    if (iters == 0) {
        const int64_t n = 3 * (int64_t)P;
        hipLaunchKernelGGL(k_dn_copy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, rgb, out, n);
        return hipGetLastError();
    }
    const dim3 blk(kDnBlock, kDnBlock), grd((W + kDnBlock - 1) / kDnBlock, (H + kDnBlock - 1) / kDnBlock);
    hipLaunchKernelGGL(k_dn_init, grd, blk, 0, s, rgb, depth, H, W, ca, va, grad);
    for (int it = 0; it < iters; ++it) {
        hipLaunchKernelGGL(k_dn_atrous, grd, blk, 0, s, ca, va, grad, depth, nrm, H, W, 1 << it, sz, sn, sl, cb, vb,
                           it + 1 == iters ? out : nullptr);
        float4 *tc = ca; ca = cb; cb = tc;
        float *tv = va; va = vb; vb = tv;
    }
    return hipGetLastError();
}

}  // namespace hg
