// hg_mis.hip -- light-importance distribution of an environment map for the
// MIS primary directions (Sec. 4.1): piecewise constant in solid angle over
// the equirectangular texels, probability proportional to Rec. 709
// luminance times the texel's solid angle; marginal CDF over rows,
// conditional CDF over the columns of each row.  Built in FP64 with the
// sums taken in a fixed order (row prefix sums per row, totals
// sequentially), so the result does not depend on the launch.
#include "hg_launch.h"

#include <hip/hip_runtime.h>

namespace hg {

constexpr int kDistThreads = 256;

#pragma clang fp contract(off)
__global__ __launch_bounds__(kDistThreads) void k_env_dist(const float *__restrict__ rgb, int H, int W,
                                                           double *__restrict__ dist) {
    double *ct = dist;
    double *marg = ct + (H + 1);
    double *cond = marg + (H + 1);
    float *dens = reinterpret_cast<float *>(cond + (size_t)H * (W + 1));
    __shared__ double s_total;
    __shared__ int s_uniform;
    const double pi = 3.14159265358979323846;
    for (int y = threadIdx.x; y <= H; y += blockDim.x) ct[y] = cos(pi * (double)y / (double)H);
    __syncthreads();
    // texel weights into cond[y][x + 1]; row sums into marg[y + 1]
    for (int y = threadIdx.x; y < H; y += blockDim.x) {
        const double omega = 2.0 * pi / (double)W * (ct[y] - ct[y + 1]);
        double *c = cond + (size_t)y * (W + 1);
        for (int x = 0; x < W; ++x) {
            const float *t = rgb + ((size_t)y * W + x) * 3;
            const double lum = 0.2126 * (double)t[0] + 0.7152 * (double)t[1] + 0.0722 * (double)t[2];
            c[x + 1] = lum * omega;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double total = 0.0;
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) total += cond[(size_t)y * (W + 1) + x + 1];
        s_uniform = !(total > 0.0);
        if (s_uniform) {
            // all-black map: weights = solid angles
            total = 0.0;
            for (int y = 0; y < H; ++y) {
                const double omega = 2.0 * pi / (double)W * (ct[y] - ct[y + 1]);
                for (int x = 0; x < W; ++x) total += omega;
            }
        }
        s_total = total;
    }
    __syncthreads();
    const double total = s_total;
    for (int y = threadIdx.x; y < H; y += blockDim.x) {
        const double omega = 2.0 * pi / (double)W * (ct[y] - ct[y + 1]);
        double *c = cond + (size_t)y * (W + 1);
        if (s_uniform)
            for (int x = 0; x < W; ++x) c[x + 1] = omega;
        double r = 0.0;
        for (int x = 0; x < W; ++x) r += c[x + 1];
        marg[y + 1] = r;
        for (int x = 0; x < W; ++x) dens[(size_t)y * W + x] = (float)(c[x + 1] / total / omega);
        c[0] = 0.0;
        double acc = 0.0;
        for (int x = 0; x < W; ++x) {
            acc += c[x + 1];
            c[x + 1] = r > 0.0 ? acc / r : (double)(x + 1) / (double)W;
        }
        c[W] = 1.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        marg[0] = 0.0;
        double acc = 0.0;
        for (int y = 0; y < H; ++y) {
            acc += marg[y + 1];
            marg[y + 1] = acc / total;
        }
        marg[H] = 1.0;
    }
}

hipError_t launch_env_dist(const float *rgb, int H, int W, double *dist, hipStream_t s) {
    hipLaunchKernelGGL(k_env_dist, dim3(1), dim3(kDistThreads), 0, s, rgb, H, W, dist);
    return hipGetLastError();
}

}  // namespace hg
