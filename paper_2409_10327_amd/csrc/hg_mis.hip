// hg_mis.hip -- light-importance distribution of an environment map for the
// MIS primary directions (Sec. 4.1): piecewise constant in solid angle over
// the equirectangular texels, probability proportional to Rec. 709
// luminance times the texel's solid angle; marginal CDF over rows,
// conditional CDF over the columns of each row.
//
// Built once per map on the host in double precision (like the level
// resolutions), then stored for the device in single precision only: each
// CDF value c as the pair (hi, lo) = (RN32(c), RN32(c - hi)), so that the
// device decides c <= u for an FP32 uniform u exactly as the double value
// does (u - hi is exact near hi, Sterbenz), and the row geometry as
// cos(theta) at the top edge, 1 - cos(theta_top), 1 + cos(theta_bottom) and
// the row's cosine span, so that sin(theta) inside a row keeps full
// relative accuracy near both poles.
#include <cmath>
#include <vector>

#include "hg_launch.h"

namespace hg {

size_t env_dist_bytes(int H, int W) {
    return (size_t)H * sizeof(float4) + (size_t)(H + 1) * sizeof(float2) + (size_t)H * (W + 1) * sizeof(float2) +
           (size_t)H * W * sizeof(float);
}

namespace {

float2 split(double c) {
    const float hi = (float)c;
    return make_float2(hi, (float)(c - (double)hi));
}

}  // namespace

void build_env_dist_host(const float *rgb, int H, int W, unsigned char *out) {
    const double pi = 3.14159265358979323846;
    float4 *rows = reinterpret_cast<float4 *>(out);
    float2 *marg = reinterpret_cast<float2 *>(rows + H);
    float2 *cond = marg + (H + 1);
    float *dens = reinterpret_cast<float *>(cond + (size_t)H * (W + 1));
    std::vector<double> edge(H + 1), solid(H), wt((size_t)H * W), rowsum(H);
    for (int y = 0; y <= H; ++y) edge[y] = std::cos(pi * (double)y / (double)H);
    for (int y = 0; y < H; ++y) {
        const double th0 = pi * (double)y / (double)H, th1 = pi * (double)(y + 1) / (double)H;
        const double s0 = std::sin(0.5 * th0), c1 = std::cos(0.5 * th1);
        // 1 - cos(th0) = 2 sin^2(th0/2); 1 + cos(th1) = 2 cos^2(th1/2);
        // cos(th0) - cos(th1) = 2 sin((th0+th1)/2) sin((th1-th0)/2)
        const double span = 2.0 * std::sin(0.5 * (th0 + th1)) * std::sin(0.5 * (th1 - th0));
        rows[y] = make_float4((float)edge[y], (float)(2.0 * s0 * s0), (float)(2.0 * c1 * c1), (float)span);
        solid[y] = 2.0 * pi / (double)W * (edge[y] - edge[y + 1]);
    }
    double total = 0.0;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            const float *t = rgb + ((size_t)y * W + x) * 3;
            const double lum = 0.2126 * (double)t[0] + 0.7152 * (double)t[1] + 0.0722 * (double)t[2];
            wt[(size_t)y * W + x] = lum * solid[y];
        }
    for (size_t i = 0; i < wt.size(); ++i) total += wt[i];
    if (!(total > 0.0)) {  // all-black map: the uniform sphere
        total = 0.0;
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) wt[(size_t)y * W + x] = solid[y];
        for (size_t i = 0; i < wt.size(); ++i) total += wt[i];
    }
    for (int y = 0; y < H; ++y) {
        const double *w = wt.data() + (size_t)y * W;
        double r = 0.0;
        for (int x = 0; x < W; ++x) r += w[x];
        rowsum[y] = r;
        float2 *c = cond + (size_t)y * (W + 1);
        c[0] = make_float2(0.0f, 0.0f);
        double acc = 0.0;
        for (int x = 0; x < W; ++x) {
            acc += w[x];
            c[x + 1] = split(r > 0.0 ? acc / r : (double)(x + 1) / (double)W);
        }
        c[W] = make_float2(1.0f, 0.0f);
        for (int x = 0; x < W; ++x) dens[(size_t)y * W + x] = (float)(w[x] / total / solid[y]);
    }
    marg[0] = make_float2(0.0f, 0.0f);
    double acc = 0.0;
    for (int y = 0; y < H; ++y) {
        acc += rowsum[y];
        marg[y + 1] = split(acc / total);
    }
    marg[H] = make_float2(1.0f, 0.0f);
}

}  // namespace hg
