// hg_launch.h -- host-side launchers shared between the translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

#include "../../include/hg.h"
#include "hg_device.h"

namespace hg {

// Compute-unit count of the calling thread's current device, cached per
// device ordinal (a relaxed atomic: concurrent first calls store the same
// value).  Devices beyond the cache are queried on every call.
inline hipError_t current_device_cus(int &out) {
    constexpr int kMaxDev = 64;
    static std::atomic<int> cache[kMaxDev];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev >= 0 && dev < kMaxDev) {
        const int c = cache[dev].load(std::memory_order_relaxed);
        if (c > 0) {
            out = c;
            return hipSuccess;
        }
    }
    int c = 0;
    e = hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    if (c < 1) return hipErrorInvalidDevice;
    if (dev >= 0 && dev < kMaxDev) cache[dev].store(c, std::memory_order_relaxed);
    out = c;
    return hipSuccess;
}

// Workspace of the backward: one record per encoding the loss depends on
// (R = 2 per query with the bounce: x and x'; 1 without): the point, the
// gradient of the loss with respect to the features there, and a Morton key
// of the point with the record's id (and their sorted copies), so that the
// table scatter runs in spatial order, decoupled from the per-query work.
struct BounceWs {
    float4 *xb;        // [R n] point (w unused)
    float *gf;         // [R n][kNF] d loss / d f(point)
    uint32_t *key, *id;          // [R n] Morton key, record id
    uint32_t *key_sorted, *id_sorted;
    void *sort_tmp;
    size_t sort_tmp_bytes;
    uint4 *tiles;      // BF16 weight tiles of the mixed MLP backward
    float *wrep;       // replicated MLP-gradient accumulators of the mixed backward
};

struct BwdK {
    RenderK r;
    const float *g_rgb, *g_vis, *g_dep;
    float *g_table;
    float *gb[6];
    float *gi[6];
    float *g_pos;
    BounceWs ws;
    int64_t p_begin, p_end;  // the queries [p_begin, p_end) of this launch
    const uint4 *tiles;      // BF16 weight tiles (mixed MLPs), in the workspace
};

// Layout of the backward's workspace for n queries with R records each
// inside `base` (sort_tmp_bytes: what the radix sort of the R n keys needs);
// returns the bytes used.
size_t backward_ws_layout(int64_t n, int R, size_t sort_tmp_bytes, void *base, BounceWs *ws);
// Temporary bytes the radix sort of `records` keys needs (a host query).
hipError_t backward_sort_bytes(int64_t records, size_t &bytes);

hipError_t launch_encode(const GridK &g, bool f16, const float *pos, int64_t n, float *feat, hipStream_t s);
hipError_t launch_encode_index(const GridK &g, const float *pos, int64_t n, uint32_t *idx, float *w, hipStream_t s);
hipError_t launch_render_f32_mma(const RenderK &a, bool indirect, bool query, hipStream_t s);
hipError_t launch_render_mixed(const RenderK &a, bool indirect, bool query, hipStream_t s);
hipError_t launch_backward(const BwdK &a, bool f16, bool bf16_mlp, bool indirect, hipStream_t s);
hipError_t launch_l2_loss(const float *rgb, const float *vis, const float *dep, const float *tgt, int64_t n,
                          float *loss, float *g_rgb, float *g_vis, float *g_dep, hipStream_t s);
size_t denoise_workspace_floats(int H, int W);
hipError_t denoise_scratch(hipStream_t s, float **ptr, size_t *floats);
size_t env_dist_bytes(int H, int W);
void build_env_dist_host(const float *rgb, int H, int W, unsigned char *out);
hipError_t launch_denoise(const float *rgb, const float *depth, const float *nrm, int H, int W, int iters, float sz,
                          float sn, float sl, float *out, float *work, hipStream_t s);
hipError_t launch_adam(float *param, const float *grad, float *m, float *v, int64_t n, float lr, float b1,
                       float b2, float eps, float wd, float bc1, float bc2, void *shadow, int shadow_kind,
                       hipStream_t s);

}  // namespace hg
