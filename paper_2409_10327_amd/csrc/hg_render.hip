// hg_render.hip -- FP32 forward kernels (one query per lane, vector ALU).
//
// encode:  f = H(x) per (point, level) pair.
// render:  Eq. (1) / Eq. (2) with the recursive bounce, shade mode with fewer
//          than 16 directions per point (the matrix-core kernel takes the rest).
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

// --------------------------------------------------------------------------
// Incoming radiance along (x, w) for one lane: Eq. (2) with the bounce.
// --------------------------------------------------------------------------
template <bool INDIRECT>
__device__ __forceinline__ void incoming(const RenderK &a, const float (&f)[kNF], float3 x, float3 w, uint32_t pid,
                                         uint32_t q, float *hbuf, int lane, float3 &Lin, float &V, float &d) {
    float z[kNI], h[kH], o[2];
#pragma unroll
    for (int i = 0; i < kNF; ++i) z[i] = f[i];
    z[kNF] = w.x; z[kNF + 1] = w.y; z[kNF + 2] = w.z;
    mlp_fwd<kNI, 2, float>(a.irt, z, hbuf, hbuf, lane, h, o);
    const bool hard = (a.s.flags & 2u) != 0;
    V = hard ? (o[0] > 0.0f ? 1.0f : 0.0f) : sigmoidf_(o[0]);
    d = fminf(softplusf_(o[1]), 1.0f);
    const float3 Le = env_lookup(a.env, w.x, w.y, w.z);
    if (!INDIRECT || (hard && V == 1.0f)) {
        Lin = make_float3(V * Le.x, V * Le.y, V * Le.z);
        return;
    }
    const float t = fmaf(a.t_span, d, a.t_near);
    const float3 xb = make_float3(fmaf(t, w.x, x.x), fmaf(t, w.y, x.y), fmaf(t, w.z, x.z));
    float fb[kNF];
    encode<float>(a.g, xb.x, xb.y, xb.z, fb);
    float ob[8];
    mlp_fwd<kNF, 8, float>(a.brdf, fb, hbuf, hbuf, lane, h, ob, a.brdf_out);
    const float3 ab = make_float3(sigmoidf_(ob[0]), sigmoidf_(ob[1]), sigmoidf_(ob[2]));
    const float rb = 0.09f + 0.91f * sigmoidf_(ob[3]);
    const float mb = sigmoidf_(ob[4]);
    // secondary view -w; normal from the decoder's normal head if it has one,
    // else the facing normal -w
    const float3 vb = make_float3(-w.x, -w.y, -w.z);
    const bool nhead = a.brdf_out == 8;
    const float3 nb = nhead ? head_normal(ob[5], ob[6], ob[7], vb) : vb;
    const Frame fr = make_frame(nb);
    const bool diffuse = (a.s.flags & 1u) != 0;
    FacingBrdf fb_;
    fb_.set(ab, rb, mb, a.f0, diffuse);
#pragma unroll
    for (int i = 0; i < kNF; ++i) z[i] = fb[i];
    float Lx = 0.f, Ly = 0.f, Lz = 0.f;
    uint4 words = make_uint4(0, 0, 0, 0);
    for (uint32_t j = 0; j < a.s.n_dirs2; ++j) {
        if ((j & 3u) == 0) words = philox4x32_10(pid, q, j >> 2, 1u, a.s.key0, a.s.key1);
        const float3 wj = sample_dir(pick4(words, j), j, a.s.nb2_shift, a.s.inv_na2, a.s.inv_nb2, fr);
        z[kNF] = wj.x; z[kNF + 1] = wj.y; z[kNF + 2] = wj.z;
        mlp_fwd<kNI, 2, float>(a.irt, z, hbuf, hbuf, lane, h, o);
        const float vj = hard ? (o[0] > 0.0f ? 1.0f : 0.0f) : sigmoidf_(o[0]);
        const float3 Ej = env_lookup(a.env, wj.x, wj.y, wj.z);
        const float3 c = nhead ? pi_brdf(nb, vb, wj, ab, rb, mb, a.f0, diffuse) : fb_.eval(dot3(nb, wj));
        Lx = fmaf(c.x * vj, Ej.x, Lx);
        Ly = fmaf(c.y * vj, Ej.y, Ly);
        Lz = fmaf(c.z * vj, Ej.z, Lz);
    }
    const float inv = 1.0f / (float)a.s.n_dirs2;
    const float om = 1.0f - V;
    Lin = make_float3(fmaf(V, Le.x, om * Lx * inv), fmaf(V, Le.y, om * Ly * inv), fmaf(V, Le.z, om * Lz * inv));
}

// --------------------------------------------------------------------------
// Shade mode: G = min(N, 64) lanes per pixel, 64/G pixels per wave; each lane
// sums N/G directions with Kahan compensation, then the G lanes of a pixel
// combine their (sum, compensation) pairs with TwoSum in a fixed butterfly.
// The result is bit-reproducible run to run.
// --------------------------------------------------------------------------
template <bool INDIRECT, bool MIS>
__global__ __launch_bounds__(128) void k_render_shade(const RenderK a) {
    extern __shared__ float lds[];
    const int lane = threadIdx.x & 63;
    float *hbuf = lds + (threadIdx.x >> 6) * kHBuf;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t gs = a.s.g_shift;
    const uint32_t G = 1u << gs;
    const int64_t p_raw = wave * (64 >> gs) + (lane >> gs);
    const bool live = p_raw < a.n;
    const int64_t p = live ? p_raw : a.n - 1;
    const uint32_t i0 = lane & (G - 1);
    const uint32_t N = a.s.n_dirs;
    const float3 x = make_float3(a.pos[3 * p], a.pos[3 * p + 1], a.pos[3 * p + 2]);
    const float3 n = make_float3(a.nrm[3 * p], a.nrm[3 * p + 1], a.nrm[3 * p + 2]);
    const float3 v = make_float3(a.wo[3 * p], a.wo[3 * p + 1], a.wo[3 * p + 2]);
    float f[kNF];
    encode<float>(a.g, x.x, x.y, x.z, f);
    float h[kH], ob[5];
    mlp_fwd<kNF, 5, float>(a.brdf, f, hbuf, hbuf, lane, h, ob);
    const float3 al = make_float3(sigmoidf_(ob[0]), sigmoidf_(ob[1]), sigmoidf_(ob[2]));
    const float rr = 0.09f + 0.91f * sigmoidf_(ob[3]);
    const float mm = sigmoidf_(ob[4]);
    const Frame fr = make_frame(n);
    const bool diffuse = (a.s.flags & 1u) != 0;
    const float3 vl = MIS ? ggx_view(fr, v) : v;
    KSum sx{0.f, 0.f}, sy{0.f, 0.f}, sz{0.f, 0.f};
    uint4 words = make_uint4(0, 0, 0, 0);
    for (uint32_t i = i0; i < N; i += G) {
        float3 wi;
        float wfac = 1.0f;
        if (MIS) {
            wi = mis_direction(a, fr, vl, rr, (uint32_t)p, i, wfac);
        } else {
            // four consecutive samples share one Philox call; with G >= 4
            // lanes per pixel each lane's samples are spaced G apart, so each
            // call serves the lane's sample only.
            words = philox4x32_10((uint32_t)p, 0u, i >> 2, 0u, a.s.key0, a.s.key1);
            wi = sample_dir(pick4(words, i), i, a.s.nb_shift, a.s.inv_na, a.s.inv_nb, fr);
        }
        float3 Lin;
        float V, d;
        incoming<INDIRECT>(a, f, x, wi, (uint32_t)p, i, hbuf, lane, Lin, V, d);
        float3 c = pi_brdf(n, v, wi, al, rr, mm, a.f0, diffuse);
        if (MIS) c = make_float3(c.x * wfac, c.y * wfac, c.z * wfac);
        sx.add(c.x * Lin.x);
        sy.add(c.y * Lin.y);
        sz.add(c.z * Lin.z);
        if (live && a.vis) {
            a.vis[p * N + i] = V;
            a.depth[p * N + i] = d;
        }
    }
    // butterfly over the G lanes of the pixel
    for (uint32_t off = G >> 1; off > 0; off >>= 1) {
        KSum *ks[3] = {&sx, &sy, &sz};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float os = __shfl_xor(ks[c]->s, (int)off);
            const float oc = __shfl_xor(ks[c]->c, (int)off);
            float s, e;
            // order the pair by lane so both partners compute the same value
            if (lane & off) two_sum(os, ks[c]->s, s, e);
            else two_sum(ks[c]->s, os, s, e);
            ks[c]->c = (lane & off) ? (oc + ks[c]->c) - e : (ks[c]->c + oc) - e;
            ks[c]->s = s;
        }
    }
    if (live && i0 == 0) {
        const float inv = 1.0f / (float)N;
        a.rgb[3 * p] = (sx.s - sx.c) * inv;
        a.rgb[3 * p + 1] = (sy.s - sy.c) * inv;
        a.rgb[3 * p + 2] = (sz.s - sz.c) * inv;
    }
}

hipError_t launch_render_f32_shade(const RenderK &a, bool indirect, hipStream_t s) {
    // 128-thread blocks: two waves, 2 x 16.6 KB of per-lane activation columns
    const size_t lds = 2 * kHBuf * sizeof(float);
    const int64_t ppw = 64 >> a.s.g_shift;
    const int64_t waves = (a.n + ppw - 1) / ppw;
    const unsigned blocks = (unsigned)((waves + 1) / 2);
    const bool mis = (a.s.flags & 4u) != 0;
    if (indirect) {
        if (mis) hipLaunchKernelGGL((k_render_shade<true, true>), dim3(blocks), dim3(128), lds, s, a);
        else hipLaunchKernelGGL((k_render_shade<true, false>), dim3(blocks), dim3(128), lds, s, a);
    } else {
        if (mis) hipLaunchKernelGGL((k_render_shade<false, true>), dim3(blocks), dim3(128), lds, s, a);
        else hipLaunchKernelGGL((k_render_shade<false, false>), dim3(blocks), dim3(128), lds, s, a);
    }
    return hipGetLastError();
}

}  // namespace hg
