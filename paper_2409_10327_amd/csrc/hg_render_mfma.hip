// hg_render_mfma.hip -- mixed-precision forward on the CDNA4 matrix cores.
//
// FP16 hash tables gathered with FP32 interpolation; both MLPs run as
// v_mfma_f32_16x16x32_bf16 tiles (BF16 operands, FP32 accumulation); the
// light-direction sum is compensated FP32.
//
// Work decomposition.  A wave owns 64 queries (one per lane) for the scalar
// work: direction sampling, hash-grid gathers, environment lookups, BRDF.
// Each MLP evaluation of the 64 queries is four 16-column N-tiles of
// matrix-core products with the units of a layer as rows (M) and the
// queries as columns (N):
//   layer output D (16x16 per M-tile): lane l holds rows 4*(l/16)+r,
//   column l%16 -- so the fp32 accumulators of one layer, after ReLU and
//   conversion to BF16, are already the B operand of the next layer once the
//   weight columns are permuted accordingly (no data movement between
//   layers).
//   head rows are replicated so that every lane group receives the outputs
//   of its column; lane l keeps N-tile l/16, which is its own query.
// Inputs that come from other lanes (features, directions) go through LDS.
// The tracer's first layer is split into a per-point part (W0f f + b0,
// computed once per point and kept in registers as the accumulator input)
// and a direction part (one matrix-core step with the direction split into
// BF16 high and low halves).
// Weight tiles are built once per workgroup in LDS in operand order; the
// tracer's hot tiles are then held in registers.
#include <hip/hip_bf16.h>

#include "hg_device.h"
#include "hg_launch.h"

namespace hg {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short s16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ f32x4 mfma(const uint4 &a, const uint4 &b, const f32x4 &c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b),
                                                    c, 0, 0, 0);
}

// Round-to-nearest-even FP32 -> BF16 of two values, packed (lo = a).
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
    const __bf16 ha = (__bf16)a, hb = (__bf16)b;
    return (uint32_t)__builtin_bit_cast(uint16_t, ha) | ((uint32_t)__builtin_bit_cast(uint16_t, hb) << 16);
}

// ReLU on two packed BF16 values: as signed 16-bit integers, every negative
// BF16 (sign bit set) is below zero, so an integer max with 0 is the ReLU.
__device__ __forceinline__ uint32_t relu_bf16x2(uint32_t v) {
    s16x2 s = __builtin_bit_cast(s16x2, v);
    s = __builtin_elementwise_max(s, (s16x2){0, 0});
    return __builtin_bit_cast(uint32_t, s);
}

// Two accumulator tiles (M-tiles 2s and 2s+1 of one N-tile) -> B operand of
// K-step s of the next layer, with ReLU.
__device__ __forceinline__ uint4 act_pack(const f32x4 &d0, const f32x4 &d1) {
    uint4 r;
    r.x = relu_bf16x2(pack_bf16(d0[0], d0[1]));
    r.y = relu_bf16x2(pack_bf16(d0[2], d0[3]));
    r.z = relu_bf16x2(pack_bf16(d1[0], d1[1]));
    r.w = relu_bf16x2(pack_bf16(d1[2], d1[3]));
    return r;
}

// Physical hidden unit feeding logical input k = 32 s + 8 g + e of a layer
// whose input is the previous layer's accumulator tiles.
__device__ __forceinline__ int unit_of(int s, int g, int e) { return 16 * (2 * s + (e >> 2)) + 4 * g + (e & 3); }

// ----------------------------------------------------------------------------
// Operand tiles in LDS: 64 lanes x 16 bytes each.
// ----------------------------------------------------------------------------
enum : int {
    T_W0W = 0,     // tracer direction part, 4 M-tiles
    T_W0F = 4,     // tracer feature part, 4 M-tiles
    T_W1 = 8,      // tracer hidden layer, 4 M-tiles x 2 K-steps (m*2+s)
    T_W2 = 16,     // tracer head, 2 K-steps
    B_W0 = 18,     // decoder first layer, 4 M-tiles
    B_W1 = 22,     // decoder hidden layer, 4 x 2
    B_W2A = 30,    // decoder head outputs 0..3, 2 K-steps
    B_W2B = 32,    // decoder head output 4, 2 K-steps
    N_TILES = 34
};

__device__ __forceinline__ float wbf(const void *W, int idx) {
    return __uint_as_float((uint32_t) static_cast<const uint16_t *>(W)[idx] << 16);
}

// Value of operand tile `t` for lane position (i = row, g = k-group, e).
__device__ float tile_value(const RenderK &a, int t, int i, int g, int e) {
    if (t < T_W0F) {  // direction part: k-group 0 holds (w_hi, w_lo) coefficients
        const int m = t - T_W0W;
        if (g != 0 || e >= 6) return 0.0f;
        return wbf(a.irt.W0, (16 * m + i) * kNI + kNF + (e % 3));
    }
    if (t < T_W1) {
        const int m = t - T_W0F;
        return wbf(a.irt.W0, (16 * m + i) * kNI + 8 * g + e);
    }
    if (t < T_W2) {
        const int m = (t - T_W1) >> 1, s = (t - T_W1) & 1;
        return wbf(a.irt.W1, (16 * m + i) * kH + unit_of(s, g, e));
    }
    if (t < B_W0) {
        const int s = t - T_W2, r = i & 3;
        return r < 2 ? wbf(a.irt.W2, r * kH + unit_of(s, g, e)) : 0.0f;
    }
    if (t < B_W1) {
        const int m = t - B_W0;
        return wbf(a.brdf.W0, (16 * m + i) * kNF + 8 * g + e);
    }
    if (t < B_W2A) {
        const int m = (t - B_W1) >> 1, s = (t - B_W1) & 1;
        return wbf(a.brdf.W1, (16 * m + i) * kH + unit_of(s, g, e));
    }
    if (t < B_W2B) {
        const int s = t - B_W2A;
        return wbf(a.brdf.W2, (i & 3) * kH + unit_of(s, g, e));
    }
    const int s = t - B_W2B;
    return (i & 3) == 0 ? wbf(a.brdf.W2, 4 * kH + unit_of(s, g, e)) : 0.0f;
}

// BF16 values are copied bit-exactly (they already are the shadow weights).
__device__ __forceinline__ uint32_t to_bits(float v) { return __float_as_uint(v) >> 16; }

__device__ void build_tiles(const RenderK &a, uint4 *tiles) {
    for (int q = threadIdx.x; q < N_TILES * 64; q += blockDim.x) {
        const int t = q >> 6, l = q & 63;
        const int i = l & 15, g = l >> 4;
        uint32_t w[4];
#pragma unroll
        for (int p = 0; p < 4; ++p)
            w[p] = to_bits(tile_value(a, t, i, g, 2 * p)) | (to_bits(tile_value(a, t, i, g, 2 * p + 1)) << 16);
        tiles[q] = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

// Bias of unit row 16 m + 4 g + r as an accumulator tile input.
__device__ __forceinline__ f32x4 bias_tile(const float *b, int m, int g) {
    const float4 v = *reinterpret_cast<const float4 *>(b + 16 * m + 4 * g);
    return f32x4{v.x, v.y, v.z, v.w};
}
__device__ __forceinline__ f32x4 head_bias(const float *b, int nout, int base) {
    f32x4 r;
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] = (base + k < nout) ? b[base + k] : 0.0f;
    return r;
}

// ----------------------------------------------------------------------------
// Per-wave LDS scratch
// ----------------------------------------------------------------------------
struct WaveLds {
    uint4 x[64][4];      // per-query input features (32 BF16) -- f(x) or f(x')
    uint4 om[64];        // per-query direction operand (w_hi, w_lo)
    float ax[4][kH];     // per-pixel tracer first-layer point part (shade mode)
    float mat[4][8];     // per-pixel decoder outputs (shade mode)
};

// Hidden and head layers of the tracer for one N-tile, starting from the
// first-layer accumulators d[4].  Returns the head tile (row r: output r).
struct TracerRegs {
    uint4 w0w[4];
    uint4 w1[8];
    uint4 w2[2];
    f32x4 b1[4];
    f32x4 b2;
};

__device__ __forceinline__ f32x4 tracer_rest(const TracerRegs &T, const f32x4 (&d)[4]) {
    const uint4 h0 = act_pack(d[0], d[1]), h1 = act_pack(d[2], d[3]);
    f32x4 e[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        e[m] = mfma(T.w1[2 * m], h0, T.b1[m]);
        e[m] = mfma(T.w1[2 * m + 1], h1, e[m]);
    }
    const uint4 k0 = act_pack(e[0], e[1]), k1 = act_pack(e[2], e[3]);
    f32x4 o = mfma(T.w2[0], k0, T.b2);
    return mfma(T.w2[1], k1, o);
}

// Decoder B on the features in x[16n..16n+15] for N-tile n; returns the two
// head tiles (outputs 0..3 in oa, output 4 in ob row 0).
__device__ __forceinline__ void decoder_tile(const uint4 *tiles, const float *b0, const float *b1, const float *b2,
                                             const uint4 &xb, int g, f32x4 &oa, f32x4 &ob) {
    f32x4 d[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) d[m] = mfma(tiles[(B_W0 + m) * 64 + (threadIdx.x & 63)], xb, bias_tile(b0, m, g));
    const uint4 h0 = act_pack(d[0], d[1]), h1 = act_pack(d[2], d[3]);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        d[m] = mfma(tiles[(B_W1 + 2 * m) * 64 + (threadIdx.x & 63)], h0, bias_tile(b1, m, g));
        d[m] = mfma(tiles[(B_W1 + 2 * m + 1) * 64 + (threadIdx.x & 63)], h1, d[m]);
    }
    const uint4 k0 = act_pack(d[0], d[1]), k1 = act_pack(d[2], d[3]);
    oa = mfma(tiles[B_W2A * 64 + (threadIdx.x & 63)], k0, head_bias(b2, 5, 0));
    oa = mfma(tiles[(B_W2A + 1) * 64 + (threadIdx.x & 63)], k1, oa);
    ob = mfma(tiles[B_W2B * 64 + (threadIdx.x & 63)], k0, head_bias(b2, 5, 4));
    ob = mfma(tiles[(B_W2B + 1) * 64 + (threadIdx.x & 63)], k1, ob);
}

__device__ __forceinline__ uint4 dir_operand(float3 w) {
    const __bf16 hx = (__bf16)w.x, hy = (__bf16)w.y, hz = (__bf16)w.z;
    const float lx = w.x - (float)hx, ly = w.y - (float)hy, lz = w.z - (float)hz;
    uint4 r;
    r.x = pack_bf16((float)hx, (float)hy);
    r.y = pack_bf16((float)hz, lx);
    r.z = pack_bf16(ly, lz);
    r.w = 0u;
    return r;
}

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Features of one query packed to BF16 into x[row] (4 x uint4).
__device__ __forceinline__ void store_feat(WaveLds &W, int row, const float (&f)[kNF]) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
        W.x[row][q] = make_uint4(pack_bf16(f[8 * q], f[8 * q + 1]), pack_bf16(f[8 * q + 2], f[8 * q + 3]),
                                 pack_bf16(f[8 * q + 4], f[8 * q + 5]), pack_bf16(f[8 * q + 6], f[8 * q + 7]));
}

// ----------------------------------------------------------------------------
// The kernel.  QUERY: one query per lane with its own point and direction;
// otherwise shade mode with G = min(N, 64) lanes per pixel.
// ----------------------------------------------------------------------------
constexpr int kMixThreads = 256;

template <bool INDIRECT, bool QUERY>
__global__ __launch_bounds__(kMixThreads) void k_render_mixed(const RenderK a, int64_t n_items) {
    __shared__ uint4 tiles[N_TILES * 64];
    __shared__ WaveLds wl[kMixThreads / 64];
    build_tiles(a, tiles);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, jcol = lane & 15;
    WaveLds &W = wl[threadIdx.x >> 6];

    TracerRegs T;
#pragma unroll
    for (int m = 0; m < 4; ++m) T.w0w[m] = tiles[(T_W0W + m) * 64 + lane];
#pragma unroll
    for (int k = 0; k < 8; ++k) T.w1[k] = tiles[(T_W1 + k) * 64 + lane];
    T.w2[0] = tiles[T_W2 * 64 + lane];
    T.w2[1] = tiles[(T_W2 + 1) * 64 + lane];
#pragma unroll
    for (int m = 0; m < 4; ++m) T.b1[m] = bias_tile(a.irt.b1, m, g);
    T.b2 = head_bias(a.irt.b2, 2, 0);

    const bool diffuse = (a.s.flags & 1u) != 0;
    const uint32_t gs = a.s.g_shift;
    const uint32_t G = 1u << gs;
    const int ppw = 64 >> gs;  // pixels per wave (shade mode)
    const int64_t waves_total = (int64_t)gridDim.x * (kMixThreads / 64);
    const int64_t wave_id = (int64_t)blockIdx.x * (kMixThreads / 64) + (threadIdx.x >> 6);

    for (int64_t item = wave_id; item < n_items; item += waves_total) {
        // ---------------- per-lane query identity ----------------
        int64_t p_raw;
        if (QUERY) p_raw = item * 64 + lane;
        else p_raw = item * ppw + (lane >> gs);
        const bool live = p_raw < a.n;
        const int64_t p = live ? p_raw : a.n - 1;
        const float3 x = make_float3(a.pos[3 * p], a.pos[3 * p + 1], a.pos[3 * p + 2]);

        // ---------------- primary point: features, decoder, point part ----------------
        f32x4 apt[4][4];  // point part of the tracer's first layer, per (M-tile, N-tile)
        float3 n_ = make_float3(0.f, 0.f, 1.f), v_ = n_, alb = n_;
        float rr = 0.5f, mm = 0.f;
        if (QUERY) {
            float f[kNF];
            encode<__half>(a.g, x.x, x.y, x.z, f);
            store_feat(W, lane, f);
            wave_sync_lds();
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const uint4 xb = W.x[16 * nt + jcol][g];
#pragma unroll
                for (int m = 0; m < 4; ++m)
                    apt[m][nt] = mfma(tiles[(T_W0F + m) * 64 + lane], xb, bias_tile(a.irt.b0, m, g));
            }
        } else {
            // lane l encodes level l % 16 of pixel slot l / 16 (one pass:
            // N >= 16 gives at most four pixels per wave)
            const int slot = lane >> 4, lvl = lane & 15;
            const int64_t ps_raw = item * ppw + slot;
            const int64_t ps = ps_raw < a.n ? ps_raw : a.n - 1;
            if (slot < ppw) {
                float u[3];
                bool in[3];
                pos_to_u(a.g, a.pos[3 * ps], a.pos[3 * ps + 1], a.pos[3 * ps + 2], u, in);
                uint32_t c[3];
                float w[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) cell_of(u[d], a.g.resf[lvl], a.g.nm1f[lvl], c[d], w[d]);
                uint32_t ix[8];
                corner_idx(a.g, lvl, c, ix);
                const void *lv = TabLoad<__half>::level(a.g.table, lvl, a.g.log2T);
                float f0 = 0.f, f1 = 0.f;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const float2 e = TabLoad<__half>::ld(lv, ix[k]);
                    const float wt = ((k & 1) ? w[0] : 1.f - w[0]) * (((k >> 1) & 1) ? w[1] : 1.f - w[1]) *
                                     (((k >> 2) & 1) ? w[2] : 1.f - w[2]);
                    f0 = fmaf(wt, e.x, f0);
                    f1 = fmaf(wt, e.y, f1);
                }
                reinterpret_cast<uint32_t *>(&W.x[slot][0])[lvl] = pack_bf16(f0, f1);
            }
            wave_sync_lds();
            // N-tile 0 holds the pixels in columns 0..ppw-1
            const uint4 xb = W.x[jcol][g];
            f32x4 oa, ob;
            decoder_tile(tiles, a.brdf.b0, a.brdf.b1, a.brdf.b2, xb, g, oa, ob);
            f32x4 ax[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) ax[m] = mfma(tiles[(T_W0F + m) * 64 + lane], xb, bias_tile(a.irt.b0, m, g));
            if (jcol < ppw) {
#pragma unroll
                for (int m = 0; m < 4; ++m)
#pragma unroll
                    for (int r = 0; r < 4; ++r) W.ax[jcol][16 * m + 4 * g + r] = ax[m][r];
                if (g == 0) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) W.mat[jcol][r] = oa[r];
                    W.mat[jcol][4] = ob[0];
                }
            }
            wave_sync_lds();
            const int myslot = lane >> gs;
            n_ = make_float3(a.nrm[3 * p], a.nrm[3 * p + 1], a.nrm[3 * p + 2]);
            v_ = make_float3(a.wo[3 * p], a.wo[3 * p + 1], a.wo[3 * p + 2]);
            alb = make_float3(sigmoidf_(W.mat[myslot][0]), sigmoidf_(W.mat[myslot][1]), sigmoidf_(W.mat[myslot][2]));
            rr = 0.09f + 0.91f * sigmoidf_(W.mat[myslot][3]);
            mm = sigmoidf_(W.mat[myslot][4]);
        }
        const Frame fr = make_frame(n_);
        const uint32_t N = QUERY ? 1u : a.s.n_dirs;
        const uint32_t i0 = QUERY ? 0u : (uint32_t)(lane & (G - 1));
        const uint32_t step = QUERY ? 1u : G;
        KSum sx{0.f, 0.f}, sy{0.f, 0.f}, sz{0.f, 0.f};

        for (uint32_t i = i0; i < N; i += step) {
            // ---------------- primary direction ----------------
            float3 w;
            if (QUERY) {
                w = make_float3(a.dir[3 * p], a.dir[3 * p + 1], a.dir[3 * p + 2]);
            } else {
                const uint4 words = philox4x32_10((uint32_t)p, 0u, i >> 2, 0u, a.s.key0, a.s.key1);
                w = sample_dir(pick4(words, i), i, a.s.nb_shift, a.s.inv_na, a.s.inv_nb, fr);
            }
            W.om[lane] = dir_operand(w);
            wave_sync_lds();
            float o0 = 0.f, o1 = 0.f;
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const uint4 ob_ = W.om[16 * nt + jcol];
                f32x4 d[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    f32x4 c0;
                    if (QUERY) {
                        c0 = apt[m][nt];
                    } else {
                        // columns of N-tile nt belong to pixel slot (16 nt) >> gs
                        const float4 v4 = *reinterpret_cast<const float4 *>(&W.ax[(16 * nt) >> gs][16 * m + 4 * g]);
                        c0 = f32x4{v4.x, v4.y, v4.z, v4.w};
                    }
                    d[m] = mfma(T.w0w[m], ob_, c0);
                }
                const f32x4 h = tracer_rest(T, d);
                if (g == nt) {
                    o0 = h[0];
                    o1 = h[1];
                }
            }
            const float V = sigmoidf_(o0);
            const float dd = fminf(softplusf_(o1), 1.0f);
            const float3 Le = env_lookup(a.env, w.x, w.y, w.z);
            float3 Lin;
            if (!INDIRECT) {
                Lin = make_float3(V * Le.x, V * Le.y, V * Le.z);
            } else {
                // ---------------- bounce point ----------------
                const float t = fmaf(a.t_span, dd, a.t_near);
                const float3 xb = make_float3(fmaf(t, w.x, x.x), fmaf(t, w.y, x.y), fmaf(t, w.z, x.z));
                float fb[kNF];
                encode<__half>(a.g, xb.x, xb.y, xb.z, fb);
                wave_sync_lds();  // previous readers of W.x are done
                store_feat(W, lane, fb);
                wave_sync_lds();
                f32x4 bpt[4][4];
                float ob0 = 0.f, ob1 = 0.f, ob2 = 0.f, ob3 = 0.f, ob4 = 0.f;
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    const uint4 xb_ = W.x[16 * nt + jcol][g];
#pragma unroll
                    for (int m = 0; m < 4; ++m)
                        bpt[m][nt] = mfma(tiles[(T_W0F + m) * 64 + lane], xb_, bias_tile(a.irt.b0, m, g));
                    f32x4 oa, obb;
                    decoder_tile(tiles, a.brdf.b0, a.brdf.b1, a.brdf.b2, xb_, g, oa, obb);
                    if (g == nt) {
                        ob0 = oa[0]; ob1 = oa[1]; ob2 = oa[2]; ob3 = oa[3]; ob4 = obb[0];
                    }
                }
                const float3 ab = make_float3(sigmoidf_(ob0), sigmoidf_(ob1), sigmoidf_(ob2));
                const float rb = 0.09f + 0.91f * sigmoidf_(ob3);
                const float mb = sigmoidf_(ob4);
                const float3 nb = make_float3(-w.x, -w.y, -w.z);
                const Frame frb = make_frame(nb);
                const uint32_t q = QUERY ? 0u : i;
                float Lx = 0.f, Ly = 0.f, Lz = 0.f;
                uint4 words2 = make_uint4(0, 0, 0, 0);
                for (uint32_t j = 0; j < a.s.n_dirs2; ++j) {
                    if ((j & 3u) == 0) words2 = philox4x32_10((uint32_t)p, q, j >> 2, 1u, a.s.key0, a.s.key1);
                    const float3 wj = sample_dir(pick4(words2, j), j, a.s.nb2_shift, a.s.inv_na2, a.s.inv_nb2, frb);
                    wave_sync_lds();
                    W.om[lane] = dir_operand(wj);
                    wave_sync_lds();
                    float vo = 0.f;
#pragma unroll
                    for (int nt = 0; nt < 4; ++nt) {
                        const uint4 ob_ = W.om[16 * nt + jcol];
                        f32x4 d[4];
#pragma unroll
                        for (int m = 0; m < 4; ++m) d[m] = mfma(T.w0w[m], ob_, bpt[m][nt]);
                        const f32x4 h = tracer_rest(T, d);
                        if (g == nt) vo = h[0];
                    }
                    const float vj = sigmoidf_(vo);
                    const float3 Ej = env_lookup(a.env, wj.x, wj.y, wj.z);
                    const float3 c = pi_brdf(nb, nb, wj, ab, rb, mb, a.f0, diffuse);
                    Lx = fmaf(c.x * vj, Ej.x, Lx);
                    Ly = fmaf(c.y * vj, Ej.y, Ly);
                    Lz = fmaf(c.z * vj, Ej.z, Lz);
                }
                const float inv = 1.0f / (float)a.s.n_dirs2;
                const float om = 1.0f - V;
                Lin = make_float3(fmaf(V, Le.x, om * Lx * inv), fmaf(V, Le.y, om * Ly * inv),
                                  fmaf(V, Le.z, om * Lz * inv));
            }
            if (QUERY) {
                if (live) {
                    a.rgb[3 * p] = Lin.x;
                    a.rgb[3 * p + 1] = Lin.y;
                    a.rgb[3 * p + 2] = Lin.z;
                    if (a.vis) {
                        a.vis[p] = V;
                        a.depth[p] = dd;
                    }
                }
            } else {
                const float3 c = pi_brdf(n_, v_, w, alb, rr, mm, a.f0, diffuse);
                sx.add(c.x * Lin.x);
                sy.add(c.y * Lin.y);
                sz.add(c.z * Lin.z);
                if (live && a.vis) {
                    a.vis[p * N + i] = V;
                    a.depth[p * N + i] = dd;
                }
            }
            wave_sync_lds();
        }
        if (!QUERY) {
            for (uint32_t off = G >> 1; off > 0; off >>= 1) {
                KSum *ks[3] = {&sx, &sy, &sz};
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float os = __shfl_xor(ks[c]->s, (int)off);
                    const float oc = __shfl_xor(ks[c]->c, (int)off);
                    float s, e;
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
        wave_sync_lds();
    }
}

static int g_num_cus = 0;

hipError_t launch_render_mixed(const RenderK &a, bool indirect, bool query, hipStream_t s) {
    if (!query && a.s.n_dirs < 16) return hipErrorNotSupported;
    if (g_num_cus == 0) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&g_num_cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
    }
    const int64_t ppw = query ? 64 : (64 >> a.s.g_shift);
    const int64_t items = (a.n + ppw - 1) / ppw;
    const int64_t want = (items + 3) / 4;
    const int64_t cap = (int64_t)g_num_cus * 2;
    const unsigned blocks = (unsigned)(want < cap ? want : cap);
    if (query) {
        if (indirect) hipLaunchKernelGGL((k_render_mixed<true, true>), dim3(blocks), dim3(kMixThreads), 0, s, a, items);
        else hipLaunchKernelGGL((k_render_mixed<false, true>), dim3(blocks), dim3(kMixThreads), 0, s, a, items);
    } else {
        if (indirect) hipLaunchKernelGGL((k_render_mixed<true, false>), dim3(blocks), dim3(kMixThreads), 0, s, a, items);
        else hipLaunchKernelGGL((k_render_mixed<false, false>), dim3(blocks), dim3(kMixThreads), 0, s, a, items);
    }
    return hipGetLastError();
}

}  // namespace hg
