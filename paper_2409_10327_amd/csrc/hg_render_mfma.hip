// hg_render_mfma.hip -- forward on the CDNA4 matrix cores, FP32 and mixed.
//
// Two precisions share one kernel body:
//   FP32:  FP32 tables, FP32 weights, v_mfma_f32_16x16x4f32 (K = 4 per step);
//   mixed: FP16 tables (FP32 interpolation), BF16 weights and activations,
//          v_mfma_f32_16x16x32_bf16 (K = 32 per step), FP32 accumulation.
// The light-direction sum is compensated FP32 in both.
//
// Work decomposition.  A wave owns 64 queries (one per lane) for the scalar
// work: direction sampling, hash-grid gathers, environment lookups, BRDF.
// Each MLP evaluation of the 64 queries is four 16-column N-tiles of
// matrix-core products with the units of a layer as rows (M) and the
// queries as columns (N):
//   layer output D (16x16 per M-tile): lane l holds rows 4*(l/16)+r,
//   column l%16 -- so the accumulators of one layer, after ReLU (and, mixed,
//   conversion to BF16), are already the B operand of the next layer once
//   the weight columns are permuted accordingly (no data movement between
//   layers);
//   head rows are replicated so that every lane group receives the outputs
//   of its column; lane l keeps N-tile l/16, which is its own query.
// Inputs that come from other lanes (features, directions) go through LDS.
// The tracer's first layer is split into a per-point part (W0f f + b0,
// computed once per point and used as the accumulator input) and a
// direction part (one matrix-core step; the mixed path splits the direction
// into BF16 high and low halves).
#include <hip/hip_bf16.h>

#include "hg_device.h"
#include "hg_launch.h"

namespace hg {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short s16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ f32x4 mfma_bf16(const uint4 &a, const uint4 &b, const f32x4 &c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b),
                                                    c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma_f32(float a, float b, const f32x4 &c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
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

// Two accumulator tiles (M-tiles 2s and 2s+1 of one N-tile) -> BF16 B
// operand of K-step s of the next layer, with ReLU.
__device__ __forceinline__ uint4 act_pack(const f32x4 &d0, const f32x4 &d1) {
    uint4 r;
    r.x = relu_bf16x2(pack_bf16(d0[0], d0[1]));
    r.y = relu_bf16x2(pack_bf16(d0[2], d0[3]));
    r.z = relu_bf16x2(pack_bf16(d1[0], d1[1]));
    r.w = relu_bf16x2(pack_bf16(d1[2], d1[3]));
    return r;
}

// Physical hidden unit feeding logical input k of a layer whose input is the
// previous layer's accumulator tiles.  BF16 (K-step s of 32, lane group g,
// element e): k = 32 s + 8 g + e.  FP32 (K-step s of 4, lane group g):
// k = 4 s + g.
__device__ __forceinline__ int unit_bf16(int s, int g, int e) { return 16 * (2 * s + (e >> 2)) + 4 * g + (e & 3); }
__device__ __forceinline__ int unit_f32(int s, int g) { return 16 * (s >> 2) + 4 * g + (s & 3); }

__device__ __forceinline__ float wbf(const void *W, int idx) {
    return __uint_as_float((uint32_t) static_cast<const uint16_t *>(W)[idx] << 16);
}
__device__ __forceinline__ float wf(const void *W, int idx) { return static_cast<const float *>(W)[idx]; }

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

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Weight pointers the tile builders read, copied out of the kernel argument
// once: selecting among them then selects values, never addresses inside
// the argument block (which would make the compiler copy the whole block to
// private memory).
struct WSrc {
    const void *iW0, *iW1, *iW2, *bW0, *bW1, *bW2;
    int nout;
};
__device__ __forceinline__ WSrc wsrc(const RenderK &a) {
    return WSrc{a.irt.W0, a.irt.W1, a.irt.W2, a.brdf.W0, a.brdf.W1, a.brdf.W2, a.brdf_out};
}

// ============================================================================
// Mixed path: BF16 operands, K = 32 per matrix-core step.
// ============================================================================
struct Bf16Path {
    typedef __half Table;
    enum : int {
        T_W0W = 0, T_W0F = 4, T_W1 = 8, T_W2 = 16,       // tracer
        B_W0 = 18, B_W1 = 22, B_W2A = 30, B_W2B = 32,    // decoder
        N_TILES = 34
    };
    typedef uint4 Tile;  // 8 BF16 per lane

    struct Wave {
        uint4 x[64][4];   // per-query input features (32 BF16)
        uint4 om[2][64];  // per-query direction operand (w_hi, w_lo), two buffers
        float ax[4][kH];  // per-pixel tracer point part (shade mode)
        float mat[4][8];  // per-pixel decoder outputs (shade mode)
        uint16_t qi[128]; // queued shadow rays (hard visibility): direction index
        float qd[128];    // and normalised depth
    };

    static __device__ __forceinline__ float tile_value(const WSrc &a, int t, int i, int g, int e) {
        if (t < T_W0F) {
            const int m = t - T_W0W;
            if (g != 0 || e >= 6) return 0.0f;
            return wbf(a.iW0, (16 * m + i) * kNI + kNF + (e % 3));
        }
        if (t < T_W1) return wbf(a.iW0, (16 * (t - T_W0F) + i) * kNI + 8 * g + e);
        if (t < T_W2) {
            const int m = (t - T_W1) >> 1, s = (t - T_W1) & 1;
            return wbf(a.iW1, (16 * m + i) * kH + unit_bf16(s, g, e));
        }
        if (t < B_W0) {
            const int s = t - T_W2, r = i & 3;
            return r < 2 ? wbf(a.iW2, r * kH + unit_bf16(s, g, e)) : 0.0f;
        }
        if (t < B_W1) return wbf(a.bW0, (16 * (t - B_W0) + i) * kNF + 8 * g + e);
        if (t < B_W2A) {
            const int m = (t - B_W1) >> 1, s = (t - B_W1) & 1;
            return wbf(a.bW1, (16 * m + i) * kH + unit_bf16(s, g, e));
        }
        if (t < B_W2B) return wbf(a.bW2, (i & 3) * kH + unit_bf16(t - B_W2A, g, e));
        return 4 + (i & 3) < a.nout ? wbf(a.bW2, (4 + (i & 3)) * kH + unit_bf16(t - B_W2B, g, e)) : 0.0f;
    }

    static __device__ __forceinline__ void build_tiles(const RenderK &ka, Tile *tiles) {
        const WSrc a = wsrc(ka);
        for (int q = threadIdx.x; q < N_TILES * 64; q += blockDim.x) {
            const int t = q >> 6, l = q & 63, i = l & 15, g = l >> 4;
            uint32_t w[4];
#pragma unroll
            for (int p = 0; p < 4; ++p)
                w[p] = (__float_as_uint(tile_value(a, t, i, g, 2 * p)) >> 16) |
                       (__float_as_uint(tile_value(a, t, i, g, 2 * p + 1)) & 0xffff0000u);
            tiles[q] = make_uint4(w[0], w[1], w[2], w[3]);
        }
    }

    // hot tracer operands held in registers
    struct Tracer {
        uint4 w0w[4], w1[8], w2[2];
        f32x4 b1[4], b2;
        __device__ void load(const Tile *tiles, const RenderK &a, int lane, int g) {
#pragma unroll
            for (int m = 0; m < 4; ++m) w0w[m] = tiles[(T_W0W + m) * 64 + lane];
#pragma unroll
            for (int k = 0; k < 8; ++k) w1[k] = tiles[(T_W1 + k) * 64 + lane];
            w2[0] = tiles[T_W2 * 64 + lane];
            w2[1] = tiles[(T_W2 + 1) * 64 + lane];
#pragma unroll
            for (int m = 0; m < 4; ++m) b1[m] = bias_tile(a.irt.b1, m, g);
            b2 = head_bias(a.irt.b2, 2, 0);
        }
    };

    static __device__ __forceinline__ void store_feat(Wave &W, int row, const float (&f)[kNF]) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            W.x[row][q] = make_uint4(pack_bf16(f[8 * q], f[8 * q + 1]), pack_bf16(f[8 * q + 2], f[8 * q + 3]),
                                     pack_bf16(f[8 * q + 4], f[8 * q + 5]), pack_bf16(f[8 * q + 6], f[8 * q + 7]));
    }
    static __device__ __forceinline__ void store_level(Wave &W, int row, int lvl, float f0, float f1) {
        reinterpret_cast<uint32_t *>(&W.x[row][0])[lvl] = pack_bf16(f0, f1);
    }
    static __device__ __forceinline__ void store_dir(Wave &W, int buf, int lane, float3 w) {
        const __bf16 hx = (__bf16)w.x, hy = (__bf16)w.y, hz = (__bf16)w.z;
        const float lx = w.x - (float)hx, ly = w.y - (float)hy, lz = w.z - (float)hz;
        W.om[buf][lane] = make_uint4(pack_bf16((float)hx, (float)hy), pack_bf16((float)hz, lx), pack_bf16(ly, lz), 0u);
    }

    // tracer point part W0f x + b0 of N-tile nt
    static __device__ __forceinline__ void point_part(const Tile *tiles, const RenderK &a, const Wave &W, int nt,
                                                      int lane, int g, f32x4 (&d)[4]) {
        const uint4 xb = W.x[16 * nt + (lane & 15)][g];
#pragma unroll
        for (int m = 0; m < 4; ++m) d[m] = mfma_bf16(tiles[(T_W0F + m) * 64 + lane], xb, bias_tile(a.irt.b0, m, g));
    }

    // decoder on the features of N-tile nt: oa rows 0..3 = outputs 0..3,
    // ob row 0 = output 4
    static __device__ __forceinline__ void decoder(const Tile *tiles, const RenderK &a, const Wave &W, int nt,
                                                   int lane, int g, f32x4 &oa, f32x4 &ob) {
        const uint4 xb = W.x[16 * nt + (lane & 15)][g];
        f32x4 d[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) d[m] = mfma_bf16(tiles[(B_W0 + m) * 64 + lane], xb, bias_tile(a.brdf.b0, m, g));
        const uint4 h0 = act_pack(d[0], d[1]), h1 = act_pack(d[2], d[3]);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            d[m] = mfma_bf16(tiles[(B_W1 + 2 * m) * 64 + lane], h0, bias_tile(a.brdf.b1, m, g));
            d[m] = mfma_bf16(tiles[(B_W1 + 2 * m + 1) * 64 + lane], h1, d[m]);
        }
        const uint4 k0 = act_pack(d[0], d[1]), k1 = act_pack(d[2], d[3]);
        oa = mfma_bf16(tiles[B_W2A * 64 + lane], k0, head_bias(a.brdf.b2, 5, 0));
        oa = mfma_bf16(tiles[(B_W2A + 1) * 64 + lane], k1, oa);
        ob = mfma_bf16(tiles[B_W2B * 64 + lane], k0, head_bias(a.brdf.b2, a.brdf_out, 4));
        ob = mfma_bf16(tiles[(B_W2B + 1) * 64 + lane], k1, ob);
    }

    // tracer for N-tile nt from the point part c: returns the head tile
    static __device__ __forceinline__ f32x4 tracer(const Tracer &T, const Tile *, const Wave &W, int buf, int nt,
                                                   int lane, const f32x4 (&c)[4]) {
        const uint4 ob_ = W.om[buf][16 * nt + (lane & 15)];
        f32x4 d[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) d[m] = mfma_bf16(T.w0w[m], ob_, c[m]);
        const uint4 h0 = act_pack(d[0], d[1]), h1 = act_pack(d[2], d[3]);
        f32x4 e[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            e[m] = mfma_bf16(T.w1[2 * m], h0, T.b1[m]);
            e[m] = mfma_bf16(T.w1[2 * m + 1], h1, e[m]);
        }
        const uint4 k0 = act_pack(e[0], e[1]), k1 = act_pack(e[2], e[3]);
        f32x4 o = mfma_bf16(T.w2[0], k0, T.b2);
        return mfma_bf16(T.w2[1], k1, o);
    }
};

// ============================================================================
// FP32 path: FP32 operands, K = 4 per matrix-core step.
// ============================================================================
struct F32Path {
    typedef float Table;
    // tracer and decoder operand tiles in LDS (62.5 KB)
    enum : int {
        T_W0W = 0,       // tracer: 4 M-tiles, one K-step (w_x, w_y, w_z, 0)
        T_W0F = 4,       // 4 M-tiles x 8 K-steps (m*8 + s)
        T_W1 = 36,       // 4 M-tiles x 16 K-steps (m*16 + s)
        T_W2 = 100,      // 16 K-steps
        D_W0 = 116,      // decoder: 4 M-tiles x 8 K-steps (m*8 + s)
        D_W1 = 148,      // 4 M-tiles x 16 K-steps (m*16 + s)
        D_W2A = 212,     // outputs 0..3, 16 K-steps
        D_W2B = 228,     // outputs 4..7, 16 K-steps
        N_TILES = 244
    };
    typedef float Tile;
    static constexpr int kXS = 36;  // row stride of the feature rows (16-byte aligned, 2-way banks)

    struct Wave {
        float x[64][kXS];
        float4 om[2][64];
        float ax[4][kH];
        float mat[4][8];
        uint16_t qi[128];
        float qd[128];
    };

    static __device__ __forceinline__ float tile_value(const WSrc &a, int t, int i, int g) {
        if (t < T_W0F) {
            const int m = t - T_W0W;
            return g < 3 ? wf(a.iW0, (16 * m + i) * kNI + kNF + g) : 0.0f;
        }
        if (t < T_W1) {
            const int m = (t - T_W0F) >> 3, s = (t - T_W0F) & 7;
            return wf(a.iW0, (16 * m + i) * kNI + 4 * s + g);
        }
        if (t < T_W2) {
            const int m = (t - T_W1) >> 4, s = (t - T_W1) & 15;
            return wf(a.iW1, (16 * m + i) * kH + unit_f32(s, g));
        }
        if (t < D_W0) {
            const int s = t - T_W2, r = i & 3;
            return r < 2 ? wf(a.iW2, r * kH + unit_f32(s, g)) : 0.0f;
        }
        if (t < D_W1) {
            const int m = (t - D_W0) >> 3, s = (t - D_W0) & 7;
            return wf(a.bW0, (16 * m + i) * kNF + 4 * s + g);
        }
        if (t < D_W2A) {
            const int m = (t - D_W1) >> 4, s = (t - D_W1) & 15;
            return wf(a.bW1, (16 * m + i) * kH + unit_f32(s, g));
        }
        const int r = i & 3;
        if (t < D_W2B) return wf(a.bW2, r * kH + unit_f32(t - D_W2A, g));
        return 4 + r < a.nout ? wf(a.bW2, (4 + r) * kH + unit_f32(t - D_W2B, g)) : 0.0f;
    }

    static __device__ __forceinline__ void build_tiles(const RenderK &ka, Tile *tiles) {
        const WSrc a = wsrc(ka);
        for (int q = threadIdx.x; q < N_TILES * 64; q += blockDim.x) {
            const int t = q >> 6, l = q & 63;
            tiles[q] = tile_value(a, t, l & 15, l >> 4);
        }
    }

    struct Tracer {
        f32x4 b1[4], b2;
        __device__ void load(const Tile *, const RenderK &a, int, int g) {
#pragma unroll
            for (int m = 0; m < 4; ++m) b1[m] = bias_tile(a.irt.b1, m, g);
            b2 = head_bias(a.irt.b2, 2, 0);
        }
    };

    static __device__ __forceinline__ void store_feat(Wave &W, int row, const float (&f)[kNF]) {
#pragma unroll
        for (int q = 0; q < 8; ++q)
            *reinterpret_cast<float4 *>(&W.x[row][4 * q]) = make_float4(f[4 * q], f[4 * q + 1], f[4 * q + 2], f[4 * q + 3]);
    }
    static __device__ __forceinline__ void store_level(Wave &W, int row, int lvl, float f0, float f1) {
        *reinterpret_cast<float2 *>(&W.x[row][2 * lvl]) = make_float2(f0, f1);
    }
    static __device__ __forceinline__ void store_dir(Wave &W, int buf, int lane, float3 w) {
        W.om[buf][lane] = make_float4(w.x, w.y, w.z, 0.0f);
    }

    static __device__ __forceinline__ void point_part(const Tile *tiles, const RenderK &a, const Wave &W, int nt,
                                                      int lane, int g, f32x4 (&d)[4]) {
        const float *xr = W.x[16 * nt + (lane & 15)];
#pragma unroll
        for (int m = 0; m < 4; ++m) d[m] = bias_tile(a.irt.b0, m, g);
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const float b = xr[4 * s + g];
#pragma unroll
            for (int m = 0; m < 4; ++m) d[m] = mfma_f32(tiles[(T_W0F + 8 * m + s) * 64 + lane], b, d[m]);
        }
    }

    static __device__ __forceinline__ void decoder(const Tile *tiles, const RenderK &a, const Wave &W, int nt,
                                                   int lane, int g, f32x4 &oa, f32x4 &ob) {
        const float *xr = W.x[16 * nt + (lane & 15)];
        f32x4 d[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) d[m] = bias_tile(a.brdf.b0, m, g);
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const float b = xr[4 * s + g];
#pragma unroll
            for (int m = 0; m < 4; ++m) d[m] = mfma_f32(tiles[(D_W0 + 8 * m + s) * 64 + lane], b, d[m]);
        }
        f32x4 e[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) e[m] = bias_tile(a.brdf.b1, m, g);
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const float b = fmaxf(d[s >> 2][s & 3], 0.0f);
#pragma unroll
            for (int m = 0; m < 4; ++m) e[m] = mfma_f32(tiles[(D_W1 + 16 * m + s) * 64 + lane], b, e[m]);
        }
        oa = head_bias(a.brdf.b2, 5, 0);
        ob = head_bias(a.brdf.b2, a.brdf_out, 4);
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const float b = fmaxf(e[s >> 2][s & 3], 0.0f);
            oa = mfma_f32(tiles[(D_W2A + s) * 64 + lane], b, oa);
            ob = mfma_f32(tiles[(D_W2B + s) * 64 + lane], b, ob);
        }
    }

    static __device__ __forceinline__ f32x4 tracer(const Tracer &T, const Tile *tiles, const Wave &W, int buf, int nt,
                                                   int lane, const f32x4 (&c)[4]) {
        const int g = lane >> 4;
        const float b0 = reinterpret_cast<const float *>(&W.om[buf][16 * nt + (lane & 15)])[g];
        f32x4 d[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) d[m] = mfma_f32(tiles[(T_W0W + m) * 64 + lane], b0, c[m]);
        f32x4 e[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) e[m] = T.b1[m];
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const float b = fmaxf(d[s >> 2][s & 3], 0.0f);
#pragma unroll
            for (int m = 0; m < 4; ++m) e[m] = mfma_f32(tiles[(T_W1 + 16 * m + s) * 64 + lane], b, e[m]);
        }
        f32x4 o = T.b2;
#pragma unroll
        for (int s = 0; s < 16; ++s) o = mfma_f32(tiles[(T_W2 + s) * 64 + lane], fmaxf(e[s >> 2][s & 3], 0.0f), o);
        return o;
    }
};

// BRDF at the bounce point for a secondary direction: the full microfacet
// model about the decoder's normal (normal head), else the facing form.
struct SecondaryBrdf {
    float3 n, v, a;
    float r, m, f0;
    bool diffuse;
    FacingBrdf facing;
    template <bool NHEAD>
    __device__ __forceinline__ float3 eval(float3 l) const {
        return NHEAD ? pi_brdf(n, v, l, a, r, m, f0, diffuse) : facing.eval(dot3(n, l));
    }
};

// (1/N') sum_j f_r(w_j) V(x', w_j) L_e(w_j) over the secondary directions of
// every lane's bounce point, from the tracer's point part bpt at x'.
// Software pipeline: while the matrix cores trace direction j (operand
// buffer j & 1), the vector ALU samples direction j + 1, issues its texel
// loads and evaluates its BRDF factor, all in one basic block (the sampler,
// lookup and BRDF use selects, not branches); the new operand goes to the
// other buffer after the tracer's reads.  The last iteration samples
// direction j again and drops it.
template <class PP, bool NHEAD>
__device__ __forceinline__ float3 secondary_lo(const RenderK &a, const typename PP::Tile *tiles,
                                               typename PP::Wave &W, const typename PP::Tracer &T,
                                               const f32x4 (&bpt)[4][4], int lane, int g, const Frame &frb,
                                               const SecondaryBrdf &sb, uint32_t pid, uint32_t q, bool hard) {
    const uint32_t n2 = a.s.n_dirs2;
    uint4 words2 = philox4x32_10(pid, q, 0u, 1u, a.s.key0, a.s.key1);
    const float3 w0 = sample_dir(pick4(words2, 0u), 0u, a.s.nb2_shift, a.s.inv_na2, a.s.inv_nb2, frb);
    float3 Ej = env_lookup(a.env, w0.x, w0.y, w0.z);
    float3 cj = sb.eval<NHEAD>(w0);
    wave_sync_lds();
    PP::store_dir(W, 0, lane, w0);
    wave_sync_lds();
    float Lx = 0.f, Ly = 0.f, Lz = 0.f;
    for (uint32_t j = 0; j < n2; ++j) {
        const uint32_t jn = j + 1 < n2 ? j + 1 : j;
        if ((jn & 3u) == 0) words2 = philox4x32_10(pid, q, jn >> 2, 1u, a.s.key0, a.s.key1);
        const float3 wn = sample_dir(pick4(words2, jn), jn, a.s.nb2_shift, a.s.inv_na2, a.s.inv_nb2, frb);
        const float3 En = env_lookup(a.env, wn.x, wn.y, wn.z);
        const float3 cn = sb.eval<NHEAD>(wn);
        float vo = 0.f;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const f32x4 c[4] = {bpt[0][nt], bpt[1][nt], bpt[2][nt], bpt[3][nt]};
            const f32x4 h = PP::tracer(T, tiles, W, (int)(j & 1u), nt, lane, c);
            if (g == nt) vo = h[0];
        }
        PP::store_dir(W, (int)((j + 1) & 1u), lane, wn);
        // hard visibility: only visible secondary rays contribute
        const float vj = hard ? (vo > 0.0f ? 1.0f : 0.0f) : sigmoidf_(vo);
        Lx = fmaf(cj.x * vj, Ej.x, Lx);
        Ly = fmaf(cj.y * vj, Ej.y, Ly);
        Lz = fmaf(cj.z * vj, Ej.z, Lz);
        Ej = En;
        cj = cn;
        wave_sync_lds();
    }
    const float inv = 1.0f / (float)n2;
    return make_float3(Lx * inv, Ly * inv, Lz * inv);
}

// ============================================================================
// Outgoing radiance L'_o at the bounce point x' = x + t w of each lane's query
// (all 64 lanes take part in the matrix-core products).
// ============================================================================
template <class PP, class TT>
__device__ __forceinline__ float3 bounce_lo(const RenderK &a, const typename PP::Tile *tiles, typename PP::Wave &W,
                                            const typename PP::Tracer &T, int lane, int g, float3 x, float3 w,
                                            float dd, uint32_t pid, uint32_t q, bool hard, bool diffuse) {
    const float t = fmaf(a.t_span, dd, a.t_near);
    const float3 xb = make_float3(fmaf(t, w.x, x.x), fmaf(t, w.y, x.y), fmaf(t, w.z, x.z));
    float fb[kNF];
    encode<TT>(a.g, xb.x, xb.y, xb.z, fb);
    wave_sync_lds();
    PP::store_feat(W, lane, fb);
    wave_sync_lds();
    f32x4 bpt[4][4];
    float ob0 = 0.f, ob1 = 0.f, ob2 = 0.f, ob3 = 0.f, ob4 = 0.f, on0 = 0.f, on1 = 0.f, on2 = 0.f;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        f32x4 d[4];
        PP::point_part(tiles, a, W, nt, lane, g, d);
#pragma unroll
        for (int m = 0; m < 4; ++m) bpt[m][nt] = d[m];
        f32x4 oa, obb;
        PP::decoder(tiles, a, W, nt, lane, g, oa, obb);
        if (g == nt) {
            ob0 = oa[0]; ob1 = oa[1]; ob2 = oa[2]; ob3 = oa[3]; ob4 = obb[0];
            on0 = obb[1]; on1 = obb[2]; on2 = obb[3];
        }
    }
    const float3 ab = make_float3(sigmoidf_(ob0), sigmoidf_(ob1), sigmoidf_(ob2));
    const float rb = 0.09f + 0.91f * sigmoidf_(ob3);
    const float mb = sigmoidf_(ob4);
    // secondary view -w; normal from the decoder's normal head if it has one,
    // else the facing normal -w
    const float3 vb = make_float3(-w.x, -w.y, -w.z);
    const bool nhead = a.brdf_out == 8;
    const float3 nb = nhead ? head_normal(on0, on1, on2, vb) : vb;
    const Frame frb = make_frame(nb);
    FacingBrdf fb_;
    fb_.set(ab, rb, mb, a.f0, diffuse);
    const SecondaryBrdf sb{nb, vb, ab, rb, mb, a.f0, diffuse, fb_};
    return nhead ? secondary_lo<PP, true>(a, tiles, W, T, bpt, lane, g, frb, sb, pid, q, hard)
                 : secondary_lo<PP, false>(a, tiles, W, T, bpt, lane, g, frb, sb, pid, q, hard);
}

// ============================================================================
// The kernel.  QUERY: one query per lane with its own point and direction;
// otherwise shade mode with G = min(N, 64) lanes per pixel (N >= 16, so at
// most four pixels per wave).
// ============================================================================
constexpr int kMixThreads = 256;

template <class PP, bool INDIRECT, bool QUERY, bool MIS>
__global__ __launch_bounds__(kMixThreads) void k_render_mma(const RenderK a, int64_t n_items) {
    typedef typename PP::Table TT;
    __shared__ typename PP::Tile tiles[PP::N_TILES * 64];
    __shared__ typename PP::Wave wl[kMixThreads / 64];
    PP::build_tiles(a, tiles);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, jcol = lane & 15;
    typename PP::Wave &W = wl[threadIdx.x >> 6];
    typename PP::Tracer T;
    T.load(tiles, a, lane, g);

    const bool diffuse = (a.s.flags & 1u) != 0;
    const bool hard = (a.s.flags & 2u) != 0;
    const uint32_t gs = a.s.g_shift;
    const uint32_t G = 1u << gs;
    const int ppw = 64 >> gs;
    const int64_t waves_total = (int64_t)gridDim.x * (kMixThreads / 64);
    const int64_t wave_id = (int64_t)blockIdx.x * (kMixThreads / 64) + (threadIdx.x >> 6);

    for (int64_t item = wave_id; item < n_items; item += waves_total) {
        int64_t p_raw;
        if (QUERY) p_raw = item * 64 + lane;
        else p_raw = item * ppw + (lane >> gs);
        const bool live = p_raw < a.n;
        const int64_t p = live ? p_raw : a.n - 1;
        const float3 x = make_float3(a.pos[3 * p], a.pos[3 * p + 1], a.pos[3 * p + 2]);

        // ---------------- primary point ----------------
        f32x4 apt[4][4];  // query mode: tracer point part at x per (M-tile, N-tile)
        float3 n_ = make_float3(0.f, 0.f, 1.f), v_ = n_, alb = n_;
        float rr = 0.5f, mm = 0.f;
        if (QUERY) {
            float f[kNF];
            encode<TT>(a.g, x.x, x.y, x.z, f);
            PP::store_feat(W, lane, f);
            wave_sync_lds();
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                f32x4 d[4];
                PP::point_part(tiles, a, W, nt, lane, g, d);
#pragma unroll
                for (int m = 0; m < 4; ++m) apt[m][nt] = d[m];
            }
        } else {
            // lane l encodes level l % 16 of pixel slot l / 16
            const int slot = lane >> 4, lvl = lane & 15;
            const int64_t ps_raw = item * ppw + slot;
            const int64_t ps = ps_raw < a.n ? ps_raw : a.n - 1;
            if (slot < ppw && lvl < (int)a.g.L) {
                float u[3];
                bool in[3];
                pos_to_u(a.g, a.pos[3 * ps], a.pos[3 * ps + 1], a.pos[3 * ps + 2], u, in);
                uint32_t c[3];
                float w[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) cell_of(u[d], a.g.resf[lvl], a.g.nm1f[lvl], c[d], w[d]);
                uint32_t ix[8];
                corner_idx(a.g, lvl, c, ix);
                const void *lv = TabLoad<TT>::level(a.g.table, lvl, a.g.log2T);
                float f0 = 0.f, f1 = 0.f;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const float2 e = TabLoad<TT>::ld(lv, ix[k]);
                    const float wt = ((k & 1) ? w[0] : 1.f - w[0]) * (((k >> 1) & 1) ? w[1] : 1.f - w[1]) *
                                     (((k >> 2) & 1) ? w[2] : 1.f - w[2]);
                    f0 = fmaf(wt, e.x, f0);
                    f1 = fmaf(wt, e.y, f1);
                }
                PP::store_level(W, slot, lvl, f0, f1);
            } else if (slot < ppw) {
                PP::store_level(W, slot, lvl, 0.0f, 0.0f);  // slot of a level the grid does not have
            }
            wave_sync_lds();
            f32x4 oa, ob, ax[4];
            PP::decoder(tiles, a, W, 0, lane, g, oa, ob);
            PP::point_part(tiles, a, W, 0, lane, g, ax);
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
        const float3 vl = MIS ? ggx_view(fr, v_) : v_;
        const uint32_t N = QUERY ? 1u : a.s.n_dirs;
        const uint32_t i0 = QUERY ? 0u : (uint32_t)(lane & (G - 1));
        const uint32_t step = QUERY ? 1u : G;
        KSum sx{0.f, 0.f}, sy{0.f, 0.f}, sz{0.f, 0.f};
        // Under hard visibility with one pixel per wave, only shadow rays
        // need the bounce: they are queued in LDS and bounced 64 at a time.
        const bool compact = INDIRECT && !QUERY && hard && ppw == 1;
        uint32_t i_next = i0;
        bool more = i_next < N;
        int cnt = 0;
        while (true) {
            // ---------------- primary directions of the next chunk ----------------
            float3 w_own = make_float3(0.f, 0.f, 1.f), Le_own = w_own;
            float V_own = 0.f, d_own = 0.f, wf_own = 1.0f;
            const uint32_t i_own = i_next;
            const bool had = more;
            if (more) {
                if (QUERY) {
                    w_own = make_float3(a.dir[3 * p], a.dir[3 * p + 1], a.dir[3 * p + 2]);
                } else if (MIS) {
                    w_own = mis_direction(a, fr, vl, rr, (uint32_t)p, i_own, wf_own);
                } else {
                    const uint4 words = philox4x32_10((uint32_t)p, 0u, i_own >> 2, 0u, a.s.key0, a.s.key1);
                    w_own = sample_dir(pick4(words, i_own), i_own, a.s.nb_shift, a.s.inv_na, a.s.inv_nb, fr);
                }
                Le_own = env_lookup(a.env, w_own.x, w_own.y, w_own.z);  // overlaps the tracer
                wave_sync_lds();
                PP::store_dir(W, 0, lane, w_own);
                wave_sync_lds();
                float o0 = 0.f, o1 = 0.f;
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    f32x4 c[4];
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        if (QUERY) {
                            c[m] = apt[m][nt];
                        } else {
                            // columns of N-tile nt belong to pixel slot (16 nt) >> gs
                            const float4 v4 =
                                *reinterpret_cast<const float4 *>(&W.ax[(16 * nt) >> gs][16 * m + 4 * g]);
                            c[m] = f32x4{v4.x, v4.y, v4.z, v4.w};
                        }
                    }
                    const f32x4 h = PP::tracer(T, tiles, W, 0, nt, lane, c);
                    if (g == nt) {
                        o0 = h[0];
                        o1 = h[1];
                    }
                }
                V_own = hard ? (o0 > 0.0f ? 1.0f : 0.0f) : sigmoidf_(o0);
                d_own = fminf(softplusf_(o1), 1.0f);
                if (!QUERY && live && a.vis) {
                    a.vis[p * N + i_own] = V_own;
                    a.depth[p * N + i_own] = d_own;
                }
                if (compact) {
                    // visible rays are finished here; shadow rays are queued
                    const bool vis1 = V_own == 1.0f;
                    if (vis1) {
                        float3 c = pi_brdf(n_, v_, w_own, alb, rr, mm, a.f0, diffuse);
                        if (MIS) c = make_float3(c.x * wf_own, c.y * wf_own, c.z * wf_own);
                        sx.add(c.x * Le_own.x);
                        sy.add(c.y * Le_own.y);
                        sz.add(c.z * Le_own.z);
                    }
                    const uint64_t qm = __ballot(!vis1);
                    const int pos = cnt + __popcll(qm & ((1ull << lane) - 1ull));
                    if (!vis1) {
                        W.qi[pos] = (uint16_t)i_own;
                        W.qd[pos] = d_own;
                    }
                    cnt += __popcll(qm);
                }
                i_next += step;
                more = i_next < N;
            }
            const bool flush = compact ? (cnt >= 64 || (!more && cnt > 0)) : had;
            if (!flush) {
                if (!more) break;
                continue;
            }
            // ---------------- bounce for 64 lanes ----------------
            bool active = true;
            uint32_t ie = i_own;
            float de = d_own, Ve = V_own, wfe = wf_own;
            float3 we = w_own;
            if (compact) {
                wave_sync_lds();
                active = lane < cnt;
                const int slot = active ? lane : 0;
                ie = W.qi[slot];
                de = W.qd[slot];
                Ve = 0.0f;
                if (MIS) {
                    we = mis_direction(a, fr, vl, rr, (uint32_t)p, ie, wfe);
                } else {
                    const uint4 words = philox4x32_10((uint32_t)p, 0u, ie >> 2, 0u, a.s.key0, a.s.key1);
                    we = sample_dir(pick4(words, ie), ie, a.s.nb_shift, a.s.inv_na, a.s.inv_nb, fr);
                }
            }
            float3 Lin;
            if (!INDIRECT) {
                Lin = make_float3(Ve * Le_own.x, Ve * Le_own.y, Ve * Le_own.z);
            } else {
                const float3 Lo = bounce_lo<PP, TT>(a, tiles, W, T, lane, g, x, we, de, (uint32_t)p,
                                                    QUERY ? 0u : ie, hard, diffuse);
                const float om = 1.0f - Ve;
                Lin = make_float3(fmaf(Ve, Le_own.x, om * Lo.x), fmaf(Ve, Le_own.y, om * Lo.y),
                                  fmaf(Ve, Le_own.z, om * Lo.z));
            }
            if (QUERY) {
                if (live) {
                    a.rgb[3 * p] = Lin.x;
                    a.rgb[3 * p + 1] = Lin.y;
                    a.rgb[3 * p + 2] = Lin.z;
                    if (a.vis) {
                        a.vis[p] = V_own;
                        a.depth[p] = d_own;
                    }
                }
            } else if (active) {
                float3 c = pi_brdf(n_, v_, we, alb, rr, mm, a.f0, diffuse);
                if (MIS) c = make_float3(c.x * wfe, c.y * wfe, c.z * wfe);
                sx.add(c.x * Lin.x);
                sy.add(c.y * Lin.y);
                sz.add(c.z * Lin.z);
            }
            if (compact) {
                // drop the 64 entries just bounced; move the rest to the front
                wave_sync_lds();
                const int rest = cnt - 64;
                uint16_t ti = 0;
                float td = 0.f;
                if (lane < rest) {
                    ti = W.qi[64 + lane];
                    td = W.qd[64 + lane];
                }
                wave_sync_lds();
                if (lane < rest) {
                    W.qi[lane] = ti;
                    W.qd[lane] = td;
                }
                cnt = rest > 0 ? rest : 0;
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

template <class PP>
static hipError_t launch_mma(const RenderK &a, bool indirect, bool query, hipStream_t s) {
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
    const dim3 grid(blocks), block(kMixThreads);
    const bool mis = (a.s.flags & 4u) != 0;
    if (query) {
        if (indirect) hipLaunchKernelGGL((k_render_mma<PP, true, true, false>), grid, block, 0, s, a, items);
        else hipLaunchKernelGGL((k_render_mma<PP, false, true, false>), grid, block, 0, s, a, items);
    } else if (mis) {
        if (indirect) hipLaunchKernelGGL((k_render_mma<PP, true, false, true>), grid, block, 0, s, a, items);
        else hipLaunchKernelGGL((k_render_mma<PP, false, false, true>), grid, block, 0, s, a, items);
    } else {
        if (indirect) hipLaunchKernelGGL((k_render_mma<PP, true, false, false>), grid, block, 0, s, a, items);
        else hipLaunchKernelGGL((k_render_mma<PP, false, false, false>), grid, block, 0, s, a, items);
    }
    return hipGetLastError();
}

hipError_t launch_render_mixed(const RenderK &a, bool indirect, bool query, hipStream_t s) {
    return launch_mma<Bf16Path>(a, indirect, query, s);
}

hipError_t launch_render_f32_mma(const RenderK &a, bool indirect, bool query, hipStream_t s) {
    return launch_mma<F32Path>(a, indirect, query, s);
}

}  // namespace hg
