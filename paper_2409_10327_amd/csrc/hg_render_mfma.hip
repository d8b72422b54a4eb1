// hg_render_mfma.hip -- forward on the CDNA4 matrix cores, FP32 and mixed.
//
// Two precisions share one kernel body:
//   FP32:  FP32 tables, FP32 weights, v_mfma_f32_32x32x2f32 (K = 2 per step),
//          output heads on the vector ALU;
//   mixed: FP16 tables (FP32 interpolation), BF16 weights and activations,
//          v_mfma_f32_16x16x32_bf16 (K = 32 per step), FP32 accumulation.
// The light-direction sum is compensated FP32 in both.
//
// Work decomposition.  A wave owns 64 queries (one per lane) for the scalar
// work: direction sampling, hash-grid gathers, environment lookups, BRDF.
// Each MLP evaluation of the 64 queries is a set of matrix-core products
// with the units of a layer as rows (M) and the queries as columns (N):
// two 32-column N-tiles (FP32) or four 16-column N-tiles (mixed).  In both,
// the accumulators of one layer, after ReLU (and, mixed, conversion to
// BF16), are already the B operand of the next layer once the weight columns
// are permuted accordingly (no data movement between layers).  Mixed: the
// 16x16 output D of an M-tile gives lane l rows 4*(l/16)+r of column l%16,
// head rows are replicated so that every lane group receives the outputs of
// its column, and lane l keeps N-tile l/16, which is its own query.
// Inputs that come from other lanes (features, directions) go through LDS.
// The tracer's first layer is split into a per-point part (W0f f + b0,
// the accumulator input) and a direction part (two K-steps in FP32; one in
// the mixed path, which splits the direction into BF16 high and low
// halves).  The FP32 path computes the per-point part once per point; the
// mixed path recomputes it at the bounce points in every secondary tracer
// call (registers, below).
//
// Occupancy.  Both paths run two waves per SIMD (at most 256 registers per
// wave), so that one wave's gathers and vector work overlap the other's
// matrix-core work.  The FP32 path runs 512-thread blocks and bounces a
// wave's 64 queries in two halves of 32 points (bounce_lo_half); the mixed
// path runs two 256-thread blocks per CU with the whole-wave bounce
// (bounce_lo) and reads its tracer operands from LDS at each use instead of
// holding them in registers.  The FP32 path, and the mixed one on moderate
// grids below 256 directions per pixel (its bounce tracer only), raise a
// wave's issue priority for the tracer's matrix-core steps, so that the vector work of the SIMD's
// other wave fills the matrix pipe's gaps rather than delaying its next
// step; the priority changes also bound a scheduling region, which is most
// of their effect.  The mixed path is compiled with and without that fence
// (Bf16PathT<FENCED>) and launch_render_mixed picks the variant.
#include "hg_bf16.h"
#include "hg_device.h"
#include "hg_launch.h"

namespace hg {

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
    const float *ib0, *ib1, *bb0, *bb1;
    int nout;
};
__device__ __forceinline__ WSrc wsrc(const RenderK &a) {
    return WSrc{a.irt.W0, a.irt.W1, a.irt.W2, a.brdf.W0, a.brdf.W1, a.brdf.W2,
                a.irt.b0, a.irt.b1, a.brdf.b0, a.brdf.b1, a.brdf_out};
}

// ============================================================================
// Mixed path: BF16 operands, K = 32 per matrix-core step.  FENCED: the
// bounce tracer's matrix-core steps form a scheduling region of their own,
// at raised issue priority (the launch picks the variant per grid and
// direction count).
// ============================================================================
template <bool FENCED>
struct Bf16PathT {
    typedef __half Table;
    enum : int {
        T_W0W = 0, T_W0F = 4, T_W1 = 8, T_W2 = 16,       // tracer
        B_W0 = 18, B_W1 = 22, B_W2A = 30, B_W2B = 32,    // decoder
        N_TILES = 34,
        // the tracer's biases in accumulator order, four FP32 per lane
        T_B0 = 34, T_B1 = 38, T_B2 = 42,
        N_ALL = 43
    };
    typedef uint4 Tile;  // 8 BF16 per lane (or four FP32 for a bias tile)
    static constexpr int kTileFloats = N_ALL * 64;  // LDS array length in Tiles
    static constexpr int kThreads = 256;  // two blocks per CU: two waves per SIMD (kernel held to 256 registers)
    static constexpr bool kHalfBounce = false;        // bounce of all 64 points at once
    static constexpr bool kFenced = FENCED;

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
        for (int q = threadIdx.x; q < N_ALL * 64; q += blockDim.x) {
            const int t = q >> 6, l = q & 63, i = l & 15, g = l >> 4;
            if (t >= T_B0) {
                const f32x4 v = t < T_B1 ? bias_tile(ka.irt.b0, t - T_B0, g)
                                         : (t < T_B2 ? bias_tile(ka.irt.b1, t - T_B1, g) : head_bias(ka.irt.b2, 2, 0));
                tiles[q] = make_uint4(__float_as_uint(v[0]), __float_as_uint(v[1]), __float_as_uint(v[2]),
                                      __float_as_uint(v[3]));
                continue;
            }
            uint32_t w[4];
#pragma unroll
            for (int p = 0; p < 4; ++p)
                w[p] = (__float_as_uint(tile_value(a, t, i, g, 2 * p)) >> 16) |
                       (__float_as_uint(tile_value(a, t, i, g, 2 * p + 1)) & 0xffff0000u);
            tiles[q] = make_uint4(w[0], w[1], w[2], w[3]);
        }
    }

    static __device__ __forceinline__ f32x4 ftile(const Tile *tiles, int t, int lane) {
        const uint4 u = tiles[t * 64 + lane];
        return f32x4{__uint_as_float(u.x), __uint_as_float(u.y), __uint_as_float(u.z), __uint_as_float(u.w)};
    }

    // The tracer's operand and bias tiles are read from LDS at each use
    // rather than held in registers across calls: that keeps the kernel
    // within 256 registers, two waves per SIMD, so that one wave's gathers
    // and vector work overlap the other's (LDS traffic of the reads: about
    // 0.5 MB per wave and 64-query chunk, a small part of the LDS rate).
    struct Tracer {
        __device__ void load(const Tile *, const RenderK &, int) {}
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
    static __device__ __forceinline__ void point_part_nt(const Tile *tiles, const RenderK &a, const Wave &W, int nt,
                                                         int lane, int g, f32x4 (&d)[4]) {
        const uint4 xb = W.x[16 * nt + (lane & 15)][g];
#pragma unroll
        for (int m = 0; m < 4; ++m)
            d[m] = mfma_bf16(tiles[(T_W0F + m) * 64 + lane], xb, ftile(tiles, T_B0 + m, lane));
    }

    // decoder on the features of N-tile nt: oa rows 0..3 = outputs 0..3,
    // ob row 0 = output 4
    static __device__ __forceinline__ void decoder_nt(const Tile *tiles, const RenderK &a, const Wave &W, int nt,
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
    // (FENCE: the fenced variant's region and priority; the primary-point
    // tracer runs without them, measured faster: 33.9 -> 33.5 ms at N = 128)
    template <bool FENCE>
    static __device__ __forceinline__ f32x4 tracer_nt(const Tracer &T, const Tile *tiles, const Wave &W, int buf, int nt,
                                                      int lane, const f32x4 (&c)[4]) {
        const uint4 ob_ = W.om[buf][16 * nt + (lane & 15)];
        // FENCED: raised issue priority over the tracer's matrix-core steps,
        // so that the SIMD's other wave fills their gaps with its vector work
        // instead of delaying them (raising it over the decoder and the point
        // part too starved the other wave's encoder: slower); the priority
        // changes also bound a scheduling region, which is most of the effect
        if constexpr (FENCED && FENCE) __builtin_amdgcn_s_setprio(1);
        f32x4 d[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) d[m] = mfma_bf16(tiles[(T_W0W + m) * 64 + lane], ob_, c[m]);
        const uint4 h0 = act_pack(d[0], d[1]), h1 = act_pack(d[2], d[3]);
        f32x4 e[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            e[m] = mfma_bf16(tiles[(T_W1 + 2 * m) * 64 + lane], h0, ftile(tiles, T_B1 + m, lane));
            e[m] = mfma_bf16(tiles[(T_W1 + 2 * m + 1) * 64 + lane], h1, e[m]);
        }
        const uint4 k0 = act_pack(e[0], e[1]), k1 = act_pack(e[2], e[3]);
        f32x4 o = mfma_bf16(tiles[T_W2 * 64 + lane], k0, ftile(tiles, T_B2, lane));
        o = mfma_bf16(tiles[(T_W2 + 1) * 64 + lane], k1, o);
        if constexpr (FENCED && FENCE) __builtin_amdgcn_s_setprio(0);
        return o;
    }

    // ---- whole-wave interface (four 16-column N-tiles) ----
    struct PointPart {
        f32x4 v[4][4];  // [M-tile][N-tile]
    };
    static __device__ __forceinline__ void point_part(const Tile *tiles, const RenderK &a, const Wave &W, int lane,
                                                      PointPart &pp) {
        const int g = lane >> 4;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            f32x4 d[4];
            point_part_nt(tiles, a, W, nt, lane, g, d);
#pragma unroll
            for (int m = 0; m < 4; ++m) pp.v[m][nt] = d[m];
        }
    }
    // query mode: the point part of the 64 lanes' own features f
    static __device__ __forceinline__ void query_point_part(const Tile *tiles, const RenderK &a, Wave &W, int lane,
                                                            const float (&f)[kNF], PointPart &pp) {
        wave_sync_lds();
        store_feat(W, lane, f);
        wave_sync_lds();
        point_part(tiles, a, W, lane, pp);
    }
    // decoder outputs of the lane's own query (N-tile l / 16)
    static __device__ __forceinline__ void decoder(const Tile *tiles, const RenderK &a, const Wave &W, int lane,
                                                   float (&o)[8]) {
        const int g = lane >> 4;
#pragma unroll
        for (int k = 0; k < 8; ++k) o[k] = 0.0f;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            f32x4 oa, ob;
            decoder_nt(tiles, a, W, nt, lane, g, oa, ob);
            if (g == nt) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    o[r] = oa[r];
                    o[4 + r] = ob[r];
                }
            }
        }
    }
    // per-lane mode: decoder outputs of the 64 lanes' own features f
    static __device__ __forceinline__ void query_material(const Tile *tiles, const RenderK &a, Wave &W, int lane,
                                                          const float (&f)[kNF], float (&o)[8]) {
        wave_sync_lds();
        store_feat(W, lane, f);
        wave_sync_lds();
        decoder(tiles, a, W, lane, o);
        wave_sync_lds();
    }

    // shade mode: decoder outputs and tracer point part of the pixel slots
    // (feature rows 0 .. ppw - 1) into W.mat / W.ax
    static __device__ __forceinline__ void pixel_setup(const Tile *tiles, const RenderK &a, Wave &W, int lane,
                                                       int ppw) {
        const int g = lane >> 4, jcol = lane & 15;
        f32x4 oa, ob, ax[4];
        decoder_nt(tiles, a, W, 0, lane, g, oa, ob);
        point_part_nt(tiles, a, W, 0, lane, g, ax);
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
    }
    // shade mode: columns of N-tile nt belong to pixel slot sbase + ((16 nt) >> gs)
    static __device__ __forceinline__ void pixel_point_part(const Wave &W, int lane, uint32_t gs, int sbase,
                                                            PointPart &pp) {
        const int g = lane >> 4;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const float4 v4 = *reinterpret_cast<const float4 *>(&W.ax[sbase + ((16 * nt) >> gs)][16 * m + 4 * g]);
                pp.v[m][nt] = f32x4{v4.x, v4.y, v4.z, v4.w};
            }
    }
    // tracer logits of the lane's own query (N-tile nt uses pp.v[.][nt])
    template <bool DEPTH, bool SHARED>
    static __device__ __forceinline__ float2 tracer(const Tracer &T, const Tile *tiles, const Wave &W, int buf,
                                                    int lane, const PointPart &pp) {
        const int g = lane >> 4;
        float o0 = 0.f, o1 = 0.f;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const f32x4 c[4] = {pp.v[0][nt], pp.v[1][nt], pp.v[2][nt], pp.v[3][nt]};
            const f32x4 hh = tracer_nt<false>(T, tiles, W, buf, nt, lane, c);
            if (g == nt) {
                o0 = hh[0];
                o1 = hh[1];
            }
        }
        return make_float2(o0, DEPTH ? o1 : 0.0f);
    }

    // Tracer at the bounce points for the secondary directions: the point
    // part b0 + W0f x' is recomputed in each call from the features in W.x
    // (the same products in the same order, so the same values) instead of
    // being kept in 64 registers across the secondary loop.
    struct NoPart {};
    typedef NoPart BouncePart;
    static __device__ __forceinline__ void bounce_part(const Tile *, const RenderK &, const Wave &, int, NoPart &) {}
    template <bool DEPTH>
    static __device__ __forceinline__ float2 tracer_bounce(const Tracer &T, const Tile *tiles, const RenderK &a,
                                                           const Wave &W, int buf, int lane, const NoPart &) {
        const int g = lane >> 4;
        float o0 = 0.f, o1 = 0.f;
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            f32x4 c[4];
            point_part_nt(tiles, a, W, nt, lane, g, c);
            const f32x4 hh = tracer_nt<true>(T, tiles, W, buf, nt, lane, c);
            if (g == nt) {
                o0 = hh[0];
                o1 = hh[1];
            }
        }
        return make_float2(o0, DEPTH ? o1 : 0.0f);
    }
};

// ============================================================================
// FP32 path: FP32 operands on v_mfma_f32_32x32x2f32 (K = 2 per step).
// One wave's 64 queries are two 32-column N-tiles; a 64-unit layer is two
// 32-row M-tiles.  Lane l supplies A[l % 32][l / 32] and B[l / 32][l % 32]
// and receives, in accumulator register r, row 8 (r / 4) + 4 (l / 32) +
// r % 4 of column l % 32.  With only four accumulator chains per layer
// (2 M-tiles x 2 N-tiles) this shape keeps the matrix pipe at its full rate
// from one wave, where the 16x16x4 shape needs four times as many chains.
// The output heads (2 tracer logits, 5 or 8 decoder outputs) are dot
// products on the vector ALU over the 32 units a lane holds, completed by
// one exchange between the two lane halves.
// ============================================================================
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ f32x16 mfma32(float a, float b, const f32x16 &c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}
// max(x, 0) in one instruction: as a signed integer every negative float
// (sign bit set) is below zero, so an integer max with 0 is the ReLU (and
// needs no NaN canonicalisation, which a float max does)
__device__ __forceinline__ float relu1(float x) { return __int_as_float(max(__float_as_int(x), 0)); }
// row of accumulator register r in lane half h, within a 32-row M-tile
__device__ __forceinline__ int row32(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }
// physical hidden unit fed by K-step s (0..31) in lane half h: M-tile s / 16,
// accumulator register s % 16 of the previous layer
__device__ __forceinline__ int unit32(int s, int h) { return 32 * (s >> 4) + row32(s & 15, h); }

struct F32Path {
    typedef float Table;
    // 512 threads per block, two waves per SIMD: with at most 256 registers
    // per wave, one wave's vector-ALU and memory work overlaps the other's
    // matrix-core work
    static constexpr int kThreads = 512;
    static constexpr bool kHalfBounce = true;  // bounce in two halves of 32 points
    static constexpr bool kFenced = true;      // the tracer's priority changes bound its region
    // operand tiles (64 floats each: lane l holds A[l % 32][l / 32])
    enum : int {
        T_W0W = 0,    // tracer direction part: 2 M-tiles x 2 K-steps (m*2 + s), components 2s + h
        T_W0F = 4,    // tracer point part: 2 x 16 K-steps (m*16 + s), feature 16h + s
        T_W1 = 36,    // tracer hidden layer: 2 x 32 K-steps (m*32 + s)
        D_W0 = 100,   // decoder first layer: 2 x 16 K-steps, feature 16h + s
        D_W1 = 132,   // decoder hidden layer: 2 x 32 K-steps
        N_TILES = 196
    };
    // Bias region (after the operand tiles, 256 floats used of 8 x 64): a
    // layer's accumulators start at its bias, loaded from LDS in accumulator
    // order, so no bias stays in registers and no matrix-core step adds it.
    enum : int {
        B_TB0 = N_TILES,      // tracer first-layer bias, 2 M-tiles
        B_TB1 = N_TILES + 2,  // tracer hidden bias
        B_DB0 = N_TILES + 4,  // decoder first-layer bias
        B_DB1 = N_TILES + 6,  // decoder hidden bias
        N_ALL = N_TILES + 8
    };
    // after the tiles: head weights for the vector ALU, [half][output][16 m + r]
    static constexpr int HT_OFF = N_ALL * 64;        // tracer: 2 halves x 2 outputs x 32
    static constexpr int HD_OFF = HT_OFF + 128;      // decoder: 2 halves x 8 outputs x 32
    static constexpr int N_FLOATS = HD_OFF + 512;
    typedef float Tile;
    static constexpr int kTileFloats = N_FLOATS;
    static constexpr int kXS = 36;  // row stride of the feature rows (16-byte aligned)

    struct Wave {
        float x[32][kXS];   // input features of 32 points (one N-tile)
        float4 om[2][64];   // per-lane direction (x, y, z, 0), two buffers
        float ax[4][kH];    // per-pixel tracer point part (shade mode)
        float mat[4][8];    // per-pixel decoder outputs (shade mode)
        float4 bpx[64];     // every lane's bounce point x' and point id (bits)
        float4 bpw[64];     // its direction w and sample index (bits)
        uint16_t qi[128];   // queued shadow rays (hard visibility): direction index
        float qd[128];      // and normalised depth
    };

    struct PointPart {
        f32x16 c[2][2];     // [M-tile][N-tile]
    };

    static __device__ __forceinline__ float tile_value(const WSrc &a, int q) {
        if (q >= HD_OFF) {
            const int t = q - HD_OFF, h = t >> 8, o = (t >> 5) & 7, mr = t & 31;
            return o < a.nout ? wf(a.bW2, o * kH + 32 * (mr >> 4) + row32(mr & 15, h)) : 0.0f;
        }
        if (q >= HT_OFF) {
            const int t = q - HT_OFF, h = t >> 6, o = (t >> 5) & 1, mr = t & 31;
            return wf(a.iW2, o * kH + 32 * (mr >> 4) + row32(mr & 15, h));
        }
        const int t = q >> 6, l = q & 63, i = l & 31, h = l >> 5;
        if (t >= N_TILES) {
            // biases in accumulator order: [layer][M-tile][lane half][register]
            const int qq = q - N_TILES * 64;
            if (qq >= 256) return 0.0f;
            const int which = qq >> 6, m = (qq >> 5) & 1, hh = (qq >> 4) & 1, r = qq & 15;
            const float *b = which == 0 ? a.ib0 : (which == 1 ? a.ib1 : (which == 2 ? a.bb0 : a.bb1));
            return b[32 * m + row32(r, hh)];
        }
        if (t < T_W0F) {
            const int m = (t - T_W0W) >> 1, c = 2 * ((t - T_W0W) & 1) + h;
            return c < 3 ? wf(a.iW0, (32 * m + i) * kNI + kNF + c) : 0.0f;
        }
        if (t < T_W1) {
            const int m = (t - T_W0F) >> 4, st = (t - T_W0F) & 15;
            return wf(a.iW0, (32 * m + i) * kNI + 16 * h + st);
        }
        if (t < D_W0) {
            const int m = (t - T_W1) >> 5, st = (t - T_W1) & 31;
            return wf(a.iW1, (32 * m + i) * kH + unit32(st, h));
        }
        if (t < D_W1) {
            const int m = (t - D_W0) >> 4, st = (t - D_W0) & 15;
            return wf(a.bW0, (32 * m + i) * kNF + 16 * h + st);
        }
        const int m = (t - D_W1) >> 5, st = (t - D_W1) & 31;
        return wf(a.bW1, (32 * m + i) * kH + unit32(st, h));
    }

    static __device__ __forceinline__ void build_tiles(const RenderK &ka, Tile *tiles) {
        const WSrc a = wsrc(ka);
        for (int q = threadIdx.x; q < N_FLOATS; q += blockDim.x) tiles[q] = tile_value(a, q);
    }

    static __device__ __forceinline__ f32x16 from4(const float4 (&v)[4]) {
        f32x16 r;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            r[4 * q] = v[q].x;
            r[4 * q + 1] = v[q].y;
            r[4 * q + 2] = v[q].z;
            r[4 * q + 3] = v[q].w;
        }
        return r;
    }
    // accumulators of M-tile m started at the bias of layer bt (one of the
    // B_* ids): register r of lane half h holds the bias of row
    // 8 (r / 4) + 4 h + r % 4, read as four broadcast 16-byte LDS loads
    static __device__ __forceinline__ f32x16 bias_start(const Tile *tiles, int bt, int m, int lane) {
        const float *bp = &tiles[N_TILES * 64 + ((((bt - N_TILES) >> 1) * 2 + m) * 2 + (lane >> 5)) * 16];
        float4 v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = *reinterpret_cast<const float4 *>(bp + 4 * q);
        return from4(v);
    }

    struct Tracer {
        float hb0, hb1;
        __device__ void load(const Tile *, const RenderK &a, int) {
            hb0 = a.irt.b2[0];
            hb1 = a.irt.b2[1];
        }
    };

    static __device__ __forceinline__ void store_level(Wave &W, int row, int lvl, float f0, float f1) {
        *reinterpret_cast<float2 *>(&W.x[row][2 * lvl]) = make_float2(f0, f1);
    }
    // features 16 hl .. 16 hl + 15 of row `row`
    static __device__ __forceinline__ void store_feat16(Wave &W, int row, int hl, const float (&f)[16]) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            *reinterpret_cast<float4 *>(&W.x[row][16 * hl + 4 * q]) =
                make_float4(f[4 * q], f[4 * q + 1], f[4 * q + 2], f[4 * q + 3]);
    }
    static __device__ __forceinline__ void store_dir(Wave &W, int buf, int lane, float3 w) {
        W.om[buf][lane] = make_float4(w.x, w.y, w.z, 0.0f);
    }

    // first layer over the features of the 32 rows: out[m] = b + W x (bias bt)
    static __device__ __forceinline__ void feat_layer(const Tile *tiles, int base, int bt, const Wave &W, int lane,
                                                      f32x16 (&out)[2]) {
        const int h = lane >> 5;
        const float *xr = &W.x[lane & 31][16 * h];
        float xv[16];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float4 v = *reinterpret_cast<const float4 *>(xr + 4 * q);
            xv[4 * q] = v.x;
            xv[4 * q + 1] = v.y;
            xv[4 * q + 2] = v.z;
            xv[4 * q + 3] = v.w;
        }
        out[0] = bias_start(tiles, bt, 0, lane);
        out[1] = bias_start(tiles, bt, 1, lane);
#pragma unroll
        for (int st = 0; st < 16; ++st)
#pragma unroll
            for (int m = 0; m < 2; ++m) out[m] = mfma32(tiles[(base + 16 * m + st) * 64 + lane], xv[st], out[m]);
    }

    // hidden layer: out[m] = b + W relu(in) (bias bt)
    static __device__ __forceinline__ void hidden_layer(const Tile *tiles, int base, int bt, const f32x16 (&in)[2],
                                                        int lane, f32x16 (&out)[2]) {
        out[0] = bias_start(tiles, bt, 0, lane);
        out[1] = bias_start(tiles, bt, 1, lane);
#pragma unroll
        for (int st = 0; st < 32; ++st) {
            // the operand tiles of eight K-steps at a time are loaded ahead, not all 64
            if ((st & 7) == 0) __builtin_amdgcn_sched_barrier(0);
            const float b = relu1(in[st >> 4][st & 15]);
#pragma unroll
            for (int m = 0; m < 2; ++m) out[m] = mfma32(tiles[(base + 32 * m + st) * 64 + lane], b, out[m]);
        }
    }

    // this lane's part of a head output over its 32 units: sum of w relu(e)
    static __device__ __forceinline__ float head_part(const float *hw, const f32x16 (&e)[2]) {
        float p = 0.f;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const float4 w = *reinterpret_cast<const float4 *>(hw + 4 * q);
            const int m = q >> 2, r = 4 * (q & 3);
            p = fmaf(relu1(e[m][r]), w.x, p);
            p = fmaf(relu1(e[m][r + 1]), w.y, p);
            p = fmaf(relu1(e[m][r + 2]), w.z, p);
            p = fmaf(relu1(e[m][r + 3]), w.w, p);
        }
        return p;
    }
    // head output of column lane % 32 of one N-tile: the two lane halves' parts
    static __device__ __forceinline__ float head_one(float p) { return p + __shfl_xor(p, 32); }
    // head output of the lane's own column of two N-tiles (N-tile l / 32)
    static __device__ __forceinline__ float head_two(float p0, float p1, int lane) {
        const bool hi = (lane >> 5) != 0;
        return (hi ? p1 : p0) + __shfl_xor(hi ? p0 : p1, 32);
    }

    // tracer point part W0f f + b0 of the 32 feature rows -> c[m][0]
    static __device__ __forceinline__ void point_part(const Tile *tiles, const RenderK &a, const Wave &W, int lane,
                                                      PointPart &pp) {
        f32x16 c[2];
        feat_layer(tiles, T_W0F, B_TB0, W, lane, c);
        pp.c[0][0] = c[0];
        pp.c[1][0] = c[1];
    }

    // query mode: the point part of the 64 lanes' own features f, rows of
    // lanes 32 nt .. 32 nt + 31 -> c[m][nt]
    static __device__ __forceinline__ void query_point_part(const Tile *tiles, const RenderK &a, Wave &W, int lane,
                                                            const float (&f)[kNF], PointPart &pp) {
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            wave_sync_lds();
            if ((lane >> 5) == nt) {
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    *reinterpret_cast<float4 *>(&W.x[lane & 31][4 * q]) =
                        make_float4(f[4 * q], f[4 * q + 1], f[4 * q + 2], f[4 * q + 3]);
            }
            wave_sync_lds();
            f32x16 c[2];
            feat_layer(tiles, T_W0F, B_TB0, W, lane, c);
            pp.c[0][nt] = c[0];
            pp.c[1][nt] = c[1];
        }
    }

    // decoder outputs (up to 8) of point lane % 32 of the 32 feature rows
    static __device__ __forceinline__ void decoder(const Tile *tiles, const RenderK &a, const Wave &W, int lane,
                                                   float (&o)[8]) {
        const int h = lane >> 5;
        f32x16 d[2], e[2];
        feat_layer(tiles, D_W0, B_DB0, W, lane, d);
        hidden_layer(tiles, D_W1, B_DB1, d, lane, e);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            o[k] = 0.0f;
            if (k < a.brdf_out) o[k] = head_one(head_part(&tiles[HD_OFF + (8 * h + k) * 32], e)) + a.brdf.b2[k];
        }
    }

    // per-lane mode: decoder outputs of the 64 lanes' own features f, in two
    // passes of 32 feature rows (lanes 32 nt .. 32 nt + 31 in pass nt)
    static __device__ __forceinline__ void query_material(const Tile *tiles, const RenderK &a, Wave &W, int lane,
                                                          const float (&f)[kNF], float (&o)[8]) {
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            wave_sync_lds();
            if ((lane >> 5) == nt) {
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    *reinterpret_cast<float4 *>(&W.x[lane & 31][4 * q]) =
                        make_float4(f[4 * q], f[4 * q + 1], f[4 * q + 2], f[4 * q + 3]);
            }
            wave_sync_lds();
            float t[8];
            decoder(tiles, a, W, lane, t);
            if ((lane >> 5) == nt) {
#pragma unroll
                for (int k = 0; k < 8; ++k) o[k] = t[k];
            }
        }
        wave_sync_lds();
    }

    // shade mode: decoder outputs and tracer point part of the pixel slots
    // (feature rows 0 .. ppw - 1) into W.mat / W.ax
    static __device__ __forceinline__ void pixel_setup(const Tile *tiles, const RenderK &a, Wave &W, int lane,
                                                       int ppw) {
        const int h = lane >> 5, j = lane & 31;
        float o[8];
        decoder(tiles, a, W, lane, o);
        f32x16 c[2];
        feat_layer(tiles, T_W0F, B_TB0, W, lane, c);
        if (j < ppw) {
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int r = 0; r < 16; ++r) W.ax[j][32 * m + row32(r, h)] = c[m][r];
            if (h == 0) {
#pragma unroll
                for (int k = 0; k < 5; ++k) W.mat[j][k] = o[k];
            }
        }
    }

    // shade mode: the point part of each query's pixel slot sbase + ((32 nt + l % 32) >> gs)
    static __device__ __forceinline__ void pixel_point_part(const Wave &W, int lane, uint32_t gs, int sbase,
                                                            PointPart &pp) {
        const int h = lane >> 5, j = lane & 31;
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const float *ar = W.ax[sbase + ((32 * nt + j) >> gs)];
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                float4 v[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = *reinterpret_cast<const float4 *>(ar + 32 * m + 8 * q + 4 * h);
                pp.c[m][nt] = from4(v);
            }
        }
    }

    // tracer logits (visibility, and depth if DEPTH) of the lane's own query:
    // N-tile nt holds the directions of lanes 32 nt .. 32 nt + 31 (operand
    // buffer buf); SHARED: both N-tiles use the point part c[m][0] (the same
    // 32 points with two directions each), else N-tile nt uses c[m][nt].
    // The two N-tiles run one after the other (two accumulator chains each).
    // The wave raises its issue priority for the matrix-core steps, so that
    // the other wave of the SIMD does not delay them with its vector work
    // (800x800 frame 82.4 -> 80.1 ms; raising it for the head dot products
    // too, or for the decoder, measured no better).
    template <bool DEPTH, bool SHARED>
    static __device__ __forceinline__ float2 tracer(const Tracer &T, const Tile *tiles, const Wave &W, int buf,
                                                    int lane, const PointPart &pp) {
        const int h = lane >> 5, j = lane & 31;
        float p0[2], p1[2];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            // one N-tile at a time (register pressure)
            __builtin_amdgcn_sched_barrier(0);
            const float4 w = W.om[buf][32 * nt + j];
            const float bd0 = h ? w.y : w.x, bd1 = h ? w.w : w.z;
            __builtin_amdgcn_s_setprio(1);
            f32x16 d[2], e[2];
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                d[m] = mfma32(tiles[(T_W0W + 2 * m) * 64 + lane], bd0, pp.c[m][SHARED ? 0 : nt]);
                d[m] = mfma32(tiles[(T_W0W + 2 * m + 1) * 64 + lane], bd1, d[m]);
            }
            hidden_layer(tiles, T_W1, B_TB1, d, lane, e);
            __builtin_amdgcn_s_setprio(0);
            p0[nt] = head_part(&tiles[HT_OFF + (2 * h) * 32], e);
            p1[nt] = DEPTH ? head_part(&tiles[HT_OFF + (2 * h + 1) * 32], e) : 0.0f;
        }
        const float o0 = head_two(p0[0], p0[1], lane) + T.hb0;
        const float o1 = DEPTH ? head_two(p1[0], p1[1], lane) + T.hb1 : 0.0f;
        return make_float2(o0, o1);
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
                                               const typename PP::BouncePart &bpt, int lane, const Frame &frb,
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
        // without the tracer's fence, a region boundary after the texel load
        // keeps it ahead of the tracer's steps (paper's grid: 35.3 -> 33.4 ms;
        // with the fence it changes nothing)
        if constexpr (!PP::kFenced) __builtin_amdgcn_sched_barrier(0);
        const float3 cn = sb.eval<NHEAD>(wn);
        const float vo = PP::template tracer_bounce<false>(T, tiles, a, W, (int)(j & 1u), lane, bpt).x;
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
                                            const typename PP::Tracer &T, int lane, float3 x, float3 w,
                                            float dd, uint32_t pid, uint32_t q, bool hard, bool diffuse) {
    const float t = fmaf(a.t_span, dd, a.t_near);
    const float3 xb = make_float3(fmaf(t, w.x, x.x), fmaf(t, w.y, x.y), fmaf(t, w.z, x.z));
    float fb[kNF];
    encode<TT>(a.g, xb.x, xb.y, xb.z, fb);
    wave_sync_lds();
    PP::store_feat(W, lane, fb);
    wave_sync_lds();
    typename PP::BouncePart bpt;
    PP::bounce_part(tiles, a, W, lane, bpt);
    float od[8];
    PP::decoder(tiles, a, W, lane, od);
    const float3 ab = make_float3(sigmoidf_(od[0]), sigmoidf_(od[1]), sigmoidf_(od[2]));
    const float rb = 0.09f + 0.91f * sigmoidf_(od[3]);
    const float mb = sigmoidf_(od[4]);
    // secondary view -w; normal from the decoder's normal head if it has one,
    // else the facing normal -w
    const float3 vb = make_float3(-w.x, -w.y, -w.z);
    const bool nhead = a.brdf_out == 8;
    const float3 nb = nhead ? head_normal(od[5], od[6], od[7], vb) : vb;
    const Frame frb = make_frame(nb);
    FacingBrdf fb_;
    fb_.set(ab, rb, mb, a.f0, diffuse);
    const SecondaryBrdf sb{nb, vb, ab, rb, mb, a.f0, diffuse, fb_};
    return nhead ? secondary_lo<PP, true>(a, tiles, W, T, bpt, lane, frb, sb, pid, q, hard)
                 : secondary_lo<PP, false>(a, tiles, W, T, bpt, lane, frb, sb, pid, q, hard);
}


// Levels 8 hl .. 8 hl + 7 of H(x) (features 16 hl .. 16 hl + 15): the two
// lane halves of a wave encode the same 32 points, half of the levels each.
// The level parameters are selected per lane half; a gather addresses the
// table by a 32-bit byte offset from its base (below 2^31: 16 levels x 2^24
// entries x 8 bytes).  Gathers are issued two levels at a time, and a slot
// past the grid's L levels reads entry 0 of level 0 and yields zeros.
template <typename TT>
__device__ __forceinline__ void encode_half(const GridK &g, float x, float y, float z, int hl, float (&f)[16]) {
    float u[3];
    bool in[3];
    pos_to_u(g, x, y, z, u, in);
    const bool hi = hl != 0;
    const uint32_t esh = sizeof(TT) == 4 ? 3u : 2u;  // log2 bytes per entry (two features)
#pragma unroll
    for (int l0 = 0; l0 < 8; l0 += 2) {
        __builtin_amdgcn_sched_barrier(0);
        float w[2][3];
        float2 e[2][8];
        bool have[2];
#pragma unroll
        for (int li = 0; li < 2; ++li) {
            const int lu = l0 + li;
            const int l = hi ? lu + 8 : lu;
            have[li] = l < (int)g.L;
            const float resf = hi ? g.resf[lu + 8] : g.resf[lu];
            const float nm1f = hi ? g.nm1f[lu + 8] : g.nm1f[lu];
            const uint32_t st = hi ? g.stride[lu + 8] : g.stride[lu];
            const bool dense = ((g.dense_mask >> l) & 1u) != 0;
            uint32_t c[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) cell_of_sel(u[d], resf, nm1f, c[d], w[li][d]);
            uint32_t idx[8];
            corner_idx_p(dense, st, g.Tmask, c, idx);
            const uint32_t lbase = (uint32_t)l << (g.log2T + esh);
#pragma unroll
            for (int k = 0; k < 8; ++k) e[li][k] = TabLoad<TT>::ld_byte(g.table, have[li] ? lbase + (idx[k] << esh) : 0u);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int li = 0; li < 2; ++li) {
            const float wx0 = 1.0f - w[li][0], wy0 = 1.0f - w[li][1], wz0 = 1.0f - w[li][2];
            float f0 = 0.0f, f1 = 0.0f;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const float wt = ((k & 1) ? w[li][0] : wx0) * (((k >> 1) & 1) ? w[li][1] : wy0) *
                                 (((k >> 2) & 1) ? w[li][2] : wz0);
                f0 = fmaf(wt, e[li][k].x, f0);
                f1 = fmaf(wt, e[li][k].y, f1);
            }
            f[2 * (l0 + li)] = have[li] ? f0 : 0.0f;
            f[2 * (l0 + li) + 1] = have[li] ? f1 : 0.0f;
        }
    }
    __builtin_amdgcn_sched_barrier(0);
}

// Sum over this lane's secondary directions j = 2 k + (l / 32) of
// f_r(w_j) V(x', w_j) L_e(w_j) at point l % 32 of the 32 points whose point
// part is bpt: a tracer call's two N-tiles are the 32 points with directions
// 2 k and 2 k + 1 (lane halves), sharing one point part.  Software pipeline
// as in secondary_lo; the Philox block (j / 4 = k / 2) is wave-uniform.  With
// N' = 1 the upper half traces a copy of direction 0 with weight zero.
template <class PP, bool NHEAD, bool OPQ>
__device__ __forceinline__ float3 secondary_pair(const RenderK &a, const typename PP::Tile *tiles,
                                                 typename PP::Wave &W, const typename PP::Tracer &T,
                                                 const typename PP::PointPart &bpt, int lane, const Frame &frb,
                                                 const SecondaryBrdf &sb, uint32_t pid, uint32_t q, bool hard) {
    const uint32_t n2 = a.s.n_dirs2;
    const uint32_t hl = (uint32_t)(lane >> 5);
    const uint32_t npair = (n2 + 1u) >> 1;
    const float wgt = hl < n2 ? 1.0f : 0.0f;
    uint4 words2 = philox4x32_10<OPQ>(pid, q, 0u, 1u, a.s.key0, a.s.key1);
    const uint32_t j0 = hl < n2 ? hl : 0u;
    const float3 w0 = sample_dir(pick4(words2, j0), j0, a.s.nb2_shift, a.s.inv_na2, a.s.inv_nb2, frb);
    float3 Ej = env_lookup(a.env, w0.x, w0.y, w0.z);
    float3 cj = sb.eval<NHEAD>(w0);
    wave_sync_lds();
    PP::store_dir(W, 0, lane, w0);
    wave_sync_lds();
    float Lx = 0.f, Ly = 0.f, Lz = 0.f;
    for (uint32_t k = 0; k < npair; ++k) {
        const uint32_t kn = k + 1 < npair ? k + 1 : k;
        if (kn != k && (kn & 1u) == 0) words2 = philox4x32_10<OPQ>(pid, q, kn >> 1, 1u, a.s.key0, a.s.key1);
        const uint32_t jr = 2u * kn + hl;
        const uint32_t jn = jr < n2 ? jr : 0u;
        const float3 wn = sample_dir(pick4(words2, jn), jn, a.s.nb2_shift, a.s.inv_na2, a.s.inv_nb2, frb);
        const float3 En = env_lookup(a.env, wn.x, wn.y, wn.z);
        const float3 cn = sb.eval<NHEAD>(wn);
        const float vo = PP::template tracer<false, true>(T, tiles, W, (int)(k & 1u), lane, bpt).x;
        PP::store_dir(W, (int)((k + 1) & 1u), lane, wn);
        // hard visibility: only visible secondary rays contribute
        const float vj = (hard ? (vo > 0.0f ? 1.0f : 0.0f) : sigmoidf_(vo)) * wgt;
        Lx = fmaf(cj.x * vj, Ej.x, Lx);
        Ly = fmaf(cj.y * vj, Ej.y, Ly);
        Lz = fmaf(cj.z * vj, Ej.z, Lz);
        Ej = En;
        cj = cn;
        wave_sync_lds();
    }
    return make_float3(Lx, Ly, Lz);
}

// L'_o at the bounce points of the wave's 64 queries, in two halves of 32
// points: every lane's bounce point goes to LDS, then for each half the two
// lane halves encode the 32 points (levels 0..7 / 8..15), the decoder and
// tracer point part run on one 32-column N-tile, and the lane halves trace
// alternate secondary directions; the two halves' sums meet in the lane
// that owns the point.
// OPQ: Philox key schedule recomputed per call (shade mode; query mode
// measured faster with it hoisted)
template <class PP, class TT, bool OPQ>
__device__ __forceinline__ float3 bounce_lo_half(const RenderK &a, const typename PP::Tile *tiles,
                                                 typename PP::Wave &W, const typename PP::Tracer &T, int lane,
                                                 float3 x, float3 w, float dd, uint32_t pid, uint32_t q, bool hard,
                                                 bool diffuse) {
    const float t = fmaf(a.t_span, dd, a.t_near);
    const float3 xb = make_float3(fmaf(t, w.x, x.x), fmaf(t, w.y, x.y), fmaf(t, w.z, x.z));
    wave_sync_lds();
    W.bpx[lane] = make_float4(xb.x, xb.y, xb.z, __uint_as_float(pid));
    W.bpw[lane] = make_float4(w.x, w.y, w.z, __uint_as_float(q));
    wave_sync_lds();
    const int j = lane & 31, hl = lane >> 5;
    const bool nhead = a.brdf_out == 8;
    const float inv = 1.0f / (float)a.s.n_dirs2;
    float3 Lo = make_float3(0.f, 0.f, 0.f);
#pragma unroll 1
    for (int half = 0; half < 2; ++half) {
        const float4 bx = W.bpx[32 * half + j], bw = W.bpw[32 * half + j];
        float fb[16];
        encode_half<TT>(a.g, bx.x, bx.y, bx.z, hl, fb);
        PP::store_feat16(W, j, hl, fb);
        wave_sync_lds();
        typename PP::PointPart bpt;
        PP::point_part(tiles, a, W, lane, bpt);
        float od[8];
        PP::decoder(tiles, a, W, lane, od);
        const float3 ab = make_float3(sigmoidf_(od[0]), sigmoidf_(od[1]), sigmoidf_(od[2]));
        const float rb = 0.09f + 0.91f * sigmoidf_(od[3]);
        const float mb = sigmoidf_(od[4]);
        // secondary view -w; normal from the decoder's normal head if it has
        // one, else the facing normal -w
        const float3 vb = make_float3(-bw.x, -bw.y, -bw.z);
        const float3 nb = nhead ? head_normal(od[5], od[6], od[7], vb) : vb;
        const Frame frb = make_frame(nb);
        FacingBrdf fb_;
        fb_.set(ab, rb, mb, a.f0, diffuse);
        const SecondaryBrdf sb{nb, vb, ab, rb, mb, a.f0, diffuse, fb_};
        const uint32_t ppid = __float_as_uint(bx.w), pq = __float_as_uint(bw.w);
        const float3 L = nhead ? secondary_pair<PP, true, OPQ>(a, tiles, W, T, bpt, lane, frb, sb, ppid, pq, hard)
                               : secondary_pair<PP, false, OPQ>(a, tiles, W, T, bpt, lane, frb, sb, ppid, pq, hard);
        const float sx = L.x + __shfl_xor(L.x, 32), sy = L.y + __shfl_xor(L.y, 32), sz = L.z + __shfl_xor(L.z, 32);
        if (hl == half) Lo = make_float3(sx * inv, sy * inv, sz * inv);
        wave_sync_lds();  // the next half rewrites the feature rows and direction buffers
    }
    return Lo;
}

// ============================================================================
// The kernel.  QUERY: one query per lane with its own point and direction;
// otherwise shade mode with G = min(N, 64) lanes per pixel.  For N >= 16 (at
// most four pixels per wave) the pixels' features, material and tracer point
// part are formed once per pixel slot; PERLANE (N < 16, up to 64 pixels per
// wave): every lane forms its own pixel's, as in query mode, and the G lanes
// of a pixel then shade and sum as in shade mode.
// ============================================================================
template <class PP, bool INDIRECT, bool QUERY, bool MIS, bool PERLANE>
// at least two waves per SIMD: the register budget is 256 per wave
__global__ __launch_bounds__(PP::kThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_render_mma(const RenderK a,
                                                                                              int64_t n_items) {
    typedef typename PP::Table TT;
    constexpr int kWaves = PP::kThreads / 64;
    __shared__ typename PP::Tile tiles[PP::kTileFloats];
    __shared__ typename PP::Wave wl[kWaves];
    PP::build_tiles(a, tiles);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    typename PP::Wave &W = wl[threadIdx.x >> 6];
    typename PP::Tracer T;
    T.load(tiles, a, lane);

    const bool diffuse = (a.s.flags & 1u) != 0;
    const bool hard = (a.s.flags & 2u) != 0;
    const uint32_t gs = a.s.g_shift;
    const uint32_t G = 1u << gs;
    const int ppw = 64 >> gs;
    const int64_t waves_total = (int64_t)gridDim.x * kWaves;
    const int64_t wave_id = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6);

    // Shade mode: a work unit is 4 / ppw consecutive items, whose four pixel
    // slots share one pixel setup (encode at x, decoder, tracer point part).
    const int ipw = (QUERY || PERLANE) ? 1 : 4 / ppw;
    const int64_t n_units = (n_items + ipw - 1) / ipw;
    for (int64_t unit = wave_id; unit < n_units; unit += waves_total) {
    for (int ii = 0; ii < ipw; ++ii) {
        const int64_t item = unit * ipw + ii;
        if (item >= n_items) break;  // wave-uniform
        const int sbase = ii * ppw;  // first pixel slot of this item
        int64_t p_raw;
        if (QUERY) p_raw = item * 64 + lane;
        else p_raw = item * ppw + (lane >> gs);
        const bool live = p_raw < a.n;
        const int64_t p = live ? p_raw : a.n - 1;
        const float3 x = make_float3(a.pos[3 * p], a.pos[3 * p + 1], a.pos[3 * p + 2]);

        // ---------------- primary point ----------------
        float3 n_ = make_float3(0.f, 0.f, 1.f), v_ = n_, alb = n_;
        float rr = 0.5f, mm = 0.f;
        float fq[kNF];  // query and per-lane modes: the lane's own features at x
        if (QUERY || PERLANE) {
            encode<TT>(a.g, x.x, x.y, x.z, fq);
        } else if (ii == 0) {
            // lane l encodes level l % 16 of pixel slot l / 16 (pixel 4 unit + slot)
            const int slot = lane >> 4, lvl = lane & 15;
            const int64_t ps_raw = unit * 4 + slot;
            const int64_t ps = ps_raw < a.n ? ps_raw : a.n - 1;
            if (lvl < (int)a.g.L) {
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
            } else {
                PP::store_level(W, slot, lvl, 0.0f, 0.0f);  // slot of a level the grid does not have
            }
            wave_sync_lds();
            PP::pixel_setup(tiles, a, W, lane, 4);
            wave_sync_lds();
        }
        if (!QUERY) {
            n_ = make_float3(a.nrm[3 * p], a.nrm[3 * p + 1], a.nrm[3 * p + 2]);
            v_ = make_float3(a.wo[3 * p], a.wo[3 * p + 1], a.wo[3 * p + 2]);
            float mo[5];
            if (PERLANE) {
                float od[8];
                PP::query_material(tiles, a, W, lane, fq, od);
#pragma unroll
                for (int k = 0; k < 5; ++k) mo[k] = od[k];
            } else {
                const int myslot = sbase + (lane >> gs);
#pragma unroll
                for (int k = 0; k < 5; ++k) mo[k] = W.mat[myslot][k];
            }
            alb = make_float3(sigmoidf_(mo[0]), sigmoidf_(mo[1]), sigmoidf_(mo[2]));
            rr = 0.09f + 0.91f * sigmoidf_(mo[3]);
            mm = sigmoidf_(mo[4]);
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
                    // key schedule recomputed per call on the FP32 path (faster
                    // there), hoisted on the mixed one
                    const uint4 words = philox4x32_10<PP::kHalfBounce>((uint32_t)p, 0u, i_own >> 2, 0u,
                                                                       a.s.key0, a.s.key1);
                    w_own = sample_dir(pick4(words, i_own), i_own, a.s.nb_shift, a.s.inv_na, a.s.inv_nb, fr);
                }
                Le_own = env_lookup(a.env, w_own.x, w_own.y, w_own.z);  // overlaps the tracer
                wave_sync_lds();
                PP::store_dir(W, 0, lane, w_own);
                wave_sync_lds();
                // tracer point part at x: query mode (one chunk per item) from
                // the lanes' features, shade mode from the pixel slots
                typename PP::PointPart c;
                if (QUERY || PERLANE) PP::query_point_part(tiles, a, W, lane, fq, c);
                else PP::pixel_point_part(W, lane, gs, sbase, c);
                const float2 oo = PP::template tracer<true, false>(T, tiles, W, 0, lane, c);
                const float o0 = oo.x, o1 = oo.y;
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
                    const uint4 words = philox4x32_10<PP::kHalfBounce>((uint32_t)p, 0u, ie >> 2, 0u,
                                                                       a.s.key0, a.s.key1);
                    we = sample_dir(pick4(words, ie), ie, a.s.nb_shift, a.s.inv_na, a.s.inv_nb, fr);
                }
            }
            float3 Lin;
            if (!INDIRECT) {
                Lin = make_float3(Ve * Le_own.x, Ve * Le_own.y, Ve * Le_own.z);
            } else {
                float3 Lo;
                if constexpr (PP::kHalfBounce)
                    Lo = bounce_lo_half<PP, TT, !QUERY>(a, tiles, W, T, lane, x, we, de, (uint32_t)p,
                                                        QUERY ? 0u : ie, hard, diffuse);
                else
                    Lo = bounce_lo<PP, TT>(a, tiles, W, T, lane, x, we, de, (uint32_t)p, QUERY ? 0u : ie, hard,
                                           diffuse);
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
}

template <class PP>
static hipError_t launch_mma(const RenderK &a, bool indirect, bool query, hipStream_t s) {
    const bool perlane = !query && a.s.n_dirs < 16;
    int n_cus = 0;
    const hipError_t ec = current_device_cus(n_cus);
    if (ec != hipSuccess) return ec;
    const int64_t ppw = query ? 64 : (64 >> a.s.g_shift);
    const int64_t items = (a.n + ppw - 1) / ppw;
    constexpr int wpb = PP::kThreads / 64;
    const int64_t want = (items + wpb - 1) / wpb;
    const int64_t cap = (int64_t)n_cus * 2;
    const unsigned blocks = (unsigned)(want < cap ? want : cap);
    const dim3 grid(blocks), block(PP::kThreads);
    const bool mis = (a.s.flags & 4u) != 0;
    if (query) {
        if (indirect) hipLaunchKernelGGL((k_render_mma<PP, true, true, false, false>), grid, block, 0, s, a, items);
        else hipLaunchKernelGGL((k_render_mma<PP, false, true, false, false>), grid, block, 0, s, a, items);
    } else if (perlane) {
        if (mis) {
            if (indirect) hipLaunchKernelGGL((k_render_mma<PP, true, false, true, true>), grid, block, 0, s, a, items);
            else hipLaunchKernelGGL((k_render_mma<PP, false, false, true, true>), grid, block, 0, s, a, items);
        } else {
            if (indirect) hipLaunchKernelGGL((k_render_mma<PP, true, false, false, true>), grid, block, 0, s, a, items);
            else hipLaunchKernelGGL((k_render_mma<PP, false, false, false, true>), grid, block, 0, s, a, items);
        }
    } else if (mis) {
        if (indirect) hipLaunchKernelGGL((k_render_mma<PP, true, false, true, false>), grid, block, 0, s, a, items);
        else hipLaunchKernelGGL((k_render_mma<PP, false, false, true, false>), grid, block, 0, s, a, items);
    } else {
        if (indirect) hipLaunchKernelGGL((k_render_mma<PP, true, false, false, false>), grid, block, 0, s, a, items);
        else hipLaunchKernelGGL((k_render_mma<PP, false, false, false, false>), grid, block, 0, s, a, items);
    }
    return hipGetLastError();
}

// The fenced tracer pays on grids whose finest resolution is moderate (finest
// 2048: the 800x800 frame at N = 128 34.6 -> 33.6 ms against the unfenced
// variant, N = 32 and 64 likewise) and costs on very fine ones (finest 131072,
// the paper's grid: 33.4 -> 39.1 ms), whatever the table size (2^17 .. 2^21
// entries per level measured), and at 256 or more directions per pixel, where
// a pixel's set-up is shared by four or more chunks (N = 256 65.1 against
// 65.6 ms, N = 512 122.8 against 126.0 ms).  The resolution switch sits
// between the two measured finest resolutions.
hipError_t launch_render_mixed(const RenderK &a, bool indirect, bool query, hipStream_t s) {
    const bool very_fine = a.g.L > 0 && a.g.resf[a.g.L - 1] > 16384.0f;
    const bool many_dirs = !query && a.s.n_dirs >= 256;
    return very_fine || many_dirs ? launch_mma<Bf16PathT<false>>(a, indirect, query, s)
                                  : launch_mma<Bf16PathT<true>>(a, indirect, query, s);
}

hipError_t launch_render_f32_mma(const RenderK &a, bool indirect, bool query, hipStream_t s) {
    return launch_mma<F32Path>(a, indirect, query, s);
}

}  // namespace hg
