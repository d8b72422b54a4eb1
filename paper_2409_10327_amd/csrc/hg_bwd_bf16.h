// hg_bwd_bf16.h -- the MLP part of the backward in BF16 on the matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation), for the mixed-precision
// distillation step (BF16 MLPs, FP16 tables, FP32 masters and gradients;
// paper Sec. 3.3).  Included by hg_backward.hip, whose kernel body calls it
// through the same interface as the FP32 MLP functions.
//
// A wave holds 64 samples; sample s = 16 nt + j is column j of N-tile nt and
// lane s's own query.  Forward: as the mixed renderer -- units as rows (four
// 16-row M-tiles), samples as columns, each layer's accumulators after ReLU
// and BF16 packing the next layer's B operand in place (units in the order
// unit_bf16), head rows replicated so that lane l keeps its own outputs.
// The packed activations stay in registers for the backward.
// Backward, per layer (o = outputs, i = inputs):
//   delta = mask(act) * W^T g      matrix cores, A = transposed-weight tiles,
//                                  B = the next layer's packed deltas in place
//   dW[o][i] = sum_s delta[o][s] act[i][s]   matrix cores with K = samples:
//                                  A and B read from LDS rows [unit][s'],
//                                  s' = 4 (s % 16) + s / 16 (a lane writes the
//                                  four samples it holds as one 8-byte store)
//   db[o] = sum_s delta[o][s]      FP32, a transposed butterfly over 16 lanes
// and d/d(features) = W0f^T delta1 goes back to lane = sample through LDS.
// Weight tiles (A operands, 8 BF16 per lane) are built once per call into the
// workspace by k_bwd_tiles and read from global memory (L2-resident).
#pragma once
#include "hg_bf16.h"

namespace hg {

// ---- weight tiles: index t, 64 lanes x 16 bytes each ----
enum : int {
    BT_IW0W = 0, BT_IW0F = 4, BT_IW1 = 8, BT_IW2 = 16, BT_IW2T = 18, BT_IW1T = 22, BT_IW0T = 30,  // tracer
    BT_BW0 = 34, BT_BW1 = 38, BT_BW2A = 46, BT_BW2B = 48, BT_BW2T = 50, BT_BW1T = 54, BT_BW0T = 62,  // decoder
    BT_N = 66
};

__device__ __forceinline__ uint32_t wraw(const void *W, int idx) { return static_cast<const uint16_t *>(W)[idx]; }

// Raw BF16 bits of element e of lane (i = row in the M-tile, g = lane group)
// of tile t (tracer 35 -> 64 -> 64 -> 2, decoder 32 -> 64 -> 64 -> 5).
__device__ __forceinline__ uint32_t btile_value(const MlpK &irt, const MlpK &brdf, int t, int i, int g, int e) {
    if (t < BT_IW0F) {  // tracer first layer, direction part: hi and lo halves
        if (g != 0 || e >= 6) return 0u;
        return wraw(irt.W0, (16 * (t - BT_IW0W) + i) * kNI + kNF + (e % 3));
    }
    if (t < BT_IW1) return wraw(irt.W0, (16 * (t - BT_IW0F) + i) * kNI + 8 * g + e);
    if (t < BT_IW2) {
        const int m = (t - BT_IW1) >> 1, s = (t - BT_IW1) & 1;
        return wraw(irt.W1, (16 * m + i) * kH + unit_bf16(s, g, e));
    }
    if (t < BT_IW2T) {
        const int s = t - BT_IW2, r = i & 3;
        return r < 2 ? wraw(irt.W2, r * kH + unit_bf16(s, g, e)) : 0u;
    }
    if (t < BT_IW1T) {  // W2^T: rows = units, K = outputs
        const int o = 8 * g + e;
        return o < 2 ? wraw(irt.W2, o * kH + 16 * (t - BT_IW2T) + i) : 0u;
    }
    if (t < BT_IW0T) {  // W1^T: rows = inputs (physical), K = outputs (chain order)
        const int m = (t - BT_IW1T) >> 1, s = (t - BT_IW1T) & 1;
        return wraw(irt.W1, unit_bf16(s, g, e) * kH + 16 * m + i);
    }
    if (t < BT_BW0) {  // W0f^T: rows = features, K = units (chain order)
        const int m = (t - BT_IW0T) >> 1, s = (t - BT_IW0T) & 1;
        return wraw(irt.W0, unit_bf16(s, g, e) * kNI + 16 * m + i);
    }
    if (t < BT_BW1) return wraw(brdf.W0, (16 * (t - BT_BW0) + i) * kNF + 8 * g + e);
    if (t < BT_BW2A) {
        const int m = (t - BT_BW1) >> 1, s = (t - BT_BW1) & 1;
        return wraw(brdf.W1, (16 * m + i) * kH + unit_bf16(s, g, e));
    }
    if (t < BT_BW2B) return wraw(brdf.W2, (i & 3) * kH + unit_bf16(t - BT_BW2A, g, e));
    if (t < BT_BW2T) return 4 + (i & 3) < 5 ? wraw(brdf.W2, (4 + (i & 3)) * kH + unit_bf16(t - BT_BW2B, g, e)) : 0u;
    if (t < BT_BW1T) {
        const int o = 8 * g + e;
        return o < 5 ? wraw(brdf.W2, o * kH + 16 * (t - BT_BW2T) + i) : 0u;
    }
    if (t < BT_BW0T) {
        const int m = (t - BT_BW1T) >> 1, s = (t - BT_BW1T) & 1;
        return wraw(brdf.W1, unit_bf16(s, g, e) * kH + 16 * m + i);
    }
    const int m = (t - BT_BW0T) >> 1, s = (t - BT_BW0T) & 1;
    return wraw(brdf.W0, unit_bf16(s, g, e) * kNF + 16 * m + i);
}

__global__ __launch_bounds__(256) void k_bwd_tiles(const MlpK irt, const MlpK brdf, uint4 *__restrict__ tiles) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= BT_N * 64) return;
    const int t = q >> 6, l = q & 63, i = l & 15, g = l >> 4;
    uint32_t w[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) w[p] = btile_value(irt, brdf, t, i, g, 2 * p) | (btile_value(irt, brdf, t, i, g, 2 * p + 1) << 16);
    tiles[q] = make_uint4(w[0], w[1], w[2], w[3]);
}

// ---- per-wave LDS ----
constexpr int kBRow = 72;  // BF16 per [unit][s'] row (144 bytes: 16-byte aligned reads)
constexpr int kDzRow = 36; // floats per row of the d/d(features) transpose (fits the D2 rows)
struct Bf16Lds {
    enum : int {
        XS = 0,                       // [64][4] uint4: a sample's 32 features
        OM = XS + 64 * 64,            // [64] uint4: direction hi/lo halves
        H1 = OM + 64 * 16,            // [64][kBRow] bf16: layer-1 activations
        H2 = H1 + 64 * kBRow * 2,     // [64][kBRow]: layer-2 activations, then layer-1 deltas
        D2 = H2 + 64 * kBRow * 2,     // [64][kBRow]: layer-2 deltas, then [64][kDzRow] floats
        ZT = D2 + 64 * kBRow * 2,     // [38][kBRow]: inputs by row (features, direction hi, lo)
        G = ZT + 38 * kBRow * 2,      // [5][kBRow]: output gradients by row
        GB = G + 5 * kBRow * 2,       // [64] uint4: a sample's output gradients
        BYTES = GB + 64 * 16
    };
};
static_assert(Bf16Lds::BYTES <= 40 * 1024, "four waves per CU");

struct Bf16State {
    uint4 p1[2][4], p2[2][4];  // packed activations of layers 1 and 2 [K-step][N-tile]
};

__device__ __forceinline__ f32x4 f4zero() { return f32x4{0.f, 0.f, 0.f, 0.f}; }
__device__ __forceinline__ f32x4 bias4(const float *b, int m, int g) {
    const float4 v = *reinterpret_cast<const float4 *>(b + 16 * m + 4 * g);
    return f32x4{v.x, v.y, v.z, v.w};
}
__device__ __forceinline__ f32x4 headb(const float *b, int nout, int base) {
    f32x4 r;
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] = (base + k < nout) ? b[base + k] : 0.0f;
    return r;
}
__device__ __forceinline__ uint32_t half_of(uint32_t w, int odd) { return odd ? (w >> 16) : (w & 0xffffu); }
__device__ __forceinline__ uint32_t word_of(const uint4 &v, int k) {
    return k == 0 ? v.x : (k == 1 ? v.y : (k == 2 ? v.z : v.w));
}
// ReLU mask of element e of a packed activation (zero or positive BF16)
__device__ __forceinline__ bool act_on(const uint4 &p, int e) { return half_of(word_of(p, e >> 1), e & 1) != 0u; }

// Packed chain [K-step][N-tile] -> rows [unit][s'] (unit_bf16 order of the
// chain; the lane's four N-tiles are s' = 4 j .. 4 j + 3).
__device__ __forceinline__ void store_chain(uint8_t *lds, int off, const uint4 (&c)[2][4], int g, int j) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int odd = e & 1, wk = e >> 1;
            const uint32_t lo = half_of(word_of(c[s][0], wk), odd) | (half_of(word_of(c[s][1], wk), odd) << 16);
            const uint32_t hi = half_of(word_of(c[s][2], wk), odd) | (half_of(word_of(c[s][3], wk), odd) << 16);
            *reinterpret_cast<uint2 *>(lds + off + (unit_bf16(s, g, e) * kBRow + 4 * j) * 2) = make_uint2(lo, hi);
        }
}
__device__ __forceinline__ uint4 row8(const uint8_t *lds, int off, int row, int col) {
    return *reinterpret_cast<const uint4 *>(lds + off + (row * kBRow + col) * 2);
}

// Sum of v[q] over the 16 lanes of a lane group, left on the lane whose
// index within the group is q (a transposed butterfly: 15 exchanges).
__device__ __forceinline__ float group_sum16(const float (&v)[16], int j) {
    float b8[8], b4[4], b2[2];
    const bool m8 = j & 8, m4 = j & 4, m2 = j & 2, m1 = j & 1;
#pragma unroll
    for (int i = 0; i < 8; ++i) b8[i] = (m8 ? v[i + 8] : v[i]) + __shfl_xor(m8 ? v[i] : v[i + 8], 8);
#pragma unroll
    for (int i = 0; i < 4; ++i) b4[i] = (m4 ? b8[i + 4] : b8[i]) + __shfl_xor(m4 ? b8[i] : b8[i + 4], 4);
#pragma unroll
    for (int i = 0; i < 2; ++i) b2[i] = (m2 ? b4[i + 2] : b4[i]) + __shfl_xor(m2 ? b4[i] : b4[i + 2], 2);
    return (m1 ? b2[1] : b2[0]) + __shfl_xor(m1 ? b2[0] : b2[1], 1);
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int k = 32; k >= 1; k >>= 1) v += __shfl_xor(v, k);
    return v;
}

struct Bf16Mlp {
    static constexpr int kLdsBytes = Bf16Lds::BYTES;
    typedef Bf16State State;
    // Forward of one MLP (W = 0 tracer, 1 decoder) for the wave's 64 samples;
    // new_x: the first kNF inputs (features) differ from the previous call's.
    template <int NIN, int NOUT, int W>
    static __device__ void fwd(const MlpK &m, const uint4 *__restrict__ tiles, uint8_t *lds, const float (&z)[NIN],
                               bool new_x, Bf16State &st, float (&out)[NOUT], int lane) {
        const int g = lane >> 4, j = lane & 15;
        constexpr int T0F = W == 0 ? BT_IW0F : BT_BW0, T1 = W == 0 ? BT_IW1 : BT_BW1;
        constexpr int T2 = W == 0 ? BT_IW2 : BT_BW2A;
        wave_sync();
        if (new_x) {
            uint4 *xs = reinterpret_cast<uint4 *>(lds + Bf16Lds::XS) + 4 * lane;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                xs[q] = make_uint4(pack_bf16(z[8 * q], z[8 * q + 1]), pack_bf16(z[8 * q + 2], z[8 * q + 3]),
                                   pack_bf16(z[8 * q + 4], z[8 * q + 5]), pack_bf16(z[8 * q + 6], z[8 * q + 7]));
        }
        if constexpr (W == 0) {
            const float wx = z[kNF], wy = z[kNF + 1], wz = z[kNF + 2];
            const __bf16 hx = (__bf16)wx, hy = (__bf16)wy, hz = (__bf16)wz;
            const float lx = wx - (float)hx, ly = wy - (float)hy, lz = wz - (float)hz;
            reinterpret_cast<uint4 *>(lds + Bf16Lds::OM)[lane] =
                make_uint4(pack_bf16((float)hx, (float)hy), pack_bf16((float)hz, lx), pack_bf16(ly, lz), 0u);
        }
        wave_sync();
        const uint4 *xs = reinterpret_cast<const uint4 *>(lds + Bf16Lds::XS);
        const uint4 *om = reinterpret_cast<const uint4 *>(lds + Bf16Lds::OM);
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const uint4 xb = xs[4 * (16 * nt + j) + g];
            f32x4 d[4];
#pragma unroll
            for (int mm = 0; mm < 4; ++mm) d[mm] = mfma_bf16(tiles[(T0F + mm) * 64 + lane], xb, bias4(m.b0, mm, g));
            if constexpr (W == 0) {
                const uint4 ob = om[16 * nt + j];
#pragma unroll
                for (int mm = 0; mm < 4; ++mm) d[mm] = mfma_bf16(tiles[(BT_IW0W + mm) * 64 + lane], ob, d[mm]);
            }
            st.p1[0][nt] = act_pack(d[0], d[1]);
            st.p1[1][nt] = act_pack(d[2], d[3]);
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            f32x4 e[4];
#pragma unroll
            for (int mm = 0; mm < 4; ++mm) {
                e[mm] = mfma_bf16(tiles[(T1 + 2 * mm) * 64 + lane], st.p1[0][nt], bias4(m.b1, mm, g));
                e[mm] = mfma_bf16(tiles[(T1 + 2 * mm + 1) * 64 + lane], st.p1[1][nt], e[mm]);
            }
            st.p2[0][nt] = act_pack(e[0], e[1]);
            st.p2[1][nt] = act_pack(e[2], e[3]);
            f32x4 o = mfma_bf16(tiles[T2 * 64 + lane], st.p2[0][nt], headb(m.b2, NOUT, 0));
            o = mfma_bf16(tiles[(T2 + 1) * 64 + lane], st.p2[1][nt], o);
            if (g == nt) {
#pragma unroll
                for (int r = 0; r < (NOUT < 4 ? NOUT : 4); ++r) out[r] = o[r];
            }
            if constexpr (NOUT > 4) {
                f32x4 o2 = mfma_bf16(tiles[BT_BW2B * 64 + lane], st.p2[0][nt], headb(m.b2, NOUT, 4));
                o2 = mfma_bf16(tiles[(BT_BW2B + 1) * 64 + lane], st.p2[1][nt], o2);
                if (g == nt) {
#pragma unroll
                    for (int r = 4; r < NOUT; ++r) out[r] = o2[r - 4];
                }
            }
        }
    }

    // Backward of the MLP evaluation just run by fwd (state st), for upstream
    // gradients gout of the lane's own sample: adds the parameter gradients
    // to gp = W0,b0,W1,b1,W2,b2 (FP32 atomics) and returns d/d(features) in
    // dz.  new_x: the features differ from those of the previous backward.
    template <int NIN, int NOUT, int W>
    static __device__ void bwd(const MlpK &, const uint4 *__restrict__ tiles, uint8_t *lds, float *const *gp,
                               const float (&z)[NIN], const float (&gout)[NOUT], bool new_x, Bf16State &st,
                               float (&dz)[kNF], int lane) {
        const int g = lane >> 4, j = lane & 15;
        const int sp = 4 * j + g;  // column s' of the lane's own sample
        constexpr int TW2T = W == 0 ? BT_IW2T : BT_BW2T, TW1T = W == 0 ? BT_IW1T : BT_BW1T;
        constexpr int TW0T = W == 0 ? BT_IW0T : BT_BW0T;
        constexpr int NZ = W == 0 ? kNF + 6 : kNF;  // rows of ZT in use (features, direction hi and lo)
        uint16_t *zt = reinterpret_cast<uint16_t *>(lds + Bf16Lds::ZT);
        uint16_t *gr = reinterpret_cast<uint16_t *>(lds + Bf16Lds::G);
        wave_sync();
        // ---- rows: output gradients, inputs, layer activations
        {
            uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
            for (int o = 0; o < NOUT; ++o) {
                const uint32_t b = pack_bf16(gout[o], 0.0f) & 0xffffu;
                w[o >> 1] |= (o & 1) ? (b << 16) : b;
                gr[o * kBRow + sp] = (uint16_t)b;
            }
            reinterpret_cast<uint4 *>(lds + Bf16Lds::GB)[lane] = make_uint4(w[0], w[1], w[2], w[3]);
        }
        if (new_x) {
#pragma unroll
            for (int k = 0; k < kNF; ++k) zt[k * kBRow + sp] = (uint16_t)(pack_bf16(z[k], 0.0f) & 0xffffu);
        }
        if constexpr (W == 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const __bf16 hi = (__bf16)z[kNF + c];
                const float lo = z[kNF + c] - (float)hi;
                zt[(kNF + c) * kBRow + sp] = __builtin_bit_cast(uint16_t, hi);
                zt[(kNF + 3 + c) * kBRow + sp] = (uint16_t)(pack_bf16(lo, 0.0f) & 0xffffu);
            }
        }
        store_chain(lds, Bf16Lds::H2, st.p2, g, j);
        store_chain(lds, Bf16Lds::H1, st.p1, g, j);
        // ---- layer 2: out = W2 h2 + b2
#pragma unroll
        for (int o = 0; o < NOUT; ++o) {
            const float sb = wave_sum(gout[o]);
            if (lane == o) atomic_addf(gp[5] + o, sb);
        }
        wave_sync();
#pragma unroll
        for (int nu = 0; nu < 4; ++nu) {
            f32x4 acc = f4zero();
#pragma unroll
            for (int kt = 0; kt < 2; ++kt) {
                const uint4 av = j < NOUT ? row8(lds, Bf16Lds::G, j, 8 * g + 32 * kt) : make_uint4(0u, 0u, 0u, 0u);
                acc = mfma_bf16(av, row8(lds, Bf16Lds::H2, 16 * nu + j, 8 * g + 32 * kt), acc);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int o = 4 * g + r;
                if (o < NOUT) atomic_addf(gp[4] + o * kH + 16 * nu + j, acc[r]);
            }
        }
        // delta2 = mask(h2) * W2^T g (rows = units, N-tiles = samples)
        uint4 q2[2][4];
        {
            const uint4 *gb = reinterpret_cast<const uint4 *>(lds + Bf16Lds::GB);
            float db[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) db[k] = 0.0f;
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const uint4 bg = g == 0 ? gb[16 * nt + j] : make_uint4(0u, 0u, 0u, 0u);
                f32x4 t[4];
#pragma unroll
                for (int mm = 0; mm < 4; ++mm) {
                    t[mm] = mfma_bf16(tiles[(TW2T + mm) * 64 + lane], bg, f4zero());
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        t[mm][r] = act_on(st.p2[mm >> 1][nt], 4 * (mm & 1) + r) ? t[mm][r] : 0.0f;
                        db[4 * mm + r] += t[mm][r];
                    }
                }
                q2[0][nt] = make_uint4(pack_bf16(t[0][0], t[0][1]), pack_bf16(t[0][2], t[0][3]),
                                       pack_bf16(t[1][0], t[1][1]), pack_bf16(t[1][2], t[1][3]));
                q2[1][nt] = make_uint4(pack_bf16(t[2][0], t[2][1]), pack_bf16(t[2][2], t[2][3]),
                                       pack_bf16(t[3][0], t[3][1]), pack_bf16(t[3][2], t[3][3]));
            }
            const float s = group_sum16(db, j);  // unit 16 (j / 4) + 4 g + j % 4
            atomic_addf(gp[3] + 16 * (j >> 2) + 4 * g + (j & 3), s);
        }
        store_chain(lds, Bf16Lds::D2, q2, g, j);
        wave_sync();
        // ---- layer 1: dW1[o][i] = sum_s delta2[o][s] h1[i][s]
#pragma unroll 1
        for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                f32x4 acc = f4zero();
#pragma unroll
                for (int kt = 0; kt < 2; ++kt)
                    acc = mfma_bf16(row8(lds, Bf16Lds::D2, 16 * mt + j, 8 * g + 32 * kt),
                                    row8(lds, Bf16Lds::H1, 16 * nt + j, 8 * g + 32 * kt), acc);
#pragma unroll
                for (int r = 0; r < 4; ++r) atomic_addf(gp[2] + (16 * mt + 4 * g + r) * kH + 16 * nt + j, acc[r]);
            }
        }
        // delta1 = mask(h1) * W1^T delta2
        uint4 q1[2][4];
        {
            float db[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) db[k] = 0.0f;
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                f32x4 t[4];
#pragma unroll
                for (int mm = 0; mm < 4; ++mm) {
                    t[mm] = mfma_bf16(tiles[(TW1T + 2 * mm) * 64 + lane], q2[0][nt], f4zero());
                    t[mm] = mfma_bf16(tiles[(TW1T + 2 * mm + 1) * 64 + lane], q2[1][nt], t[mm]);
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        t[mm][r] = act_on(st.p1[mm >> 1][nt], 4 * (mm & 1) + r) ? t[mm][r] : 0.0f;
                        db[4 * mm + r] += t[mm][r];
                    }
                }
                q1[0][nt] = make_uint4(pack_bf16(t[0][0], t[0][1]), pack_bf16(t[0][2], t[0][3]),
                                       pack_bf16(t[1][0], t[1][1]), pack_bf16(t[1][2], t[1][3]));
                q1[1][nt] = make_uint4(pack_bf16(t[2][0], t[2][1]), pack_bf16(t[2][2], t[2][3]),
                                       pack_bf16(t[3][0], t[3][1]), pack_bf16(t[3][2], t[3][3]));
            }
            const float s = group_sum16(db, j);
            atomic_addf(gp[1] + 16 * (j >> 2) + 4 * g + (j & 3), s);
        }
        wave_sync();  // H2 (layer-2 activations) read above: free now
        store_chain(lds, Bf16Lds::H2, q1, g, j);
        wave_sync();
        // ---- layer 0: dW0[o][k] = sum_s delta1[o][s] z[k][s]
        constexpr int NKT = (NZ + 15) / 16;
#pragma unroll 1
        for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
            for (int nk = 0; nk < NKT; ++nk) {
                f32x4 acc = f4zero();
#pragma unroll
                for (int kt = 0; kt < 2; ++kt) {
                    // rows past the NZ in use read as zero (the ZT rows stop at NZ)
                    const uint4 bz = 16 * nk + j < NZ ? row8(lds, Bf16Lds::ZT, 16 * nk + j, 8 * g + 32 * kt)
                                                      : make_uint4(0u, 0u, 0u, 0u);
                    acc = mfma_bf16(row8(lds, Bf16Lds::H2, 16 * mt + j, 8 * g + 32 * kt), bz, acc);
                }
                if (nk < 2) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) atomic_addf(gp[0] + (16 * mt + 4 * g + r) * NIN + 16 * nk + j, acc[r]);
                } else {
                    // direction columns: hi (rows 32..34) + lo (rows 35..37)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const float v = acc[r] + __shfl_down(acc[r], 3, 16);
                        if (j < 3) atomic_addf(gp[0] + (16 * mt + 4 * g + r) * NIN + kNF + j, v);
                    }
                }
            }
        }
        // d/d(features) = W0f^T delta1 (rows = features, N-tiles = samples)
        float *dzt = reinterpret_cast<float *>(lds + Bf16Lds::D2);  // delta2 rows: read above
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int mm = 0; mm < 2; ++mm) {
                f32x4 t = mfma_bf16(tiles[(TW0T + 2 * mm) * 64 + lane], q1[0][nt], f4zero());
                t = mfma_bf16(tiles[(TW0T + 2 * mm + 1) * 64 + lane], q1[1][nt], t);
                *reinterpret_cast<float4 *>(dzt + (16 * nt + j) * kDzRow + 16 * mm + 4 * g) =
                    make_float4(t[0], t[1], t[2], t[3]);
            }
        wave_sync();
#pragma unroll
        for (int k = 0; k < kNF; k += 2) {
            const float2 v = *reinterpret_cast<const float2 *>(dzt + lane * kDzRow + k);
            dz[k] = v.x;
            dz[k + 1] = v.y;
        }
    }
};

}  // namespace hg
