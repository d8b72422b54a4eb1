// hg_backward.hip -- hand-written backward of query mode (distillation).
//
// One query per lane.  Every activation of the recursive bounce is
// recomputed here; nothing is stored by the forward.  Weight gradients of
// the two MLPs are reduced over the 64 queries of a wave from LDS (on the
// matrix cores for the 64-output layers) and then added to global memory
// with FP32 atomics; table gradients are scattered with FP32 atomics
// through the trilinear weights, summed first over the lanes of a wave that
// share a cell (coarse levels).
#include <hipcub/hipcub.hpp>


#include "hg_device.h"
#include "hg_launch.h"

namespace hg {

constexpr int kDelStride = 68;  // del[s][k]: 16-byte aligned rows for broadcast reads

// Replicated MLP-gradient accumulators.  Every wave adds the weight
// gradients of its 64 samples into one of kWRep copies of
// [tracer W0, b0, W1, b1, W2, b2 | decoder W0, b0, W1, b1, W2, b2], picked by
// its block index, instead of into the caller's arrays: with one copy all
// waves add into the same 13k addresses and those atomics queue behind each
// other (the backward at 2^18 queries, 128 copies against one: BF16 MLPs
// 3.9 against 5.2 ms, FP32 MLPs 3.56 against 3.66 ms, with FP16 tables 3.54
// against 3.79 ms).  k_zero_wrep clears the copies first and k_reduce_wrep
// adds their sum to the caller's arrays afterwards.
constexpr int kWRep = 128;
constexpr int kRepSize[12] = {kH * kNI, kH, kH * kH, kH, 2 * kH, 2, kH * kNF, kH, kH * kH, kH, 5 * kH, 5};
constexpr int rep_off(int k) { return k == 0 ? 0 : rep_off(k - 1) + kRepSize[k - 1]; }
constexpr int kRepTotal = rep_off(12);
constexpr int kRepStride = (kRepTotal + 255) / 256 * 256;  // floats per copy
struct GradArrays {
    float *p[12];  // tracer W0..b2, decoder W0..b2
};
// Per-wave LDS of the FP32 MLP backward: two buffers, each of which holds
// in turn an activation layout ([unit][kHS]) or delta rows
// ([sample][kDelStride]), and the upstream-gradient rows of the output layer
// (at most 8 per sample): 36 KB, so four waves fit in a CU.
constexpr int kBufF = kHBuf > 64 * kDelStride ? kHBuf : 64 * kDelStride;
constexpr int kGoStride = 8;
constexpr int kWaveLds = 2 * kBufF + 64 * kGoStride;
constexpr int kBwdThreads = 64;

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void atomic_addf(float *p, float v) { unsafeAtomicAdd(p, v); }

// dW[o][col] += sum_s del[s][o] * act[col][s] over the wave's 64 samples
// (act in the [unit][kHS] layout of the forward, del in [sample][DS]);
// lane == col owns column col.  Bias gradients db[o] = sum_s del[s][o] are
// added by lane == o.
template <int NOUT, int NIN, int DS>
__device__ __forceinline__ void reduce_layer(const float *act, const float *del, float *gW, float *gb, int lane) {
    constexpr int CH = NOUT < 16 ? NOUT : 16;
    if (lane < NIN) {
#pragma unroll 1
        for (int ob = 0; ob < NOUT; ob += CH) {
            float acc[CH];
#pragma unroll
            for (int k = 0; k < CH; ++k) acc[k] = 0.0f;
#pragma unroll 4
            for (int s = 0; s < 64; ++s) {
                const float a = act[lane * kHS + s];
                const float *row = del + s * DS + ob;
                if constexpr (CH % 4 == 0) {
#pragma unroll
                    for (int k = 0; k < CH; k += 4) {
                        const float4 d4 = *reinterpret_cast<const float4 *>(row + k);
                        acc[k] = fmaf(d4.x, a, acc[k]);
                        acc[k + 1] = fmaf(d4.y, a, acc[k + 1]);
                        acc[k + 2] = fmaf(d4.z, a, acc[k + 2]);
                        acc[k + 3] = fmaf(d4.w, a, acc[k + 3]);
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < CH; ++k) acc[k] = fmaf(row[k], a, acc[k]);
                }
            }
#pragma unroll
            for (int k = 0; k < CH; ++k) atomic_addf(gW + (size_t)(ob + k) * NIN + lane, acc[k]);
        }
    }
    if (lane < NOUT) {
        float acc = 0.0f;
#pragma unroll 8
        for (int s = 0; s < 64; ++s) acc += del[s * DS + lane];
        atomic_addf(gb + lane, acc);
    }
}

typedef float f32x16 __attribute__((ext_vector_type(16)));

// dW[o][i] += sum_s del[s][o] * act[i][s] for the 64 outputs of a hidden
// layer, as v_mfma_f32_32x32x2f32 products: M = outputs (two 32-row tiles),
// N = inputs (32-column tiles), K = the wave's 64 samples, with
// A[o][s] = del[s][o] and B[s][i] = act[i][s] read straight from the LDS
// layouts above (lanes read contiguous floats of a del row, and act columns
// at the odd stride kHS: no bank conflicts).  Lane l then holds
// dW[32 mo + 8 (r / 4) + 4 (l / 32) + r % 4][32 ni + l % 32] in accumulator
// register r; columns past NIN (stale rows of the act buffer) are dropped.
// Bias gradients db[o] = sum_s del[s][o] are added by lane == o.
template <int NIN>
__device__ __forceinline__ void reduce_layer_mma(const float *act, const float *del, float *gW, float *gb, int lane) {
    constexpr int NT = (NIN + 31) / 32;
    const int h = lane >> 5, j = lane & 31;
    // one 32-row output tile at a time (register pressure)
#pragma unroll 1
    for (int mo = 0; mo < 2; ++mo) {
        f32x16 acc[NT];
#pragma unroll
        for (int ni = 0; ni < NT; ++ni)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[ni][r] = 0.0f;
#pragma unroll 8
        for (int st = 0; st < 32; ++st) {
            const int smp = 2 * st + h;
            const float av = del[smp * kDelStride + 32 * mo + j];
#pragma unroll
            for (int ni = 0; ni < NT; ++ni)
                acc[ni] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, act[(32 * ni + j) * kHS + smp], acc[ni], 0, 0, 0);
        }
#pragma unroll
        for (int ni = 0; ni < NT; ++ni) {
            const int i = 32 * ni + j;
            if (i < NIN) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int o = 32 * mo + 8 * (r >> 2) + 4 * h + (r & 3);
                    atomic_addf(gW + (size_t)o * NIN + i, acc[ni][r]);
                }
            }
        }
    }
    float accb = 0.0f;
#pragma unroll 8
    for (int smp = 0; smp < 64; ++smp) accb += del[smp * kDelStride + lane];
    atomic_addf(gb + lane, accb);
}

// T[s][i] = sum_k W[k][i] del[s][k] for i < NI (W row-major with row length
// ldw, 64 rows k): the input gradient of a 64-output layer for the wave's 64
// samples, as v_mfma_f32_32x32x2f32 products with M = inputs, N = samples,
// K = outputs: A[i][k] = W[k][i] from global memory (cached), B[k][s] =
// del[s][k] from LDS.  Lane l holds T[32 mi + 8 (r / 4) + 4 (l / 32) + r % 4]
// [32 ns + l % 32] in register r and writes it to the transpose buffer T
// (row stride kHS), from which each lane then reads its own sample's row.
template <int NI>
__device__ __forceinline__ void wt_times_del(const float *W, int ldw, const float *del, float *T, int lane) {
    constexpr int MT = (NI + 31) / 32;
    const int h = lane >> 5, j = lane & 31;
#pragma unroll 1
    for (int ns = 0; ns < 2; ++ns) {
        f32x16 acc[MT];
#pragma unroll
        for (int mi = 0; mi < MT; ++mi)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[mi][r] = 0.0f;
#pragma unroll 8
        for (int st = 0; st < 32; ++st) {
            const int k = 2 * st + h;
            const float bv = del[(32 * ns + j) * kDelStride + k];
#pragma unroll
            for (int mi = 0; mi < MT; ++mi) {
                const int i = 32 * mi + j;
                const float av = i < NI ? W[k * ldw + i] : 0.0f;
                acc[mi] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc[mi], 0, 0, 0);
            }
        }
#pragma unroll
        for (int mi = 0; mi < MT; ++mi)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int i = 32 * mi + 8 * (r >> 2) + 4 * h + (r & 3);
                if (i < NI) T[(32 * ns + j) * kHS + i] = acc[mi][r];
            }
    }
}

// Forward of one MLP evaluation for the wave's 64 samples on the matrix
// cores (v_mfma_f32_32x32x2f32; M = units, N = samples, K = inputs), leaving
// the ReLU activations in the [unit][sample] layouts the backward reads
// (h1buf, h2buf; they may alias when h1 is not needed).  The inputs z go
// through h2buf first (B[k][s] = z_s[k]); the first layer's accumulators,
// after ReLU, are the second layer's B operand in place (K-step st takes
// register st % 16 of M-tile st / 16, i.e. unit 32 (st / 16) + 8 ((st % 16) / 4)
// + 4 (l / 32) + st % 4, so W1 is read with its columns in that order).
// Weights come from global memory (cached).  Returns h2 of the lane's own
// sample in h and the outputs in out (vector ALU, one row per output).
template <int NIN, int NOUT>
__device__ __forceinline__ void mlp_fwd_mma(const MlpK &m, const float (&z)[NIN], float *h1buf, float *h2buf, int lane,
                                            float (&h)[kH], float (&out)[NOUT]) {
    const float *W0 = static_cast<const float *>(m.W0);
    const float *W1 = static_cast<const float *>(m.W1);
    const int hh = lane >> 5, j = lane & 31;
    wave_sync();
#pragma unroll
    for (int i = 0; i < NIN; ++i) h2buf[i * kHS + lane] = z[i];
    wave_sync();
    constexpr int KS0 = (NIN + 1) / 2;
#pragma unroll 1
    for (int ns = 0; ns < 2; ++ns) {
        const int col = 32 * ns + j;
        f32x16 a0[2], a1[2];
#pragma unroll
        for (int mo = 0; mo < 2; ++mo)
#pragma unroll
            for (int r = 0; r < 16; ++r) a0[mo][r] = m.b0[32 * mo + 8 * (r >> 2) + 4 * hh + (r & 3)];
#pragma unroll
        for (int st = 0; st < KS0; ++st) {
            // operands of eight K-steps at a time in flight (register pressure)
            if ((st & 7) == 0) __builtin_amdgcn_sched_barrier(0);
            const int k = 2 * st + hh;
            const float bv = k < NIN ? h2buf[k * kHS + col] : 0.0f;
#pragma unroll
            for (int mo = 0; mo < 2; ++mo) {
                const float av = k < NIN ? W0[(32 * mo + j) * NIN + k] : 0.0f;
                a0[mo] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, a0[mo], 0, 0, 0);
            }
        }
#pragma unroll
        for (int mo = 0; mo < 2; ++mo)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                a0[mo][r] = fmaxf(a0[mo][r], 0.0f);
                h1buf[(32 * mo + 8 * (r >> 2) + 4 * hh + (r & 3)) * kHS + col] = a0[mo][r];
            }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int mo = 0; mo < 2; ++mo)
#pragma unroll
            for (int r = 0; r < 16; ++r) a1[mo][r] = m.b1[32 * mo + 8 * (r >> 2) + 4 * hh + (r & 3)];
#pragma unroll
        for (int st = 0; st < 32; ++st) {
            if ((st & 7) == 0) __builtin_amdgcn_sched_barrier(0);
            const int u = 32 * (st >> 4) + 8 * ((st & 15) >> 2) + 4 * hh + (st & 3);
            const float bv = a0[st >> 4][st & 15];
#pragma unroll
            for (int mo = 0; mo < 2; ++mo)
                a1[mo] = __builtin_amdgcn_mfma_f32_32x32x2f32(W1[(32 * mo + j) * kH + u], bv, a1[mo], 0, 0, 0);
        }
#pragma unroll
        for (int mo = 0; mo < 2; ++mo)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                h2buf[(32 * mo + 8 * (r >> 2) + 4 * hh + (r & 3)) * kHS + col] = fmaxf(a1[mo][r], 0.0f);
    }
    wave_sync();
#pragma unroll
    for (int k = 0; k < kH; ++k) h[k] = h2buf[k * kHS + lane];
    const WPtr<float> W2(m.W2);
    const BPtr b2(m.b2);
#pragma unroll
    for (int o = 0; o < NOUT; ++o) {
        float acc = b2[o];
#pragma unroll
        for (int k = 0; k < kH; ++k) acc = fmaf(W2[o * kH + k], h[k], acc);
        out[o] = acc;
    }
}

__device__ __forceinline__ void store_row(float *del, int lane, const float (&v)[kH]) {
#pragma unroll
    for (int k = 0; k < kH; k += 4)
        *reinterpret_cast<float4 *>(del + lane * kDelStride + k) = make_float4(v[k], v[k + 1], v[k + 2], v[k + 3]);
}

// Backward of one MLP evaluation for every lane of the wave (all lanes call
// it together), given the forward just run by mlp_fwd_mma with h1 in bufA
// and h2 in bufB and h = the lane's own h2: accumulates parameter gradients
// (gp = W0,b0,W1,b1,W2,b2) and returns d/d(input) for the first kNF inputs.
// The delta rows, the transposed products and the restaged inputs take
// their turns in the two buffers as those fall free (h1 is needed after its
// weight gradient only as the lane's ReLU mask, kept as 64 bits), so a wave
// needs two buffers rather than three.
template <int NIN, int NOUT>
__device__ __forceinline__ void mlp_bwd_stored(const MlpK &m, float *const *gp, const float (&z)[NIN],
                                               const float (&gout)[NOUT], float (&h)[kH], float *bufA, float *bufB,
                                               float *go, int lane, float (&dz)[kNF]) {
    // ---- layer 2: out = W2 h2 + b2 (upstream gradient rows in go)
#pragma unroll
    for (int k = 0; k < NOUT; ++k) go[lane * kGoStride + k] = gout[k];
    wave_sync();
    reduce_layer<NOUT, kH, kGoStride>(bufB, go, gp[4], gp[5], lane);
    {
        const WPtr<float> W2(m.W2);
#pragma unroll
        for (int k = 0; k < kH; ++k) {
            float s = 0.0f;
#pragma unroll
            for (int oo = 0; oo < NOUT; ++oo) s = fmaf(W2[oo * kH + k], gout[oo], s);
            h[k] = h[k] > 0.0f ? s : 0.0f;  // h now holds d/d(pre-activation 2)
        }
    }
    wave_sync();  // h2 (bufB) read by every lane
    // ---- layer 1: pre2 = W1 h1 + b1; delta2 rows into bufB
    store_row(bufB, lane, h);
    wave_sync();
    reduce_layer_mma<kH>(bufA, bufB, gp[2], gp[3], lane);
    uint64_t m1 = 0;  // ReLU mask of the lane's own h1
#pragma unroll
    for (int j = 0; j < kH; ++j) m1 |= (uint64_t)(bufA[j * kHS + lane] > 0.0f) << j;
    wave_sync();  // h1 (bufA) read by every lane
    // d/d(pre-activation 1) = mask(h1) * W1^T delta2, transposed through bufA
    wt_times_del<kH>(static_cast<const float *>(m.W1), kH, bufB, bufA, lane);
    wave_sync();
#pragma unroll
    for (int j = 0; j < kH; ++j) h[j] = ((m1 >> j) & 1u) ? bufA[lane * kHS + j] : 0.0f;
    wave_sync();
    // ---- layer 0: pre1 = W0 z + b0; delta1 rows into bufB, z into bufA
    store_row(bufB, lane, h);
#pragma unroll
    for (int i = 0; i < NIN; ++i) bufA[i * kHS + lane] = z[i];
    wave_sync();
    reduce_layer_mma<NIN>(bufA, bufB, gp[0], gp[1], lane);
    wave_sync();
    // d/d(features) = W0f^T delta1, transposed through bufA
    wt_times_del<kNF>(static_cast<const float *>(m.W0), NIN, bufB, bufA, lane);
    wave_sync();
#pragma unroll
    for (int i = 0; i < kNF; ++i) dz[i] = bufA[lane * kHS + i];
}

// The FP32 MLP functions behind the interface the kernel body calls (the
// BF16 ones are in hg_bwd_bf16.h): per-wave LDS = two buffers and the
// upstream-gradient rows; the state kept from forward to backward is the
// lane's own last hidden layer.
struct F32Mlp {
    static constexpr int kLdsBytes = kWaveLds * (int)sizeof(float);
    struct State {
        float h[kH];
    };
    template <int NIN, int NOUT, int W>
    static __device__ void fwd(const MlpK &m, const uint4 *, uint8_t *lds, const float (&z)[NIN], bool, State &st,
                               float (&out)[NOUT], int lane) {
        float *h1 = reinterpret_cast<float *>(lds);
        mlp_fwd_mma<NIN, NOUT>(m, z, h1, h1 + kBufF, lane, st.h, out);
    }
    template <int NIN, int NOUT, int W>
    static __device__ void bwd(const MlpK &m, const uint4 *, uint8_t *lds, float *const *gp, const float (&z)[NIN],
                               const float (&gout)[NOUT], bool, State &st, float (&dz)[kNF], int lane) {
        float *h1 = reinterpret_cast<float *>(lds);
        mlp_bwd_stored<NIN, NOUT>(m, gp, z, gout, st.h, h1, h1 + kBufF, h1 + 2 * kBufF, lane, dz);
    }
};

// Adds this lane's 16 contributions v[2k + f] (corner k, feature f) into the
// table gradient of one level (gl = level base, idx = corner entries of the
// lane's cell c).  Lanes of the wave that share a cell are summed first, so
// at coarse levels -- where a wave's queries fall into a handful of cells --
// one atomic per value and cell reaches memory instead of one per lane (the
// per-address serialisation of those atomics dominated the backward).  A
// group's 16 values are summed over the wave with a transposed butterfly
// (17 lane exchanges) that leaves value q = lane >> 2 on lanes with
// lane % 4 == 0.  Once the next group has a single lane (fine levels), the
// remaining lanes add directly.  All lanes of the wave call this together.
__device__ __forceinline__ void scatter_cell(float *gl, const uint32_t (&idx)[8], const uint32_t (&c)[3],
                                             const float (&v)[16], bool live, int lane) {
    uint64_t pending = __ballot(live);
    while (pending) {
        const int leader = __builtin_ctzll(pending);  // wave-uniform
        const uint32_t l0 = __builtin_amdgcn_readlane(c[0], leader);
        const uint32_t l1 = __builtin_amdgcn_readlane(c[1], leader);
        const uint32_t l2 = __builtin_amdgcn_readlane(c[2], leader);
        const bool same = ((pending >> lane) & 1ull) && c[0] == l0 && c[1] == l1 && c[2] == l2;
        const uint64_t grp = __ballot(same);
        if (__popcll(grp) < 2) break;
        float b8[8], b4[4], b2[2];
        const bool h32 = lane & 32, h16 = lane & 16, h8 = lane & 8, h4 = lane & 4;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const float lo = same ? v[i] : 0.0f, hi = same ? v[i + 8] : 0.0f;
            b8[i] = (h32 ? hi : lo) + __shfl_xor(h32 ? lo : hi, 32);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) b4[i] = (h16 ? b8[i + 4] : b8[i]) + __shfl_xor(h16 ? b8[i] : b8[i + 4], 16);
#pragma unroll
        for (int i = 0; i < 2; ++i) b2[i] = (h8 ? b4[i + 2] : b4[i]) + __shfl_xor(h8 ? b4[i] : b4[i + 2], 8);
        float b1 = (h4 ? b2[1] : b2[0]) + __shfl_xor(h4 ? b2[0] : b2[1], 4);
        b1 += __shfl_xor(b1, 2);
        b1 += __shfl_xor(b1, 1);
        const int q = lane >> 2;  // value index held by this lane group
        uint32_t e = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint32_t ik = __builtin_amdgcn_readlane(idx[k], leader);
            e = (q >> 1) == k ? ik : e;
        }
        if ((lane & 3) == 0) atomic_addf(gl + 2 * (size_t)e + (q & 1), b1);
        pending &= ~grp;
    }
    if ((pending >> lane) & 1ull) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            atomic_addf(gl + 2 * (size_t)idx[k], v[2 * k]);
            atomic_addf(gl + 2 * (size_t)idx[k] + 1, v[2 * k + 1]);
        }
    }
}

// d/dx of the encoding at x contracted with gf (table reads only; the table
// gradient is scattered later, in spatial order, by k_scatter_records).
template <typename TT>
__device__ __forceinline__ float3 encode_dx(const GridK &g, float x, float y, float z, const float (&gf)[kNF]) {
    float u[3];
    bool in[3];
    pos_to_u(g, x, y, z, u, in);
    float gxx = 0.f, gxy = 0.f, gxz = 0.f;
#pragma unroll
    for (int l = 0; l < kL; ++l) {
        if (l >= (int)g.L) break;  // wave-uniform
        uint32_t c[3];
        float w[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) cell_of(u[d], g.resf[l], g.nm1f[l], c[d], w[d]);
        const size_t base = (size_t)l << g.log2T;
        uint32_t idx[8];
        corner_idx(g, l, c, idx);
        const float w0[3] = {1.0f - w[0], 1.0f - w[1], 1.0f - w[2]};
        const float sc = g.dscale[l];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int dx = k & 1, dy = (k >> 1) & 1, dzz = (k >> 2) & 1;
            const float fx = dx ? w[0] : w0[0], fy = dy ? w[1] : w0[1], fz = dzz ? w[2] : w0[2];
            const float2 te = TabLoad<TT>::ld(g.table, base + idx[k]);
            const float ge = (gf[2 * l] * te.x + gf[2 * l + 1] * te.y) * sc;
            gxx = fmaf(ge, (dx ? 1.0f : -1.0f) * fy * fz, gxx);
            gxy = fmaf(ge, fx * (dy ? 1.0f : -1.0f) * fz, gxy);
            gxz = fmaf(ge, fx * fy * (dzz ? 1.0f : -1.0f), gxz);
        }
    }
    return make_float3(in[0] ? gxx : 0.f, in[1] ? gxy : 0.f, in[2] ? gxz : 0.f);
}

// 30-bit Morton code of x over the grid's box, 10 bits per axis
__device__ __forceinline__ uint32_t spread10(uint32_t v) {
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    return (v | (v << 2)) & 0x09249249u;
}
__device__ __forceinline__ uint32_t morton30(const GridK &g, float3 x) {
    const float q[3] = {clamp01((x.x - g.lo) * g.inv_ext), clamp01((x.y - g.lo) * g.inv_ext),
                        clamp01((x.z - g.lo) * g.inv_ext)};
    uint32_t k = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) k |= spread10(min((uint32_t)(q[d] * 1024.0f), 1023u)) << d;
    return k;
}

// One record of the table scatter: the point, its feature gradient, the
// Morton key and the record's own index.
__device__ __forceinline__ void put_record(const BounceWs &ws, const GridK &g, int64_t rec, float3 x,
                                           const float (&gf)[kNF]) {
    ws.xb[rec] = make_float4(x.x, x.y, x.z, 0.0f);
    float4 *dst = reinterpret_cast<float4 *>(ws.gf + (size_t)rec * kNF);
#pragma unroll
    for (int i = 0; i < kNF; i += 4) dst[i / 4] = make_float4(gf[i], gf[i + 1], gf[i + 2], gf[i + 3]);
    ws.key[rec] = morton30(g, x);
    ws.id[rec] = (uint32_t)rec;
}

}  // namespace hg

#include "hg_bwd_bf16.h"

namespace hg {

// pi f_r and its derivatives with respect to albedo (per channel),
// roughness and metallic.
struct BrdfGrad {
    float3 c, dca, dcr, dcm;
};
__device__ __forceinline__ BrdfGrad pi_brdf_grad(float3 n, float3 v, float3 l, float3 a, float r, float m, float f0,
                                                 bool diffuse) {
    BrdfGrad o;
    const float3 z = make_float3(0.f, 0.f, 0.f);
    if (!(dot3(n, l) > 0.0f)) {
        o.c = o.dca = o.dcr = o.dcm = z;
        return o;
    }
    if (diffuse) {
        o.c = a;
        o.dca = make_float3(1.f, 1.f, 1.f);
        o.dcr = o.dcm = z;
        return o;
    }
    const BrdfTerms t = brdf_terms(n, v, l, r, true);
    const float s = kPi * t.D * t.Vis;
    const float q = 1.0f - t.P;
    const float dsr = kPi * (t.dD_da2 * t.Vis + t.D * t.dVis_da2) * 4.0f * r * r * r;
    const float av[3] = {a.x, a.y, a.z};
    float c[3], da[3], dr[3], dm[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float F0 = f0 * (1.0f - m) + av[k] * m;
        const float F = F0 * q + t.P;
        c[k] = (1.0f - m) * av[k] + s * F;
        da[k] = (1.0f - m) + s * q * m;
        dm[k] = -av[k] + s * q * (av[k] - f0);
        dr[k] = F * dsr;
    }
    o.c = make_float3(c[0], c[1], c[2]);
    o.dca = make_float3(da[0], da[1], da[2]);
    o.dcr = make_float3(dr[0], dr[1], dr[2]);
    o.dcm = make_float3(dm[0], dm[1], dm[2]);
    return o;
}

// One query per lane; MLP = F32Mlp (FP32 matrix cores) or Bf16Mlp (BF16
// matrix cores, FP32 accumulation).  The features last staged for the MLPs
// (flags "new_x" below) are f(x) after the first tracer call, f(x') from the
// decoder at x' through the bounce, and f(x) again for the final tracer.
template <typename TT, bool INDIRECT, typename MLP>
__global__ __launch_bounds__(kBwdThreads) void k_backward(const BwdK a) {
    extern __shared__ float lds_f[];
    const int lane = threadIdx.x & 63;
    uint8_t *lds = reinterpret_cast<uint8_t *>(lds_f) + (threadIdx.x >> 6) * MLP::kLdsBytes;
    typename MLP::State st;
    // this wave's MLP weight gradients go to one of the replicated accumulators
    float *gi[6], *gb[6];
    {
        float *rep = a.ws.wrep + (size_t)(blockIdx.x & (kWRep - 1)) * kRepStride;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            gi[k] = rep + rep_off(k);
            gb[k] = rep + rep_off(6 + k);
        }
    }
    const int64_t p_raw = a.p_begin + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const RenderK &r = a.r;
    const bool live = p_raw < a.p_end;
    const int64_t p = live ? p_raw : a.p_end - 1;
    constexpr int R = INDIRECT ? 2 : 1;  // records per query: x (and x')
    const float3 x = make_float3(r.pos[3 * p], r.pos[3 * p + 1], r.pos[3 * p + 2]);
    const float3 w = make_float3(r.dir[3 * p], r.dir[3 * p + 1], r.dir[3 * p + 2]);
    float3 G = make_float3(0.f, 0.f, 0.f);
    float gV = 0.f, gd = 0.f;
    if (live) {
        G = make_float3(a.g_rgb[3 * p], a.g_rgb[3 * p + 1], a.g_rgb[3 * p + 2]);
        gV = a.g_vis[p];
        gd = a.g_dep[p];
    }
    // z = [features, direction] of the current tracer call; zf aliases its
    // features (f(x), then f(x') through the bounce, then f(x) again,
    // recomputed rather than kept live across the bounce)
    float z[kNI], o[2];
    float(&zf)[kNF] = *reinterpret_cast<float(*)[kNF]>(z);
    encode<TT>(r.g, x.x, x.y, x.z, zf);
    z[kNF] = w.x; z[kNF + 1] = w.y; z[kNF + 2] = w.z;
    MLP::template fwd<kNI, 2, 0>(r.irt, a.tiles, lds, z, true, st, o, lane);
    const float V = sigmoidf_(o[0]);
    const float o1p = o[1];
    const float sp = softplusf_(o1p);
    const float d = fminf(sp, 1.0f);
    const float t = fmaf(r.t_span, d, r.t_near);
    const float3 Le = env_lookup(r.env, w.x, w.y, w.z);
    float3 gxb = make_float3(0.f, 0.f, 0.f);
    float dz[kNF];
    if constexpr (INDIRECT) {
        const float3 xb = make_float3(fmaf(t, w.x, x.x), fmaf(t, w.y, x.y), fmaf(t, w.z, x.z));
        encode<TT>(r.g, xb.x, xb.y, xb.z, zf);
        float ob[5];
        MLP::template fwd<kNF, 5, 1>(r.brdf, a.tiles, lds, zf, true, st, ob, lane);
        const float3 ab = make_float3(sigmoidf_(ob[0]), sigmoidf_(ob[1]), sigmoidf_(ob[2]));
        const float s3 = sigmoidf_(ob[3]);
        const float rb = 0.09f + 0.91f * s3;
        const float mb = sigmoidf_(ob[4]);
        const float3 nb = make_float3(-w.x, -w.y, -w.z);
        const Frame fr = make_frame(nb);
        const bool diffuse = (r.s.flags & 1u) != 0;
        const uint32_t N2 = r.s.n_dirs2;
        const float invN2 = 1.0f / (float)N2;
        // one pass over the secondary directions: the forward of tracer j gives
        // V'_j for L'_o and, since d L / d V'_j needs only (1 - V) G, its
        // backward runs on the activations just computed
        float Lx = 0.f, Ly = 0.f, Lz = 0.f;
        const float3 gLo = make_float3((1.0f - V) * G.x, (1.0f - V) * G.y, (1.0f - V) * G.z);
        float gfb[kNF];
#pragma unroll
        for (int i = 0; i < kNF; ++i) gfb[i] = 0.f;
        float gax = 0.f, gay = 0.f, gaz = 0.f, gr = 0.f, gm = 0.f;
        uint4 words = make_uint4(0, 0, 0, 0);
        for (uint32_t j = 0; j < N2; ++j) {
            if ((j & 3u) == 0) words = philox4x32_10((uint32_t)p, 0u, j >> 2, 1u, r.s.key0, r.s.key1);
            const float3 wj = sample_dir(pick4(words, j), j, r.s.nb2_shift, r.s.inv_na2, r.s.inv_nb2, fr);
            z[kNF] = wj.x; z[kNF + 1] = wj.y; z[kNF + 2] = wj.z;
            MLP::template fwd<kNI, 2, 0>(r.irt, a.tiles, lds, z, false, st, o, lane);
            const float vj = sigmoidf_(o[0]);
            const float3 Ej = env_lookup(r.env, wj.x, wj.y, wj.z);
            const BrdfGrad bg = pi_brdf_grad(nb, nb, wj, ab, rb, mb, r.f0, diffuse);
            Lx = fmaf(bg.c.x * vj, Ej.x, Lx);
            Ly = fmaf(bg.c.y * vj, Ej.y, Ly);
            Lz = fmaf(bg.c.z * vj, Ej.z, Lz);
            const float gvj = (gLo.x * bg.c.x * Ej.x + gLo.y * bg.c.y * Ej.y + gLo.z * bg.c.z * Ej.z) * invN2;
            const float go[2] = {gvj * vj * (1.0f - vj), 0.0f};
            MLP::template bwd<kNI, 2, 0>(r.irt, a.tiles, lds, gi, z, go, j == 0, st, dz, lane);
#pragma unroll
            for (int i = 0; i < kNF; ++i) gfb[i] += dz[i];
            const float kx = gLo.x * vj * Ej.x * invN2, ky = gLo.y * vj * Ej.y * invN2, kz = gLo.z * vj * Ej.z * invN2;
            gax = fmaf(kx, bg.dca.x, gax);
            gay = fmaf(ky, bg.dca.y, gay);
            gaz = fmaf(kz, bg.dca.z, gaz);
            gr += kx * bg.dcr.x + ky * bg.dcr.y + kz * bg.dcr.z;
            gm += kx * bg.dcm.x + ky * bg.dcm.y + kz * bg.dcm.z;
        }
        Lx *= invN2; Ly *= invN2; Lz *= invN2;
        gV += G.x * (Le.x - Lx) + G.y * (Le.y - Ly) + G.z * (Le.z - Lz);
        const float gob[5] = {gax * ab.x * (1.0f - ab.x), gay * ab.y * (1.0f - ab.y), gaz * ab.z * (1.0f - ab.z),
                              gr * 0.91f * s3 * (1.0f - s3), gm * mb * (1.0f - mb)};
        MLP::template fwd<kNF, 5, 1>(r.brdf, a.tiles, lds, zf, false, st, ob, lane);
        MLP::template bwd<kNF, 5, 1>(r.brdf, a.tiles, lds, gb, zf, gob, false, st, dz, lane);
#pragma unroll
        for (int i = 0; i < kNF; ++i) gfb[i] += dz[i];
        // the table gradient at x' is scattered by k_scatter_records after the
        // queries are sorted by x'; here only d/dx' (for the depth head)
        gxb = encode_dx<TT>(r.g, xb.x, xb.y, xb.z, gfb);
        if (live) put_record(a.ws, r.g, R * p + 1, xb, gfb);
        const float gt = gxb.x * w.x + gxb.y * w.y + gxb.z * w.z;
        gd = fmaf(r.t_span, gt, gd);
    } else {
        gV += G.x * Le.x + G.y * Le.y + G.z * Le.z;
    }
    // tracer at (f(x), w)
    if constexpr (INDIRECT) encode<TT>(r.g, x.x, x.y, x.z, zf);
    z[kNF] = w.x; z[kNF + 1] = w.y; z[kNF + 2] = w.z;
    const float go2[2] = {gV * V * (1.0f - V), sp < 1.0f ? gd * sigmoidf_(o1p) : 0.0f};
    MLP::template fwd<kNI, 2, 0>(r.irt, a.tiles, lds, z, INDIRECT, st, o, lane);
    MLP::template bwd<kNI, 2, 0>(r.irt, a.tiles, lds, gi, z, go2, true, st, dz, lane);
    // the table gradient at x is scattered by k_scatter_records too
    float3 gx = make_float3(0.f, 0.f, 0.f);
    if (a.g_pos) gx = encode_dx<TT>(r.g, x.x, x.y, x.z, dz);
    if (live) put_record(a.ws, r.g, R * p, x, dz);
    if (live && a.g_pos) {
        a.g_pos[3 * p] = gx.x + gxb.x;
        a.g_pos[3 * p + 1] = gx.y + gxb.y;
        a.g_pos[3 * p + 2] = gx.z + gxb.z;
    }
}

// Table-gradient scatter, one lane per record in the order of the Morton
// keys of the record points, so that a wave's 64 points are neighbours.  Per
// level the wave sums its 64 x 8 corner contributions by 64-byte line of the
// gradient table (8 entries of two FP32 features) in a wave-private LDS hash
// table (open addressing on the line, LDS compare-and-swap on the key, LDS
// float adds into the entry's two words), lists the lines it touched and
// adds each line with one instruction of 16 lanes, i.e. one atomic request.
// The global FP32 atomic add costs the same per request whatever the
// addresses (a request being the lanes of one instruction that fall in one
// line), so the number of lines is the cost: a cell's two corners along x
// share a line in 7 of 8 cases on dense and hashed levels alike (the hash's
// x factor is 1), and neighbouring points share cells and lines; at the
// benchmark batch about 17 requests per record remain of the 256 adds.
// The table has 256 slots (18 KB of LDS per wave, so that two waves share
// each SIMD): a level whose lanes form at most 32 runs inserts the run sums
// in one pass (at most 256 entries), any other level in two passes of 32
// lanes, each pass listed and flushed before the next.
constexpr int kScatterThreads = 64;       // one wave per block
constexpr int kPassLanes = 32;            // lanes inserting in one pass of a level
constexpr int kLineSlots = kPassLanes * 8;  // >= the corner entries of one pass, so probing ends
constexpr int kSlotBits = 8;
static_assert((1 << kSlotBits) == kLineSlots, "slot count");
constexpr uint32_t kEmptySlot = 0xffffffffu;
template <typename TT>
__global__ __launch_bounds__(kScatterThreads) void k_scatter_records(const GridK g, const uint32_t *__restrict__ id,
                                                                     const float4 *__restrict__ xb,
                                                                     const float *__restrict__ gf,
                                                                     float *__restrict__ g_table, int64_t n) {
    __shared__ uint32_t K[kLineSlots];        // line index (entry / 8) or empty
    __shared__ float V[kLineSlots][16];       // the line's 8 entries x 2 features
    __shared__ uint32_t list[kLineSlots];     // occupied (line << 9 | slot) of this pass
    const int lane = threadIdx.x;
    for (int q = lane; q < kLineSlots; q += 64) {
        K[q] = kEmptySlot;
#pragma unroll
        for (int w = 0; w < 16; ++w) V[q][w] = 0.0f;
    }
    const int64_t i = (int64_t)blockIdx.x * kScatterThreads + lane;
    const bool live = i < n;
    const uint32_t p = id[live ? i : n - 1];
    const float4 x = xb[p];
    float gfp[kNF];
    const float4 *src = reinterpret_cast<const float4 *>(gf + (size_t)p * kNF);
#pragma unroll
    for (int k = 0; k < kNF; k += 4) {
        const float4 v = src[k / 4];
        gfp[k] = v.x;
        gfp[k + 1] = v.y;
        gfp[k + 2] = v.z;
        gfp[k + 3] = v.w;
    }
    float u[3];
    bool in[3];
    pos_to_u(g, x.x, x.y, x.z, u, in);
    wave_sync();
    const uint64_t below = (1ull << lane) - 1ull;
#pragma unroll 1
    for (int l = 0; l < kL; ++l) {
        if (l >= (int)g.L) break;  // wave-uniform
        uint32_t c[3];
        float w[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) cell_of(u[d], g.resf[l], g.nm1f[l], c[d], w[d]);
        uint32_t idx[8];
        corner_idx(g, l, c, idx);
        const float w0[3] = {1.0f - w[0], 1.0f - w[1], 1.0f - w[2]};
        float vx[8], vy[8];  // the lane's contributions to the two features of its eight corners
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const float wt = live ? ((k & 1) ? w[0] : w0[0]) * (((k >> 1) & 1) ? w[1] : w0[1]) *
                                        (((k >> 2) & 1) ? w[2] : w0[2])
                                  : 0.0f;
            vx[k] = wt * gfp[2 * l];
            vy[k] = wt * gfp[2 * l + 1];
        }
        // Lanes whose points lie in one cell of this level form runs (the
        // records are in Morton order).  When the wave has few runs (the
        // coarse levels), each run's sums are formed across its lanes first
        // and only its first lane inserts them: LDS atomics of many lanes on
        // one word are serialised.
        // (every lane takes part in every shuffle: a lane left out of one
        // leaves undefined values for the lanes that read from it)
        const uint32_t p0 = __shfl_up(c[0], 1), p1 = __shfl_up(c[1], 1), p2 = __shfl_up(c[2], 1);
        const bool head = lane == 0 || p0 != c[0] || p1 != c[1] || p2 != c[2];
        const uint64_t heads = __ballot(head);
        bool ins = live;
        const bool few = __popcll(heads) <= 32;  // wave-uniform
        if (few) {
            const int seg = __popcll(heads & (below | (1ull << lane)));
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int sn = __shfl_down(seg, off);
                const bool same = lane + off < 64 && sn == seg;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const float tx = __shfl_down(vx[k], off), ty = __shfl_down(vy[k], off);
                    vx[k] += same ? tx : 0.0f;
                    vy[k] += same ? ty : 0.0f;
                }
            }
            ins = head;
        }
#pragma unroll 1
        for (int pass = 0; pass < (few ? 1 : 64 / kPassLanes); ++pass) {
            if (ins && (few || lane / kPassLanes == pass)) {
                // the first probe of the eight corners in flight together,
                // then the collisions resolved one by one; at most 256
                // distinct lines in 256 slots, so every probe ends
                uint32_t h[8], prev[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    h[k] = ((idx[k] >> 3) * 2654435761u) >> (32 - kSlotBits);
                    prev[k] = atomicCAS(&K[h[k]], kEmptySlot, idx[k] >> 3);
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const uint32_t ln = idx[k] >> 3;
                    while (prev[k] != kEmptySlot && prev[k] != ln) {
                        h[k] = (h[k] + 1) & (kLineSlots - 1);
                        prev[k] = atomicCAS(&K[h[k]], kEmptySlot, ln);
                    }
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    atomicAdd(&V[h[k]][2 * (idx[k] & 7u)], vx[k]);
                    atomicAdd(&V[h[k]][2 * (idx[k] & 7u) + 1], vy[k]);
                }
            }
            wave_sync();
            // list the occupied slots (a ballot per 64 slots)
            int cnt = 0;
#pragma unroll
            for (int r = 0; r < kLineSlots / 64; ++r) {
                const int q = 64 * r + lane;
                const uint32_t ln = K[q];
                const bool occ = ln != kEmptySlot;
                const uint64_t m = __ballot(occ);
                if (occ) list[cnt + __popcll(m & below)] = (ln << 9) | (uint32_t)q;
                cnt += __popcll(m);
            }
            wave_sync();
            // one instruction of 16 lanes per line: lane 16 j + w adds word w
            // of the j-th listed line (four lines per instruction, four
            // instructions with their LDS reads issued together) and clears
            // it for the next pass
            float *gl = g_table + 2 * ((size_t)l << g.log2T);
            const int wd = lane & 15;
            for (int j0 = lane >> 4; j0 < cnt; j0 += 16) {
                uint32_t it[4];
                float v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) it[u] = j0 + 4 * u < cnt ? list[j0 + 4 * u] : kEmptySlot;
#pragma unroll
                for (int u = 0; u < 4; ++u) v[u] = it[u] != kEmptySlot ? V[it[u] & (kLineSlots - 1)][wd] : 0.0f;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (it[u] != kEmptySlot) {
                        const uint32_t q = it[u] & (kLineSlots - 1);
                        atomic_addf(gl + 16 * (size_t)(it[u] >> 9) + wd, v[u]);
                        V[q][wd] = 0.0f;
                        if (wd == 0) K[q] = kEmptySlot;
                    }
                }
            }
            wave_sync();
        }
    }
}

__global__ __launch_bounds__(256) void k_zero_wrep(float4 *__restrict__ p, int64_t n4) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n4) p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// one thread per parameter: the sum of its kWRep copies, added to the
// caller's gradient array (the only writer of that element in this call)
__global__ __launch_bounds__(256) void k_reduce_wrep(const float *__restrict__ rep, GradArrays out) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= kRepTotal) return;
    float s = 0.0f;
#pragma unroll 8
    for (int r = 0; r < kWRep; ++r) s += rep[(size_t)r * kRepStride + q];
    int k = 0;
#pragma unroll
    for (int t = 1; t < 12; ++t) k = q >= rep_off(t) ? t : k;
    int o = 0;
#pragma unroll
    for (int t = 0; t < 12; ++t) o = k == t ? rep_off(t) : o;
    out.p[k][q - o] += s;
}

hipError_t backward_sort_bytes(int64_t records, size_t &bytes) {
    bytes = 0;
    return hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const uint32_t *)nullptr, (uint32_t *)nullptr,
                                              (const uint32_t *)nullptr, (uint32_t *)nullptr, (int)records, 0, 30,
                                              (hipStream_t)0);
}

// The per-query kernel, then the sort of its records by Morton key and the
// table scatter, all on the caller's stream.  (A pipeline over chunks of
// queries with the scatter on a second stream measured slower: the two
// kernels slowed each other down and the scatter side became the critical
// path, 7.5 against 7.0 ms at 2^18 queries.)
template <typename TT, typename MLP>
static void launch_k_backward(const BwdK &c, bool indirect, unsigned blocks, hipStream_t s) {
    const size_t lds = (size_t)(kBwdThreads / 64) * MLP::kLdsBytes;
    if (indirect) hipLaunchKernelGGL((k_backward<TT, true, MLP>), dim3(blocks), dim3(kBwdThreads), lds, s, c);
    else hipLaunchKernelGGL((k_backward<TT, false, MLP>), dim3(blocks), dim3(kBwdThreads), lds, s, c);
}

hipError_t launch_backward(const BwdK &a, bool f16, bool bf16_mlp, bool indirect, hipStream_t s) {
    const int64_t n = a.r.n;
    const int R = indirect ? 2 : 1;
    BwdK c = a;
    c.p_begin = 0;
    c.p_end = n;
    c.tiles = a.ws.tiles;
    const unsigned blocks = (unsigned)((n + kBwdThreads - 1) / kBwdThreads);
    const int64_t n4 = (int64_t)kWRep * kRepStride / 4;
    hipLaunchKernelGGL(k_zero_wrep, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<float4 *>(a.ws.wrep), n4);
    if (bf16_mlp) {
        hipLaunchKernelGGL(k_bwd_tiles, dim3((BT_N * 64 + 255) / 256), dim3(256), 0, s, a.r.irt, a.r.brdf, a.ws.tiles);
        launch_k_backward<__half, Bf16Mlp>(c, indirect, blocks, s);
    } else if (f16) {
        launch_k_backward<__half, F32Mlp>(c, indirect, blocks, s);
    } else {
        launch_k_backward<float, F32Mlp>(c, indirect, blocks, s);
    }
    GradArrays ga;
    for (int k = 0; k < 6; ++k) {
        ga.p[k] = a.gi[k];
        ga.p[6 + k] = a.gb[k];
    }
    hipLaunchKernelGGL(k_reduce_wrep, dim3((kRepTotal + 255) / 256), dim3(256), 0, s, a.ws.wrep, ga);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t rn = R * n;
    size_t tmp = a.ws.sort_tmp_bytes;
    e = hipcub::DeviceRadixSort::SortPairs(a.ws.sort_tmp, tmp, a.ws.key, a.ws.key_sorted, a.ws.id, a.ws.id_sorted,
                                           (int)rn, 0, 30, s);
    if (e != hipSuccess) return e;
    const unsigned sb = (unsigned)((rn + kScatterThreads - 1) / kScatterThreads);
    if (f16)
        hipLaunchKernelGGL(k_scatter_records<__half>, dim3(sb), dim3(kScatterThreads), 0, s, a.r.g, a.ws.id_sorted,
                           a.ws.xb, a.ws.gf, a.g_table, rn);
    else
        hipLaunchKernelGGL(k_scatter_records<float>, dim3(sb), dim3(kScatterThreads), 0, s, a.r.g, a.ws.id_sorted,
                           a.ws.xb, a.ws.gf, a.g_table, rn);
    return hipGetLastError();
}

size_t backward_ws_layout(int64_t n, int R, size_t sort_tmp_bytes, void *base, BounceWs *ws) {
    auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
    const size_t un = (size_t)n * (size_t)R;
    size_t off = 0;
    const size_t o_xb = off;
    off += al(un * sizeof(float4));
    const size_t o_gf = off;
    off += al(un * kNF * sizeof(float));
    size_t o_k[4];
    for (int k = 0; k < 4; ++k) {
        o_k[k] = off;
        off += al(un * sizeof(uint32_t));
    }
    const size_t o_tmp = off;
    off += al(sort_tmp_bytes);
    const size_t o_tiles = off;
    off += al((size_t)BT_N * 64 * sizeof(uint4));
    const size_t o_wrep = off;
    off += al((size_t)kWRep * kRepStride * sizeof(float));
    if (ws && base) {
        char *b = static_cast<char *>(base);
        ws->xb = reinterpret_cast<float4 *>(b + o_xb);
        ws->gf = reinterpret_cast<float *>(b + o_gf);
        ws->key = reinterpret_cast<uint32_t *>(b + o_k[0]);
        ws->id = reinterpret_cast<uint32_t *>(b + o_k[1]);
        ws->key_sorted = reinterpret_cast<uint32_t *>(b + o_k[2]);
        ws->id_sorted = reinterpret_cast<uint32_t *>(b + o_k[3]);
        ws->sort_tmp = b + o_tmp;
        ws->sort_tmp_bytes = sort_tmp_bytes;
        ws->tiles = reinterpret_cast<uint4 *>(b + o_tiles);
        ws->wrep = reinterpret_cast<float *>(b + o_wrep);
    }
    return off;
}

}  // namespace hg
