// hg_device.h -- device building blocks of the gfx950 hash-grid renderer.
//
// Included by the .hip translation units only.  Every routine here works on
// one query per lane (64-wide wavefronts); the matrix-core MLPs live in
// hg_render_mfma.hip and hg_backward.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace hg {

constexpr int kL = 16;          // levels
constexpr int kF = 2;           // features per level
constexpr int kNF = kL * kF;    // feature width (32)
constexpr int kH = 64;          // hidden width
constexpr int kNI = kNF + 3;    // tracer input width (35)
constexpr float kPi = 3.14159265358979323846f;

// --------------------------------------------------------------------------
// Kernel-side descriptors (passed by value as kernel arguments).
// --------------------------------------------------------------------------
struct GridK {
    const void *table;      // [L][T][F] FP32 or FP16
    uint32_t L;             // levels (<= kL); feature slots of levels >= L are zero
    uint32_t log2T, Tmask;
    float lo, inv_ext;      // u = (x - lo) * inv_ext, inv_ext = 2^-k
    float resf[kL];         // N_l as float (exact)
    float nm1f[kL];         // N_l - 1 as float
    float dscale[kL];       // N_l / extent (d u N_l / dx)
    uint32_t stride[kL];    // N_l + 1 (dense levels)
    uint32_t dense_mask;    // bit l set: level l is dense
};

struct MlpK {
    const void *W0; const float *b0;
    const void *W1; const float *b1;
    const void *W2; const float *b2;
};

struct EnvK {
    const float *rgb;  // [H][W][3]
    int32_t H, W;
    float Hf, Wf;
    // light-sampling distribution (MIS): per row (cos theta_top,
    // 1 - cos theta_top, 1 + cos theta_bottom, cos span) [H]; marginal CDF
    // [H+1] and conditional CDFs [H][W+1] as (hi, lo) pairs; densities [H][W]
    const float4 *rows;
    const float2 *marg, *cond;
    const float *dens;
};

struct SampK {
    uint32_t n_dirs, n_dirs2;
    uint32_t key0, key1, flags;
    uint32_t nb_shift, nb2_shift;   // log2 of the azimuth strata count
    float inv_na, inv_nb, inv_na2, inv_nb2;
    uint32_t g_shift;               // log2(min(n_dirs, 64)) (shade reduction)
    uint32_t m_half, nbm_shift;     // MIS: M = n_dirs / 2 samples per strategy, their strata
    float inv_nam, inv_nbm;
};

struct RenderK {
    GridK g;
    MlpK brdf, irt;
    EnvK env;
    SampK s;
    float t_near, t_span, f0;
    int32_t brdf_out;       // 5, or 8 with the decoder's normal head
    const float *pos, *nrm, *wo, *dir;
    float *rgb, *vis, *depth;
    int64_t n;
};

// --------------------------------------------------------------------------
// Small helpers
// --------------------------------------------------------------------------
__device__ __forceinline__ float clamp01(float u) { return fminf(fmaxf(u, 0.0f), 1.0f); }
// Reciprocal by the hardware instruction (v_rcp_f32, 1 ulp) where a quotient
// feeds further arithmetic: a correctly rounded division is about ten
// instructions on this ISA.
__device__ __forceinline__ float rcpf_(float x) { return __builtin_amdgcn_rcpf(x); }
// Square root by the hardware instruction (v_sqrt_f32, 1 ulp; the correctly
// rounded form adds a scaling, two residual fmas and selects, about fourteen
// instructions); every argument here is zero or a normal number.
__device__ __forceinline__ float sqrtf_(float x) { return __builtin_amdgcn_sqrtf(x); }
// sin(2 pi x) and cos(2 pi x) for x in [0, 1) revolutions by the hardware
// instructions (v_sin_f32 / v_cos_f32 take revolutions): measured on an
// MI355X over 2^20 bin centres of [0, 1), the largest error is 1.24e-7 (about
// two ulp of 1; sincospif: 5.1e-8, at about thirty instructions).
__device__ __forceinline__ void sincos2pi_(float x, float &s, float &c) {
    s = __builtin_amdgcn_sinf(x);
    c = __builtin_amdgcn_cosf(x);
}
__device__ __forceinline__ float sigmoidf_(float z) { return rcpf_(1.0f + __expf(-z)); }
// log(1 + y) for y in [0, 1] from log(1 + y) = 2 atanh(s), s = y / (2 + y)
// in [0, 1/3]: s from the hardware reciprocal plus one residual correction
// (the rounding of 2 + y recovered exactly, Sterbenz), then 2 s + the odd
// series of atanh to s^15 (truncation below 2e-9 relative), all in single
// precision: within 2.1e-7 relative (mean 0.5 ulp) when emulated exactly
// (the device library's log1pf takes the exponent through double precision).
__device__ __forceinline__ float log1p01_(float y) {
#pragma clang fp contract(off)
    const float d = 2.0f + y;
    const float ed = y - (d - 2.0f);  // (2 + y) - d, exact
    const float rc = rcpf_(d);
    const float s0 = y * rc;
    float r = fmaf(-s0, d, y);
    r = fmaf(-s0, ed, r);
    const float s = fmaf(r, rc, s0);
    const float s2 = s * s;
    float q = 2.0f / 15.0f;
    q = fmaf(q, s2, 2.0f / 13.0f);
    q = fmaf(q, s2, 2.0f / 11.0f);
    q = fmaf(q, s2, 2.0f / 9.0f);
    q = fmaf(q, s2, 2.0f / 7.0f);
    q = fmaf(q, s2, 2.0f / 5.0f);
    q = fmaf(q, s2, 2.0f / 3.0f);
    return fmaf(2.0f, s, (s * s2) * q);
}
__device__ __forceinline__ float softplusf_(float z) { return fmaxf(z, 0.0f) + log1p01_(__expf(-fabsf(z))); }

// Weights are read through constant-address-space pointers so that the
// wave-uniform reads become scalar loads.  The pointer is passed through an
// empty asm statement at every MLP evaluation: this keeps the compiler from
// hoisting thousands of loop-invariant weight loads out of the bounce loop.
typedef __attribute__((address_space(4))) const float *cf32_p;
typedef __attribute__((address_space(4))) const uint32_t *cu32_p;

__device__ __forceinline__ uint64_t opaque64(const void *p) {
    uint64_t v = reinterpret_cast<uint64_t>(p);
    asm volatile("" : "+s"(v));
    return v;
}

template <typename T> struct WPtr;
template <> struct WPtr<float> {
    cf32_p p;
    __device__ __forceinline__ explicit WPtr(const void *q) : p((cf32_p)opaque64(q)) {}
    __device__ __forceinline__ float operator[](int i) const { return p[i]; }
};
// BF16 stored as raw 16-bit patterns; read as 32-bit pairs.
template <> struct WPtr<uint16_t> {
    cu32_p p;
    __device__ __forceinline__ explicit WPtr(const void *q) : p((cu32_p)opaque64(q)) {}
    __device__ __forceinline__ float operator[](int i) const {
        const uint32_t w = p[i >> 1];
        return __uint_as_float((i & 1) ? (w & 0xffff0000u) : (w << 16));
    }
};
struct BPtr {
    cf32_p p;
    __device__ __forceinline__ explicit BPtr(const float *q) : p((cf32_p)opaque64(q)) {}
    __device__ __forceinline__ float operator[](int i) const { return p[i]; }
};

// --------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64-bit
// products with the round multipliers, key bumped by the Weyl constants.
// --------------------------------------------------------------------------
// OPAQUE_KEY: the (wave-uniform) key is made opaque at the call, so that its
// schedule of 20 round keys is recomputed by scalar adds there instead of
// being hoisted out of the loops.  The two-wave FP32 render kernel, short of
// scalar registers, otherwise reloads the hoisted schedule from vector-register
// lanes (800x800 frame 79.9 -> 78.8 ms with it); every other kernel measured
// faster with the hoisted schedule.
template <bool OPAQUE_KEY = false>
__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1) {
    if (OPAQUE_KEY) asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return make_uint4(c0, c1, c2, c3);
}

// Word k % 4 of a Philox block: a two-level select on the bits of k (no
// branch; k may differ between lanes).
__device__ __forceinline__ uint32_t pick4(const uint4 &w, uint32_t k) {
    const bool b0 = (k & 1u) != 0, b1 = (k & 2u) != 0;
    const uint32_t lo = b0 ? w.y : w.x, hi = b0 ? w.w : w.z;
    return b1 ? hi : lo;
}

// Orthonormal basis about a unit normal (Duff et al., JCGT 2017).
struct Frame { float3 t, b, n; };
__device__ __forceinline__ Frame make_frame(float3 n) {
    const float sgn = copysignf(1.0f, n.z);
    const float a = -1.0f / (sgn + n.z);
    const float bb = n.x * n.y * a;
    Frame f;
    f.t = make_float3(1.0f + sgn * n.x * n.x * a, sgn * bb, -sgn * n.x);
    f.b = make_float3(bb, sgn + n.y * n.y * a, -n.y);
    f.n = n;
    return f;
}

// Stratified cosine-weighted direction for sample k of an N = n_a x n_b
// stratification; `word` holds two 16-bit uniforms (bin centres).
__device__ __forceinline__ float3 sample_dir(uint32_t word, uint32_t k, uint32_t nb_shift,
                                             float inv_na, float inv_nb, const Frame &fr) {
    const float u1 = ((float)(word & 0xffffu) + 0.5f) * (1.0f / 65536.0f);
    const float u2 = ((float)(word >> 16) + 0.5f) * (1.0f / 65536.0f);
    const uint32_t a = k >> nb_shift;
    const uint32_t b = k & ((1u << nb_shift) - 1u);
    const float s1 = ((float)a + u1) * inv_na;
    const float s2 = ((float)b + u2) * inv_nb;
    const float r = sqrtf_(s1);
    float sn, cs;
    sincos2pi_(s2, sn, cs);
    const float lx = r * cs, ly = r * sn, lz = sqrtf_(1.0f - s1);
    return make_float3(lx * fr.t.x + ly * fr.b.x + lz * fr.n.x,
                       lx * fr.t.y + ly * fr.b.y + lz * fr.n.y,
                       lx * fr.t.z + ly * fr.b.z + lz * fr.n.z);
}

// --------------------------------------------------------------------------
// Hash-grid index stage.  The cell is floor of the exact product u*N.  The
// rounded product p = fl(u N) can only cross an integer by rounding up onto
// it.  With fl = floor(p), q = fl(u N - fl) (one fma) lies in (-1, 1) and has
// the sign of u N - fl, so fl + floor(q) is the exact floor, with no compare.
// After the clamp to N - 1, w = fl(u N - fl) is the fractional position with
// one rounding (p - fl is exact and p plus the product's error is u N).
// --------------------------------------------------------------------------
__device__ __forceinline__ void cell_of(float u, float Nf, float nm1f, uint32_t &c, float &w) {
    // no contraction: p must be the rounded product
#pragma clang fp contract(off)
    const float p = u * Nf;
    float fl = floorf(p);
    fl += floorf(fmaf(u, Nf, -fl));
    fl = fminf(fl, nm1f);
    c = (uint32_t)fl;
    w = fmaf(u, Nf, -fl);
}
// The same cell and weight with the product's error e = fl(u N - p) formed
// first and the case p integral, e < 0 taken by a compare and select
// (w = (p - fl) + e).  The two-wave FP32 bounce encoder measured faster with
// this form (82.4 against 82.9 ms for the 800x800 frame), every other encoder
// with the one above.
__device__ __forceinline__ void cell_of_sel(float u, float Nf, float nm1f, uint32_t &c, float &w) {
#pragma clang fp contract(off)
    const float p = u * Nf;
    const float e = fmaf(u, Nf, -p);
    float fl = floorf(p);
    fl = (fl == p && e < 0.0f) ? fl - 1.0f : fl;
    fl = fminf(fl, nm1f);
    c = (uint32_t)fl;
    w = (p - fl) + e;
}

__device__ __forceinline__ uint32_t vidx(const GridK &g, int l, uint32_t x, uint32_t y, uint32_t z) {
    if ((g.dense_mask >> l) & 1u) {
        const uint32_t s = g.stride[l];
        return x + s * (y + s * z);
    }
    return (x ^ (y * 2654435761u) ^ (z * 805459861u)) & g.Tmask;
}

// Table entry loads.  `lvl` is the wave-uniform base of one level and the
// entry offset is a 32-bit byte offset, so the loads use the scalar-base +
// 32-bit vector-offset addressing form (one VGPR per address).
template <typename TT> struct TabLoad;
template <> struct TabLoad<float> {
    static __device__ __forceinline__ const void *level(const void *t, int l, uint32_t log2T) {
        return static_cast<const char *>(t) + ((size_t)l << (log2T + 3));
    }
    static __device__ __forceinline__ float2 ld(const void *lvl, uint32_t idx) {
        return *reinterpret_cast<const float2 *>(static_cast<const char *>(lvl) + (idx << 3));
    }
    static __device__ __forceinline__ float2 ld_byte(const void *t, uint32_t off) {
        return *reinterpret_cast<const float2 *>(static_cast<const char *>(t) + off);
    }
    static __device__ __forceinline__ float2 ld(const void *t, size_t e) {
        return static_cast<const float2 *>(t)[e];
    }
};
template <> struct TabLoad<__half> {
    static __device__ __forceinline__ const void *level(const void *t, int l, uint32_t log2T) {
        return static_cast<const char *>(t) + ((size_t)l << (log2T + 2));
    }
    static __device__ __forceinline__ float2 ld(const void *lvl, uint32_t idx) {
        return __half22float2(*reinterpret_cast<const __half2 *>(static_cast<const char *>(lvl) + (idx << 2)));
    }
    static __device__ __forceinline__ float2 ld_byte(const void *t, uint32_t off) {
        return __half22float2(*reinterpret_cast<const __half2 *>(static_cast<const char *>(t) + off));
    }
    static __device__ __forceinline__ float2 ld(const void *t, size_t e) {
        return __half22float2(static_cast<const __half2 *>(t)[e]);
    }
};

// Per-level cell record (enough to recompute weights and indices).
struct LevelCell {
    uint32_t c[3];
    float w[3];
};

__device__ __forceinline__ void pos_to_u(const GridK &g, float x, float y, float z, float u[3],
                                         bool inside[3]) {
    const float r[3] = {(x - g.lo) * g.inv_ext, (y - g.lo) * g.inv_ext, (z - g.lo) * g.inv_ext};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        inside[d] = (r[d] > 0.0f) && (r[d] < 1.0f);
        u[d] = clamp01(r[d]);
    }
}

// Table indices of the 8 corners of cell c of a level that is dense (row
// stride s) or hashed (mask Tmask); corner bit 0 = +x, bit 1 = +y, bit 2 = +z.
// Both index forms are computed and selected, keeping the encoder free of
// branches (one straight-line scheduling region per group of levels).
__device__ __forceinline__ void corner_idx_p(bool dense, uint32_t s, uint32_t Tmask, const uint32_t (&c)[3],
                                             uint32_t (&idx)[8]) {
    // dense form with 24-bit multiplies (full rate; the 32-bit multiply is
    // quarter rate): a dense level has s^3 <= T <= 2^24, so s <= 256 and every
    // operand is below 2^24 and every product below 2^32 (for a hashed level
    // this form is not selected)
    const uint32_t b = c[0] + __umul24(s, c[1] + __umul24(s, c[2]));
    const uint32_t s2 = __umul24(s, s);
    const uint32_t hy0 = c[1] * 2654435761u, hy1 = hy0 + 2654435761u;
    const uint32_t hz0 = c[2] * 805459861u, hz1 = hz0 + 805459861u;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t di = b + (k & 1) + ((k >> 1) & 1) * s + ((k >> 2) & 1) * s2;
        const uint32_t hi = ((c[0] + (k & 1)) ^ ((k >> 1) & 1 ? hy1 : hy0) ^ ((k >> 2) & 1 ? hz1 : hz0)) & Tmask;
        idx[k] = dense ? di : hi;
    }
}
// the same at level l of grid g (the dense/hashed choice is wave-uniform)
__device__ __forceinline__ void corner_idx(const GridK &g, int l, const uint32_t (&c)[3], uint32_t (&idx)[8]) {
    corner_idx_p(((g.dense_mask >> l) & 1u) != 0, g.stride[l], g.Tmask, c, idx);
}

// f = H(x), features level-major.  Levels are processed in groups (two
// levels for FP32 tables, one for FP16): the gathers of a group are all
// issued before a scheduling barrier and interpolated after it.  Deeper
// groups (more gathers in flight) measured slower for the FP16 tables, whose
// random gathers are bound by cache-line throughput, not latency.  The level
// loop has no branch: a slot past the grid's L levels takes the hashed form
// with a zero mask, i.e. gathers entry 0 of level 0 (always in the table), and
// its features are set to zero by a select.
template <typename TT>
__device__ __forceinline__ void encode(const GridK &g, float x, float y, float z, float (&f)[kNF]) {
    float u[3];
    bool in[3];
    pos_to_u(g, x, y, z, u, in);
    constexpr int GRP = sizeof(TT) == 4 ? 2 : 1;
#pragma unroll
    for (int l0 = 0; l0 < kL; l0 += GRP) {
        __builtin_amdgcn_sched_barrier(0);
        float w[GRP][3];
        float2 e[GRP][8];
#pragma unroll
        for (int li = 0; li < GRP; ++li) {
            const int l = l0 + li;
            const bool have = l < (int)g.L;  // wave-uniform
            uint32_t c[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) cell_of(u[d], g.resf[l], g.nm1f[l], c[d], w[li][d]);
            uint32_t idx[8];
            corner_idx_p(have && ((g.dense_mask >> l) & 1u) != 0, g.stride[l], have ? g.Tmask : 0u, c, idx);
            const void *lvl = TabLoad<TT>::level(g.table, have ? l : 0, g.log2T);
#pragma unroll
            for (int k = 0; k < 8; ++k) e[li][k] = TabLoad<TT>::ld(lvl, idx[k]);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int li = 0; li < GRP; ++li) {
            const int l = l0 + li;
            const float wx0 = 1.0f - w[li][0], wy0 = 1.0f - w[li][1], wz0 = 1.0f - w[li][2];
            float f0 = 0.0f, f1 = 0.0f;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const float wt = ((k & 1) ? w[li][0] : wx0) * (((k >> 1) & 1) ? w[li][1] : wy0) *
                                 (((k >> 2) & 1) ? w[li][2] : wz0);
                f0 = fmaf(wt, e[li][k].x, f0);
                f1 = fmaf(wt, e[li][k].y, f1);
            }
            const bool have = l < (int)g.L;
            f[2 * l] = have ? f0 : 0.0f;
            f[2 * l + 1] = have ? f1 : 0.0f;
        }
    }
    __builtin_amdgcn_sched_barrier(0);
}

// --------------------------------------------------------------------------
// atan2 from a polynomial approximation of atan on [0, 1]:
// atan(t) ~ t * P(t^2), P of degree 7, the coefficients printed by
// fit_atan_poly.py beside this file (Lawson-reweighted least squares on 4000
// Chebyshev nodes towards the minimax absolute error); |error| < 1.4e-7 rad
// when evaluated in FP32 (about one ulp of pi).  Octant reduction: t = min(|x|,|y|) / max(|x|,|y|), formed with the
// hardware reciprocal (relative error about 1.5 ulp, which moves atan(t) by
// at most t / (1 + t^2) * 1.8e-7 <= 9e-8 rad): |error| < 2.5e-7 rad.
// --------------------------------------------------------------------------
__device__ __forceinline__ float atan2_poly(float y, float x) {
    const float ax = fabsf(x), ay = fabsf(y);
    const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
    const float t = mx > 0.0f ? mn * rcpf_(mx) : 0.0f;
    const float s = t * t;
    float p = -0.00405456731f;
    p = fmaf(p, s, 0.0218629576f);
    p = fmaf(p, s, -0.055912327f);
    p = fmaf(p, s, 0.0964219719f);
    p = fmaf(p, s, -0.139086291f);
    p = fmaf(p, s, 0.199465662f);
    p = fmaf(p, s, -0.333298594f);
    p = fmaf(p, s, 0.999999344f);
    float r = p * t;
    if (ay > ax) r = 1.57079632679489662f - r;
    if (x < 0.0f) r = kPi - r;
    return copysignf(r, y);
}

// --------------------------------------------------------------------------
// Environment lookup: y up, azimuth atan2(w_z, w_x), polar angle from +y,
// texel centres at +1/2, bilinear, columns wrap, rows clamp.  Indices are
// clamped so that any input (including NaN) stays inside the map.
// --------------------------------------------------------------------------
__device__ __forceinline__ float3 env_lookup(const EnvK &e, float wx, float wy, float wz) {
    const float phi = atan2_poly(wz, wx);
    const float th = atan2_poly(sqrtf_(wx * wx + wz * wz), wy);
    const float s = (phi + kPi) * (e.Wf * (0.5f / kPi)) - 0.5f;
    const float q = th * (e.Hf * (1.0f / kPi)) - 0.5f;
    const float xf = floorf(s), yf = floorf(q);
    const float fx = s - xf, fy = q - yf;
    int x0 = (int)xf, y0 = (int)yf;
    if (x0 < 0) x0 += e.W;
    x0 = min(max(x0, 0), e.W - 1);
    const int x1 = (x0 + 1 == e.W) ? 0 : x0 + 1;
    const int y1 = min(max(y0 + 1, 0), e.H - 1);
    y0 = min(max(y0, 0), e.H - 1);
    const float *r0 = e.rgb + (size_t)y0 * e.W * 3;
    const float *r1 = e.rgb + (size_t)y1 * e.W * 3;
    const float w00 = (1.0f - fy) * (1.0f - fx), w01 = (1.0f - fy) * fx;
    const float w10 = fy * (1.0f - fx), w11 = fy * fx;
    float3 o;
    o.x = w00 * r0[x0 * 3 + 0] + w01 * r0[x1 * 3 + 0] + w10 * r1[x0 * 3 + 0] + w11 * r1[x1 * 3 + 0];
    o.y = w00 * r0[x0 * 3 + 1] + w01 * r0[x1 * 3 + 1] + w10 * r1[x0 * 3 + 1] + w11 * r1[x1 * 3 + 1];
    o.z = w00 * r0[x0 * 3 + 2] + w01 * r0[x1 * 3 + 2] + w10 * r1[x0 * 3 + 2] + w11 * r1[x1 * 3 + 2];
    return o;
}

// --------------------------------------------------------------------------
// Microfacet BRDF: Lambert (1-m) a/pi + GGX D (alpha = r^2) * Schlick F
// (F0 = mix(f0, a, m)) * height-correlated Smith visibility.
// --------------------------------------------------------------------------
__device__ __forceinline__ float dot3(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

struct BrdfTerms {
    float D, Vis, P;         // specular factors and Schlick weight (1 - VdotH)^5
    float dD_da2, dVis_da2;  // derivatives w.r.t. alpha^2
    bool live;               // n.l > 0
};

__device__ __forceinline__ BrdfTerms brdf_terms(float3 n, float3 v, float3 l, float r, bool want_d) {
    BrdfTerms t;
    const float NdotL = dot3(n, l);
    t.live = NdotL > 0.0f;
    float NdotV = fmaxf(dot3(n, v), 1e-4f);
    float3 h = make_float3(l.x + v.x, l.y + v.y, l.z + v.z);
    const float hh = dot3(h, h);
    {
        const float inv = rsqrtf(hh);
        const bool ok = hh > 0.0f;
        h = make_float3(ok ? h.x * inv : n.x, ok ? h.y * inv : n.y, ok ? h.z * inv : n.z);
    }
    const float NdotH = fmaxf(dot3(n, h), 0.0f);
    const float VdotH = fmaxf(dot3(v, h), 0.0f);
    const float al = r * r, a2 = al * al;
    const float Q = NdotH * NdotH * (a2 - 1.0f) + 1.0f;
    t.D = a2 * rcpf_(kPi * Q * Q);
    const float sv = sqrtf_(NdotV * NdotV * (1.0f - a2) + a2);
    const float sl = sqrtf_(NdotL * NdotL * (1.0f - a2) + a2);
    const float A = NdotL * sv, B = NdotV * sl;
    t.Vis = 0.5f * rcpf_(A + B);
    const float om = 1.0f - VdotH;
    const float om2 = om * om;
    t.P = om2 * om2 * om;
    if (want_d) {
        t.dD_da2 = (Q - 2.0f * a2 * NdotH * NdotH) / (kPi * Q * Q * Q);
        const float dA = NdotL * (1.0f - NdotV * NdotV) / (2.0f * sv);
        const float dB = NdotV * (1.0f - NdotL * NdotL) / (2.0f * sl);
        t.dVis_da2 = -0.5f * (dA + dB) / ((A + B) * (A + B));
    } else {
        t.dD_da2 = t.dVis_da2 = 0.0f;
    }
    return t;
}

// pi * f_r per channel (zero where n.l <= 0).  Written with selects only, so
// that it can share a basic block with matrix-core work.
__device__ __forceinline__ float3 pi_brdf(float3 n, float3 v, float3 l, float3 a, float r, float m, float f0,
                                          bool diffuse_only) {
    const BrdfTerms t = brdf_terms(n, v, l, r, false);
    // diffuse only: metalness and specular factor zero, which returns a exactly
    const float me = diffuse_only ? 0.0f : m;
    const float s = diffuse_only ? 0.0f : kPi * t.D * t.Vis;
    const float q = 1.0f - t.P;
    const float F0x = f0 * (1.0f - me) + a.x * me, F0y = f0 * (1.0f - me) + a.y * me,
                F0z = f0 * (1.0f - me) + a.z * me;
    const float3 o = make_float3((1.0f - me) * a.x + s * (F0x * q + t.P), (1.0f - me) * a.y + s * (F0y * q + t.P),
                                 (1.0f - me) * a.z + s * (F0z * q + t.P));
    return make_float3(t.live ? o.x : 0.f, t.live ? o.y : 0.f, t.live ? o.z : 0.f);
}

// Unit normal from the decoder's normal head (n / |n|); `fallback` when the
// head outputs the zero vector.
__device__ __forceinline__ float3 head_normal(float x, float y, float z, float3 fallback) {
    const float nn = x * x + y * y + z * z;
    if (!(nn > 0.0f)) return fallback;
    const float inv = rsqrtf(nn);
    return make_float3(x * inv, y * inv, z * inv);
}

// pi * f_r at a surface seen along its own normal (v = n, the bounce point's
// facing reading): NdotV = 1, |l + n|^2 = 2 (1 + NdotL), so
// NdotH^2 = VdotH^2 = (1 + NdotL) / 2 and the view term of the
// height-correlated Smith visibility is 1.  Per-point factors are set once.
struct FacingBrdf {
    float3 kd, F0;     // (1-m) a and mix(f0, a, m)
    float a2, a2m1;    // alpha^2 and alpha^2 - 1
    bool diffuse;
    __device__ __forceinline__ void set(float3 a, float r, float m, float f0, bool diffuse_only) {
        diffuse = diffuse_only;
        kd = diffuse_only ? a : make_float3((1.0f - m) * a.x, (1.0f - m) * a.y, (1.0f - m) * a.z);
        F0 = make_float3(f0 * (1.0f - m) + a.x * m, f0 * (1.0f - m) + a.y * m, f0 * (1.0f - m) + a.z * m);
        const float al = r * r;
        a2 = al * al;
        a2m1 = a2 - 1.0f;
    }
    // selects only (no branch), zero where n.l <= 0
    __device__ __forceinline__ float3 eval(float NdotL) const {
        const float h2 = 0.5f * (1.0f + NdotL);
        const float Q = fmaf(h2, a2m1, 1.0f);
        const float D = a2 * rcpf_(kPi * Q * Q);
        const float sl = sqrtf_(fmaf(NdotL * NdotL, -a2m1, a2));
        const float Vis = 0.5f * rcpf_(NdotL + sl);
        const float om = 1.0f - sqrtf_(h2);
        const float om2 = om * om;
        const float P = om2 * om2 * om;
        // diffuse only: specular factor zero, which returns kd exactly
        const float sp = diffuse ? 0.0f : kPi * D * Vis, q = 1.0f - P;
        const float3 o = make_float3(fmaf(sp, fmaf(F0.x, q, P), kd.x), fmaf(sp, fmaf(F0.y, q, P), kd.y),
                                     fmaf(sp, fmaf(F0.z, q, P), kd.z));
        const bool live = NdotL > 0.0f;
        return make_float3(live ? o.x : 0.f, live ? o.y : 0.f, live ? o.z : 0.f);
    }
};

// --------------------------------------------------------------------------
// Per-lane activation storage in LDS (the backward's FP32 MLPs): column
// `lane` of a [64][kHS] array, the odd stride letting both the per-lane rows
// and the per-unit columns be read without bank conflicts.
// --------------------------------------------------------------------------
constexpr int kHS = 65;
constexpr int kHBuf = kH * kHS;   // floats per wave per activation buffer

// --------------------------------------------------------------------------
// Multiple importance sampling of the primary directions (Sec. 4.1): light
// samples from the environment's piecewise-constant distribution and GGX
// samples of the visible normals (Heitz, JCGT 2018), balance heuristic.
// The CDFs come as (hi, lo) single-precision pairs of double values; the
// test u - hi >= lo decides c <= u for an FP32 uniform exactly as the double
// c would (u - hi is exact when u is within a factor two of hi, and
// otherwise its sign already decides), so texel choices do not depend on
// rounding.  Everything here is FP32.
// --------------------------------------------------------------------------
// largest i in [0, n-1] with c[i] <= u (c nondecreasing, c[0] = 0 <= u)
__device__ __forceinline__ int cdf_find(const float2 *c, int n, float u) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const float2 v = c[mid];
        if (u - v.x >= v.y) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// position of u in [a, b) as a fraction of the interval
__device__ __forceinline__ float cdf_frac(float2 a, float2 b, float u) {
    const float num = (u - a.x) - a.y;
    const float den = (b.x - a.x) + (b.y - a.y);
    return den > 0.0f ? clamp01(num / den) : 0.5f;
}

// light sample for the stratified uniforms (s1, s2); returns the direction
// and its density (per steradian)
__device__ __forceinline__ float3 env_light_sample(const EnvK &e, float s1, float s2, float &dens) {
    const int H = e.H, W = e.W;
    const int y = cdf_find(e.marg, H, s1);
    const float fv = cdf_frac(e.marg[y], e.marg[y + 1], s1);
    const float2 *c = e.cond + (size_t)y * (W + 1);
    const int x = cdf_find(c, W, s2);
    const float fu = cdf_frac(c[x], c[x + 1], s2);
    // uniform in cos(theta) inside the row: cos = cos_top - fv span, with
    // 1 - cos and 1 + cos each formed without cancellation
    const float4 row = e.rows[y];
    const float omc = fmaf(fv, row.w, row.y);
    const float opc = fmaf(1.0f - fv, row.w, row.z);
    const float cth = fv < 0.5f ? fmaf(-fv, row.w, row.x) : opc - 1.0f;
    const float sth = sqrtf_(omc * opc);
    // phi = -pi + 2 pi r with r = (x + fu) / W in [0, 1] revolutions, so
    // (cos phi, sin phi) = -(cos 2 pi r, sin 2 pi r)
    const float r = ((float)x + fu) / (float)W;
    float sn, cs;
    sincos2pi_(r, sn, cs);
    dens = e.dens[(size_t)y * W + x];
    return make_float3(-sth * cs, cth, -sth * sn);
}

// density of the light distribution at a direction (texel lookup)
__device__ __forceinline__ float env_light_density(const EnvK &e, float3 w) {
    const float phi = atan2_poly(w.z, w.x);
    const float th = atan2_poly(sqrtf_(w.x * w.x + w.z * w.z), w.y);
    int x = (int)floorf((phi + kPi) * (e.Wf * (0.5f / kPi)));
    int y = (int)floorf(th * (e.Hf * (1.0f / kPi)));
    x = min(max(x, 0), e.W - 1);
    y = min(max(y, 0), e.H - 1);
    return e.dens[(size_t)y * e.W + x];
}

// view in the frame of the normal, normal component clamped to 1e-4, unit
__device__ __forceinline__ float3 ggx_view(const Frame &fr, float3 v) {
    float3 vl = make_float3(dot3(v, fr.t), dot3(v, fr.b), fmaxf(dot3(v, fr.n), 1e-4f));
    const float inv = rsqrtf(dot3(vl, vl));
    return make_float3(vl.x * inv, vl.y * inv, vl.z * inv);
}

// density of the GGX visible-normal reflection at world direction l
__device__ __forceinline__ float ggx_density(const Frame &fr, float3 vl, float r, float3 l) {
    const float3 ll = make_float3(dot3(l, fr.t), dot3(l, fr.b), dot3(l, fr.n));
    float3 h = make_float3(vl.x + ll.x, vl.y + ll.y, vl.z + ll.z);
    const float hh = dot3(h, h);
    if (!(hh > 0.0f)) return 0.0f;
    const float inv = rsqrtf(hh);
    h = make_float3(h.x * inv, h.y * inv, h.z * inv);
    if (!(dot3(vl, h) > 0.0f) || !(h.z > 0.0f)) return 0.0f;
    const float al = r * r, a2 = al * al;
    const float Q = fmaf(h.z * h.z, a2 - 1.0f, 1.0f);
    const float D = a2 / (kPi * Q * Q);
    const float G1 = 2.0f * vl.z / (vl.z + sqrtf_(fmaf(1.0f - a2, vl.z * vl.z, a2)));
    return G1 * D / (4.0f * vl.z);
}

// GGX visible-normal sample, reflected about the sampled normal; world space
__device__ __forceinline__ float3 ggx_sample(const Frame &fr, float3 vl, float r, float s1, float s2) {
    const float al = r * r;
    float3 vh = make_float3(al * vl.x, al * vl.y, vl.z);
    const float iv = rsqrtf(dot3(vh, vh));
    vh = make_float3(vh.x * iv, vh.y * iv, vh.z * iv);
    const float lensq = vh.x * vh.x + vh.y * vh.y;
    float3 T1 = make_float3(1.0f, 0.0f, 0.0f);
    if (lensq > 0.0f) {
        const float il = rsqrtf(lensq);
        T1 = make_float3(-vh.y * il, vh.x * il, 0.0f);
    }
    const float3 T2 = make_float3(vh.y * T1.z - vh.z * T1.y, vh.z * T1.x - vh.x * T1.z, vh.x * T1.y - vh.y * T1.x);
    const float rr = sqrtf_(s1);
    float sn, cs;
    sincos2pi_(s2, sn, cs);
    const float t1 = rr * cs;
    float t2 = rr * sn;
    const float sv = 0.5f * (1.0f + vh.z);
    t2 = (1.0f - sv) * sqrtf_(fmaxf(1.0f - t1 * t1, 0.0f)) + sv * t2;
    const float tz = sqrtf_(fmaxf(1.0f - t1 * t1 - t2 * t2, 0.0f));
    const float3 nh = make_float3(t1 * T1.x + t2 * T2.x + tz * vh.x, t1 * T1.y + t2 * T2.y + tz * vh.y,
                                  t1 * T1.z + t2 * T2.z + tz * vh.z);
    float3 ne = make_float3(al * nh.x, al * nh.y, fmaxf(nh.z, 0.0f));
    const float ie = rsqrtf(dot3(ne, ne));
    ne = make_float3(ne.x * ie, ne.y * ie, ne.z * ie);
    const float vn2 = 2.0f * dot3(vl, ne);
    const float3 ll = make_float3(vn2 * ne.x - vl.x, vn2 * ne.y - vl.y, vn2 * ne.z - vl.z);
    return make_float3(ll.x * fr.t.x + ll.y * fr.b.x + ll.z * fr.n.x, ll.x * fr.t.y + ll.y * fr.b.y + ll.z * fr.n.y,
                       ll.x * fr.t.z + ll.y * fr.b.z + ll.z * fr.n.z);
}

// Primary direction i of a point under MIS and the factor that turns pi f_r
// into its balance-heuristic weight, 2 (n.w) / (pi (p_env + p_ggx)).
__device__ __forceinline__ float3 mis_direction(const RenderK &a, const Frame &fr, float3 vl, float r, uint32_t pid,
                                                uint32_t i, float &wfac) {
    const uint32_t M = a.s.m_half;
    const bool light = i < M;
    const uint32_t k = light ? i : i - M;
    const uint4 words = philox4x32_10(pid, 0u, k >> 2, light ? 2u : 3u, a.s.key0, a.s.key1);
    const uint32_t w = pick4(words, k);
    const uint32_t sa = k >> a.s.nbm_shift, sb = k & ((1u << a.s.nbm_shift) - 1u);
    // (stratum + uniform at its bin centre) / strata: exact in FP32 and FP64
    const float s1 = ((float)sa + ((float)(w & 0xffffu) + 0.5f) * (1.0f / 65536.0f)) * a.s.inv_nam;
    const float s2 = ((float)sb + ((float)(w >> 16) + 0.5f) * (1.0f / 65536.0f)) * a.s.inv_nbm;
    float3 d;
    float pe;
    if (light) {
        d = env_light_sample(a.env, s1, s2, pe);
    } else {
        d = ggx_sample(fr, vl, r, s1, s2);
        pe = env_light_density(a.env, d);
    }
    const float nl = dot3(fr.n, d);
    const float den = pe + ggx_density(fr, vl, r, d);
    wfac = (nl > 0.0f && den > 0.0f) ? 2.0f * nl / (kPi * den) : 0.0f;
    return d;
}

// Compensated accumulation (Kahan) and exact pairwise combination (TwoSum).
struct KSum {
    float s, c;
    __device__ __forceinline__ void add(float x) {
        const float y = x - c;
        const float t = s + y;
        c = (t - s) - y;
        s = t;
    }
};
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

}  // namespace hg
