// hg_membench.hip -- microbenchmarks of the ceilings the renderer's kernels
// are measured against (include/hg_membench.h): random gathers, random and
// grouped FP32 atomics, matrix-core throughput loops.
#include <hip/hip_runtime.h>

#include "../../include/hg_membench.h"

namespace {

constexpr int kThreads = 256;

// 32-bit integer hash (a bijection: xor-shifts and odd multipliers, the
// "lowbias32" constants of C. Wellons' hash-prospector search)
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

template <int E>
struct Item;
template <>
struct Item<4> {
    typedef uint32_t T;
    static __device__ __forceinline__ uint32_t fold(T v) { return v; }
};
template <>
struct Item<8> {
    typedef uint2 T;
    static __device__ __forceinline__ uint32_t fold(T v) { return v.x ^ v.y; }
};
template <>
struct Item<16> {
    typedef uint4 T;
    static __device__ __forceinline__ uint32_t fold(T v) { return v.x ^ v.y ^ v.z ^ v.w; }
};

template <int E>
__global__ __launch_bounds__(kThreads) void k_gather(const typename Item<E>::T *__restrict__ table, uint32_t mask,
                                                     uint32_t rounds, uint32_t seed, uint32_t *__restrict__ sink) {
    const uint32_t tid = blockIdx.x * kThreads + threadIdx.x;
    const uint32_t nthr = gridDim.x * kThreads;
    uint32_t acc = 0;
    for (uint32_t r = 0; r < rounds; ++r) {
        typename Item<E>::T v[8];
        const uint32_t base = (r * nthr + tid) * 8u;
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = table[mix32((base + u) ^ seed) & mask];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc ^= Item<E>::fold(v[u]);
    }
    sink[tid] = acc;
}

// Persistent replay: thread t walks the eight-item groups g = t, t + nthr,
// ... (consecutive lanes on consecutive groups, as the encoder's threads
// are), gathers table[idx[8g .. 8g+7]] with all eight loads in flight and
// prefetches the next group's indices behind them, so that one memory
// latency is exposed per group; the tail (n mod 8 items) goes one item per
// thread at the end.
template <int E>
__global__ __launch_bounds__(kThreads) void k_gather_indexed(const typename Item<E>::T *__restrict__ table,
                                                             const uint32_t *__restrict__ idx, int64_t n,
                                                             uint32_t *__restrict__ sink) {
    const int64_t tid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int64_t nthr = (int64_t)gridDim.x * kThreads;
    const int64_t groups = n >> 3;
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 *ix4 = reinterpret_cast<const u32x4 *>(idx);
    uint32_t acc = 0;
    int64_t g = tid;
    u32x4 a = u32x4(0u), b = a;
    // the index stream is read non-temporally so that it does not displace
    // table lines from the caches
    if (g < groups) {
        a = __builtin_nontemporal_load(ix4 + 2 * g);
        b = __builtin_nontemporal_load(ix4 + 2 * g + 1);
    }
    for (; g < groups; g += nthr) {
        const int64_t gn = g + nthr;
        u32x4 an = u32x4(0u), bn = an;
        if (gn < groups) {
            an = __builtin_nontemporal_load(ix4 + 2 * gn);
            bn = __builtin_nontemporal_load(ix4 + 2 * gn + 1);
        }
        const uint32_t ix[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
        typename Item<E>::T v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = table[ix[u]];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc ^= Item<E>::fold(v[u]);
        a = an;
        b = bn;
    }
    const int64_t i = (groups << 3) + tid;
    if (i < n) acc ^= Item<E>::fold(table[idx[i]]);
    sink[tid] = acc;
}

__global__ __launch_bounds__(kThreads) void k_atomic(float *__restrict__ table, uint32_t mask, uint32_t rounds,
                                                     uint32_t group_shift, uint32_t seed) {
    const uint32_t tid = blockIdx.x * kThreads + threadIdx.x;
    const uint32_t ngroups = (gridDim.x * kThreads) >> group_shift;
    const uint32_t g = tid >> group_shift;
    for (uint32_t r = 0; r < rounds; ++r) {
        const uint32_t base = (r * ngroups + g) * 4u;
#pragma unroll
        for (int u = 0; u < 4; ++u) unsafeAtomicAdd(&table[mix32((base + u) ^ seed) & mask], 1.0f);
    }
}

// Groups of G = 2^gs consecutive lanes add to G adjacent words of one
// G-word-aligned block at a random place: for G <= 16 the group's words lie
// in one 64-byte line.
__global__ __launch_bounds__(kThreads) void k_atomic_lines(float *__restrict__ table, uint32_t log2_items,
                                                           uint32_t rounds, uint32_t gs, uint32_t seed) {
    const uint32_t tid = blockIdx.x * kThreads + threadIdx.x;
    const uint32_t ngroups = (gridDim.x * kThreads) >> gs;
    const uint32_t grp = tid >> gs, sub = tid & ((1u << gs) - 1u);
    const uint32_t emask = (1u << (log2_items - gs)) - 1u;
    for (uint32_t r = 0; r < rounds; ++r) {
        const uint32_t base = (r * ngroups + grp) * 4u;
#pragma unroll
        for (int u = 0; u < 4; ++u) unsafeAtomicAdd(&table[((mix32((base + u) ^ seed) & emask) << gs) + sub], 1.0f);
    }
}

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int C>
__global__ __launch_bounds__(kThreads) void k_mfma_f32(uint32_t iters, float *__restrict__ sink) {
    const float a = 1.0f + 1e-3f * (float)(threadIdx.x & 63), b = 1.0f - 1e-3f * (float)(threadIdx.x & 7);
    f32x16 acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = f32x16(0.0f);
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[c], 0, 0, 0);
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int k = 0; k < 16; ++k) s += acc[c][k];
    sink[blockIdx.x * kThreads + threadIdx.x] = s;
}

template <int C>
__global__ __launch_bounds__(kThreads) void k_mfma_bf16(uint32_t iters, float *__restrict__ sink) {
    bf16x8 a, b;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        a[k] = (__bf16)(1.0f + 0.0625f * (float)k);
        b[k] = (__bf16)(1.0f - 0.03125f * (float)((threadIdx.x + k) & 7));
    }
    f32x4 acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = f32x4(0.0f);
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < C; ++c)
#pragma unroll
        for (int k = 0; k < 4; ++k) s += acc[c][k];
    sink[blockIdx.x * kThreads + threadIdx.x] = s;
}

bool aligned16(const void *p) { return p != nullptr && (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
int launched() { return hipGetLastError() == hipSuccess ? 0 : 4; }

}  // namespace

extern "C" {

int hgmb_gather(const void *table, int32_t log2_items, int32_t item_bytes, int32_t blocks, int32_t rounds,
                uint32_t seed, uint32_t *sink, hipStream_t stream) {
    const int lb = item_bytes == 4 ? 2 : item_bytes == 8 ? 3 : item_bytes == 16 ? 4 : -1;
    if (lb < 0 || !aligned16(table) || sink == nullptr) return 1;
    if (log2_items < 4 || log2_items > 31 - lb || blocks < 1 || blocks > (1 << 20) || rounds < 1 ||
        rounds > (1 << 16))
        return 1;
    const uint32_t mask = (uint32_t)((uint64_t(1) << log2_items) - 1);
    const dim3 g((unsigned)blocks), b(kThreads);
    if (lb == 2)
        hipLaunchKernelGGL(k_gather<4>, g, b, 0, stream, static_cast<const uint32_t *>(table), mask, (uint32_t)rounds,
                           seed, sink);
    else if (lb == 3)
        hipLaunchKernelGGL(k_gather<8>, g, b, 0, stream, static_cast<const uint2 *>(table), mask, (uint32_t)rounds,
                           seed, sink);
    else
        hipLaunchKernelGGL(k_gather<16>, g, b, 0, stream, static_cast<const uint4 *>(table), mask, (uint32_t)rounds,
                           seed, sink);
    return launched();
}

int hgmb_gather_indexed(const void *table, int32_t item_bytes, const uint32_t *idx, int64_t n, int32_t blocks,
                        uint32_t *sink, hipStream_t stream) {
    if ((item_bytes != 4 && item_bytes != 8 && item_bytes != 16) || !aligned16(table) || sink == nullptr ||
        n < 0 || n > (int64_t(1) << 40) || (n > 0 && !aligned16(idx)) || blocks < 1 || blocks > (1 << 20))
        return 1;
    if (n == 0) return 0;
    const dim3 g((unsigned)blocks), b(kThreads);
    if (item_bytes == 4)
        hipLaunchKernelGGL(k_gather_indexed<4>, g, b, 0, stream, static_cast<const uint32_t *>(table), idx, n, sink);
    else if (item_bytes == 8)
        hipLaunchKernelGGL(k_gather_indexed<8>, g, b, 0, stream, static_cast<const uint2 *>(table), idx, n, sink);
    else
        hipLaunchKernelGGL(k_gather_indexed<16>, g, b, 0, stream, static_cast<const uint4 *>(table), idx, n, sink);
    return launched();
}

int hgmb_atomic(float *table, int32_t log2_items, int32_t blocks, int32_t rounds, int32_t lanes_per_address,
                uint32_t seed, hipStream_t stream) {
    int shift = -1;
    for (int s = 0; s <= 6; ++s)
        if (lanes_per_address == (1 << s)) shift = s;
    if (shift < 0 || !aligned16(table) || log2_items < 4 || log2_items > 29 || blocks < 1 || blocks > (1 << 20) ||
        rounds < 1 || rounds > (1 << 16))
        return 1;
    const uint32_t mask = (uint32_t)((uint64_t(1) << log2_items) - 1);
    hipLaunchKernelGGL(k_atomic, dim3((unsigned)blocks), dim3(kThreads), 0, stream, table, mask, (uint32_t)rounds,
                       (uint32_t)shift, seed);
    return launched();
}

int hgmb_atomic_lines(float *table, int32_t log2_items, int32_t blocks, int32_t rounds, int32_t lanes_per_line,
                      uint32_t seed, hipStream_t stream) {
    int shift = -1;
    for (int s = 0; s <= 4; ++s)
        if (lanes_per_line == (1 << s)) shift = s;
    if (shift < 0 || !aligned16(table) || log2_items < 4 || log2_items > 29 || blocks < 1 || blocks > (1 << 20) ||
        rounds < 1 || rounds > (1 << 16))
        return 1;
    hipLaunchKernelGGL(k_atomic_lines, dim3((unsigned)blocks), dim3(kThreads), 0, stream, table, (uint32_t)log2_items,
                       (uint32_t)rounds, (uint32_t)shift, seed);
    return launched();
}

int hgmb_mfma(int32_t kind, int32_t blocks, int32_t iters, int32_t chains, float *sink, hipStream_t stream) {
    if ((kind != 0 && kind != 1) || sink == nullptr || blocks < 1 || blocks > (1 << 20) || iters < 1 ||
        iters > (1 << 20))
        return 1;
    const dim3 g((unsigned)blocks), b(kThreads);
    const uint32_t it = (uint32_t)iters;
#define HGMB_CASE(C)                                                                   \
    case C:                                                                            \
        if (kind == 0) hipLaunchKernelGGL(k_mfma_f32<C>, g, b, 0, stream, it, sink);   \
        else hipLaunchKernelGGL(k_mfma_bf16<C>, g, b, 0, stream, it, sink);           \
        break;
    switch (chains) {
        HGMB_CASE(1)
        HGMB_CASE(2)
        HGMB_CASE(4)
        HGMB_CASE(8)
        HGMB_CASE(16)
        default:
            return 1;
    }
#undef HGMB_CASE
    return launched();
}

}  // extern "C"
