// Z-order (Morton) permutation of a batch of points: hg_morton_order.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include "hg_order.h"

namespace hg {

// --------------------------------------------------------------------------
// Order of a batch of points along a Z-order (Morton) curve: 21 bits per
// axis over the grid's domain box, one 63-bit key per point, sorted with the
// point's index by a stable radix sort.  A training batch drawn at random and
// rendered in this order gives each wave neighbouring points, whose gathers
// share cells and cache lines.
// --------------------------------------------------------------------------
__device__ __forceinline__ uint64_t spread21(uint32_t v) {
    uint64_t x = v & 0x1fffffu;
    x = (x | (x << 32)) & 0x001f00000000ffffull;
    x = (x | (x << 16)) & 0x001f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

// key: bits 3b, 3b+1, 3b+2 hold bit b of the x, y, z cell; the cell along an
// axis is trunc((p - lo) * 2^21 / extent) clamped to [0, 2^21 - 1] (a NaN
// coordinate takes cell 0)
__global__ __launch_bounds__(256) void k_morton63(const float *__restrict__ pos, int64_t n, float lo, float scale,
                                                  uint64_t *__restrict__ key, int32_t *__restrict__ idx) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    uint64_t k = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float f = fminf(fmaxf((pos[3 * i + d] - lo) * scale, 0.0f), 2097151.0f);
        k |= spread21((uint32_t)f) << d;
    }
    key[i] = k;
    idx[i] = (int32_t)i;
}

hipError_t morton_sort_bytes(int64_t n, size_t &bytes) {
    bytes = 0;
    return hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const uint64_t *)nullptr, (uint64_t *)nullptr,
                                              (const int32_t *)nullptr, (int32_t *)nullptr, (int)n, 0, 63,
                                              (hipStream_t)0);
}

// workspace: keys, sorted keys, indices, the sort's temporary storage
size_t morton_ws_layout(int64_t n, size_t sort_tmp_bytes) {
    auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
    return 2 * al((size_t)n * sizeof(uint64_t)) + al((size_t)n * sizeof(int32_t)) + al(sort_tmp_bytes);
}

hipError_t launch_morton_order(const float *pos, int64_t n, float lo, float extent, int32_t *perm, void *ws,
                               size_t sort_tmp_bytes, hipStream_t s) {
    auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
    char *b = static_cast<char *>(ws);
    uint64_t *key = reinterpret_cast<uint64_t *>(b);
    uint64_t *key_sorted = reinterpret_cast<uint64_t *>(b + al((size_t)n * sizeof(uint64_t)));
    int32_t *idx = reinterpret_cast<int32_t *>(b + 2 * al((size_t)n * sizeof(uint64_t)));
    void *tmp = b + 2 * al((size_t)n * sizeof(uint64_t)) + al((size_t)n * sizeof(int32_t));
    hipLaunchKernelGGL(k_morton63, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pos, n, lo,
                       2097152.0f / extent, key, idx);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    size_t bytes = sort_tmp_bytes;
    return hipcub::DeviceRadixSort::SortPairs(tmp, bytes, key, key_sorted, idx, perm, (int)n, 0, 63, s);
}

}  // namespace hg
