// Host-side launch interface of the batch ordering (hg_order.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace hg {
// temporary storage the radix sort needs for n keys
hipError_t morton_sort_bytes(int64_t n, size_t &bytes);
// workspace bytes: keys, sorted keys, indices, the sort's storage
size_t morton_ws_layout(int64_t n, size_t sort_tmp_bytes);
// keys of pos [n][3] over the box (lo, extent), then the stable sort of
// (key, index) into perm [n]; ws holds morton_ws_layout(n, sort_tmp_bytes)
hipError_t launch_morton_order(const float *pos, int64_t n, float lo, float extent, int32_t *perm, void *ws,
                               size_t sort_tmp_bytes, hipStream_t s);
}  // namespace hg
