// hg_bf16.h -- BF16 matrix-core helpers shared by the mixed-precision
// forward and backward: v_mfma_f32_16x16x32_bf16 (lane l supplies
// A[l%16][8(l/16)..+8] and B[8(l/16)..+8][l%16] and receives
// D[4(l/16)+r][l%16] in register r), FP32 -> BF16 packing, ReLU on packed
// BF16, and the unit order in which a layer's accumulator tiles are the next
// layer's B operand.
#pragma once
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hg {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short s16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ f32x4 mfma_bf16(const uint4 &a, const uint4 &b, const f32x4 &c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b),
                                                    c, 0, 0, 0);
}

// Round-to-nearest-even FP32 -> BF16 of two values, packed (lo = a).  Written
// as one two-element conversion so that it is a single v_cvt_pk_bf16_f32
// (two scalar conversions become two instructions plus a merge).
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
    const f32x2_t v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
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

// Physical hidden unit feeding logical input k = 32 s + 8 g + e of a BF16
// layer (K-step s, lane group g, element e) whose input is the previous
// layer's accumulator tiles.
__device__ __forceinline__ int unit_bf16(int s, int g, int e) { return 16 * (2 * s + (e >> 2)) + 4 * g + (e & 3); }


}  // namespace hg
