// Gram-form frame cost on the matrix cores (gfx950):
//   C(i,j) = sqrt(max(0, |x_i|^2 + |y_j|^2 - 2 x_i . y_j))
// with x, y rounded to bf16 (or fp16), the dot products from
// v_mfma_f32_32x32x16_bf16 (or _f16; FP32 accumulation) and the squared norms
// of the rounded frames in FP32.
//
// Lane layout of v_mfma_f32_32x32x16_bf16 and _f16 (checked on the device): lane l
// supplies A[l % 32][8*(l/32) .. 8*(l/32)+7] and B[8*(l/32) .. +7][l % 32];
// accumulator register r of lane l holds C[8*(r/4) + 4*(l/32) + r%4][l % 32].
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dtw {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

__device__ __forceinline__ bf16x8_t load_bf16x8(const uint16_t* p) {
  return __builtin_bit_cast(bf16x8_t, *reinterpret_cast<const uint4*>(p));
}

// One 32x32x16 product of 16-bit frames held as raw bit patterns: bf16 for
// kBf16, else fp16.
template <bool kBf16>
__device__ __forceinline__ f32x16_t mfma_16bit_32x32x16(bf16x8_t a, bf16x8_t b, f32x16_t c) {
  if constexpr (kBf16) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  } else {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8_t, a), __builtin_bit_cast(f16x8_t, b), c,
                                                  0, 0, 0);
  }
}

__device__ __forceinline__ f32x16_t f32x16_zero() {
  f32x16_t z = {};
  return z;
}

}  // namespace dtw
