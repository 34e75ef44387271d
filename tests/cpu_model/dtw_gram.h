// CPU-model stand-in for dtw_gram.h (tests only): the 32x32x16 matrix
// core operation of a wave (bf16 or fp16 operands), computed from the 64 lanes' operands exchanged
// through a shared buffer, with the lane layout that the device uses (see the
// real header).  Products are summed in FP32 in k order.
#pragma once
#include <cstdint>
#include <cmath>
#include <cstring>

#include "hip/hip_runtime.h"

namespace dtw {

struct bf16x8_t {
  uint16_t v[8];
};
struct f32x16_t {
  float v[16];
  float& operator[](int i) { return v[i]; }
  float operator[](int i) const { return v[i]; }
};

extern uint16_t cpu_mfma_a[16][64][8];
extern uint16_t cpu_mfma_b[16][64][8];

inline float cpu_bf16_to_float(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

inline bf16x8_t load_bf16x8(const uint16_t* p) {
  bf16x8_t r;
  std::memcpy(r.v, p, 16);
  return r;
}

inline f32x16_t f32x16_zero() {
  f32x16_t z;
  for (int i = 0; i < 16; ++i) z.v[i] = 0.0f;
  return z;
}

inline float cpu_f16_to_float(uint16_t h) {
  const int e = (h >> 10) & 0x1f, m = h & 0x3ff;
  const float v = e == 0 ? std::ldexp((float)m, -24) : std::ldexp((float)(m | 0x400), e - 25);
  return (h & 0x8000) ? -v : v;
}

template <bool kBf16>
inline f32x16_t mfma_16bit_32x32x16(bf16x8_t a, bf16x8_t b, f32x16_t c) {
  const int wv = threadIdx.x / 64, l = threadIdx.x % 64;
  std::memcpy(cpu_mfma_a[wv][l], a.v, 16);
  std::memcpy(cpu_mfma_b[wv][l], b.v, 16);
  cpu_wave_barrier->arrive_and_wait();
  for (int r = 0; r < 16; ++r) {
    const int row = 8 * (r / 4) + 4 * (l / 32) + r % 4, col = l % 32;
    float s = c.v[r];
    for (int k = 0; k < 16; ++k) {
      // A[row][k] comes from lane (k/8)*32 + row, element k%8; B[k][col] from lane (k/8)*32 + col
      const uint16_t ah = cpu_mfma_a[wv][(k / 8) * 32 + row][k % 8];
      const uint16_t bh = cpu_mfma_b[wv][(k / 8) * 32 + col][k % 8];
      const float av = kBf16 ? cpu_bf16_to_float(ah) : cpu_f16_to_float(ah);
      const float bv = kBf16 ? cpu_bf16_to_float(bh) : cpu_f16_to_float(bh);
      s += av * bv;
    }
    c.v[r] = s;
  }
  cpu_wave_barrier->arrive_and_wait();
  return c;
}

}  // namespace dtw
