// bf16_split.h -- BF16 and FP16 pieces of FP32 / FP64 values for the split
// M2L forms.
//
// x is carried as np BF16 pieces x = x0 + x1 (+ x2), x0 = bf16(x),
// x1 = bf16(x - x0), x2 = bf16(x - x0 - x1), each rounded to nearest even.
// Each difference is exact (x and its BF16 rounding lie within a factor 2 of
// each other), so three pieces reproduce an FP32 value exactly (8 + 8 + 8
// significant bits).  Pieces are packed two per 32-bit word, low half first;
// a 16-byte quad holds 8 consecutive k values.
#ifndef FMM_BF16_SPLIT_H_
#define FMM_BF16_SPLIT_H_

#include "fmm_internal.h"

namespace fmm {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));  // one 16-byte quad

// FP32 -> BF16, round to nearest even (finite inputs).
__host__ __device__ inline uint32_t bf16_bits(float x) {
  uint32_t u = __builtin_bit_cast(uint32_t, x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
__host__ __device__ inline float bf16_value(uint32_t b) { return __builtin_bit_cast(float, b << 16); }

template <int NP>
__host__ __device__ inline void split_f32(float x, uint32_t* piece) {
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    piece[i] = bf16_bits(x);
    x -= bf16_value(piece[i]);
  }
}
// FP64 input: the first rounding goes through FP32; three pieces hold about
// 24 significant bits.
template <int NP>
__host__ __device__ inline void split_f64(double x, uint32_t* piece) {
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    piece[i] = bf16_bits((float)x);
    x -= (double)bf16_value(piece[i]);
  }
}

// FP16 pieces: x = h + l with h = fp16(x), l = fp16(x - h), round to nearest
// even (callers scale x into the FP16 range first); about 22 significant bits.
__device__ inline uint32_t f16_bits(float x) { return __builtin_bit_cast(uint16_t, (_Float16)x); }
__device__ inline float f16_value(uint32_t b) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)b);
}
__device__ inline void split_f16_f32(float x, uint32_t* piece) {
  piece[0] = f16_bits(x);
  piece[1] = f16_bits(x - f16_value(piece[0]));
}
__device__ inline void split_f16_f64(double x, uint32_t* piece) {
  piece[0] = f16_bits((float)x);
  piece[1] = f16_bits((float)(x - (double)f16_value(piece[0])));
}

// The NP quads of 8 values given as pieces pc[j][i] (value j, piece i).
template <int NP>
__host__ __device__ inline void pack_quads(const uint32_t (*pc)[NP], u32x4* q) {
#pragma unroll
  for (int i = 0; i < NP; ++i)
#pragma unroll
    for (int w = 0; w < 4; ++w) q[i][w] = pc[2 * w][i] | pc[2 * w + 1][i] << 16;
}

}  // namespace fmm

#endif  // FMM_BF16_SPLIT_H_
