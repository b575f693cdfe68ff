// bfloat16 storage of FP32 values (the 16-bit direction vector of the
// SW_MIXED_FP16 inner CG): the upper half of the FP32 bit pattern, rounded
// to nearest with ties to even; a NaN stays a (quiet) NaN.  bfloat16 keeps
// FP32's exponent range, so a direction that shrinks with the residual over
// an inner solve needs no scaling.
#pragma once

#include <stdint.h>

#if defined(__HIP__)
#define SW_BF16_HD __host__ __device__ __forceinline__
#else
#define SW_BF16_HD inline
#endif

namespace sw {

SW_BF16_HD uint32_t f32_bits(float f) {
  uint32_t u;
  __builtin_memcpy(&u, &f, sizeof u);
  return u;
}

SW_BF16_HD float f32_from_bits(uint32_t u) {
  float f;
  __builtin_memcpy(&f, &u, sizeof f);
  return f;
}

SW_BF16_HD uint16_t bf16_round(float f) {
  const uint32_t u = f32_bits(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x0040u);
  // adding 0x7fff, plus one when the kept part is odd, carries into the kept
  // half exactly when the dropped half is above one half ulp, or equal to it
  // with an odd kept part
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

SW_BF16_HD float bf16_value(uint16_t h) { return f32_from_bits((uint32_t)h << 16); }

}  // namespace sw
