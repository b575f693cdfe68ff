// C entry points to the bfloat16 conversions of csrc/sw_bf16.h for the CPU
// test in tests/test_bf16.py (built there with g++).
#include <stdint.h>

#include "sw_bf16.h"

extern "C" {

void to_bf16(int64_t n, const float* x, uint16_t* h) {
  for (int64_t i = 0; i < n; ++i) h[i] = sw::bf16_round(x[i]);
}

void from_bf16(int64_t n, const uint16_t* h, float* x) {
  for (int64_t i = 0; i < n; ++i) x[i] = sw::bf16_value(h[i]);
}
}
