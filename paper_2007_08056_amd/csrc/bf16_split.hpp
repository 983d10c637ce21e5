// Split of a binary32 value into two bfloat16 parts, x = hi + lo + O(2^-16 x):
// hi = bf16(x), lo = bf16(x - hi), both rounded to nearest even (the split-bf16
// product form).  Shared by the transforms that write hi/lo planes and by the
// product that splits U's elements in registers, so both give the same bits.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace symt {

// bfloat16 rounded to nearest even: the gfx950 conversion (v_cvt_pk_bf16_f32),
// the same instruction the wide product uses when it splits U in registers.
__device__ __forceinline__ uint16_t bf16_rne(float x) {
  return __builtin_bit_cast(uint16_t, static_cast<__bf16>(x));
}
__device__ __forceinline__ float bf16_as_f32(uint16_t h) {
  return __uint_as_float(static_cast<uint32_t>(h) << 16);
}
// x is taken in binary32 first (a binary64 input is rounded to nearest).  The
// empty asm keeps that binary32 value: the compiler would otherwise fold the two
// conversions into one rounding of the binary64 value to bfloat16, which can
// differ by one unit in hi.
__device__ __forceinline__ void bf16_split(double x, uint16_t& hi, uint16_t& lo) {
  float f = static_cast<float>(x);
  asm("" : "+v"(f));
  hi = bf16_rne(f);
  lo = bf16_rne(f - bf16_as_f32(hi));
}

}  // namespace symt
