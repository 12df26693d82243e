// Near-FP32 products on the FP16 matrix cores.
//
// A float x is split into two FP16 values, x ~= h + l, h the round-to-
// nearest FP16 of x and l that of the residual x - h (exact in FP32):
// |x - h| <= 2^-11 |x| and |x - (h + l)| <= 2^-22 |x| while x - h stays in
// FP16's normal range.  A product x*y is taken as hh + hl + lh; the dropped
// ll is below 2^-22 |x y|, so a product carries at most ~3 * 2^-22
// relative error, and every FP16 x FP16 product is exact in the FP32
// accumulator (subnormal FP16 inputs included, checked on the device).
// A three-way BF16 split (h + m + l, six partial products) reaches FP32
// accuracy over FP32's range but takes twice the matrix-core work and about
// twice the VALU work per value; the cost of FP16 is its range: operands
// must be scaled into it by the caller (a power of two, exact both ways).
//
// Operand layout of v_mfma_f32_32x32x16_f16 (checked on the device): lane l
// holds A[l%32][8(l/32) + j] and B[8(l/32) + j][l%32] in element j of its
// 8-wide FP16 vectors; the 32x32 FP32 result is laid out as for
// v_mfma_f32_32x32x2_f32 (register r: row 8(r/4) + 4(l/32) + r%4, column
// l%32).
#pragma once

#include "dev_common.h"

namespace rtc {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx2 __attribute__((ext_vector_type(2)));

struct Split2 {
  halfx8 h, l;
};

// two floats -> packed FP16 pair (round to nearest even); element 0 low
RTC_DEV unsigned pack_f16(float a, float b) {
  halfx2 v = __builtin_convertvector((floatx2){a, b}, halfx2);
  return __builtin_bit_cast(unsigned, v);
}

// x - h with h the low (LO) or high FP16 half of w, in one v_fma_mix_f32
// (x * 1 - h, one rounding of an exactly representable difference) instead
// of a conversion and a subtraction.
template <bool LO>
RTC_DEV float sub_f16(float x, unsigned w) {
  float r;
  if constexpr (LO)
    asm("v_fma_mix_f32 %0, %1, 1.0, -%2 op_sel_hi:[0,0,1]" : "=v"(r) : "v"(x), "v"(w));
  else
    asm("v_fma_mix_f32 %0, %1, 1.0, -%2 op_sel:[0,0,1] op_sel_hi:[0,0,1]" : "=v"(r)
        : "v"(x), "v"(w));
  return r;
}

RTC_DEV Split2 split2(const float (&x)[8]) {
  u32x4 H, L;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float a = x[2 * j], b = x[2 * j + 1];
    const unsigned wh = pack_f16(a, b);
    H[j] = wh;
    L[j] = pack_f16(sub_f16<true>(a, wh), sub_f16<false>(b, wh));
  }
  Split2 s;
  s.h = __builtin_bit_cast(halfx8, H);
  s.l = __builtin_bit_cast(halfx8, L);
  return s;
}

RTC_DEV floatx16 mfma_f16(halfx8 a, halfx8 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// c += A B with both operands split; small terms first.
RTC_DEV floatx16 mac3(const Split2& a, const Split2& b, floatx16 c) {
  c = mfma_f16(a.l, b.h, c);
  c = mfma_f16(a.h, b.l, c);
  c = mfma_f16(a.h, b.h, c);
  return c;
}

}  // namespace rtc
