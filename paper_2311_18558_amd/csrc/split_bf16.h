// FP32-accurate products on the BF16 matrix cores.
//
// A float x is split into three BF16 values, x ~= h + m + l, each the
// round-to-nearest BF16 of what the previous ones leave (the residuals are
// exact in FP32, so |x - (h + m + l)| <= 2^-24 |x|).  A product x*y is then
// the sum of the six partial products whose weights reach 2^-24:
//     hh + hm + mh + hl + lh + mm
// (the dropped ml, lm, ll are below 2^-24 |x y|).  Every BF16 x BF16 product
// is exact in FP32 and the matrix core accumulates in FP32, so the result
// carries FP32-level error at the BF16 instruction rate.
//
// Operand layout of v_mfma_f32_32x32x16_bf16 (checked on the device): lane l
// holds A[l%32][8(l/32) + j] and B[8(l/32) + j][l%32] in element j of its
// 8-wide BF16 vectors; the 32x32 FP32 result is laid out as for
// v_mfma_f32_32x32x2_f32 (register r: row 8(r/4) + 4(l/32) + r%4, column
// l%32).
#pragma once

#include "dev_common.h"

namespace rtc {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

struct Split3 {
  bf16x8 h, m, l;
};

// two floats -> packed BF16 pair (round to nearest even); element 0 low
RTC_DEV unsigned pack_bf16(float a, float b) {
  bf16x2 v = __builtin_convertvector((floatx2){a, b}, bf16x2);
  return __builtin_bit_cast(unsigned, v);
}
RTC_DEV float bf16_lo(unsigned w) { return __builtin_bit_cast(float, w << 16); }
RTC_DEV float bf16_hi(unsigned w) { return __builtin_bit_cast(float, w & 0xffff0000u); }

RTC_DEV Split3 split3(const float (&x)[8]) {
  u32x4 H, M, L;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float a = x[2 * j], b = x[2 * j + 1];
    const unsigned wh = pack_bf16(a, b);
    const float ra = a - bf16_lo(wh), rb = b - bf16_hi(wh);
    const unsigned wm = pack_bf16(ra, rb);
    const float sa = ra - bf16_lo(wm), sb = rb - bf16_hi(wm);
    H[j] = wh;
    M[j] = wm;
    L[j] = pack_bf16(sa, sb);
  }
  Split3 s;
  s.h = __builtin_bit_cast(bf16x8, H);
  s.m = __builtin_bit_cast(bf16x8, M);
  s.l = __builtin_bit_cast(bf16x8, L);
  return s;
}

// -x, exactly (sign bits flipped)
RTC_DEV bf16x8 neg_bf16x8(bf16x8 v) {
  u32x4 w = __builtin_bit_cast(u32x4, v);
  w ^= 0x80008000u;
  return __builtin_bit_cast(bf16x8, w);
}
RTC_DEV Split3 neg3(const Split3& s) {
  Split3 r;
  r.h = neg_bf16x8(s.h);
  r.m = neg_bf16x8(s.m);
  r.l = neg_bf16x8(s.l);
  return r;
}

RTC_DEV floatx16 mfma_bf16(bf16x8 a, bf16x8 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// c += A B with both operands split; small terms first.
RTC_DEV floatx16 mac6(const Split3& a, const Split3& b, floatx16 c) {
  c = mfma_bf16(a.m, b.m, c);
  c = mfma_bf16(a.l, b.h, c);
  c = mfma_bf16(a.h, b.l, c);
  c = mfma_bf16(a.m, b.h, c);
  c = mfma_bf16(a.h, b.m, c);
  c = mfma_bf16(a.h, b.h, c);
  return c;
}

}  // namespace rtc
