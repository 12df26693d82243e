// Device pieces shared by the CFR kernels (cfr.hip) and the fused step
// kernel (fused.hip).
#pragma once

#include "dev_common.h"

namespace rtc {

constexpr double kInv2Pi = 0.15915494309189533577;

// v of lane (lane ^ O) within each 32-lane half, O < 32: ds_swizzle in its
// bit mode (and mask 0x1f, xor mask O) takes the pattern as an immediate, so
// no per-lane address is formed (or held in a register)
template <int O>
RTC_DEV float swz_xor(float v) {
  static_assert(O > 0 && O < 32, "within a 32-lane half");
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), (O << 10) | 0x1f));
}

// Butterfly sum over the 32 lanes of each half-wave (fixed order; every
// lane of the half gets its half's total).
RTC_DEV float half_sum_f32(float v) {
  v += swz_xor<16>(v);
  v += swz_xor<8>(v);
  v += swz_xor<4>(v);
  v += swz_xor<2>(v);
  v += swz_xor<1>(v);
  return v;
}

RTC_DEV float wave_max_f32(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

// Power-of-two scale that brings the A operand of link [off0, off1) into
// FP16's range: |Re|, |Im| of a_i g_m exp(j phase) are at most |a_i| |g_m|
// <= 2 max(|Re a|, |Im a|) max(|Re g|, |Im g|) =: b < 2^e, and the scale
// 2^(14 - e) puts every value below 2^14 (FP16 holds up to 65504), so
// values down to 2^-28 of the largest stay normal.  A zero link gets 1;
// the exponent is clamped so the scale and its inverse are finite FP32.
RTC_DEV int cfr_link_scale_exp(const float2* a, int64_t off0, int64_t off1, float2 gm, int lane) {
  float am = 0.0f;
  for (int64_t p = off0 + lane; p < off1; p += 64) {
    const float2 v = a[p];
    am = fmaxf(am, fmaxf(fabsf(v.x), fabsf(v.y)));
  }
  am = wave_max_f32(am);
  const float gx = wave_max_f32(fmaxf(fabsf(gm.x), fabsf(gm.y)));
  int e = 0;
  frexpf(2.0f * am * gx, &e);  // b = f 2^e, 0.5 <= f < 1
  return min(max(e, -100), 100);
}

}  // namespace rtc
