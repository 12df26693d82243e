// Device pieces shared by the CFR kernels (cfr.hip) and the fused step
// kernel (fused.hip).
#pragma once

#include "dev_common.h"

namespace rtc {

constexpr double kInv2Pi = 0.15915494309189533577;

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
