// Device pieces shared by the CFR kernels (cfr.hip) and the fused step
// kernel (fused.hip).
#pragma once

#include "dev_common.h"
#include "split_f16.h"

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

// The same butterfly in FP64 (each half of the double swizzled alike).
template <int O>
RTC_DEV double swz_xor_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_ds_swizzle((int)(unsigned)(b & 0xffffffffll), (O << 10) | 0x1f);
  const int hi = __builtin_amdgcn_ds_swizzle((int)(b >> 32), (O << 10) | 0x1f);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
RTC_DEV double half_sum_f64(double v) {
  v += swz_xor_f64<16>(v);
  v += swz_xor_f64<8>(v);
  v += swz_xor_f64<4>(v);
  v += swz_xor_f64<2>(v);
  v += swz_xor_f64<1>(v);
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

// The forward product's path operand A'[i, m] = a_i g_m exp(j psi_i (m - c))
// exp(-j 2 pi f_ref tau_i), formed once per workgroup and shared through LDS
// (cfr_kernel, cfr_fused_kernel).  A stage holds nt/8 paths for nt threads:
// thread t forms the values of element t % 32 for paths 2 kp + e, kp = t / 32
// + (nt / 32) s (s, e in {0, 1}), splits them into FP16 parts and stores them
// in the lane layout of the MFMA operand -- path i of a 16-path chunk goes to
// lane m + 32 ((i % 16) / 8), element i % 8 of the part's 8-vector, parts
// re_h, re_l, im_h, im_l, 4 x 64 x 16 bytes per chunk -- and the stage's
// delays after them.  The path data of the next stage are fetched into
// registers (PathFetch) while the current stage's products run.
// nt is a multiple of 128, so that a stage is whole 16-path chunks.
struct PathFetch {
  float2 a[4];
  float psi[4];
  double tau[4];
};

constexpr int path_stage_paths(int nt) { return nt / 8; }
constexpr int path_stage_opnd_bytes(int nt) { return nt / 8 / 16 * 4 * 64 * 16; }
constexpr int path_stage_bytes(int nt) {
  return path_stage_opnd_bytes(nt) + path_stage_paths(nt) * 8;
}

// value v = 2 s + e of the thread: stage path 2 (t/32 + (nt/32) s) + e
RTC_DEV int path_stage_k(int v, int nt) {
  return 2 * ((int)(threadIdx.x >> 5) + (nt >> 5) * (v >> 1)) + (v & 1);
}

// loads clamp to the link's last path (a valid address); the store zeroes
// the paths past it
RTC_DEV void path_fetch(const float2* a, const float* psi, const double* tau, int64_t s0,
                        int64_t off1, int nt, PathFetch& F) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t p = s0 + path_stage_k(v, nt);
    const int64_t pc = p < off1 ? p : off1 - 1;
    F.a[v] = a[pc];
    F.psi[v] = psi[pc];
    F.tau[v] = tau[pc];
  }
}

// col = t % 32, gm = g_m times the link's power-of-two scale, mc_cyc = (m - c)
// / (2 pi); opnd and tau_s: the stage's LDS areas
RTC_DEV void path_stage_store(const PathFetch& F, int64_t s0, int64_t off1, int nt, double fref,
                              double mc_cyc, float2 gm, int col, unsigned* opnd, double* tau_s) {
#pragma unroll
  for (int sp = 0; sp < 2; ++sp) {
    float re[2], im[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int v = 2 * sp + e;
      const int64_t p = s0 + path_stage_k(v, nt);
      float2 b = make_float2(0.0f, 0.0f);
      if (p < off1) {
        // exp(j psi_i (m - c)) c_i as one phase, in cycles
        const float2 ph = expm2pi_f64_hw(fma(fref, F.tau[v], -(double)F.psi[v] * mc_cyc));
        b = cmul(cmul(F.a[v], gm), ph);
      }
      re[e] = b.x;
      im[e] = b.y;
      if (col == 0) tau_s[path_stage_k(v, nt)] = p < off1 ? F.tau[v] : 0.0;  // any finite phase
    }
    const int k = path_stage_k(2 * sp, nt);  // even
    const unsigned wr = pack_f16(re[0], re[1]);
    const unsigned wi = pack_f16(im[0], im[1]);
    const unsigned lr = pack_f16(sub_f16<true>(re[0], wr), sub_f16<false>(re[1], wr));
    const unsigned li = pack_f16(sub_f16<true>(im[0], wi), sub_f16<false>(im[1], wi));
    const int c = k >> 4;
    const int sl = col + 32 * ((k & 15) >> 3);
    const int w32 = (k & 7) >> 1;
    opnd[((c * 4 + 0) * 64 + sl) * 4 + w32] = wr;
    opnd[((c * 4 + 1) * 64 + sl) * 4 + w32] = lr;
    opnd[((c * 4 + 2) * 64 + sl) * 4 + w32] = wi;
    opnd[((c * 4 + 3) * 64 + sl) * 4 + w32] = li;
  }
}

// chunk c of the stage: the lane's A' parts
RTC_DEV void path_stage_read(const unsigned* opnd, int c, int lane, Split2& AR, Split2& AI) {
  const u32x4* ob = reinterpret_cast<const u32x4*>(opnd) + (c * 4) * 64 + lane;
  AR.h = __builtin_bit_cast(halfx8, ob[0]);
  AR.l = __builtin_bit_cast(halfx8, ob[64]);
  AI.h = __builtin_bit_cast(halfx8, ob[128]);
  AI.l = __builtin_bit_cast(halfx8, ob[192]);
}

}  // namespace rtc
