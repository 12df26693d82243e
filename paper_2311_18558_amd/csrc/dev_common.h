// Device-side helpers shared by the rtcal kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define RTC_DEV __device__ __forceinline__

// ---------------------------------------------------------------- complex
RTC_DEV float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
RTC_DEV float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
RTC_DEV float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
RTC_DEV float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
RTC_DEV float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// conj(a) * b
RTC_DEV float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
RTC_DEV float cabs2(float2 a) { return a.x * a.x + a.y * a.y; }
RTC_DEV float2 cdiv(float2 a, float2 b) {
  // scaled to keep |b|^2 in range for large permittivities
  float s = fmaxf(fabsf(b.x), fabsf(b.y));
  float inv = 1.0f / s;
  float2 bs = make_float2(b.x * inv, b.y * inv);
  float2 as = make_float2(a.x * inv, a.y * inv);
  float d = 1.0f / (bs.x * bs.x + bs.y * bs.y);
  return make_float2((as.x * bs.x + as.y * bs.y) * d, (as.y * bs.x - as.x * bs.y) * d);
}
// Principal square root (Re >= 0), written to avoid cancellation.
RTC_DEV float2 csqrt_principal(float2 z) {
  float r = hypotf(z.x, z.y);
  if (r == 0.0f) return make_float2(0.0f, 0.0f);
  if (z.x >= 0.0f) {
    float t = sqrtf(0.5f * (r + z.x));
    return make_float2(t, z.y / (2.0f * t));
  }
  float t = sqrtf(0.5f * (r - z.x));
  return make_float2(fabsf(z.y) / (2.0f * t), copysignf(t, z.y));
}

// ---------------------------------------------------------------- vectors
struct v3 {
  float x, y, z;
};
RTC_DEV v3 mk3(float x, float y, float z) { return v3{x, y, z}; }
RTC_DEV v3 sub3(v3 a, v3 b) { return v3{a.x - b.x, a.y - b.y, a.z - b.z}; }
RTC_DEV v3 add3(v3 a, v3 b) { return v3{a.x + b.x, a.y + b.y, a.z + b.z}; }
RTC_DEV v3 scl3(v3 a, float s) { return v3{a.x * s, a.y * s, a.z * s}; }
RTC_DEV float dot3(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
RTC_DEV v3 cross3(v3 a, v3 b) {
  return v3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
RTC_DEV v3 unit3(v3 a) { return scl3(a, 1.0f / sqrtf(dot3(a, a))); }

// theta_hat and phi_hat of the spherical basis at unit direction k, built
// without trigonometry: with rho = sqrt(kx^2+ky^2),
//   phi_hat = (-ky, kx, 0)/rho,  theta_hat = (kz kx/rho, kz ky/rho, -rho);
// at the poles phi = 0 is taken (phi_hat = y, theta_hat = (kz, 0, 0)).
RTC_DEV void sph_basis(v3 k, v3* th, v3* ph) {
  float rho = sqrtf(k.x * k.x + k.y * k.y);
  if (rho > 1e-20f) {
    float ir = 1.0f / rho;
    *ph = v3{-k.y * ir, k.x * ir, 0.0f};
    *th = v3{k.z * k.x * ir, k.z * k.y * ir, -rho};
  } else {
    *ph = v3{0.0f, 1.0f, 0.0f};
    *th = v3{k.z, 0.0f, 0.0f};
  }
}

// ------------------------------------------------------ trigonometry (2 pi)
// sin(2 pi x), cos(2 pi x) for any float x: exact reduction to the nearest
// quarter turn, then Taylor polynomials of sin/cos(2 pi r) on |r| <= 1/8
// (truncation error < 2e-9; coefficients (-1)^k (2 pi)^n / n!).
RTC_DEV void sincos2pi(float x, float* s_out, float* c_out) {
  float q = rintf(4.0f * x);
  float r = fmaf(q, -0.25f, x);  // exact
  int qi = (int)q;
  float r2 = r * r;
  float ps = 42.058693944897634f;
  ps = fmaf(ps, r2, -76.70585975306136f);
  ps = fmaf(ps, r2, 81.60524927607504f);
  ps = fmaf(ps, r2, -41.341702240399755f);
  ps = fmaf(ps, r2, 6.283185307179586f);
  ps = ps * r;
  float pc = -26.426256783374388f;
  pc = fmaf(pc, r2, 60.24464137187664f);
  pc = fmaf(pc, r2, -85.45681720669371f);
  pc = fmaf(pc, r2, 64.93939402266828f);
  pc = fmaf(pc, r2, -19.739208802178716f);
  pc = fmaf(pc, r2, 1.0f);
  // rotate by qi quarter turns
  float s = ps, c = pc;
  if (qi & 1) {
    float t = s;
    s = c;
    c = -t;
  }
  if (qi & 2) {
    s = -s;
    c = -c;
  }
  *s_out = s;
  *c_out = c;
}

// exp(-j 2 pi x) for an FP64 phase in cycles on the transcendental unit:
// v_fract_f64 reduces to [0, 1) exactly (a result that would round to 1 is
// returned as the largest double below it, the same phase), the remainder
// is rounded to FP32 and v_sin_f32 / v_cos_f32 take it in revolutions
// (measured on the device: max abs error 1.3e-7 over 2^20 points of
// [0, 1), against ~6e-8 for sincos2pi, at two instructions instead of ~20).
RTC_DEV float2 expm2pi_f64_hw(double x) {
  const float f = (float)__builtin_amdgcn_fract(x);
  return make_float2(__builtin_amdgcn_cosf(f), -__builtin_amdgcn_sinf(f));
}

// --------------------------------------------------------------- reductions
// Butterfly sum over the 64 lanes of a wave; every lane gets the total.  The
// combination order is fixed, so the result is reproducible.
RTC_DEV double wave_sum_f64(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
RTC_DEV float wave_sum_f32(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum of a double over the block in a fixed order (wave butterfly, then the
// waves in index order).  All threads must call; result valid on thread 0.
RTC_DEV double block_sum_f64(double v, double* red) {
  v = wave_sum_f64(v);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  __syncthreads();
  return s;
}
