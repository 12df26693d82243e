// Workgroup-wide radix-2 FFT in LDS and a fixed-order workgroup sum, for
// CFR rows longer than one wave's register FFT handles.
#pragma once

#include "dev_common.h"

namespace rtc {

// tw[k] = exp(-j 2 pi k / N), k < N/2
RTC_DEV void make_twiddles(float2* tw, int N) {
  for (int k = threadIdx.x; k < N / 2; k += blockDim.x) {
    float s, c;
    sincos2pi((float)k / (float)N, &s, &c);  // k/N exact for N = 2^k
    tw[k] = make_float2(c, -s);
  }
}

// In-place radix-2 decimation-in-time FFT on bit-reversed input.
// SIGN = -1: X_k = sum x_n e^{-j 2 pi nk/N}; SIGN = +1: e^{+j...}.
template <int SIGN>
RTC_DEV void fft_lds(float2* x, const float2* tw, int N, int logN) {
  for (int s = 1; s <= logN; ++s) {
    const int mh = 1 << (s - 1);
    const int tstride = N >> s;
    for (int b = threadIdx.x; b < N / 2; b += blockDim.x) {
      const int k = b & (mh - 1);
      const int i0 = ((b >> (s - 1)) << s) + k;
      const int i1 = i0 + mh;
      float2 w = tw[k * tstride];
      if (SIGN > 0) w.y = -w.y;
      float2 u = x[i0];
      float2 v = cmul(x[i1], w);
      x[i0] = cadd(u, v);
      x[i1] = csub(u, v);
    }
    __syncthreads();
  }
}

RTC_DEV int bitrev(int i, int logN) { return (int)(__brev((unsigned)i) >> (32 - logN)); }

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

}  // namespace rtc
