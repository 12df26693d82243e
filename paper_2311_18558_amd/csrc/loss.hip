// Coherent + power-delay-profile CFR loss and its gradient dL/dH.
//
// The threads of one row (one wave up to 1024 subcarriers, N/16 beyond)
// transform it to the CIR taps of the centred 1/sqrt(N) IDFT (Sec. II-A) with
// a register Stockham FFT (fft_wave.h); the power delay profile is
// p_l = |h[l]|^2 = |X_l|^2 / N with X the unnormalised inverse DFT (the
// centring multiplies taps by unit-modulus factors and reorders them, which
// changes neither |.|^2 nor the sums).
//
// With Z_c = sum|H*|^2 and Z_p = sum (p*)^2 over the batch,
//   L = w_c sum|H - H*|^2 / Z_c + w_p sum (p - p*)^2 / Z_p
//   dL/dH_n = 2 w_c (H_n - H*_n) / Z_c + FFT_n[ 4 w_p (p - p*) X / (N Z_p) ]
// (the second term is the adjoint of the unitary IDFT applied to
// dL/dh = 4 w_p (p - p*) h / Z_p).  Per-row partial sums are written in FP64
// and reduced across rows in a fixed order.
#include <cmath>
#include <mutex>

#include "api_common.h"
#include "dev_common.h"
#include "fft_wave.h"

namespace rtc {

constexpr int kRedBlock = 256;
constexpr int kRedChunk = 64;  // rows per reduction block (first two levels)

// ------------------------------------------------------- register-FFT rows
// T = fft_threads(LOGN) threads own a row: one wave up to N = 1024, N/16
// threads (one radix-16 butterfly each per pass) beyond.  The H and H* rows
// are read straight into the first FFT pass, the last inverse pass leaves
// the taps in dL/dH in the row's natural order, next to H - H* kept from the
// load.  Up to 1,024 points four waves share a workgroup, each taking its own
// rows and transforming them in place in its own LDS buffer, with the
// twiddles from the workgroup's LDS rows (fft_row_waves, fft_twiddle_tab);
// longer rows ping-pong between two buffers of the workgroup.  With PT
// the target PDP comes precomputed (p_tgt from the target statistics)
// instead of from a transform of H*.

// TGT: 0 = targets H* (p* by a transform of H*), 1 = H* and a stored p*,
// 2 = the targets' transforms X* (rtc_cfr_target_cir): then the coherent
// term is taken by Parseval, sum |H - H*|^2 = sum |X - X*|^2 / N, the PDP
// target is |X*|^2 / N, and dL/dH = IDFT(gc/N (X - X*) + gp (p - p*) X)
// (unnormalised inverse): two transforms per row and nothing of H* kept.
template <int LOGN, int TGT>
__global__ void __launch_bounds__(fft_threads(LOGN) * fft_row_waves(LOGN))
    cfr_loss_wave_kernel(const float2* H, const float2* __restrict__ Ht,
                         const float* __restrict__ Pt, int64_t n_rows, const double* Z,
                         float w_coh, float w_pdp, double* row_out, float2* dLdH) {
  constexpr int N = 1 << LOGN;
  constexpr int NP = fft_npass(LOGN);
  constexpr int RA = fft_radix(LOGN, 0), RZ = fft_radix(LOGN, NP - 1);
  constexpr int T = fft_threads(LOGN);
  constexpr int JA = fft_bpl(N, RA, T), JZ = fft_bpl(N, RZ, T);
  constexpr int BA = N / RA, BZ = N / RZ;
  RTC_FFT_ROWS_SETUP();
  const float invN = 1.0f / (float)N;
  float gc = 0.0f, gp = 0.0f;
  if (dLdH) {
    gc = (float)(2.0 * (double)w_coh / Z[0]);
    gp = (float)(4.0 * (double)w_pdp / (Z[1] * (double)N));
  }
  for (int64_t row = (int64_t)blockIdx.x * W + wv; row < n_rows; row += (int64_t)gridDim.x * W) {
    int lane = lane0;
    asm volatile("" : "+v"(lane));  // twiddles per row, not held across rows
    const float2* hs = H + row * N;
    const float2* ts = Ht + row * N;
    float ec = 0.0f, et = 0.0f;
    if constexpr (TGT == 2) {
      // X* in the last pass's layout (natural tap order j + r BZ)
      float2 xs[JZ][RZ];
#pragma unroll
      for (int i = 0; i < JZ; ++i) {
        const int j = lane + T * i;
#pragma unroll
        for (int r = 0; r < RZ; ++r)
          xs[i][r] = (BZ % T == 0 || j < BZ) ? ts[j + r * BZ] : make_float2(0.0f, 0.0f);
      }
      float2 vh[JA][RA];
#pragma unroll
      for (int i = 0; i < JA; ++i) {
        const int j = lane + T * i;
#pragma unroll
        for (int r = 0; r < RA; ++r)
          vh[i][r] = (BA % T == 0 || j < BA) ? hs[j + r * BA] : make_float2(0.0f, 0.0f);
      }
      float2 xh[JZ][RZ];
      fft_full<LOGN, +1, +1, SY, T, TAB>(vh, xh, b0, b1, lane, twr);
      const float gcn = gc * invN;
      float ep = 0.0f, eq = 0.0f;
#pragma unroll
      for (int i = 0; i < JZ; ++i) {
        const int j = lane + T * i;
        if (BZ % T == 0 || j < BZ) {
#pragma unroll
          for (int r = 0; r < RZ; ++r) {
            const float2 dx = csub(xh[i][r], xs[i][r]);
            ec += cabs2(dx);
            const float pt = cabs2(xs[i][r]) * invN;
            et += pt;
            const float d = cabs2(xh[i][r]) * invN - pt;
            ep += d * d;
            eq += pt * pt;
            xh[i][r] = cadd(cscale(dx, gcn), cscale(xh[i][r], gp * d));
          }
        }
      }
      double s1 = group_sum_f64<T>((double)ec * (double)invN, red);
      double s2 = group_sum_f64<T>((double)et, red);
      double s3 = group_sum_f64<T>((double)ep, red);
      double s4 = group_sum_f64<T>((double)eq, red);
      if (lane == 0) {
        row_out[row * 4 + 0] = s1;
        row_out[row * 4 + 1] = s2;
        row_out[row * 4 + 2] = s3;
        row_out[row * 4 + 3] = s4;
      }
      if (dLdH) {
        float2 G[JA][RA];
        fft_full<LOGN, -1, -1, SY, T, TAB>(xh, G, b0, b1, lane, twr);
        float2* out = dLdH + row * N;
#pragma unroll
        for (int i = 0; i < JA; ++i) {
          const int j = lane + T * i;
          if (BA % T == 0 || j < BA) {
#pragma unroll
            for (int r = 0; r < RA; ++r) out[j + r * BA] = G[i][r];
          }
        }
      }
      continue;
    }
    float pt[JZ][RZ];
    if constexpr (TGT == 1) {
      const float* ps = Pt + row * N;
#pragma unroll
      for (int i = 0; i < JZ; ++i) {
        const int j = lane + T * i;
#pragma unroll
        for (int r = 0; r < RZ; ++r)
          pt[i][r] = (BZ % T == 0 || j < BZ) ? ps[j + r * BZ] : 0.0f;
      }
    } else {
      float2 vt[JA][RA], xt[JZ][RZ];
#pragma unroll
      for (int i = 0; i < JA; ++i) {
        const int j = lane + T * i;
#pragma unroll
        for (int r = 0; r < RA; ++r)
          vt[i][r] = (BA % T == 0 || j < BA) ? ts[j + r * BA] : make_float2(0.0f, 0.0f);
      }
      fft_full<LOGN, +1, +1, SY, T, TAB>(vt, xt, b0, b1, lane, twr);
#pragma unroll
      for (int i = 0; i < JZ; ++i) {
#pragma unroll
        for (int r = 0; r < RZ; ++r) pt[i][r] = cabs2(xt[i][r]) * invN;
      }
    }
    float2 vh[JA][RA], diff[JA][RA];
#pragma unroll
    for (int i = 0; i < JA; ++i) {
      const int j = lane + T * i;
#pragma unroll
      for (int r = 0; r < RA; ++r) {
        const float2 h = (BA % T == 0 || j < BA) ? hs[j + r * BA] : make_float2(0.0f, 0.0f);
        const float2 t = (BA % T == 0 || j < BA) ? ts[j + r * BA] : make_float2(0.0f, 0.0f);
        vh[i][r] = h;
        diff[i][r] = csub(h, t);
        ec += cabs2(diff[i][r]);
        et += cabs2(t);
      }
    }
    float2 xh[JZ][RZ];
    fft_full<LOGN, +1, +1, SY, T, TAB>(vh, xh, b0, b1, lane, twr);
    float ep = 0.0f, eq = 0.0f;
#pragma unroll
    for (int i = 0; i < JZ; ++i) {
      const int j = lane + T * i;
      if (BZ % T == 0 || j < BZ) {
#pragma unroll
        for (int r = 0; r < RZ; ++r) {
          const float p = cabs2(xh[i][r]) * invN;
          const float d = p - pt[i][r];
          ep += d * d;
          eq += pt[i][r] * pt[i][r];
          xh[i][r] = cscale(xh[i][r], gp * d);  // gradient source
        }
      }
    }
    double s1 = group_sum_f64<T>((double)ec, red);
    double s2 = group_sum_f64<T>((double)et, red);
    double s3 = group_sum_f64<T>((double)ep, red);
    double s4 = group_sum_f64<T>((double)eq, red);
    if (lane == 0) {
      row_out[row * 4 + 0] = s1;
      row_out[row * 4 + 1] = s2;
      row_out[row * 4 + 2] = s3;
      row_out[row * 4 + 3] = s4;
    }
    if (dLdH) {
      float2 G[JA][RA];
      fft_full<LOGN, -1, -1, SY, T, TAB>(xh, G, b0, b1, lane, twr);
      float2* out = dLdH + row * N;
#pragma unroll
      for (int i = 0; i < JA; ++i) {
        const int j = lane + T * i;
        if (BA % T == 0 || j < BA) {
#pragma unroll
          for (int r = 0; r < RA; ++r) out[j + r * BA] = cadd(cscale(diff[i][r], gc), G[i][r]);
        }
      }
    }
  }
}

// Target statistics per row {sum |H*|^2, sum (p*)^2}; with Pt also the
// target PDP p* (natural tap order) for later loss calls, with Xt the
// transform X* itself (natural tap order).
template <int LOGN>
__global__ void __launch_bounds__(fft_threads(LOGN) * fft_row_waves(LOGN))
    target_stats_wave_kernel(const float2* __restrict__ Ht, int64_t n_rows, double* row_out,
                             float* Pt, float2* Xt) {
  constexpr int N = 1 << LOGN;
  constexpr int NP = fft_npass(LOGN);
  constexpr int RA = fft_radix(LOGN, 0), RZ = fft_radix(LOGN, NP - 1);
  constexpr int T = fft_threads(LOGN);
  constexpr int JA = fft_bpl(N, RA, T), JZ = fft_bpl(N, RZ, T);
  constexpr int BA = N / RA, BZ = N / RZ;
  RTC_FFT_ROWS_SETUP();
  const int lane = lane0;
  const float invN = 1.0f / (float)N;
  for (int64_t row = (int64_t)blockIdx.x * W + wv; row < n_rows; row += (int64_t)gridDim.x * W) {
    const float2* ts = Ht + row * N;
    float2 vt[JA][RA];
    float et = 0.0f;
#pragma unroll
    for (int i = 0; i < JA; ++i) {
      const int j = lane + T * i;
      if (BA % T == 0 || j < BA) {
#pragma unroll
        for (int r = 0; r < RA; ++r) {
          vt[i][r] = ts[j + r * BA];
          et += cabs2(vt[i][r]);
        }
      }
    }
    float2 xt[JZ][RZ];
    fft_full<LOGN, +1, +1, SY, T, TAB>(vt, xt, b0, b1, lane, twr);
    float eq = 0.0f;
#pragma unroll
    for (int i = 0; i < JZ; ++i) {
      const int j = lane + T * i;
      if (BZ % T == 0 || j < BZ) {
#pragma unroll
        for (int r = 0; r < RZ; ++r) {
          const float pt = cabs2(xt[i][r]) * invN;
          eq += pt * pt;
          if (Pt) Pt[row * N + j + r * BZ] = pt;
          if (Xt) Xt[row * N + j + r * BZ] = xt[i][r];
        }
      }
    }
    double se = group_sum_f64<T>((double)et, red);
    double sq = group_sum_f64<T>((double)eq, red);
    if (lane == 0) {
      row_out[row * 2 + 0] = se;
      row_out[row * 2 + 1] = sq;
    }
  }
}

// Fixed-order reduction of [R][K] doubles: block b sums rows
// [b C, min(R, (b + 1) C)) into out[b][K].  For K <= kRedBlock thread t
// takes column t % K on row lane t / K (a row is read by K neighbouring
// threads) and the lanes' partial sums are added in lane order; wider rows
// are walked column by column by one thread each.
__global__ void __launch_bounds__(kRedBlock)
    reduce_rows_kernel(const double* in, int64_t R, int K, int64_t C, double* out) {
  __shared__ double part[kRedBlock];
  const int64_t r0 = (int64_t)blockIdx.x * C;
  const int64_t r1 = r0 + C < R ? r0 + C : R;
  const int t = threadIdx.x;
  double* dst = out + (int64_t)blockIdx.x * K;
  if (K > kRedBlock) {
    for (int c = t; c < K; c += kRedBlock) {
      double v = 0.0;
      for (int64_t r = r0; r < r1; ++r) v += in[r * K + c];
      dst[c] = v;
    }
    return;
  }
  const int lanes = kRedBlock / K;
  const int c = t % K, lane = t / K;
  double v = 0.0;
  if (lane < lanes)
    for (int64_t r = r0 + lane; r < r1; r += lanes) v += in[r * K + c];
  part[t] = v;
  __syncthreads();
  if (t < K) {
    double s = 0.0;
    for (int i = 0; i < lanes; ++i) s += part[i * K + t];
    dst[t] = s;
  }
}

__global__ void loss_finish_kernel(const double* sums, const double* Z, float w_coh, float w_pdp,
                                   double* loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double zc = Z ? Z[0] : sums[1];
  double zp = Z ? Z[1] : sums[3];
  double coh = sums[0] / zc;
  double pdp = sums[2] / zp;
  loss[0] = (double)w_coh * coh + (double)w_pdp * pdp;
  loss[1] = coh;
  loss[2] = pdp;
}

__global__ void copy2_kernel(const double* src, double* dst) {
  if (threadIdx.x < 2 && blockIdx.x == 0) dst[threadIdx.x] = src[threadIdx.x];
}

static int ilog2(int n) {
  int k = 0;
  while ((1 << k) < n) ++k;
  return k;
}

static int64_t n_red1(int64_t R) { return (R + kRedChunk - 1) / kRedChunk; }

// Reduce rows -> [K] in `dst` using `tmp` (n_red1(R)*K doubles, and a second
// level if needed).
size_t reduce_tmp_doubles(int64_t R, int K) {
  int64_t R1 = n_red1(R), R2 = n_red1(R1);
  return (size_t)((R1 + R2 + 1) * K);
}

rtc_status reduce_all(const double* rows, int64_t R, int K, double* tmp, double* dst,
                      hipStream_t s, const char* fn) {
  const int64_t C = kRedChunk;
  int64_t R1 = n_red1(R);
  hipLaunchKernelGGL(reduce_rows_kernel, dim3((unsigned)R1), dim3(kRedBlock), 0, s, rows, R, K, C,
                     R1 == 1 ? dst : tmp);
  rtc_status st = check_launch(fn);
  if (st != RTC_OK || R1 == 1) return st;
  int64_t R2 = n_red1(R1);
  double* tmp2 = tmp + R1 * K;
  hipLaunchKernelGGL(reduce_rows_kernel, dim3((unsigned)R2), dim3(kRedBlock), 0, s, tmp, R1, K, C,
                     R2 == 1 ? dst : tmp2);
  if ((st = check_launch(fn)) != RTC_OK || R2 == 1) return st;
  // the last level is one block over all R2 rows, whatever their number
  hipLaunchKernelGGL(reduce_rows_kernel, dim3(1), dim3(kRedBlock), 0, s, tmp2, R2, K, R2, dst);
  return check_launch(fn);
}

// Workspace layout (doubles): rows[R*4] | red[(R1 + R2 + 1) * 4] | Z[2] | sums[4]
static size_t ws_doubles(int64_t R) {
  int64_t R1 = n_red1(R), R2 = n_red1(R1);
  return (size_t)(R * 4 + (R1 + R2 + 1) * 4 + 2 + 4);
}

size_t ws_cfr_loss(const rtc_radio* r, int32_t n_links) {
  int64_t R = (int64_t)(n_links > 0 ? n_links : 1) * (r->n_elem > 0 ? r->n_elem : 1);
  return ws_doubles(R) * sizeof(double);
}

size_t ws_target_stats(const rtc_radio* r, int32_t n_links) { return ws_cfr_loss(r, n_links); }

// workgroups for R rows of 2^logn points (fft_row_waves rows in flight each)
static unsigned wave_grid(int64_t R, int logn) {
  const int w = fft_row_waves(logn);
  int64_t g = (R + w - 1) / w;
  g = g < 40960 / w ? g : 40960 / w;
  return (unsigned)(g > 0 ? g : 1);
}
static unsigned row_block(int logn) { return (unsigned)(fft_threads(logn) * fft_row_waves(logn)); }

static void launch_target_stats(int logN, const float2* Ht, int64_t R, double* rows, float* Pt,
                                float2* Xt, hipStream_t s) {
  switch (logN) {
#define RTC_TS(L)                                                                            \
  case L:                                                                                    \
    hipLaunchKernelGGL(target_stats_wave_kernel<L>, dim3(wave_grid(R, L)),                      \
                       dim3(row_block(L)), 0, s, Ht, R, rows, Pt, Xt);                     \
    return;
    RTC_TS(1) RTC_TS(2) RTC_TS(3) RTC_TS(4) RTC_TS(5) RTC_TS(6) RTC_TS(7) RTC_TS(8) RTC_TS(9)
    RTC_TS(10) RTC_TS(11) RTC_TS(12)
#undef RTC_TS
    default:
      return;  // n_sc is checked by the entry points
  }
}

// tgt: the TGT mode of cfr_loss_wave_kernel (Ht is X* for mode 2)
static void launch_loss(int logN, int tgt, const float2* H, const float2* Ht, const float* Pt,
                        int64_t R, const double* Z, float w_coh, float w_pdp, double* rows,
                        float2* dLdH, hipStream_t s) {
  switch (logN) {
#define RTC_LW(L)                                                                             \
  case L:                                                                                     \
    if (tgt == 2)                                                                             \
      hipLaunchKernelGGL((cfr_loss_wave_kernel<L, 2>), dim3(wave_grid(R, L)),                    \
                         dim3(row_block(L)), 0, s, H, Ht, Pt, R, Z, w_coh, w_pdp, rows,     \
                         dLdH);                                                               \
    else if (tgt == 1)                                                                        \
      hipLaunchKernelGGL((cfr_loss_wave_kernel<L, 1>), dim3(wave_grid(R, L)),                    \
                         dim3(row_block(L)), 0, s, H, Ht, Pt, R, Z, w_coh, w_pdp, rows,     \
                         dLdH);                                                               \
    else                                                                                      \
      hipLaunchKernelGGL((cfr_loss_wave_kernel<L, 0>), dim3(wave_grid(R, L)),                    \
                         dim3(row_block(L)), 0, s, H, Ht, Pt, R, Z, w_coh, w_pdp, rows,     \
                         dLdH);                                                               \
    return;
    RTC_LW(1) RTC_LW(2) RTC_LW(3) RTC_LW(4) RTC_LW(5) RTC_LW(6) RTC_LW(7) RTC_LW(8) RTC_LW(9)
    RTC_LW(10) RTC_LW(11) RTC_LW(12)
#undef RTC_LW
    default:
      return;  // n_sc is checked by the entry points
  }
}

}  // namespace rtc

using namespace rtc;

static rtc_status check_fft_n(const rtc_radio* r, const char* fn) {
  RTC_REQUIRE(is_pow2(r->n_sc) && r->n_sc >= 2 && r->n_sc <= kMaxFFT, RTC_ERR_UNSUPPORTED,
              "%s: n_sc must be a power of two in [2, %d]", fn, kMaxFFT);
  return RTC_OK;
}

extern "C" rtc_status rtc_cfr_target_stats(const rtc_radio* radio, int32_t n_links,
                                           const void* H_tgt, double* stats, float* p_tgt,
                                           void* ws, size_t ws_bytes, void* stream) {
  const char* fn = "rtc_cfr_target_stats";
  rtc_status st;
  if ((st = check_radio(radio, fn)) != RTC_OK) return st;
  if ((st = check_fft_n(radio, fn)) != RTC_OK) return st;
  RTC_REQUIRE(n_links >= 1, RTC_ERR_SHAPE, "%s: n_links must be >= 1", fn);
  RTC_REQUIRE(H_tgt && stats, RTC_ERR_INVALID_ARG, "%s: H_tgt and stats are required", fn);
  int64_t R = (int64_t)n_links * radio->n_elem;
  size_t need = ws_target_stats(radio, n_links);
  RTC_REQUIRE(ws != nullptr && ws_bytes >= need, RTC_ERR_WORKSPACE,
              "%s: workspace of %zu bytes required", fn, need);
  hipStream_t s = as_stream(stream);
  double* rows = reinterpret_cast<double*>(ws);
  double* red = rows + R * 4;
  int N = radio->n_sc, logN = ilog2(N);
  (void)N;
  launch_target_stats(logN, reinterpret_cast<const float2*>(H_tgt), R, rows, p_tgt, nullptr, s);
  if ((st = check_launch(fn)) != RTC_OK) return st;
  return reduce_all(rows, R, 2, red, stats, s, fn);
}

extern "C" rtc_status rtc_cfr_target_cir(const rtc_radio* radio, int32_t n_links,
                                         const void* H_tgt, double* stats, void* X_tgt, void* ws,
                                         size_t ws_bytes, void* stream) {
  const char* fn = "rtc_cfr_target_cir";
  rtc_status st;
  if ((st = check_radio(radio, fn)) != RTC_OK) return st;
  if ((st = check_fft_n(radio, fn)) != RTC_OK) return st;
  RTC_REQUIRE(n_links >= 1, RTC_ERR_SHAPE, "%s: n_links must be >= 1", fn);
  RTC_REQUIRE(H_tgt && stats && X_tgt, RTC_ERR_INVALID_ARG,
              "%s: H_tgt, stats and X_tgt are required", fn);
  RTC_REQUIRE(X_tgt != H_tgt, RTC_ERR_INVALID_ARG, "%s: X_tgt must not alias H_tgt", fn);
  int64_t R = (int64_t)n_links * radio->n_elem;
  size_t need = ws_target_stats(radio, n_links);
  RTC_REQUIRE(ws != nullptr && ws_bytes >= need, RTC_ERR_WORKSPACE,
              "%s: workspace of %zu bytes required", fn, need);
  hipStream_t s = as_stream(stream);
  double* rows = reinterpret_cast<double*>(ws);
  double* red = rows + R * 4;
  launch_target_stats(ilog2(radio->n_sc), reinterpret_cast<const float2*>(H_tgt), R, rows,
                      nullptr, reinterpret_cast<float2*>(X_tgt), s);
  if ((st = check_launch(fn)) != RTC_OK) return st;
  return reduce_all(rows, R, 2, red, stats, s, fn);
}

// The loss pass of rtc_cfr_loss over a workspace of ws_bytes bytes (checked
// by the caller).
static rtc_status cfr_loss_run(const char* fn, const rtc_radio* radio, int32_t n_links,
                               const void* H, const void* H_tgt, const double* tgt_stats,
                               const float* p_tgt, float w_coh, float w_pdp, double* loss,
                               void* dLdH, double* rows, hipStream_t s) {
  rtc_status st;
  int64_t R = (int64_t)n_links * radio->n_elem;
  int64_t R1 = n_red1(R), R2 = n_red1(R1);
  double* red = rows + R * 4;
  double* Z = red + (R1 + R2 + 1) * 4;
  double* sums = Z + 2;
  int logN = ilog2(radio->n_sc);
  const double* Zuse = tgt_stats;
  if (dLdH && !tgt_stats) {
    launch_target_stats(logN, reinterpret_cast<const float2*>(H_tgt), R, rows, nullptr, nullptr,
                        s);
    if ((st = check_launch(fn)) != RTC_OK) return st;
    if ((st = reduce_all(rows, R, 2, red, Z, s, fn)) != RTC_OK) return st;
    Zuse = Z;
  }
  launch_loss(logN, p_tgt ? 1 : 0, reinterpret_cast<const float2*>(H),
              reinterpret_cast<const float2*>(H_tgt), p_tgt, R, Zuse, w_coh, w_pdp, rows,
              reinterpret_cast<float2*>(dLdH), s);
  if ((st = check_launch(fn)) != RTC_OK) return st;
  if ((st = reduce_all(rows, R, 4, red, sums, s, fn)) != RTC_OK) return st;
  hipLaunchKernelGGL(loss_finish_kernel, dim3(1), dim3(64), 0, s, sums, Zuse, w_coh, w_pdp, loss);
  return check_launch(fn);
}

static rtc_status cfr_loss_check(const char* fn, const rtc_radio* radio, int32_t n_links,
                                 const void* H, const void* H_tgt, double* loss,
                                 const void* dLdH) {
  rtc_status st;
  if ((st = check_radio(radio, fn)) != RTC_OK) return st;
  if ((st = check_fft_n(radio, fn)) != RTC_OK) return st;
  RTC_REQUIRE(n_links >= 1, RTC_ERR_SHAPE, "%s: n_links must be >= 1", fn);
  RTC_REQUIRE(H && H_tgt && loss, RTC_ERR_INVALID_ARG, "%s: H, H_tgt and loss are required", fn);
  RTC_REQUIRE(dLdH != H_tgt, RTC_ERR_INVALID_ARG, "%s: dLdH must not alias H_tgt", fn);
  return RTC_OK;
}

extern "C" rtc_status rtc_cfr_loss(const rtc_radio* radio, int32_t n_links, const void* H,
                                   const void* H_tgt, const double* tgt_stats,
                                   const float* p_tgt, float w_coh, float w_pdp, double* loss,
                                   void* dLdH, void* ws, size_t ws_bytes, void* stream) {
  const char* fn = "rtc_cfr_loss";
  rtc_status st;
  if ((st = cfr_loss_check(fn, radio, n_links, H, H_tgt, loss, dLdH)) != RTC_OK) return st;
  size_t need = ws_cfr_loss(radio, n_links);
  RTC_REQUIRE(ws != nullptr && ws_bytes >= need, RTC_ERR_WORKSPACE,
              "%s: workspace of %zu bytes required", fn, need);
  return cfr_loss_run(fn, radio, n_links, H, H_tgt, tgt_stats, p_tgt, w_coh, w_pdp, loss, dLdH,
                      reinterpret_cast<double*>(ws), as_stream(stream));
}

extern "C" rtc_status rtc_cfr_loss_cir(const rtc_radio* radio, int32_t n_links, const void* H,
                                       const void* X_tgt, const double* tgt_stats, float w_coh,
                                       float w_pdp, double* loss, void* dLdH, void* ws,
                                       size_t ws_bytes, void* stream) {
  const char* fn = "rtc_cfr_loss_cir";
  rtc_status st;
  if ((st = check_radio(radio, fn)) != RTC_OK) return st;
  if ((st = check_fft_n(radio, fn)) != RTC_OK) return st;
  RTC_REQUIRE(n_links >= 1, RTC_ERR_SHAPE, "%s: n_links must be >= 1", fn);
  RTC_REQUIRE(H && X_tgt && loss, RTC_ERR_INVALID_ARG, "%s: H, X_tgt and loss are required", fn);
  RTC_REQUIRE(dLdH != X_tgt, RTC_ERR_INVALID_ARG, "%s: dLdH must not alias X_tgt", fn);
  RTC_REQUIRE(tgt_stats || !dLdH, RTC_ERR_INVALID_ARG,
              "%s: tgt_stats (rtc_cfr_target_cir) is required for dLdH", fn);
  const size_t need = ws_cfr_loss(radio, n_links);
  RTC_REQUIRE(ws != nullptr && ws_bytes >= need, RTC_ERR_WORKSPACE,
              "%s: workspace of %zu bytes required", fn, need);
  hipStream_t s = as_stream(stream);
  const int64_t R = (int64_t)n_links * radio->n_elem;
  double* rows = reinterpret_cast<double*>(ws);
  double* red = rows + R * 4;
  double* sums = red + (n_red1(R) + n_red1(n_red1(R)) + 1) * 4 + 2;
  launch_loss(ilog2(radio->n_sc), 2, reinterpret_cast<const float2*>(H),
              reinterpret_cast<const float2*>(X_tgt), nullptr, R, tgt_stats, w_coh, w_pdp, rows,
              reinterpret_cast<float2*>(dLdH), s);
  if ((st = check_launch(fn)) != RTC_OK) return st;
  if ((st = reduce_all(rows, R, 4, red, sums, s, fn)) != RTC_OK) return st;
  hipLaunchKernelGGL(loss_finish_kernel, dim3(1), dim3(64), 0, s, sums, tgt_stats, w_coh, w_pdp,
                     loss);
  return check_launch(fn);
}

// ------------------------------------------------ the allocation-free variant
// rtc_cfr_loss_noalloc runs the same kernels with their workspace in a
// file-scope device array, one copy per GPU, so that it needs no memory
// beyond its inputs and outputs.  The array's device address on each GPU is
// looked up once (hipGetSymbolAddress, with that GPU current) and kept; host
// code never passes the array's own name to a kernel.
namespace rtc {
constexpr int64_t kNoAllocRows = int64_t(1) << 19;  // links x elements
constexpr int64_t kNoAllocDoubles =
    kNoAllocRows * 4 + ((kNoAllocRows + kRedChunk - 1) / kRedChunk +
                        ((kNoAllocRows + kRedChunk - 1) / kRedChunk + kRedChunk - 1) / kRedChunk +
                        1) * 4 + 2 + 4;
constexpr int kNoAllocMaxDevices = 64;
}  // namespace rtc

static __device__ __align__(256) double scratch[rtc::kNoAllocDoubles];

static std::mutex g_scratch_mu;
static double* g_scratch_ptr[rtc::kNoAllocMaxDevices];

static rtc_status scratch_on_current_device(const char* fn, double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  RTC_REQUIRE(e == hipSuccess, RTC_ERR_HIP, "%s: hipGetDevice failed: %s", fn,
              hipGetErrorString(e));
  RTC_REQUIRE(dev >= 0 && dev < rtc::kNoAllocMaxDevices, RTC_ERR_RANGE,
              "%s: device %d beyond the %d devices supported", fn, dev, rtc::kNoAllocMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    RTC_REQUIRE(e == hipSuccess && p != nullptr, RTC_ERR_HIP,
                "%s: hipGetSymbolAddress of the scratch array failed on device %d: %s", fn, dev,
                hipGetErrorString(e));
    g_scratch_ptr[dev] = reinterpret_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return RTC_OK;
}

extern "C" int64_t rtc_cfr_loss_noalloc_max_rows(void) { return rtc::kNoAllocRows; }

extern "C" rtc_status rtc_cfr_loss_noalloc(const rtc_radio* radio, int32_t n_links,
                                           const void* H, const void* H_tgt,
                                           const double* tgt_stats, const float* p_tgt,
                                           float w_coh, float w_pdp, double* loss, void* dLdH,
                                           void* stream) {
  const char* fn = "rtc_cfr_loss_noalloc";
  rtc_status st;
  if ((st = cfr_loss_check(fn, radio, n_links, H, H_tgt, loss, dLdH)) != RTC_OK) return st;
  const int64_t R = (int64_t)n_links * radio->n_elem;
  RTC_REQUIRE(R <= rtc::kNoAllocRows, RTC_ERR_RANGE,
              "%s: %lld rows (links x elements) exceed the %lld of its fixed scratch; use "
              "rtc_cfr_loss with a workspace",
              fn, (long long)R, (long long)rtc::kNoAllocRows);
  RTC_REQUIRE(ws_cfr_loss(radio, n_links) <= sizeof(double) * (size_t)rtc::kNoAllocDoubles,
              RTC_ERR_RANGE, "%s: workspace beyond the fixed scratch", fn);
  double* ws = nullptr;
  if ((st = scratch_on_current_device(fn, &ws)) != RTC_OK) return st;
  return cfr_loss_run(fn, radio, n_links, H, H_tgt, tgt_stats, p_tgt, w_coh, w_pdp, loss, dLdH,
                      ws, as_stream(stream));
}
