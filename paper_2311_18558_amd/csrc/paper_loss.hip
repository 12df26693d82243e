// The paper's calibration loss on CIR statistics with the measurement scale
// estimate (Sec. III-E Eqs. loss, smape, delay_spread, channel_gain;
// Sec. III-F Eqs. scaling_param, alpha_hat), and the evaluation metrics of
// Sec. IV-C.
//
// Every CIR row (link, element) of N subcarriers is one example.  Its taps
// come from the unnormalised inverse DFT X of the row in storage order:
// p_l = |X_k|^2 / N at k = l mod N, the delay index l centred in
// [-N/2, N/2) (a path of delay tau lands at l = tau W, W = N df).  Per row
//   S0 = sum p,  tbar = sum l p / S0,  v = sum (l - tbar)^2 p / S0  (taps^2)
//   P^ = S0,  tau^ = sqrt(v) / W.
// With the measured (P_b, tau_b), the scale alpha and B rows,
//   L = (1/B) sum_b [w_t l(tau_b, tau^_b) + w_g l(alpha P_b, P^_b)]
//   l(x, y) = |x - y| / (x + y),   dl/dy = sgn(y - x) 2x / (x + y)^2
//   dL/dp_l = (1/B) [w_g g_g + w_t g_t ((l - tbar)^2 - v) / (2 W sqrt(v) S0)]
// (the derivative through tbar vanishes because sum (l - tbar) p = 0), and
// with p_l = |X_k|^2 / N and X the inverse DFT of H,
//   dL/dH_n = sum_k (2 dL/dp_k X_k / N) exp(-j 2 pi n k / N),
// one forward transform back.  alpha is a constant of the gradient.
//
// The least-squares scale uses P^_b = sum_n |H_n|^2 (equal to sum_l p_l by
// Parseval), so it needs no transform.
#include <cmath>

#include "api_common.h"
#include "dev_common.h"
#include "fft_wave.h"

namespace rtc {


struct PaperLossArgs {
  const double* tgt;    // [R][2] measured {P, tau_RMS}; loss only
  const double* alpha;  // [2] {alpha, updates}; loss only
  double* row_out;      // [R][2] {l_tau, l_gain}; loss only
  double* pred;         // [R][2] {P^, tau^} or null
  float2* dLdH;         // [R][N] or null
  double inv_B;         // 1 / rows
  double inv_W;         // 1 / bandwidth
  float w_tau, w_gain;
};

RTC_DEV float centred_tap(int k, int N) { return (float)(k < N / 2 ? k : k - N); }

RTC_DEV double smape_val(double x, double y) {
  const double s = x + y;
  return s > 0.0 ? fabs(x - y) / s : 0.0;
}

// d/dy |x - y| / (x + y); 0 at y = x and where x + y = 0
RTC_DEV double smape_dy(double x, double y) {
  const double s = x + y;
  if (!(s > 0.0) || y == x) return 0.0;
  const double g = 2.0 * x / (s * s);
  return y > x ? g : -g;
}

// Per-row loss terms and the coefficients of dL/dp_l = a0 + a1 ((l - tbar)^2
// - v), pre-multiplied by 2/N for the gradient source 2 dL/dp X / N.
struct RowGrad {
  float a0, a1;
};

RTC_DEV RowGrad row_loss(const PaperLossArgs& A, int64_t row, double alpha, double S0,
                         double v, double tau_hat, int N, bool write) {
  const double Pm = alpha * A.tgt[row * 2 + 0];
  const double tm = A.tgt[row * 2 + 1];
  if (write) {
    A.row_out[row * 2 + 0] = smape_val(tm, tau_hat);
    A.row_out[row * 2 + 1] = smape_val(Pm, S0);
  }
  const double c0 = A.inv_B * (double)A.w_gain * smape_dy(Pm, S0);
  const double c1 = (v > 0.0 && S0 > 0.0)
                        ? A.inv_B * (double)A.w_tau * smape_dy(tm, tau_hat) * A.inv_W /
                              (2.0 * sqrt(v) * S0)
                        : 0.0;
  return RowGrad{(float)(2.0 * c0 / N), (float)(2.0 * c1 / N)};
}

// ------------------------------------------------------- register-FFT rows
// T = fft_threads(LOGN) threads own a row (one wave up to N = 1024, four
// rows per workgroup then; N/16 threads beyond, fft_row_waves); the row is
// read straight into the first FFT pass and the gradient's transform leaves
// dL/dH in natural order.
template <int LOGN, bool LOSS>
__global__ void __launch_bounds__(fft_threads(LOGN) * fft_row_waves(LOGN))
    paper_loss_wave_kernel(const float2* H, int64_t n_rows, PaperLossArgs A) {
  constexpr int N = 1 << LOGN;
  constexpr int NP = fft_npass(LOGN);
  constexpr int RA = fft_radix(LOGN, 0), RZ = fft_radix(LOGN, NP - 1);
  constexpr int T = fft_threads(LOGN);
  constexpr int JA = fft_bpl(N, RA, T), JZ = fft_bpl(N, RZ, T);
  constexpr int BA = N / RA, BZ = N / RZ;
  RTC_FFT_ROWS_SETUP();
  const float invN = 1.0f / (float)N;
  const double alpha = LOSS ? A.alpha[0] : 1.0;
  for (int64_t row = (int64_t)blockIdx.x * W + wv; row < n_rows; row += (int64_t)gridDim.x * W) {
    int lane = lane0;
    asm volatile("" : "+v"(lane));  // twiddles per row, not held across rows
    const float2* hs = H + row * N;
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
    float s0 = 0.0f, s1 = 0.0f;
#pragma unroll
    for (int i = 0; i < JZ; ++i) {
      const int j = lane + T * i;
      if (BZ % T == 0 || j < BZ) {
#pragma unroll
        for (int r = 0; r < RZ; ++r) {
          const float p = cabs2(xh[i][r]) * invN;
          s0 += p;
          s1 = fmaf(centred_tap(j + r * BZ, N), p, s1);
        }
      }
    }
    const double S0 = group_sum_f64<T>((double)s0, red);
    const double S1 = group_sum_f64<T>((double)s1, red);
    const double tbar = S0 > 0.0 ? S1 / S0 : 0.0;
    const float tb = (float)tbar;
    float s2 = 0.0f;
#pragma unroll
    for (int i = 0; i < JZ; ++i) {
      const int j = lane + T * i;
      if (BZ % T == 0 || j < BZ) {
#pragma unroll
        for (int r = 0; r < RZ; ++r) {
          const float d = centred_tap(j + r * BZ, N) - tb;
          s2 = fmaf(d * d, cabs2(xh[i][r]) * invN, s2);
        }
      }
    }
    const double S2 = group_sum_f64<T>((double)s2, red);
    const double v = S0 > 0.0 ? S2 / S0 : 0.0;
    const double tau_hat = sqrt(v) * A.inv_W;
    if (A.pred && lane == 0) {
      A.pred[row * 2 + 0] = S0;
      A.pred[row * 2 + 1] = tau_hat;
    }
    if constexpr (LOSS) {
      const RowGrad c = row_loss(A, row, alpha, S0, v, tau_hat, N, lane == 0);
      if (A.dLdH) {
        const float vf = (float)v;
#pragma unroll
        for (int i = 0; i < JZ; ++i) {
          const int j = lane + T * i;
#pragma unroll
          for (int r = 0; r < RZ; ++r) {
            const float d = centred_tap(j + r * BZ, N) - tb;
            xh[i][r] = cscale(xh[i][r], fmaf(c.a1, fmaf(d, d, -vf), c.a0));
          }
        }
        float2 G[JA][RA];
        fft_full<LOGN, -1, -1, SY, T, TAB>(xh, G, b0, b1, lane, twr);
        float2* out = A.dLdH + row * N;
#pragma unroll
        for (int i = 0; i < JA; ++i) {
          const int j = lane + T * i;
          if (BA % T == 0 || j < BA) {
#pragma unroll
            for (int r = 0; r < RA; ++r) out[j + r * BA] = G[i][r];
          }
        }
      }
    }
  }
}

// ------------------------------------------------------------ scale alpha
// One wave per row: rows_out[r] = {P_r E_r, P_r^2} with E_r = sum_n |H_n|^2
// and P_r the measured gain.  16-byte loads (two taps; N is even), unrolled
// so that a wave has its row's loads in flight together.
__global__ void __launch_bounds__(256)
    gain_products_kernel(const float2* __restrict__ H, int64_t n_rows, int N,
                         const double* __restrict__ tgt, double* rows_out) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n_rows) return;
  const float4* hs = reinterpret_cast<const float4*>(H + row * N);
  float e = 0.0f;
#pragma unroll 8
  for (int n = lane; n < N / 2; n += 64) {
    const float4 v = hs[n];
    e += v.x * v.x + v.y * v.y + v.z * v.z + v.w * v.w;
  }
  const double E = wave_sum_f64((double)e);
  if (lane == 0) {
    const double P = tgt[row * 2];
    rows_out[row * 2 + 0] = P * E;
    rows_out[row * 2 + 1] = P * P;
  }
}

__global__ void alpha_update_kernel(const double* sums, double* alpha, double delta) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (!(sums[1] > 0.0)) return;
  const double ah = sums[0] / sums[1];
  const double n = alpha[1];
  alpha[0] = n > 0.0 ? delta * alpha[0] + (1.0 - delta) * ah : ah;
  alpha[1] = n + 1.0;
}

__global__ void paper_loss_finish_kernel(const double* sums, double inv_B, float w_tau,
                                         float w_gain, double* loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double lt = sums[0] * inv_B, lg = sums[1] * inv_B;
  loss[0] = (double)w_tau * lt + (double)w_gain * lg;
  loss[1] = lt;
  loss[2] = lg;
}

// ------------------------------------------------------ evaluation metrics
__global__ void ale_rae_kernel(int n_links, int n_elem, const double* meas, const double* pred,
                               const double* scale, double* out) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= n_links) return;
  double Pm = 0.0, Pp = 0.0, tm = 0.0, tp = 0.0;
  for (int m = 0; m < n_elem; ++m) {
    const int64_t r = (int64_t)l * n_elem + m;
    Pm += meas[r * 2];
    tm += meas[r * 2 + 1];
    Pp += pred[r * 2];
    tp += pred[r * 2 + 1];
  }
  const double inv = 1.0 / (double)n_elem;
  Pm *= inv;
  Pp *= inv;
  tm *= inv;
  tp *= inv;
  if (scale) Pm *= scale[0];
  out[(int64_t)l * 2 + 0] = fabs(10.0 * log10(Pm) - 10.0 * log10(Pp));
  out[(int64_t)l * 2 + 1] = fabs(tm - tp) / tm;
}

// ------------------------------------------------------------------ host
static int ilog2_pl(int n) {
  int k = 0;
  while ((1 << k) < n) ++k;
  return k;
}

// workgroups for R rows of 2^logn points (fft_row_waves rows in flight each)
static unsigned pl_wave_grid(int64_t R, int logn) {
  const int w = fft_row_waves(logn);
  int64_t g = (R + w - 1) / w;
  g = g < 40960 / w ? g : 40960 / w;
  return (unsigned)(g > 0 ? g : 1);
}

template <bool LOSS>
static void launch_paper_rows(int logN, const float2* H, int64_t R, const PaperLossArgs& A,
                              hipStream_t s) {
  switch (logN) {
#define RTC_PL(L)                                                                            \
  case L:                                                                                    \
    hipLaunchKernelGGL((paper_loss_wave_kernel<L, LOSS>), dim3(pl_wave_grid(R, L)),          \
                       dim3(fft_threads(L) * fft_row_waves(L)), 0, s, H, R, A);             \
    return;
    RTC_PL(1) RTC_PL(2) RTC_PL(3) RTC_PL(4) RTC_PL(5) RTC_PL(6) RTC_PL(7) RTC_PL(8) RTC_PL(9)
    RTC_PL(10) RTC_PL(11) RTC_PL(12)
#undef RTC_PL
    default:
      return;  // n_sc is checked by the entry points
  }
}

// Workspace (doubles): rows[R*2] | reduction scratch | sums[2]
size_t ws_paper_loss(const rtc_radio* r, int32_t n_links) {
  const int64_t R = (int64_t)(n_links > 0 ? n_links : 1) * (r->n_elem > 0 ? r->n_elem : 1);
  return (size_t)(R * 2 + reduce_tmp_doubles(R, 2) + 2) * sizeof(double);
}

}  // namespace rtc

using namespace rtc;

static rtc_status check_rows(const rtc_radio* radio, int32_t n_links, const char* fn) {
  rtc_status st;
  if ((st = check_radio(radio, fn)) != RTC_OK) return st;
  RTC_REQUIRE(is_pow2(radio->n_sc) && radio->n_sc >= 2 && radio->n_sc <= kMaxFFT,
              RTC_ERR_UNSUPPORTED, "%s: n_sc must be a power of two in [2, %d]", fn, kMaxFFT);
  RTC_REQUIRE(n_links >= 1, RTC_ERR_SHAPE, "%s: n_links must be >= 1", fn);
  return RTC_OK;
}

extern "C" rtc_status rtc_cir_stats(const rtc_radio* radio, int32_t n_links, const void* H,
                                    double* stats, void* stream) {
  const char* fn = "rtc_cir_stats";
  rtc_status st;
  if ((st = check_rows(radio, n_links, fn)) != RTC_OK) return st;
  RTC_REQUIRE(H && stats, RTC_ERR_INVALID_ARG, "%s: H and stats are required", fn);
  const int64_t R = (int64_t)n_links * radio->n_elem;
  PaperLossArgs A{};
  A.pred = stats;
  A.inv_B = 1.0 / (double)R;
  A.inv_W = 1.0 / ((double)radio->n_sc * radio->df_hz);
  launch_paper_rows<false>(ilog2_pl(radio->n_sc), reinterpret_cast<const float2*>(H), R, A,
                           as_stream(stream));
  return check_launch(fn);
}

extern "C" rtc_status rtc_paper_loss(const rtc_radio* radio, int32_t n_links, const void* H,
                                     const double* tgt_stats, double* alpha,
                                     int32_t update_alpha, double delta, float w_tau,
                                     float w_gain, double* loss, double* pred_stats, void* dLdH,
                                     void* ws, size_t ws_bytes, void* stream) {
  const char* fn = "rtc_paper_loss";
  rtc_status st;
  if ((st = check_rows(radio, n_links, fn)) != RTC_OK) return st;
  RTC_REQUIRE(H && tgt_stats && alpha && loss, RTC_ERR_INVALID_ARG,
              "%s: H, tgt_stats, alpha and loss are required", fn);
  RTC_REQUIRE(!update_alpha || (delta >= 0.0 && delta <= 1.0), RTC_ERR_INVALID_ARG,
              "%s: delta must lie in [0, 1]", fn);
  const int64_t R = (int64_t)n_links * radio->n_elem;
  const size_t need = ws_paper_loss(radio, n_links);
  RTC_REQUIRE(ws != nullptr && ws_bytes >= need, RTC_ERR_WORKSPACE,
              "%s: workspace of %zu bytes required", fn, need);
  hipStream_t s = as_stream(stream);
  double* rows = reinterpret_cast<double*>(ws);
  double* red = rows + R * 2;
  double* sums = red + reduce_tmp_doubles(R, 2);
  const int N = radio->n_sc;
  if (update_alpha) {
    const unsigned blocks = (unsigned)((R + 3) / 4);
    hipLaunchKernelGGL(gain_products_kernel, dim3(blocks), dim3(256), 0, s,
                       reinterpret_cast<const float2*>(H), R, N, tgt_stats, rows);
    if ((st = check_launch(fn)) != RTC_OK) return st;
    if ((st = reduce_all(rows, R, 2, red, sums, s, fn)) != RTC_OK) return st;
    hipLaunchKernelGGL(alpha_update_kernel, dim3(1), dim3(64), 0, s, sums, alpha, delta);
    if ((st = check_launch(fn)) != RTC_OK) return st;
  }
  PaperLossArgs A{};
  A.tgt = tgt_stats;
  A.alpha = alpha;
  A.row_out = rows;
  A.pred = pred_stats;
  A.dLdH = reinterpret_cast<float2*>(dLdH);
  A.inv_B = 1.0 / (double)R;
  A.inv_W = 1.0 / ((double)N * radio->df_hz);
  A.w_tau = w_tau;
  A.w_gain = w_gain;
  launch_paper_rows<true>(ilog2_pl(N), reinterpret_cast<const float2*>(H), R, A, s);
  if ((st = check_launch(fn)) != RTC_OK) return st;
  if ((st = reduce_all(rows, R, 2, red, sums, s, fn)) != RTC_OK) return st;
  hipLaunchKernelGGL(paper_loss_finish_kernel, dim3(1), dim3(64), 0, s, sums, A.inv_B, w_tau,
                     w_gain, loss);
  return check_launch(fn);
}

extern "C" rtc_status rtc_eval_ale_rae(int32_t n_links, int32_t n_elem, const double* meas,
                                       const double* pred, const double* scale, double* out,
                                       void* stream) {
  const char* fn = "rtc_eval_ale_rae";
  RTC_REQUIRE(n_links >= 1 && n_elem >= 1, RTC_ERR_SHAPE,
              "%s: n_links and n_elem must be >= 1", fn);
  RTC_REQUIRE(meas && pred && out, RTC_ERR_INVALID_ARG, "%s: meas, pred and out are required",
              fn);
  const unsigned blocks = (unsigned)((n_links + 255) / 256);
  hipLaunchKernelGGL(ale_rae_kernel, dim3(blocks), dim3(256), 0, as_stream(stream), n_links,
                     n_elem, meas, pred, scale, out);
  return check_launch(fn);
}
