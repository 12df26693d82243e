// Material embeddings (Sec. III-C, Eqs. trainable_materials_1-4).  Each
// material m has four embeddings w_{m,1..4} in R^L; one read-out vector v in
// R^L is shared by all materials.  u_{m,j} = v . w_{m,j} is the raw scalar
// of sigma (j = 1, log domain), eps_r (j = 2, log of eps_r - 1), S (j = 3,
// logit) and K_x (j = 4, logit).  The read-out writes the u where the field
// kernels take raw material values: the per-id rows (eps_r, sigma, S) and
// column 0 (K_x) of the per-material pattern rows.
//
// The operation is a few thousand multiply-adds: one thread per output, FP64
// sums rounded once, so that the result does not depend on the launch.
#include "api_common.h"
#include "dev_common.h"

namespace rtc {

constexpr int kEmbedMaxL = 1024;
constexpr int kEmbedMaxMat = 4096;
constexpr int kEmbedBlock = 256;

// Column of the per-id raw row that embedding j (0-based, paper order sigma,
// eps_r, S, K_x) feeds; -1 for K_x, which goes to the pattern row.
RTC_DEV int raw_col(int j) { return j == 0 ? 1 : (j == 1 ? 0 : (j == 2 ? 2 : -1)); }

__global__ void __launch_bounds__(kEmbedBlock)
    embed_readout_kernel(int n_mat, int L, const float* __restrict__ v,
                         const float* __restrict__ W, float* __restrict__ raw,
                         float* __restrict__ pat) {
  const int i = blockIdx.x * kEmbedBlock + threadIdx.x;  // i = 4 m + j
  if (i >= 4 * n_mat) return;
  const float* w = W + (size_t)i * L;
  double s = 0.0;
  for (int l = 0; l < L; ++l) s = fma((double)v[l], (double)w[l], s);
  const int m = i >> 2, c = raw_col(i & 3);
  if (c >= 0)
    raw[3 * m + c] = (float)s;
  else if (pat)
    pat[6 * m] = (float)s;
}

RTC_DEV float upstream(int i, const float* __restrict__ g_raw, const float* __restrict__ g_pat) {
  const int m = i >> 2, c = raw_col(i & 3);
  return c >= 0 ? g_raw[3 * m + c] : (g_pat ? g_pat[6 * m] : 0.0f);
}

// dL/dW[m, j, l] = v[l] dL/du[m, j]
__global__ void __launch_bounds__(kEmbedBlock)
    embed_grad_w_kernel(int n_mat, int L, const float* __restrict__ v,
                        const float* __restrict__ g_raw, const float* __restrict__ g_pat,
                        float* __restrict__ dW) {
  const int64_t n = (int64_t)4 * n_mat * L;
  for (int64_t k = (int64_t)blockIdx.x * kEmbedBlock + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * kEmbedBlock) {
    const int i = (int)(k / L), l = (int)(k - (int64_t)i * L);
    dW[k] = v[l] * upstream(i, g_raw, g_pat);
  }
}

// dL/dv[l] = sum over (m, j) of W[m, j, l] dL/du[m, j]; one block per l,
// FP64 partial sums in a fixed order.
__global__ void __launch_bounds__(kEmbedBlock)
    embed_grad_v_kernel(int n_mat, int L, const float* __restrict__ W,
                        const float* __restrict__ g_raw, const float* __restrict__ g_pat,
                        float* __restrict__ dv) {
  __shared__ double red[kEmbedBlock / 64];
  const int l = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < 4 * n_mat; i += kEmbedBlock)
    s = fma((double)W[(size_t)i * L + l], (double)upstream(i, g_raw, g_pat), s);
  s = block_sum_f64(s, red);
  if (threadIdx.x == 0) dv[l] = (float)s;
}

static rtc_status check_embed(int32_t n_mat, int32_t L, const float* v, const float* W,
                              const char* fn) {
  RTC_REQUIRE(n_mat >= 1 && n_mat <= kEmbedMaxMat, RTC_ERR_RANGE, "%s: n_mat must be in [1, %d]",
              fn, kEmbedMaxMat);
  RTC_REQUIRE(L >= 1 && L <= kEmbedMaxL, RTC_ERR_RANGE, "%s: L must be in [1, %d]", fn,
              kEmbedMaxL);
  RTC_REQUIRE(v && W, RTC_ERR_INVALID_ARG, "%s: v and W are required", fn);
  return RTC_OK;
}

}  // namespace rtc

using namespace rtc;

extern "C" rtc_status rtc_embed_readout(int32_t n_mat, int32_t L, const float* v, const float* W,
                                        float* raw, float* pat_raw, void* stream) {
  const char* fn = "rtc_embed_readout";
  rtc_status st;
  if ((st = check_embed(n_mat, L, v, W, fn)) != RTC_OK) return st;
  RTC_REQUIRE(raw, RTC_ERR_INVALID_ARG, "%s: raw is NULL", fn);
  const int blocks = (4 * n_mat + kEmbedBlock - 1) / kEmbedBlock;
  hipLaunchKernelGGL(embed_readout_kernel, dim3(blocks), dim3(kEmbedBlock), 0, as_stream(stream),
                     (int)n_mat, (int)L, v, W, raw, pat_raw);
  return check_launch(fn);
}

extern "C" rtc_status rtc_embed_readout_backward(int32_t n_mat, int32_t L, const float* v,
                                                 const float* W, const float* dLd_raw,
                                                 const float* dLd_pat, float* dLd_v,
                                                 float* dLd_W, void* stream) {
  const char* fn = "rtc_embed_readout_backward";
  rtc_status st;
  if ((st = check_embed(n_mat, L, v, W, fn)) != RTC_OK) return st;
  RTC_REQUIRE(dLd_raw, RTC_ERR_INVALID_ARG, "%s: dLd_raw is NULL", fn);
  hipStream_t s = as_stream(stream);
  if (dLd_W) {
    int64_t blocks = ((int64_t)4 * n_mat * L + kEmbedBlock - 1) / kEmbedBlock;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(embed_grad_w_kernel, dim3((unsigned)blocks), dim3(kEmbedBlock), 0, s,
                       (int)n_mat, (int)L, v, dLd_raw, dLd_pat, dLd_W);
    if ((st = check_launch(fn)) != RTC_OK) return st;
  }
  if (dLd_v) {
    hipLaunchKernelGGL(embed_grad_v_kernel, dim3(L), dim3(kEmbedBlock), 0, s, (int)n_mat, (int)L,
                       W, dLd_raw, dLd_pat, dLd_v);
    return check_launch(fn);
  }
  return RTC_OK;
}
