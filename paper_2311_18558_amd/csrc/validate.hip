// Device-side validation of a path store: counts of entries that break the
// contract of rtc_paths, one count per category, without atomics (per-block
// partial counts, then a fixed-order sum).  The field kernels themselves
// clamp material ids and never read past the arrays, so an invalid store
// gives wrong numbers rather than faults; this check names what is wrong.
#include <cmath>

#include "api_common.h"
#include "dev_common.h"

namespace rtc {

constexpr int kValBlock = 256;
constexpr int kValMaxBlocks = 2048;

size_t ws_validate_paths() { return (size_t)kValMaxBlocks * RTC_N_VALIDATE * sizeof(int64_t); }

RTC_DEV bool finite3(float x, float y, float z) {
  return isfinite(x) && isfinite(y) && isfinite(z);
}

__global__ void __launch_bounds__(kValBlock)
    validate_paths_kernel(rtc_paths P, int32_t n_mat, int64_t* part) {
  __shared__ int64_t red[kValBlock / 64][RTC_N_VALIDATE];
  int64_t c[RTC_N_VALIDATE];
#pragma unroll
  for (int k = 0; k < RTC_N_VALIDATE; ++k) c[k] = 0;
  const int64_t n_items = P.n_paths > P.n_links + 1 ? P.n_paths : P.n_links + 1;
  for (int64_t i = (int64_t)blockIdx.x * kValBlock + threadIdx.x; i < n_items;
       i += (int64_t)gridDim.x * kValBlock) {
    if (i <= P.n_links) {
      const int64_t o = P.link_off[i];
      const bool bad = (i == 0 && o != 0) || (i == P.n_links && o != P.n_paths) ||
                       (i > 0 && o < P.link_off[i - 1]) || o < 0 || o > P.n_paths;
      c[RTC_VAL_LINK_OFF] += bad;
      if (i < P.n_links) {
        c[RTC_VAL_NONFINITE] += !finite3(P.tx_pos[3 * i], P.tx_pos[3 * i + 1], P.tx_pos[3 * i + 2]);
        c[RTC_VAL_NONFINITE] += !finite3(P.rx_pos[3 * i], P.rx_pos[3 * i + 1], P.rx_pos[3 * i + 2]);
      }
    }
    if (i < P.n_paths) {
      const int64_t p = i;
      int d = P.depth[p];
      c[RTC_VAL_DEPTH] += d > P.max_depth;
      d = d < P.max_depth ? d : P.max_depth;
      const double t = P.tau[p];
      c[RTC_VAL_TAU] += !(isfinite(t) && t > 0.0);
      for (int k = 0; k < d; ++k) {
        const int64_t s = (int64_t)k * P.n_paths + p;
        c[RTC_VAL_MAT] += n_mat > 0 && (int)P.mat[s] >= n_mat;
        c[RTC_VAL_NONFINITE] += !finite3(P.px[s], P.py[s], P.pz[s]);
        const float nn = P.nx[s] * P.nx[s] + P.ny[s] * P.ny[s] + P.nz[s] * P.nz[s];
        c[RTC_VAL_UNIT] += !(fabsf(nn - 1.0f) <= 1e-2f);
        if (P.kind) {
          const int kd = P.kind[s];
          c[RTC_VAL_KIND] += kd > 2;
          if (kd == 1) c[RTC_VAL_RANGE] += !(isfinite(P.dA[s]) && P.dA[s] >= 0.0f);
        }
      }
      if (P.edge && P.kind && d == 1 && P.kind[p] == 2) {
        const float ex = P.edge[p], ey = P.edge[P.n_paths + p], ez = P.edge[2 * (int64_t)P.n_paths + p];
        const float nw = P.edge[3 * (int64_t)P.n_paths + p];
        c[RTC_VAL_UNIT] += !(fabsf(ex * ex + ey * ey + ez * ez - 1.0f) <= 1e-2f);
        c[RTC_VAL_RANGE] += !(nw > 0.0f && nw <= 2.0f);
        c[RTC_VAL_MAT] += n_mat > 0 && P.mat_n != nullptr && (int)P.mat_n[p] >= n_mat;
      }
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < RTC_N_VALIDATE; ++k) {
    int64_t v = c[k];
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) red[wave][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < RTC_N_VALIDATE) {
    int64_t v = 0;
    for (int w = 0; w < kValBlock / 64; ++w) v += red[w][threadIdx.x];
    part[(int64_t)blockIdx.x * RTC_N_VALIDATE + threadIdx.x] = v;
  }
}

__global__ void validate_sum_kernel(const int64_t* part, int n_blocks, int64_t* counts) {
  if (threadIdx.x < RTC_N_VALIDATE) {
    int64_t v = 0;
    for (int b = 0; b < n_blocks; ++b) v += part[(int64_t)b * RTC_N_VALIDATE + threadIdx.x];
    counts[threadIdx.x] = v;
  }
}

}  // namespace rtc

using namespace rtc;

extern "C" rtc_status rtc_validate_paths(const rtc_paths* paths, int32_t n_mat, int64_t* counts,
                                         void* ws, size_t ws_bytes, void* stream) {
  const char* fn = "rtc_validate_paths";
  rtc_status st;
  if ((st = check_paths(paths, fn, true)) != RTC_OK) return st;
  RTC_REQUIRE(counts != nullptr, RTC_ERR_INVALID_ARG, "%s: counts is NULL", fn);
  RTC_REQUIRE(ws != nullptr && ws_bytes >= ws_validate_paths(), RTC_ERR_WORKSPACE,
              "%s: workspace of %zu bytes required", fn, ws_validate_paths());
  const int64_t n_items = (int64_t)(paths->n_paths > paths->n_links + 1 ? paths->n_paths
                                                                        : paths->n_links + 1);
  int64_t blocks = (n_items + kValBlock - 1) / kValBlock;
  if (blocks > kValMaxBlocks) blocks = kValMaxBlocks;
  if (blocks < 1) blocks = 1;
  hipStream_t s = as_stream(stream);
  int64_t* part = reinterpret_cast<int64_t*>(ws);
  hipLaunchKernelGGL(validate_paths_kernel, dim3((unsigned)blocks), dim3(kValBlock), 0, s, *paths,
                     n_mat, part);
  if ((st = check_launch(fn)) != RTC_OK) return st;
  hipLaunchKernelGGL(validate_sum_kernel, dim3(1), dim3(64), 0, s, part, (int)blocks, counts);
  return check_launch(fn);
}
