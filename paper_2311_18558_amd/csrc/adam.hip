// Adam update on float32 parameter arrays (the optimiser of Sec. III-G).
#include <cmath>

#include "api_common.h"
#include "dev_common.h"

namespace rtc {

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, int64_t n, float lr,
                            float b1, float b2, float eps, float inv_bc1, float inv_bc2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    float gi = g[i];
    float mi = fmaf(b1, m[i], (1.0f - b1) * gi);
    float vi = fmaf(b2, v[i], (1.0f - b2) * gi * gi);
    m[i] = mi;
    v[i] = vi;
    float mhat = mi * inv_bc1;
    float vhat = vi * inv_bc2;
    p[i] -= lr * mhat / (sqrtf(vhat) + eps);
  }
}

// The same update with the step count read from device memory (t = *step +
// 1), so that a recorded HIP graph advances the bias corrections on replay.
__global__ void adam_dev_kernel(float* __restrict__ p, const float* __restrict__ g,
                                float* __restrict__ m, float* __restrict__ v, int64_t n, float lr,
                                float b1, float b2, float eps, const int32_t* __restrict__ step) {
  const double t = (double)(*step) + 1.0;
  const float inv_bc1 = (float)(1.0 / (1.0 - pow((double)b1, t)));
  const float inv_bc2 = (float)(1.0 / (1.0 - pow((double)b2, t)));
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    float gi = g[i];
    float mi = fmaf(b1, m[i], (1.0f - b1) * gi);
    float vi = fmaf(b2, v[i], (1.0f - b2) * gi * gi);
    m[i] = mi;
    v[i] = vi;
    float mhat = mi * inv_bc1;
    float vhat = vi * inv_bc2;
    p[i] -= lr * mhat / (sqrtf(vhat) + eps);
  }
}

// y += alpha x (gradient accumulation over batches)
__global__ void axpy_kernel(float* __restrict__ y, const float* __restrict__ x, float alpha,
                            int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = fmaf(alpha, x[i], y[i]);
}

__global__ void advance_step_kernel(int32_t* step) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *step += 1;
}

}  // namespace rtc

using namespace rtc;

extern "C" rtc_status rtc_adam_step_dev(float* param, const float* grad, float* m, float* v,
                                        int64_t n, int32_t* step, int32_t advance, float lr,
                                        float beta1, float beta2, float eps, void* stream) {
  const char* fn = "rtc_adam_step_dev";
  RTC_REQUIRE(n >= 0, RTC_ERR_SHAPE, "%s: n must be >= 0", fn);
  RTC_REQUIRE(step != nullptr, RTC_ERR_INVALID_ARG, "%s: step is NULL", fn);
  RTC_REQUIRE(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f,
              RTC_ERR_INVALID_ARG, "%s: betas must be in [0, 1)", fn);
  hipStream_t s = as_stream(stream);
  rtc_status st;
  if (n > 0) {
    RTC_REQUIRE(param && grad && m && v, RTC_ERR_INVALID_ARG, "%s: NULL array", fn);
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(adam_dev_kernel, dim3((unsigned)blocks), dim3(256), 0, s, param, grad, m,
                       v, n, lr, beta1, beta2, eps, step);
    if ((st = check_launch(fn)) != RTC_OK) return st;
  }
  if (advance) {
    hipLaunchKernelGGL(advance_step_kernel, dim3(1), dim3(64), 0, s, step);
    return check_launch(fn);
  }
  return RTC_OK;
}

extern "C" rtc_status rtc_adam_step(float* param, const float* grad, float* m, float* v,
                                    int64_t n, int32_t step, float lr, float beta1, float beta2,
                                    float eps, void* stream) {
  const char* fn = "rtc_adam_step";
  RTC_REQUIRE(n >= 0, RTC_ERR_SHAPE, "%s: n must be >= 0", fn);
  RTC_REQUIRE(step >= 1, RTC_ERR_INVALID_ARG, "%s: step must be >= 1", fn);
  RTC_REQUIRE(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f,
              RTC_ERR_INVALID_ARG, "%s: betas must be in [0, 1)", fn);
  if (n == 0) return RTC_OK;
  RTC_REQUIRE(param && grad && m && v, RTC_ERR_INVALID_ARG, "%s: NULL array", fn);
  // bias corrections in FP64 on the host
  double bc1 = 1.0 - std::pow((double)beta1, (double)step);
  double bc2 = 1.0 - std::pow((double)beta2, (double)step);
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)blocks), dim3(256), 0, as_stream(stream), param,
                     grad, m, v, n, lr, beta1, beta2, eps, (float)(1.0 / bc1), (float)(1.0 / bc2));
  return check_launch(fn);
}

extern "C" rtc_status rtc_axpy(float* y, const float* x, float alpha, int64_t n, void* stream) {
  const char* fn = "rtc_axpy";
  RTC_REQUIRE(n >= 0, RTC_ERR_SHAPE, "%s: n must be >= 0", fn);
  if (n == 0) return RTC_OK;
  RTC_REQUIRE(y && x, RTC_ERR_INVALID_ARG, "%s: NULL array", fn);
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(axpy_kernel, dim3((unsigned)blocks), dim3(256), 0, as_stream(stream), y, x,
                     alpha, n);
  return check_launch(fn);
}
