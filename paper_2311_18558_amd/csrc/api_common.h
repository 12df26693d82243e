// Host-side helpers shared by the entry points of librtcal.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <map>
#include <mutex>
#include <tuple>

#include "rtcal.h"

namespace rtc {

void set_error(const char* fmt, ...);
void clear_error();

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline rtc_status check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("%s: HIP launch failed: %s", what, hipGetErrorString(e));
    return RTC_ERR_HIP;
  }
  return RTC_OK;
}

// Shared validation of the radio and path-store descriptors.
rtc_status check_radio(const rtc_radio* r, const char* fn);
rtc_status check_paths(const rtc_paths* p, const char* fn, bool need_geometry);
rtc_status check_mats(const rtc_materials* m, const rtc_paths* p, const char* fn);

// Workgroups of `threads` threads of `kernel` that the current device keeps
// resident at once (its CUs times the occupancy), for persistent launches;
// looked up once per device and block size (a host query, no stream work).
inline int64_t resident_workgroups(const void* kernel, int threads) {
  static std::mutex mu;
  static std::map<std::tuple<int, const void*, int>, int64_t> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1024;
  std::lock_guard<std::mutex> lock(mu);
  const auto key = std::make_tuple(dev, kernel, threads);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int cus = 0, per_cu = 0;
  int64_t n = 1024;  // a safe number if a query fails
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) == hipSuccess &&
      cus > 0 && per_cu > 0)
    n = (int64_t)cus * per_cu;
  cache[key] = n;
  return n;
}

inline bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

// Zero n_floats floats on the stream with a fill kernel (not a memset node:
// the entry points stay safe to record into a HIP graph).
rtc_status zero_floats(float* p, int64_t n_floats, hipStream_t s, const char* fn);

// Fixed-order reduction of a [R][K] double array over rows into dst[K]
// (device), using tmp (reduce_tmp_doubles(R, K) doubles of device memory).
rtc_status reduce_all(const double* rows, int64_t R, int K, double* tmp, double* dst,
                      hipStream_t s, const char* fn);
size_t reduce_tmp_doubles(int64_t R, int K);

constexpr int kMaxMat = 512;
constexpr int kMaxDepth = 8;
constexpr int kMaxFFT = 4096;

}  // namespace rtc

#define RTC_REQUIRE(cond, code, ...)  \
  do {                                \
    if (!(cond)) {                    \
      ::rtc::set_error(__VA_ARGS__);  \
      return code;                    \
    }                                 \
  } while (0)
