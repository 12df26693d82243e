// Library-wide entry points: version, error reporting, workspace sizes and
// descriptor validation.
#include <string>

#include "api_common.h"

namespace rtc {

static thread_local std::string g_last_error;

void set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
}

void clear_error() { g_last_error.clear(); }

rtc_status check_radio(const rtc_radio* r, const char* fn) {
  RTC_REQUIRE(r != nullptr, RTC_ERR_INVALID_ARG, "%s: radio is NULL", fn);
  RTC_REQUIRE(r->fc_hz > 0.0, RTC_ERR_INVALID_ARG, "%s: fc_hz must be > 0", fn);
  RTC_REQUIRE(r->df_hz >= 0.0, RTC_ERR_INVALID_ARG, "%s: df_hz must be >= 0", fn);
  RTC_REQUIRE(r->n_sc >= 1, RTC_ERR_SHAPE, "%s: n_sc must be >= 1", fn);
  RTC_REQUIRE(r->n_elem >= 1, RTC_ERR_SHAPE, "%s: n_elem must be >= 1", fn);
  return RTC_OK;
}

__global__ void zero_floats_kernel(float* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0f;
}

rtc_status zero_floats(float* p, int64_t n_floats, hipStream_t s, const char* fn) {
  if (n_floats <= 0) return RTC_OK;
  int64_t blocks = (n_floats + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(zero_floats_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n_floats);
  return check_launch(fn);
}

rtc_status check_paths(const rtc_paths* p, const char* fn, bool need_geometry) {
  RTC_REQUIRE(p != nullptr, RTC_ERR_INVALID_ARG, "%s: paths is NULL", fn);
  RTC_REQUIRE(p->n_links >= 0 && p->n_paths >= 0, RTC_ERR_SHAPE,
              "%s: n_links and n_paths must be >= 0", fn);
  RTC_REQUIRE(p->max_depth >= 0 && p->max_depth <= kMaxDepth, RTC_ERR_RANGE,
              "%s: max_depth must be in [0, %d]", fn, kMaxDepth);
  RTC_REQUIRE(p->link_off != nullptr || p->n_links == 0, RTC_ERR_INVALID_ARG,
              "%s: link_off is NULL", fn);
  RTC_REQUIRE(p->tau != nullptr || p->n_paths == 0, RTC_ERR_INVALID_ARG, "%s: tau is NULL", fn);
  if (need_geometry && p->n_paths > 0) {
    RTC_REQUIRE(p->tx_pos && p->rx_pos && p->depth, RTC_ERR_INVALID_ARG,
                "%s: tx_pos, rx_pos and depth are required", fn);
    if (p->max_depth > 0) {
      RTC_REQUIRE(p->px && p->py && p->pz && p->nx && p->ny && p->nz && p->mat,
                  RTC_ERR_INVALID_ARG, "%s: interaction arrays are required when max_depth > 0",
                  fn);
      RTC_REQUIRE(p->kind == nullptr || p->dA != nullptr, RTC_ERR_INVALID_ARG,
                  "%s: dA is required when kind is given", fn);
      RTC_REQUIRE(p->edge == nullptr || p->kind != nullptr, RTC_ERR_INVALID_ARG,
                  "%s: edge needs kind (diffraction paths are kind 2)", fn);
    }
  }
  return RTC_OK;
}

rtc_status check_mats(const rtc_materials* m, const rtc_paths* p, const char* fn) {
  RTC_REQUIRE(m != nullptr, RTC_ERR_INVALID_ARG, "%s: materials is NULL", fn);
  RTC_REQUIRE((m->raw == nullptr) != (m->per_inter == nullptr), RTC_ERR_INVALID_ARG,
              "%s: exactly one of materials.raw and materials.per_inter must be set", fn);
  if (m->per_inter && m->inter_idx) {
    RTC_REQUIRE(m->n_inter >= 0 && m->n_inter <= (int64_t)p->max_depth * p->n_paths,
                RTC_ERR_SHAPE, "%s: n_inter must be in [0, max_depth * n_paths]", fn);
  }
  if (m->raw) {
    RTC_REQUIRE(m->n_mat >= 1 && m->n_mat <= kMaxMat, RTC_ERR_RANGE,
                "%s: n_mat must be in [1, %d]", fn, kMaxMat);
    RTC_REQUIRE(p->edge == nullptr || p->mat_n != nullptr || p->n_paths == 0,
                RTC_ERR_INVALID_ARG, "%s: per-id materials with edge need mat_n", fn);
  }
  return RTC_OK;
}

}  // namespace rtc

// Workspace layouts (bytes), kept in one place so the sizes and the users
// agree.
namespace rtc {
size_t ws_cfr_loss(const rtc_radio* r, int32_t n_links);
size_t ws_cfr_adjoint(const rtc_radio* r, int32_t n_links, int32_t n_paths);
size_t ws_trace_adjoint(int32_t n_paths, int32_t n_mat);
size_t ws_target_stats(const rtc_radio* r, int32_t n_links);
size_t ws_paper_loss(const rtc_radio* r, int32_t n_links);
size_t ws_validate_paths();
size_t ws_trace_adjoint_pat(int32_t n_paths, int32_t n_mat);
size_t ws_cfr_loss_adjoint(const rtc_radio* r, int32_t n_links);
}  // namespace rtc

extern "C" {

int rtc_abi_version(void) { return RTC_ABI_VERSION; }

const char* rtc_last_error(void) { return rtc::g_last_error.c_str(); }

size_t rtc_workspace_size(int op, const rtc_radio* radio, int32_t n_links, int32_t n_paths,
                          int32_t n_mat) {
  if (n_links < 0 || n_paths < 0) return 0;
  switch (op) {
    case RTC_OP_CFR_LOSS:
      return radio ? rtc::ws_cfr_loss(radio, n_links) : 0;
    case RTC_OP_CFR_ADJOINT:
      return radio ? rtc::ws_cfr_adjoint(radio, n_links, n_paths) : 0;
    case RTC_OP_TRACE_FIELDS_ADJOINT:
      return rtc::ws_trace_adjoint(n_paths, n_mat);
    case RTC_OP_CFR_TARGET_STATS:
      return radio ? rtc::ws_target_stats(radio, n_links) : 0;
    case RTC_OP_PAPER_LOSS:
      return radio ? rtc::ws_paper_loss(radio, n_links) : 0;
    case RTC_OP_TRACE_FIELDS_ADJOINT_PAT:
      return rtc::ws_trace_adjoint_pat(n_paths, n_mat);
    case RTC_OP_VALIDATE_PATHS:
      return rtc::ws_validate_paths();
    case RTC_OP_CFR_LOSS_ADJOINT:
      return radio ? rtc::ws_cfr_loss_adjoint(radio, n_links) : 0;
    default:
      return 0;
  }
}

}  // extern "C"
