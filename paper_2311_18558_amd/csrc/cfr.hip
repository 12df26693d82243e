// Channel frequency response and its adjoint on the FP32 matrix cores.
//
// For one link l the CFR is a complex matrix product
//     H_l[m, n] = sum_i B[m, i] E[i, n],
//     B[m, i] = a_i g_m exp(j psi_i (m - c)),  E[i, n] = exp(-j 2 pi f_n tau_i),
// with M elements, N subcarriers and P_l paths (Eq. cfr_cont, Sec. II-A).
// Both operands are generated in registers, one value per lane, and fed to
// v_mfma_f32_32x32x2_f32 (A: 32 rows x 2 k, B: 2 k x 32 columns, lane l
// holds A[l%32][l/32] and B[l/32][l%32]; D row 8(r/4)+4(l/32)+r%4, column
// l%32 in register r).  The complex product is split into four real MFMAs
// that share operands without any lane exchange: the two k-slices are two
// different paths, lane l owns path i+l/32 and computes B for row l%32 and
// E for column l%32, and
//     Re H += B_re E_re + (-B_im) E_im,   Im H += B_im E_re + B_re E_im.
// The subcarrier phase f_n tau_i (thousands of cycles) is reduced in FP64;
// within a wave, tile t+1 is tile t times exp(-j 2 pi 32 df tau_i).
//
// The adjoint G[m, i] = sum_n dLdH[m, n] conj(E[i, n]) is the same kind of
// product with the subcarriers as the contraction axis; each lane reads its
// dL/dH row directly, and E advances by exp(-j 2 pi df tau_i) from an FP64
// anchor every 32 subcarriers.
#include <cmath>

#include "api_common.h"
#include "dev_common.h"

namespace rtc {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kCfrWaves = 4;   // waves per workgroup (forward)
constexpr int kCfrTiles = 4;   // 32-subcarrier tiles per wave (forward)
constexpr int kAdjWaves = 4;   // waves per workgroup (adjoint)
constexpr int kAdjTP = 2;      // 32-path tiles per wave (adjoint)
constexpr double kInv2Pi = 0.15915494309189533577;

RTC_DEV floatx16 mfma32(float a, float b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

struct CfrArgs {
  int n_links, M, N;
  int n_mblk, n_nchunk;
  const int64_t* link_off;
  const float2* a;
  const float* psi;
  const double* tau;
  const float2* g;
  double f0;    // frequency of subcarrier 0
  double df;    // subcarrier spacing
  double cm;    // (M-1)/2
};

__global__ void __launch_bounds__(kCfrWaves * 64) cfr_kernel(CfrArgs A, float2* __restrict__ H) {
  const int lane = threadIdx.x & 63;
  const int half = lane >> 5;
  const int col = lane & 31;
  const int64_t wt = (int64_t)blockIdx.x * kCfrWaves + (threadIdx.x >> 6);
  const int nchunk = (int)(wt % A.n_nchunk);
  const int64_t rest = wt / A.n_nchunk;
  const int mblk = (int)(rest % A.n_mblk);
  const int64_t l = rest / A.n_mblk;
  if (l >= A.n_links) return;

  const int m = mblk * 32 + col;
  const float2 gm = m < A.M ? A.g[m] : make_float2(0.0f, 0.0f);
  const double mc_cyc = ((double)m - A.cm) * kInv2Pi;
  const int n_base = nchunk * 32 * kCfrTiles;
  const double f_lane = A.f0 + (double)(n_base + col) * A.df;
  const double df32 = 32.0 * A.df;
  const int64_t off0 = A.link_off[l];
  const int64_t off1 = A.link_off[l + 1];

  floatx16 acc_re[kCfrTiles], acc_im[kCfrTiles];
#pragma unroll
  for (int t = 0; t < kCfrTiles; ++t) {
    acc_re[t] = floatx16{0};
    acc_im[t] = floatx16{0};
  }

  for (int64_t i0 = off0; i0 < off1; i0 += 2) {
    const int64_t i = i0 + half;
    float2 ai = make_float2(0.0f, 0.0f);
    float ps = 0.0f;
    double ti = 0.0;
    if (i < off1) {
      ai = A.a[i];
      ps = A.psi[i];
      ti = A.tau[i];
    }
    // A operand: B[m, i] = a_i g_m exp(j psi_i (m - c))
    double ph = (double)ps * mc_cyc;
    float2 arr = expm2pi_f64(-ph);  // exp(+j 2 pi ph)
    float2 b = cmul(cmul(ai, gm), arr);
    // B operand: E[i, n] for the lane's subcarrier in each tile
    float2 e = expm2pi_f64(f_lane * ti);
    float2 w = expm2pi_f64(df32 * ti);
#pragma unroll
    for (int t = 0; t < kCfrTiles; ++t) {
      if (t > 0) e = cmul(e, w);
      acc_re[t] = mfma32(b.x, e.x, acc_re[t]);
      acc_re[t] = mfma32(-b.y, e.y, acc_re[t]);
      acc_im[t] = mfma32(b.y, e.x, acc_im[t]);
      acc_im[t] = mfma32(b.x, e.y, acc_im[t]);
    }
  }

  float2* Hl = H + (int64_t)l * A.M * A.N;
#pragma unroll
  for (int t = 0; t < kCfrTiles; ++t) {
    const int n = n_base + t * 32 + col;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = mblk * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
      if (row < A.M && n < A.N) Hl[(int64_t)row * A.N + n] = make_float2(acc_re[t][r], acc_im[t][r]);
    }
  }
}

// ------------------------------------------------------------------ adjoint
// One wave per (link, group of kAdjTP 32-path tiles), found by binary search
// in a per-link exclusive scan of wave counts.  For each 32-row element
// block the wave contracts over subcarriers: MFMA step s of a 64-subcarrier
// chunk takes subcarriers n0 + s (k = 0) and n0 + 32 + s (k = 1), so lane l
// reads a contiguous run of its own row (16-byte loads) and advances its
// exponential by exp(-j 2 pi df tau) from an FP64 anchor per half-chunk.
struct AdjArgs {
  int n_links, M, N;
  int64_t max_waves;
  const int64_t* link_off;
  const int64_t* wave_off;  // [n_links + 1] exclusive scan of waves per link
  const float2* a;
  const float* psi;
  const double* tau;
  const float2* g;
  const float2* dH;
  float2* dLda;    // may be null
  double* g_part;  // [max_waves][M][2] per-wave dL/dg partials, or null
  double f0, df, cm;
};

__device__ __forceinline__ int adj_waves_of(const int64_t* off, int l) {
  const int64_t P = off[l + 1] - off[l];
  const int64_t tiles = (P + 31) / 32;
  return (int)((tiles + kAdjTP - 1) / kAdjTP);
}

// Exclusive scan of waves per link (one block, fixed order).
__global__ void __launch_bounds__(1024) adj_wave_scan_kernel(const int64_t* link_off, int n_links,
                                                              int64_t* wave_off) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int per = (n_links + 1023) / 1024;
  const int l0 = t * per, l1 = min(n_links, l0 + per);
  int64_t s = 0;
  for (int l = l0; l < l1; ++l) s += adj_waves_of(link_off, l);
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    int64_t acc = 0;
    for (int i = 0; i < 1024; ++i) {
      int64_t v = part[i];
      part[i] = acc;
      acc += v;
    }
  }
  __syncthreads();
  int64_t acc = part[t];
  for (int l = l0; l < l1; ++l) {
    wave_off[l] = acc;
    acc += adj_waves_of(link_off, l);
  }
  if (t == 1023) wave_off[n_links] = acc;
}

__device__ __forceinline__ void load4(const float2* row, int n, int N, bool vec, float2 h[4]) {
  if (vec && n + 3 < N) {
    const float4* p = reinterpret_cast<const float4*>(row + n);
    float4 x = p[0], y = p[1];
    h[0] = make_float2(x.x, x.y);
    h[1] = make_float2(x.z, x.w);
    h[2] = make_float2(y.x, y.y);
    h[3] = make_float2(y.z, y.w);
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) h[q] = (n + q < N) ? row[n + q] : make_float2(0.0f, 0.0f);
  }
}

__global__ void __launch_bounds__(kAdjWaves * 64) cfr_adjoint_kernel(AdjArgs A) {
  const int lane = threadIdx.x & 63;
  const int half = lane >> 5;
  const int col = lane & 31;
  const int64_t w = (int64_t)blockIdx.x * kAdjWaves + (threadIdx.x >> 6);
  if (w >= A.max_waves) return;
  const int64_t total = A.wave_off[A.n_links];
  if (w >= total) {
    // surplus wave: its dL/dg partial row is zero
    if (A.g_part)
      for (int m = lane; m < A.M; m += 64) {
        A.g_part[(w * A.M + m) * 2 + 0] = 0.0;
        A.g_part[(w * A.M + m) * 2 + 1] = 0.0;
      }
    return;
  }
  int lo = 0, hi = A.n_links - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (A.wave_off[mid] <= w)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int64_t l = lo;
  const int grp = (int)(w - A.wave_off[l]);
  const int64_t off0 = A.link_off[l];
  const int64_t off1 = A.link_off[l + 1];
  const int n_tiles = (int)((off1 - off0 + 31) / 32);
  const int n_mblk = (A.M + 31) / 32;
  const bool vec = (A.N & 3) == 0;
  const float2* dHl = A.dH + l * (int64_t)A.M * A.N;

  int64_t pidx[kAdjTP];
  bool ok[kAdjTP];
  float2 ai[kAdjTP];
  float psv[kAdjTP];
  double tv[kAdjTP];
  float2 w1[kAdjTP];
#pragma unroll
  for (int u = 0; u < kAdjTP; ++u) {
    const int tile = grp * kAdjTP + u;
    pidx[u] = off0 + (int64_t)tile * 32 + col;
    ok[u] = tile < n_tiles && pidx[u] < off1;
    ai[u] = ok[u] ? A.a[pidx[u]] : make_float2(0.0f, 0.0f);
    psv[u] = ok[u] ? A.psi[pidx[u]] : 0.0f;
    tv[u] = ok[u] ? A.tau[pidx[u]] : 0.0;
    w1[u] = expm2pi_f64(A.df * tv[u]);
  }
  float2 da[kAdjTP];
#pragma unroll
  for (int u = 0; u < kAdjTP; ++u) da[u] = make_float2(0.0f, 0.0f);

  for (int mblk = 0; mblk < n_mblk; ++mblk) {
    const int row = mblk * 32 + col;
    const bool row_ok = row < A.M;
    const float2* rp = dHl + (int64_t)(row_ok ? row : 0) * A.N;
    floatx16 gre[kAdjTP], gim[kAdjTP];
#pragma unroll
    for (int u = 0; u < kAdjTP; ++u) {
      gre[u] = floatx16{0};
      gim[u] = floatx16{0};
    }
    for (int n0 = 0; n0 < A.N; n0 += 64) {
      const int nb = n0 + 32 * half;
      float2 e[kAdjTP];
#pragma unroll
      for (int u = 0; u < kAdjTP; ++u) e[u] = expm2pi_f64((A.f0 + (double)nb * A.df) * tv[u]);
      for (int s4 = 0; s4 < 32; s4 += 4) {
        float2 h[4];
        if (row_ok) {
          load4(rp, nb + s4, A.N, vec, h);
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) h[q] = make_float2(0.0f, 0.0f);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
#pragma unroll
          for (int u = 0; u < kAdjTP; ++u) {
            // G += dH conj(E):  Re: hre er + him ei,  Im: him er - hre ei
            gre[u] = mfma32(h[q].x, e[u].x, gre[u]);
            gre[u] = mfma32(h[q].y, e[u].y, gre[u]);
            gim[u] = mfma32(h[q].y, e[u].x, gim[u]);
            gim[u] = mfma32(-h[q].x, e[u].y, gim[u]);
            e[u] = cmul(e[u], w1[u]);
          }
        }
      }
    }
    // epilogue: rows m = mblk*32 + 8(r/4) + 4 half + r%4, column = path
#pragma unroll
    for (int u = 0; u < kAdjTP; ++u) {
      const double psi_cyc = (double)psv[u] * kInv2Pi;
      float gacc_re[16], gacc_im[16];
#pragma unroll
      for (int grp4 = 0; grp4 < 4; ++grp4) {
        const int mrow0 = mblk * 32 + 8 * grp4 + 4 * half;
        float2 ph = expm2pi_f64(psi_cyc * ((double)mrow0 - A.cm));  // exp(-j psi (m - c))
        const float2 step = expm2pi_f64(psi_cyc);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = grp4 * 4 + q;
          const int mrow = mrow0 + q;
          if (q > 0) ph = cmul(ph, step);
          float2 G = make_float2(gre[u][r], gim[u][r]);
          float2 gm = mrow < A.M ? A.g[mrow] : make_float2(0.0f, 0.0f);
          float2 Gph = cmul(G, ph);
          da[u] = cadd(da[u], cmulc(gm, Gph));
          float2 tg2 = cmulc(ai[u], Gph);
          gacc_re[r] = tg2.x;
          gacc_im[r] = tg2.y;
        }
      }
      if (A.g_part) {
        // sum over the 32 paths of this half (fixed butterfly), add tiles in order
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          float vr = gacc_re[r], vi = gacc_im[r];
#pragma unroll
          for (int o = 16; o >= 1; o >>= 1) {
            vr += __shfl_xor(vr, o, 64);
            vi += __shfl_xor(vi, o, 64);
          }
          const int mrow = mblk * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
          if (col == 0 && mrow < A.M) {
            double* dst = A.g_part + (w * A.M + mrow) * 2;
            if (u == 0) {
              dst[0] = (double)vr;
              dst[1] = (double)vi;
            } else {
              dst[0] += (double)vr;
              dst[1] += (double)vi;
            }
          }
        }
      }
    }
  }
  if (A.dLda) {
#pragma unroll
    for (int u = 0; u < kAdjTP; ++u) {
      float2 d = da[u];
      d.x += __shfl_xor(d.x, 32, 64);
      d.y += __shfl_xor(d.y, 32, 64);
      if (half == 0 && ok[u]) A.dLda[pidx[u]] = d;
    }
  }
}

__global__ void to_c64_kernel(const double* v, int M, float2* out) {
  int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < M) out[m] = make_float2((float)v[2 * m], (float)v[2 * m + 1]);
}

static int64_t adj_max_waves(int32_t n_links, int32_t n_paths) {
  // sum over links of ceil(ceil(P_l / 32) / TP) <= n_paths / (32 TP) + n_links
  return (int64_t)n_paths / (32 * kAdjTP) + n_links + 1;
}

// Workspace: wave_off int64 [L+1] | per-wave dL/dg partials double
// [max_waves][M][2] | reduction tmp | reduced [M][2].
size_t ws_cfr_adjoint(const rtc_radio* r, int32_t n_links, int32_t n_paths) {
  if (r->n_elem < 1) return 0;
  int64_t L = n_links > 0 ? n_links : 1;
  int64_t W = adj_max_waves(n_links, n_paths);
  int K = 2 * r->n_elem;
  return (size_t)(L + 1) * sizeof(int64_t) +
         ((size_t)W * K + reduce_tmp_doubles(W, K) + K) * sizeof(double);
}

static double subcarrier0(const rtc_radio* r) { return r->fc_hz - (double)(r->n_sc / 2) * r->df_hz; }

}  // namespace rtc

using namespace rtc;

extern "C" rtc_status rtc_cfr(const rtc_radio* radio, const rtc_paths* paths, const void* a,
                              const float* psi, const void* g, void* H, void* stream) {
  const char* fn = "rtc_cfr";
  rtc_status st;
  if ((st = check_radio(radio, fn)) != RTC_OK) return st;
  if ((st = check_paths(paths, fn, false)) != RTC_OK) return st;
  RTC_REQUIRE(H != nullptr || paths->n_links == 0, RTC_ERR_INVALID_ARG, "%s: H is NULL", fn);
  RTC_REQUIRE(g != nullptr, RTC_ERR_INVALID_ARG, "%s: g is NULL", fn);
  RTC_REQUIRE((a != nullptr && psi != nullptr) || paths->n_paths == 0, RTC_ERR_INVALID_ARG,
              "%s: a and psi are required", fn);
  if (paths->n_links == 0) return RTC_OK;
  CfrArgs A;
  A.n_links = paths->n_links;
  A.M = radio->n_elem;
  A.N = radio->n_sc;
  A.n_mblk = (A.M + 31) / 32;
  A.n_nchunk = (A.N + 32 * kCfrTiles - 1) / (32 * kCfrTiles);
  A.link_off = paths->link_off;
  A.a = reinterpret_cast<const float2*>(a);
  A.psi = psi;
  A.tau = paths->tau;
  A.g = reinterpret_cast<const float2*>(g);
  A.f0 = subcarrier0(radio);
  A.df = radio->df_hz;
  A.cm = 0.5 * (double)(radio->n_elem - 1);
  int64_t waves = (int64_t)A.n_links * A.n_mblk * A.n_nchunk;
  int64_t blocks = (waves + kCfrWaves - 1) / kCfrWaves;
  RTC_REQUIRE(blocks < (1ll << 31), RTC_ERR_RANGE, "%s: problem too large for one launch", fn);
  hipLaunchKernelGGL(cfr_kernel, dim3((unsigned)blocks), dim3(kCfrWaves * 64), 0,
                     as_stream(stream), A, reinterpret_cast<float2*>(H));
  return check_launch(fn);
}

extern "C" rtc_status rtc_cfr_adjoint(const rtc_radio* radio, const rtc_paths* paths,
                                      const void* a, const float* psi, const void* g,
                                      const void* dLdH, void* dLda, void* dLdg, void* ws,
                                      size_t ws_bytes, void* stream) {
  const char* fn = "rtc_cfr_adjoint";
  rtc_status st;
  if ((st = check_radio(radio, fn)) != RTC_OK) return st;
  if ((st = check_paths(paths, fn, false)) != RTC_OK) return st;
  RTC_REQUIRE(g != nullptr, RTC_ERR_INVALID_ARG, "%s: g is NULL", fn);
  RTC_REQUIRE(dLdH != nullptr || paths->n_links == 0, RTC_ERR_INVALID_ARG, "%s: dLdH is NULL",
              fn);
  RTC_REQUIRE((a != nullptr && psi != nullptr) || paths->n_paths == 0, RTC_ERR_INVALID_ARG,
              "%s: a and psi are required", fn);
  hipStream_t s = as_stream(stream);
  {
    size_t need = ws_cfr_adjoint(radio, paths->n_links, paths->n_paths);
    RTC_REQUIRE(ws != nullptr && ws_bytes >= need, RTC_ERR_WORKSPACE,
                "%s: workspace of %zu bytes required", fn, need);
  }
  if (paths->n_links == 0) {
    if (dLdg) {
      if (hipMemsetAsync(dLdg, 0, sizeof(float2) * radio->n_elem, s) != hipSuccess) {
        set_error("%s: hipMemsetAsync failed", fn);
        return RTC_ERR_HIP;
      }
    }
    return RTC_OK;
  }
  AdjArgs A;
  A.n_links = paths->n_links;
  A.M = radio->n_elem;
  A.N = radio->n_sc;
  A.max_waves = adj_max_waves(paths->n_links, paths->n_paths);
  A.link_off = paths->link_off;
  int64_t* wave_off = reinterpret_cast<int64_t*>(ws);
  A.wave_off = wave_off;
  A.a = reinterpret_cast<const float2*>(a);
  A.psi = psi;
  A.tau = paths->tau;
  A.g = reinterpret_cast<const float2*>(g);
  A.dH = reinterpret_cast<const float2*>(dLdH);
  A.dLda = reinterpret_cast<float2*>(dLda);
  double* gpart = reinterpret_cast<double*>(wave_off + (paths->n_links + 1));
  A.g_part = dLdg ? gpart : nullptr;
  A.f0 = subcarrier0(radio);
  A.df = radio->df_hz;
  A.cm = 0.5 * (double)(radio->n_elem - 1);
  hipLaunchKernelGGL(adj_wave_scan_kernel, dim3(1), dim3(1024), 0, s, paths->link_off,
                     paths->n_links, wave_off);
  if ((st = check_launch(fn)) != RTC_OK) return st;
  const int64_t blocks = (A.max_waves + kAdjWaves - 1) / kAdjWaves;
  RTC_REQUIRE(blocks < (1ll << 31), RTC_ERR_RANGE, "%s: problem too large for one launch", fn);
  hipLaunchKernelGGL(cfr_adjoint_kernel, dim3((unsigned)blocks), dim3(kAdjWaves * 64), 0, s, A);
  if ((st = check_launch(fn)) != RTC_OK) return st;
  if (dLdg) {
    // dL/dg_m = sum over waves (links in order) of the partials, fixed order, FP64
    const int K = 2 * A.M;
    double* tmp = A.g_part + A.max_waves * K;
    double* red = tmp + reduce_tmp_doubles(A.max_waves, K);
    if ((st = reduce_all(A.g_part, A.max_waves, K, tmp, red, s, fn)) != RTC_OK) return st;
    hipLaunchKernelGGL(to_c64_kernel, dim3((A.M + 63) / 64), dim3(64), 0, s, red, A.M,
                       reinterpret_cast<float2*>(dLdg));
    return check_launch(fn);
  }
  return RTC_OK;
}
