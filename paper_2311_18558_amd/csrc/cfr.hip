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
// product with the subcarriers as the contraction axis; dLdH is staged
// through LDS in chunks of 64 subcarriers, and E advances by a two-step
// recurrence exp(-j 2 pi 2 df tau_i), re-anchored in FP64 at every chunk.
#include <cmath>

#include "api_common.h"
#include "dev_common.h"

namespace rtc {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kCfrWaves = 4;   // waves per workgroup (forward)
constexpr int kCfrTiles = 4;   // 32-subcarrier tiles per wave (forward)
constexpr int kAdjWaves = 4;   // waves per workgroup (adjoint)
constexpr int kAdjTP = 2;      // 32-path tiles per wave (adjoint)
constexpr int kAdjChunk = 64;  // subcarriers per LDS chunk (adjoint)
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
struct AdjArgs {
  int n_links, M, N;
  const int64_t* link_off;
  const float2* a;
  const float* psi;
  const double* tau;
  const float2* g;
  const float2* dH;
  float2* dLda;     // may be null
  double* g_part;   // [n_links][M][2] per-link dL/dg partials, or null
  double f0, df, cm;
};

__global__ void __launch_bounds__(kAdjWaves * 64) cfr_adjoint_kernel(AdjArgs A) {
  __shared__ float sre[32][kAdjChunk + 1];
  __shared__ float sim[32][kAdjChunk + 1];
  __shared__ double gsum[kAdjWaves][32][2];

  const int lane = threadIdx.x & 63;
  const int half = lane >> 5;
  const int col = lane & 31;
  const int wave = threadIdx.x >> 6;
  const int64_t l = blockIdx.x;
  const int64_t off0 = A.link_off[l];
  const int64_t off1 = A.link_off[l + 1];
  const int64_t P_l = off1 - off0;
  const int n_tiles = (int)((P_l + 31) / 32);
  const int n_mblk = (A.M + 31) / 32;
  const int n_chunks = (A.N + kAdjChunk - 1) / kAdjChunk;
  const double df2 = 2.0 * A.df;
  const float2* dHl = A.dH + l * (int64_t)A.M * A.N;

  for (int mblk = 0; mblk < n_mblk; ++mblk) {
    // per-wave dL/dg partial sums for the 16 rows this lane's half reduces
    double gacc_re[16], gacc_im[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) gacc_re[r] = gacc_im[r] = 0.0;

    for (int tg = 0; tg < n_tiles; tg += kAdjWaves * kAdjTP) {
      // this wave's tiles
      int64_t pidx[kAdjTP];
      float2 ai[kAdjTP];
      float psv[kAdjTP];
      double tv[kAdjTP];
      bool any_tile = false;
#pragma unroll
      for (int u = 0; u < kAdjTP; ++u) {
        int tile = tg + wave * kAdjTP + u;
        pidx[u] = off0 + (int64_t)tile * 32 + col;
        bool ok = tile < n_tiles && pidx[u] < off1;
        any_tile |= tile < n_tiles;
        ai[u] = ok ? A.a[pidx[u]] : make_float2(0.0f, 0.0f);
        psv[u] = ok ? A.psi[pidx[u]] : 0.0f;
        tv[u] = ok ? A.tau[pidx[u]] : 0.0;
      }
      floatx16 gre[kAdjTP], gim[kAdjTP];
#pragma unroll
      for (int u = 0; u < kAdjTP; ++u) {
        gre[u] = floatx16{0};
        gim[u] = floatx16{0};
      }
      float2 w2[kAdjTP];
#pragma unroll
      for (int u = 0; u < kAdjTP; ++u) w2[u] = expm2pi_f64(df2 * tv[u]);

      for (int ch = 0; ch < n_chunks; ++ch) {
        const int n0 = ch * kAdjChunk;
        __syncthreads();  // previous chunk fully consumed
        for (int idx = threadIdx.x; idx < 32 * kAdjChunk; idx += blockDim.x) {
          int mr = idx / kAdjChunk, j = idx % kAdjChunk;
          int row = mblk * 32 + mr, n = n0 + j;
          float2 v = (row < A.M && n < A.N) ? dHl[(int64_t)row * A.N + n] : make_float2(0.0f, 0.0f);
          sre[mr][j] = v.x;
          sim[mr][j] = v.y;
        }
        __syncthreads();
        if (any_tile) {
          float2 e[kAdjTP];
#pragma unroll
          for (int u = 0; u < kAdjTP; ++u)
            e[u] = expm2pi_f64((A.f0 + (double)(n0 + half) * A.df) * tv[u]);
          const int steps = kAdjChunk / 2;
          for (int s2 = 0; s2 < steps; ++s2) {
            const float hre = sre[col][2 * s2 + half];
            const float him = sim[col][2 * s2 + half];
#pragma unroll
            for (int u = 0; u < kAdjTP; ++u) {
              // G += dH conj(E):  Re: hre er + him ei,  Im: him er - hre ei
              gre[u] = mfma32(hre, e[u].x, gre[u]);
              gre[u] = mfma32(him, e[u].y, gre[u]);
              gim[u] = mfma32(him, e[u].x, gim[u]);
              gim[u] = mfma32(-hre, e[u].y, gim[u]);
              e[u] = cmul(e[u], w2[u]);
            }
          }
        }
      }

      // epilogue: dL/da_i and dL/dg partials from G (rows m, columns paths)
#pragma unroll
      for (int u = 0; u < kAdjTP; ++u) {
        float2 da = make_float2(0.0f, 0.0f);
        const double psi_cyc = (double)psv[u] * kInv2Pi;
#pragma unroll
        for (int grp = 0; grp < 4; ++grp) {
          const int mrow0 = mblk * 32 + 8 * grp + 4 * half;
          // exp(-j psi (m - c)) for m = mrow0 .. mrow0+3 by a 1-step recurrence
          float2 ph = expm2pi_f64(psi_cyc * ((double)mrow0 - A.cm));
          float2 step = expm2pi_f64(psi_cyc);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = grp * 4 + q;
            const int mrow = mrow0 + q;
            if (q > 0) ph = cmul(ph, step);
            float2 G = make_float2(gre[u][r], gim[u][r]);
            float2 gm = mrow < A.M ? A.g[mrow] : make_float2(0.0f, 0.0f);
            float2 Gph = cmul(G, ph);
            // conj(g_m e^{j psi (m-c)}) = conj(g_m) e^{-j psi (m-c)}
            da = cadd(da, cmulc(gm, Gph));
            // conj(a_i e^{j psi (m-c)}) = conj(a_i) e^{-j psi (m-c)}
            float2 tg2 = cmulc(ai[u], Gph);
            gacc_re[r] += (double)tg2.x;
            gacc_im[r] += (double)tg2.y;
          }
        }
        da.x += __shfl_xor(da.x, 32, 64);
        da.y += __shfl_xor(da.y, 32, 64);
        int tile = tg + wave * kAdjTP + u;
        if (A.dLda && half == 0 && tile < n_tiles && pidx[u] < off1 && mblk == 0) {
          A.dLda[pidx[u]] = da;
        } else if (A.dLda && half == 0 && tile < n_tiles && pidx[u] < off1) {
          float2 prev = A.dLda[pidx[u]];
          A.dLda[pidx[u]] = cadd(prev, da);
        }
      }
    }

    // reduce dL/dg over the 32 path lanes of each half, then over waves
    if (A.g_part) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        double vr = gacc_re[r], vi = gacc_im[r];
#pragma unroll
        for (int o = 16; o >= 1; o >>= 1) {
          vr += __shfl_xor(vr, o, 64);
          vi += __shfl_xor(vi, o, 64);
        }
        if (col == 0) {
          const int mr = 8 * (r >> 2) + 4 * half + (r & 3);
          gsum[wave][mr][0] = vr;
          gsum[wave][mr][1] = vi;
        }
      }
      __syncthreads();
      if (threadIdx.x < 32) {
        const int mr = threadIdx.x;
        const int row = mblk * 32 + mr;
        if (row < A.M) {
          double sr = 0.0, si = 0.0;
          for (int w = 0; w < kAdjWaves; ++w) {
            sr += gsum[w][mr][0];
            si += gsum[w][mr][1];
          }
          A.g_part[(l * A.M + row) * 2 + 0] = sr;
          A.g_part[(l * A.M + row) * 2 + 1] = si;
        }
      }
      __syncthreads();
    }
  }
}

__global__ void to_c64_kernel(const double* v, int M, float2* out) {
  int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < M) out[m] = make_float2((float)v[2 * m], (float)v[2 * m + 1]);
}

// Workspace (doubles): per-link dL/dg partials [L][M][2] | reduction tmp |
// reduced [M][2].
size_t ws_cfr_adjoint(const rtc_radio* r, int32_t n_links) {
  if (r->n_elem < 1) return 0;
  int64_t L = n_links > 0 ? n_links : 1;
  int K = 2 * r->n_elem;
  return ((size_t)L * K + reduce_tmp_doubles(L, K) + K) * sizeof(double);
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
  if (dLdg) {
    size_t need = ws_cfr_adjoint(radio, paths->n_links);
    RTC_REQUIRE(ws != nullptr && ws_bytes >= need, RTC_ERR_WORKSPACE,
                "%s: workspace of %zu bytes required for dLdg", fn, need);
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
  A.link_off = paths->link_off;
  A.a = reinterpret_cast<const float2*>(a);
  A.psi = psi;
  A.tau = paths->tau;
  A.g = reinterpret_cast<const float2*>(g);
  A.dH = reinterpret_cast<const float2*>(dLdH);
  A.dLda = reinterpret_cast<float2*>(dLda);
  A.g_part = dLdg ? reinterpret_cast<double*>(ws) : nullptr;
  A.f0 = subcarrier0(radio);
  A.df = radio->df_hz;
  A.cm = 0.5 * (double)(radio->n_elem - 1);
  hipLaunchKernelGGL(cfr_adjoint_kernel, dim3(paths->n_links), dim3(kAdjWaves * 64), 0, s, A);
  if ((st = check_launch(fn)) != RTC_OK) return st;
  if (dLdg) {
    // dL/dg_m = sum over links of the per-link partials, fixed order, FP64
    const int K = 2 * A.M;
    double* tmp = A.g_part + (int64_t)A.n_links * K;
    double* red = tmp + reduce_tmp_doubles(A.n_links, K);
    if ((st = reduce_all(A.g_part, A.n_links, K, tmp, red, s, fn)) != RTC_OK) return st;
    hipLaunchKernelGGL(to_c64_kernel, dim3((A.M + 63) / 64), dim3(64), 0, s, red, A.M,
                       reinterpret_cast<float2*>(dLdg));
    return check_launch(fn);
  }
  return RTC_OK;
}
