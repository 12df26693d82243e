// Channel frequency response and its adjoint on the matrix cores.
//
// For one link l the CFR is a complex matrix product
//     H_l[m, n] = sum_i B[m, i] E[i, n],
//     B[m, i] = a_i g_m exp(j psi_i (m - c)),  E[i, n] = exp(-j 2 pi f_n tau_i),
// with M elements, N subcarriers and P_l paths (Eq. cfr_cont, Sec. II-A).
// Both operands are generated in registers and fed to
// v_mfma_f32_32x32x16_bf16 as three-way BF16 splits (six partial products
// per real product, FP32 accumulation; see split_bf16.h), which keeps FP32
// accuracy at the BF16 instruction rate.  A lane holds eight k values of its
// row (A) or column (B): in the forward product k runs over paths, so lane l
// generates B for row l%32 and E for column l%32 over paths 8(l/32)..+7 of a
// 16-path chunk; the complex product takes four real products,
//     Re H += B_re E_re + (-B_im) E_im,   Im H += B_re E_im + B_im E_re.
// The subcarrier phase f_n tau_i (thousands of cycles) is reduced in FP64;
// within a wave, tile t+1 is tile t times exp(-j 2 pi 32 df tau_i).
//
// The adjoint G[m, i] = sum_n dLdH[m, n] conj(E[i, n]) is the same kind of
// product with the subcarriers as the contraction axis: lane l reads eight
// consecutive subcarriers of its dL/dH row.  Within a 16-subcarrier chunk
// conj(E) factors into a per-chunk phase of the path times a pattern that is
// the same for every chunk, so the B operand is split once per wave and the
// per-chunk phase is applied to the FP32 product (see adj_wave).
#include <cmath>

#include "api_common.h"
#include "dev_common.h"
#include "split_bf16.h"

namespace rtc {

constexpr int kCfrWaves = 4;   // waves per workgroup (forward)
constexpr int kCfrTiles = 8;   // 32-subcarrier tiles per wave (forward)
constexpr int kAdjWaves = 4;   // waves per workgroup (adjoint)
constexpr int kAdjTP = 2;      // 32-path tiles per wave (adjoint)
constexpr double kInv2Pi = 0.15915494309189533577;

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

// Four accumulator chains advance together (two tiles, real and imaginary
// parts), so consecutive MFMAs are independent.
RTC_DEV void cfr_tile_pair(const Split3& BR, const Split3& BI, const Split3& NBI,
                           const Split3& ER0, const Split3& EI0, const Split3& ER1,
                           const Split3& EI1, floatx16& re0, floatx16& im0, floatx16& re1,
                           floatx16& im1) {
  re0 = mac6(BR, ER0, re0);
  im0 = mac6(BR, EI0, im0);
  re1 = mac6(BR, ER1, re1);
  im1 = mac6(BR, EI1, im1);
  re0 = mac6(NBI, EI0, re0);
  im0 = mac6(BI, ER0, im0);
  re1 = mac6(NBI, EI1, re1);
  im1 = mac6(BI, ER1, im1);
}

// One wave per (link, 32-row element block, kCfrTiles x 32 subcarriers).
__global__ void __launch_bounds__(kCfrWaves * 64) cfr_kernel(CfrArgs A, float2* __restrict__ H) {
  static_assert(kCfrTiles % 2 == 0, "tiles are processed in pairs");
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

  // The lane's eight paths of a 16-path chunk.  Software pipeline: while
  // the MFMAs of chunk k run, the wave loads the path data of chunk k+1 and
  // generates its operands (the FP64-reduced exponentials), so the matrix
  // cores are not idle during that VALU work.  Loads clamp to the link's
  // last path (always a valid address) and padding paths get a = 0.
  auto fetch = [&](int64_t c0, float2 (&pa)[8], float (&pp)[8], double (&pt)[8]) {
    const int64_t p0 = c0 + 8 * half;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int64_t p = p0 + j;
      const int64_t pc = p < off1 ? p : off1 - 1;
      const float2 av = A.a[pc];
      pa[j] = p < off1 ? av : make_float2(0.0f, 0.0f);
      pp[j] = A.psi[pc];
      pt[j] = A.tau[pc];
    }
  };
  // A operand B[m, i] = a_i g_m exp(j psi_i (m - c)); B operand anchor
  // E[i, n] at the lane's subcarrier of tile 0 and the tile step w_i
  auto operands = [&](const float2 (&pa)[8], const float (&pp)[8], const double (&pt)[8],
                      float (&br)[8], float (&bi)[8], float2 (&ev)[8], float2 (&wv)[8]) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float2 arr = expm2pi_f64(-(double)pp[j] * mc_cyc);
      const float2 b = cmul(cmul(pa[j], gm), arr);
      br[j] = b.x;
      bi[j] = b.y;
      ev[j] = expm2pi_f64(f_lane * pt[j]);
      wv[j] = expm2pi_f64(df32 * pt[j]);
    }
  };
  if (off0 < off1) {
    float br[8], bi[8];
    float2 ev[8], wv[8];
    {
      float2 pa[8];
      float pp[8];
      double pt[8];
      fetch(off0, pa, pp, pt);
      operands(pa, pp, pt, br, bi, ev, wv);
    }
    for (int64_t c0 = off0; c0 < off1; c0 += 16) {
      // next chunk (a clamped, unused load past the last chunk)
      float2 pa[8];
      float pp[8];
      double pt[8];
      fetch(c0 + 16, pa, pp, pt);
      const Split3 BR = split3(br), BI = split3(bi), NBI = neg3(BI);
#pragma unroll
      for (int t = 0; t < kCfrTiles; t += 2) {
        float er0[8], ei0[8], er1[8], ei1[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          if (t > 0) ev[j] = cmul(ev[j], wv[j]);
          er0[j] = ev[j].x;
          ei0[j] = ev[j].y;
          ev[j] = cmul(ev[j], wv[j]);
          er1[j] = ev[j].x;
          ei1[j] = ev[j].y;
        }
        const Split3 ER0 = split3(er0), EI0 = split3(ei0);
        const Split3 ER1 = split3(er1), EI1 = split3(ei1);
        cfr_tile_pair(BR, BI, NBI, ER0, EI0, ER1, EI1, acc_re[t], acc_im[t], acc_re[t + 1],
                      acc_im[t + 1]);
      }
      operands(pa, pp, pt, br, bi, ev, wv);
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

// Eight consecutive values of a dL/dH row starting at subcarrier n (zero
// beyond N or for a padding row); vec: 16-byte aligned rows.
__device__ __forceinline__ void load8(const float2* row, int n, int N, bool vec, bool ok,
                                      float2 (&h)[8]) {
  if (ok && vec && n + 7 < N) {
    const float4* p = reinterpret_cast<const float4*>(row + n);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 x = p[q];
      h[2 * q] = make_float2(x.x, x.y);
      h[2 * q + 1] = make_float2(x.z, x.w);
    }
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) h[j] = (ok && n + j < N) ? row[n + j] : make_float2(0.0f, 0.0f);
  }
}

// Contraction of one wave over NT (1 or 2) consecutive 32-path tiles of link
// l, starting at tile grp * kAdjTP; the caller picks NT = 1 for a link's
// last wave when it holds a single tile, so no MFMA runs on empty tiles.
// LDS home of a wave's B operands: [tile][VR h,m,l, VI h,m,l][lane], 16 B
// per entry, read back once per chunk (they are constant over the wave, but
// held in registers they would cost the occupancy of two waves per SIMD).
typedef bf16x8 AdjVbuf[kAdjTP][6][64];

template <int NT>
__device__ __forceinline__ void adj_wave(const AdjArgs& A, int64_t w, int64_t l, int grp,
                                         int lane, AdjVbuf& vbuf) {
  const int half = lane >> 5;
  const int col = lane & 31;
  const int64_t off0 = A.link_off[l];
  const int64_t off1 = A.link_off[l + 1];
  const int n_mblk = (A.M + 31) / 32;
  const bool vec = (A.N & 1) == 0 && (reinterpret_cast<uintptr_t>(A.dH) & 15) == 0;
  const float2* dHl = A.dH + l * (int64_t)A.M * A.N;

  // Per 16-subcarrier chunk starting at n0, conj(E[p, n0 + k]) =
  // c_p(n0) v_p(k) with c_p(n0) = exp(+j 2 pi f_n0 tau_p) and
  // v_p(k) = exp(+j 2 pi k df tau_p).  The B operand V[k, p] = v_p(k) is the
  // same for every chunk, so it is generated and split once; each chunk's
  // MFMA product P = dH_chunk V is rotated by the lane's c_p (the result
  // column is the lane's path) and added to G in FP32.
  // the lane's path in tile u (a, psi are read again in the epilogue)
  auto path_of = [&](int u) { return off0 + (int64_t)(grp * kAdjTP + u) * 32 + col; };
  double tv[NT];
  float2 w16[NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    const int64_t p = path_of(u);
    tv[u] = p < off1 ? A.tau[p] : 0.0;
    float vr[8], vi[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float2 e = expm2pi_f64((double)(8 * half + j) * A.df * tv[u]);
      vr[j] = e.x;
      vi[j] = -e.y;
    }
    const Split3 VR = split3(vr), VI = split3(vi);
    vbuf[u][0][lane] = VR.h;
    vbuf[u][1][lane] = VR.m;
    vbuf[u][2][lane] = VR.l;
    vbuf[u][3][lane] = VI.h;
    vbuf[u][4][lane] = VI.m;
    vbuf[u][5][lane] = VI.l;
    w16[u] = cconj(expm2pi_f64(16.0 * A.df * tv[u]));
  }
  // each lane reads back only what it wrote: no barrier, but the compiler
  // must not keep the values in registers
  asm volatile("" ::: "memory");
  float2 da[NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) da[u] = make_float2(0.0f, 0.0f);

  for (int mblk = 0; mblk < n_mblk; ++mblk) {
    const int row = mblk * 32 + col;
    const bool row_ok = row < A.M;
    const float2* rp = dHl + (int64_t)(row_ok ? row : 0) * A.N;
    floatx16 gre[NT], gim[NT];
    float2 c[NT];
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      gre[u] = floatx16{0};
      gim[u] = floatx16{0};
      c[u] = make_float2(1.0f, 0.0f);
    }
    // 16-subcarrier chunks: lane l holds subcarriers n0 + 8(l/32) + j of its
    // dL/dH row (A operand); the next chunk's values are loaded while the
    // current chunk's MFMAs run
    float2 hv[8];
    load8(rp, 8 * half, A.N, vec, row_ok, hv);
    for (int n0 = 0; n0 < A.N; n0 += 16) {
      float hr[8], hi[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        hr[j] = hv[j].x;
        hi[j] = hv[j].y;
      }
      if (n0 + 16 < A.N) load8(rp, n0 + 16 + 8 * half, A.N, vec, row_ok, hv);
      const Split3 HR = split3(hr), HI = split3(hi), NHI = neg3(HI);
      const bool anchor = (n0 & 63) == 0;  // FP64 re-anchor every 64 subcarriers
#pragma unroll
      for (int u = 0; u < NT; ++u) {
        asm volatile("" ::: "memory");  // reload V per chunk (see vbuf)
        Split3 VR, VI;
        VR.h = vbuf[u][0][lane];
        VR.m = vbuf[u][1][lane];
        VR.l = vbuf[u][2][lane];
        VI.h = vbuf[u][3][lane];
        VI.m = vbuf[u][4][lane];
        VI.l = vbuf[u][5][lane];
        // P = dH V:  Re: hre vr - him vi,  Im: hre vi + him vr
        floatx16 pr = mac6(HR, VR, floatx16{0});
        floatx16 pim = mac6(HR, VI, floatx16{0});
        pr = mac6(NHI, VI, pr);
        pim = mac6(HI, VR, pim);
        c[u] = anchor ? cconj(expm2pi_f64((A.f0 + (double)n0 * A.df) * tv[u]))
                      : cmul(c[u], w16[u]);
        const float2 cu = c[u];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          gre[u][r] = fmaf(cu.x, pr[r], fmaf(-cu.y, pim[r], gre[u][r]));
          gim[u][r] = fmaf(cu.x, pim[r], fmaf(cu.y, pr[r], gim[u][r]));
        }
      }
    }
    // epilogue: rows m = mblk*32 + 8(r/4) + 4 half + r%4, column = path
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      const int64_t p = path_of(u);
      const bool ok = p < off1;
      const float2 ai = ok ? A.a[p] : make_float2(0.0f, 0.0f);
      const double psi_cyc = (double)(ok ? A.psi[p] : 0.0f) * kInv2Pi;
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
          float2 tg2 = cmulc(ai, Gph);
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
    for (int u = 0; u < NT; ++u) {
      float2 d = da[u];
      d.x += __shfl_xor(d.x, 32, 64);
      d.y += __shfl_xor(d.y, 32, 64);
      const int64_t p = path_of(u);
      if (half == 0 && p < off1) A.dLda[p] = d;
    }
  }
}

__global__ void __launch_bounds__(kAdjWaves * 64, 2) cfr_adjoint_kernel(AdjArgs A) {
  __shared__ AdjVbuf vbuf[kAdjWaves];
  const int lane = threadIdx.x & 63;
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
  const int n_tiles = (int)((A.link_off[l + 1] - A.link_off[l] + 31) / 32);
  AdjVbuf& vb = vbuf[threadIdx.x >> 6];
  if constexpr (kAdjTP == 2) {
    if (grp * kAdjTP + 1 < n_tiles)
      adj_wave<2>(A, w, l, grp, lane, vb);
    else
      adj_wave<1>(A, w, l, grp, lane, vb);
  } else {
    (void)n_tiles;
    adj_wave<1>(A, w, l, grp, lane, vb);
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
