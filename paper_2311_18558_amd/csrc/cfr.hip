// Channel frequency response and its adjoint on the matrix cores.
//
// For one link l the CFR is a complex matrix product
//     H_l[m, n] = sum_i B[m, i] E[i, n],
//     B[m, i] = a_i g_m exp(j psi_i (m - c)),  E[i, n] = exp(-j 2 pi f_n tau_i),
// with M elements, N subcarriers and P_l paths (Eq. cfr_cont, Sec. II-A).
// Both operands are generated in registers and fed to
// v_mfma_f32_32x32x16_f16 as two-way FP16 splits with FP32 accumulation
// (three partial products per real product, ~2^-22 relative error per
// product; split_f16.h).  The exponentials are unit-modulus; the other
// operand is brought into FP16's range by a power-of-two scale, exact both
// ways: per link from its largest path coefficient in the forward product,
// per wave from the running maximum of the dL/dH values read so far in the
// adjoint.  A lane holds eight k values of its row (A) or column (B): in the
// forward product k runs over paths, so lane l holds the A operand for
// element row l%32 and the B operand for column l%32 over paths
// 8(l/32)..+7 of a 16-path chunk.  The forward's A operand is the same for
// every wave of a link and element block: the workgroup forms it once per
// stage of paths and shares it through LDS.
//
// The forward product uses the symmetry of the subcarrier grid about its
// midpoint: the exponentials of the subcarriers at offsets +t and -t from
// it are conjugate up to a common per-path phase, which moves into the A
// operand, so a complex-by-real product gives both subcarriers of a pair
// (see cfr_pair_tile).  The subcarrier phases (thousands of cycles) are
// reduced in FP64 for every (pair, path) of the forward product.
//
// The adjoint G[m, i] = sum_n dLdH[m, n] conj(E[i, n]) is the same kind of
// product with the subcarriers as the contraction axis: lane l reads eight
// consecutive subcarrier pairs of its dL/dH row, the workgroup forming these
// operands once in LDS for all its waves (see cfr_adjoint_kernel).
#include <algorithm>
#include <cmath>

#include "api_common.h"
#include "dev_common.h"
#include "cfr_common.h"
#include "split_f16.h"

namespace rtc {

constexpr int kCfrWaves = 8;      // waves per workgroup at most (forward): two per SIMD
constexpr int kCfrPairTiles = 2;  // tiles of 32 subcarrier pairs per wave (forward)
// the shared path operand's LDS stage at the largest workgroup (forward)
constexpr int kCfrStageBytes = path_stage_bytes(kCfrWaves * 64);
constexpr int kAdjPathsPerWave = 64;  // two 32-path tiles per wave (adjoint)
constexpr int kAdjWaves = 4;   // waves per workgroup (per-wave adjoint)
constexpr int kAdjTP = 2;      // 32-path tiles per wave (per-wave adjoint)

struct CfrArgs {
  int n_links, M, N;
  int n_mblk, n_qchunk;
  int Q;        // subcarrier pairs, ceil(N/2)
  const int64_t* link_off;
  const float2* a;
  const float* psi;
  const double* tau;
  const float2* g;
  double fref;  // midpoint of the grid, f0 + (N-1)/2 df
  double t_off; // t of pair 0: 1/2 for even N, 0 for odd N
  double df;    // subcarrier spacing
  double cm;    // (M-1)/2
};

// Conjugate pairs of subcarriers.  The grid f_n = f0 + n df is symmetric
// about its midpoint f_ref = f0 + (N-1)/2 df, and with t = n - (N-1)/2
//     E[i, n] = c_i u_i(t),  c_i = exp(-j 2 pi f_ref tau_i),
//     u_i(t) = exp(-j 2 pi t df tau_i),  u_i(-t) = conj(u_i(t)).
// Pair q (0 <= q < ceil(N/2)) joins n_hi = floor(N/2) + q and
// n_lo = N - 1 - n_hi (t = +-t_q); with A'[m, i] = B[m, i] c_i,
//     X = sum_i A' Re u_i(t_q),  Y = sum_i A' Im u_i(t_q)      (complex)
//     H[m, n_hi] = X + j Y,      H[m, n_lo] = X - j Y,
// so one complex-by-real product (four real products, as one complex
// product took before) yields two subcarriers, and only the real and
// imaginary parts of u are split.  For odd N pair 0 is the middle
// subcarrier alone (t = 0, Y = 0).
RTC_DEV void cfr_pair_tile(const Split2& AR, const Split2& AI, const Split2& UR,
                           const Split2& UI, floatx16& xr, floatx16& xi, floatx16& yr,
                           floatx16& yi) {
  xr = mac3(AR, UR, xr);
  xi = mac3(AI, UR, xi);
  yr = mac3(AR, UI, yr);
  yi = mac3(AI, UI, yi);
}

// One workgroup of NW <= kCfrWaves waves per (link, 32-row element block,
// NW x 64 subcarrier pairs): two waves per SIMD, each wave two 32-pair tiles.
// Per stage of NW x 8 paths the workgroup forms the path operand A' once
// (path_stage_store: four values per thread, FP16 parts in the MFMA lane
// layout in LDS); each wave reads it back with four 16-byte loads per 16
// paths and forms its subcarrier operand u_i(t_q) directly from FP64-reduced
// phases (no recurrence, no shuffles).
// Work items b = blockIdx.x + k gridDim.x: with short links the launch holds
// only the workgroups the device keeps resident (one per CU at this register
// count), so the H stores of one item drain while the next item's products
// run; otherwise one workgroup per item.
__global__ void __launch_bounds__(kCfrWaves * 64)
    cfr_kernel(CfrArgs A, float2* __restrict__ H, int64_t n_work) {
  __shared__ __align__(16) char smem[kCfrStageBytes];
  const int nt = blockDim.x;
  const int lane = threadIdx.x & 63;
  const int half = lane >> 5;
  const int col = lane & 31;
  const int wv = threadIdx.x >> 6;
  for (int64_t b = blockIdx.x; b < n_work; b += gridDim.x) {
  const int qg = (int)(b % A.n_qchunk);
  const int64_t rest = b / A.n_qchunk;
  const int mblk = (int)(rest % A.n_mblk);
  const int64_t l = rest / A.n_mblk;
  const int q_base = (qg * (nt >> 6) + wv) * 32 * kCfrPairTiles;
  const int m = mblk * 32 + col;
  const float2 g_row = m < A.M ? A.g[m] : make_float2(0.0f, 0.0f);
  const double mc_cyc = ((double)m - A.cm) * kInv2Pi;
  const int64_t off0 = A.link_off[l];
  const int64_t off1 = A.link_off[l + 1];
  // the A operand carries the link's scale 2^sx (exact), removed on output
  const int sx = 14 - cfr_link_scale_exp(A.a, off0, off1, g_row, lane);
  const float2 gm = make_float2(ldexpf(g_row.x, sx), ldexpf(g_row.y, sx));
  const float unscale = ldexpf(1.0f, -sx);
  // t_q df of the lane's pair column in each tile
  double tq[kCfrPairTiles];
#pragma unroll
  for (int t = 0; t < kCfrPairTiles; ++t) tq[t] = ((double)(q_base + 32 * t + col) + A.t_off) * A.df;

  floatx16 acc[kCfrPairTiles][4];
#pragma unroll
  for (int t = 0; t < kCfrPairTiles; ++t)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[t][k] = floatx16{0};

  unsigned* opnd = reinterpret_cast<unsigned*>(smem);
  double* tau_s = reinterpret_cast<double*>(smem + path_stage_opnd_bytes(nt));
  const int sp = path_stage_paths(nt);
  PathFetch pf;
  if (off0 < off1) path_fetch(A.a, A.psi, A.tau, off0, off1, nt, pf);
  for (int64_t s0 = off0; s0 < off1; s0 += sp) {
    __syncthreads();  // the previous stage's operands are consumed
    path_stage_store(pf, s0, off1, nt, A.fref, mc_cyc, gm, col, opnd, tau_s);
    __syncthreads();
    // the next stage's path data load while this stage's products run
    if (s0 + sp < off1) path_fetch(A.a, A.psi, A.tau, s0 + sp, off1, nt, pf);
    const int nch = (int)min((int64_t)(sp / 16), (off1 - s0 + 15) >> 4);
    for (int c = 0; c < nch; ++c) {
      Split2 AR, AI;
      path_stage_read(opnd, c, lane, AR, AI);
      const double* tp = tau_s + 16 * c + 8 * half;
#pragma unroll
      for (int t = 0; t < kCfrPairTiles; ++t) {
        float ur[8], ui[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const float2 u = expm2pi_f64_hw(tq[t] * tp[j]);
          ur[j] = u.x;
          ui[j] = u.y;
        }
        const Split2 UR = split2(ur), UI = split2(ui);
        cfr_pair_tile(AR, AI, UR, UI, acc[t][0], acc[t][1], acc[t][2], acc[t][3]);
      }
    }
  }

  float2* Hl = H + (int64_t)l * A.M * A.N;
#pragma unroll
  for (int t = 0; t < kCfrPairTiles; ++t) {
    const int q = q_base + t * 32 + col;
    const int n_hi = A.N / 2 + q;
    const int n_lo = A.N - 1 - n_hi;
    const bool ok = q < A.Q;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = mblk * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
      if (ok && row < A.M) {
        const float xr = acc[t][0][r] * unscale, xi = acc[t][1][r] * unscale;
        const float yr = acc[t][2][r] * unscale, yi = acc[t][3][r] * unscale;
        float2* Hr = Hl + (int64_t)row * A.N;
        Hr[n_hi] = make_float2(xr - yi, xi + yr);
        if (n_lo != n_hi) Hr[n_lo] = make_float2(xr + yi, xi - yr);
      }
    }
  }
  }  // work items
}

// ------------------------------------------------------------------ adjoint
struct AdjArgs {
  int n_links, M, N, Q;
  int64_t max_waves;        // work units of the launch (rows of g_part)
  const int64_t* link_off;
  const int64_t* wave_off;  // [n_links + 1] exclusive scan of work units per link
  const float2* a;
  const float* psi;
  const double* tau;
  const float2* g;
  const float2* dH;
  float2* dLda;    // may be null
  double* g_part;  // [max_waves][M][2] per-unit dL/dg partials, or null
  double fref, t_off, df, cm;  // grid midpoint, t of pair 0, spacing, (M-1)/2
};

// Exclusive scan of work units per link, ceil(P_l / unit) (unit = 64 NWA
// paths for the matrix-core adjoint's workgroups, kM1Block paths for the
// single-element one); one block, thread t owns a contiguous run of links.
__global__ void __launch_bounds__(1024) adj_wave_scan_kernel(const int64_t* link_off, int n_links,
                                                              int unit, int64_t* wave_off) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int per = (n_links + 1023) / 1024;
  const int l0 = t * per, l1 = min(n_links, l0 + per);
  // the thread's links in batches of eight (independent loads in flight)
  auto batch = [&](int l, int (&units)[8]) {
    int64_t o[9];
#pragma unroll
    for (int j = 0; j <= 8; ++j) o[j] = link_off[min(l + j, l1)];
#pragma unroll
    for (int j = 0; j < 8; ++j) units[j] = (int)((o[j + 1] - o[j] + unit - 1) / unit);
  };
  int64_t s = 0;
  for (int l = l0; l < l1; l += 8) {
    int units[8];
    batch(l, units);
#pragma unroll
    for (int j = 0; j < 8; ++j) s += units[j];
  }
  // inclusive scan of the 1024 thread totals (Hillis-Steele, fixed order)
  part[t] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int64_t add = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += add;
    __syncthreads();
  }
  int64_t acc = part[t] - s;  // exclusive
  for (int l = l0; l < l1; l += 8) {
    int units[8];
    batch(l, units);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (l + j < l1) wave_off[l + j] = acc;
      acc += units[j];
    }
  }
  if (t == 1023) wave_off[n_links] = acc;
}

// One workgroup of NWA waves per (link, group of NWA x 64 paths), found by
// binary search in a per-link exclusive scan of group counts; wave w takes
// the group's 32-path tiles 2w and 2w + 1.  For each 32-row element block
// the workgroup walks the subcarrier pairs in blocks of 8 NWA: it loads the
// block's dL/dH (both subcarriers of each pair, 16-byte runs; the next
// block's loads are in flight while the current block's products run),
// forms S and D, scales them with the workgroup's running power-of-two scale,
// splits them into FP16 parts and stores them in LDS in the MFMA's A-operand
// layout (double-buffered); every wave reads them back and contracts them
// with its own tiles' exponentials.  S and D are thus formed once per
// workgroup instead of once per wave, and a link's dL/dH is read by its
// ceil(P_l / (64 NWA)) groups instead of by each of its waves.
//
// Conjugate pairs of subcarriers (as in the forward product): with c_p =
// exp(-j 2 pi f_ref tau_p) and u_p(t) = exp(-j 2 pi t df tau_p),
// conj(E[p, n_hi]) = conj(c_p) conj(u_p(t_q)) and conj(E[p, n_lo]) =
// conj(c_p) u_p(t_q), so
//     G[m, p] = conj(c_p) sum_q (S[m, q] Re u_p(t_q) - j D[m, q] Im u_p(t_q))
// with S = dH[., n_hi] + dH[., n_lo] and D = dH[., n_hi] - dH[., n_lo]: two
// complex-by-real products per 16 pairs (32 subcarriers), accumulated over
// the row in the matrix cores, and the path phase conj(c_p) applied once.
template <int NWA>
struct AdjWg {
  static constexpr int NT = NWA * 64;
  static constexpr int BLK = 8 * NWA;             // pairs per block: one (row, quad) item per thread
  static constexpr int NCH = BLK / 16;            // 16-pair chunks per block
  static constexpr int OPND_U32 = NCH * 8 * 64 * 4;  // chunks x 8 parts x 64 lanes x 16 B
  static_assert(NCH >= 1 && 32 * (BLK / 4) == NT, "one staging item per thread");
};

// The four pairs q0 .. q0+3 of a dL/dH row: hi[j] = dH[n_hi(q0 + j)], lo[j] =
// dH[n_lo(q0 + j)], zero past Q, for a padding row, and on the lo side of the
// middle subcarrier of odd N (pair 0 pairs with itself and is counted on the
// n_hi side); 16-byte loads where the rows allow them.
__device__ __forceinline__ void adj_load4(const float2* row, int q0, int N, int Q, bool vec,
                                          bool ok, float2 (&hi)[4], float2 (&lo)[4]) {
  const int nh = N / 2;
  if (ok && vec && q0 + 3 < Q && q0 > 0) {
    const float4* ph = reinterpret_cast<const float4*>(row + nh + q0);
    const float4* pl = reinterpret_cast<const float4*>(row + (N - 4 - nh - q0));
    const float4 a = ph[0], b = ph[1], c = pl[0], d = pl[1];
    hi[0] = make_float2(a.x, a.y);
    hi[1] = make_float2(a.z, a.w);
    hi[2] = make_float2(b.x, b.y);
    hi[3] = make_float2(b.z, b.w);
    lo[3] = make_float2(c.x, c.y);
    lo[2] = make_float2(c.z, c.w);
    lo[1] = make_float2(d.x, d.y);
    lo[0] = make_float2(d.z, d.w);
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = q0 + j;
      const bool use = ok && q < Q;
      hi[j] = use ? row[nh + q] : make_float2(0.0f, 0.0f);
      lo[j] = (use && !((N & 1) && q == 0)) ? row[N - 1 - nh - q] : make_float2(0.0f, 0.0f);
    }
  }
}

template <int NWA>
__global__ void __launch_bounds__(NWA * 64) cfr_adjoint_kernel(AdjArgs A) {
  using C = AdjWg<NWA>;
  __shared__ __align__(16) unsigned opnd[2][C::OPND_U32];
  __shared__ float smax[2][NWA];
  __shared__ double gsh[NWA][32][2];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int half = lane >> 5;
  const int col = lane & 31;
  // XCD-aware order: workgroups go to the eight XCDs in turn, so the first
  // 8 nb workgroups (nb = the real groups per XCD) give XCD b % 8 the
  // (b % 8)-th eighth of the real groups, in order; the groups of one link
  // then sit on one XCD and share its L2 for the link's dL/dH.  The surplus
  // workgroups come after them (the grid is a multiple of eight, sized for
  // the most groups possible).
  const int64_t total = A.wave_off[A.n_links];
  const int64_t nb = (total + 7) / 8;
  const int64_t b = blockIdx.x, x = b & 7, bs = b >> 3;
  const int64_t unit = bs < nb ? x * nb + bs : 8 * nb + (bs - nb) * 8 + x;
  if (unit >= A.max_waves) return;
  if (unit >= total) {
    // surplus group: its dL/dg partial row is zero
    if (A.g_part)
      for (int i = tid; i < 2 * A.M; i += C::NT) A.g_part[unit * 2 * A.M + i] = 0.0;
    return;
  }
  int lo_l = 0, hi_l = A.n_links - 1;
  while (lo_l < hi_l) {
    const int mid = (lo_l + hi_l + 1) >> 1;
    if (A.wave_off[mid] <= unit)
      lo_l = mid;
    else
      hi_l = mid - 1;
  }
  const int64_t l = lo_l;
  const int grp = (int)(unit - A.wave_off[l]);
  const int64_t off0 = A.link_off[l];
  const int64_t off1 = A.link_off[l + 1];
  const int N = A.N, Q = A.Q, M = A.M;
  const int n_mblk = (M + 31) / 32;
  const bool vec = (N & 3) == 0 && (reinterpret_cast<uintptr_t>(A.dH) & 15) == 0;
  const float2* dHl = A.dH + l * (int64_t)M * N;
  // this wave's tiles (0, 1 or 2 of them; the same on every lane)
  const int64_t wp0 = off0 + (int64_t)grp * C::NT + 64 * wv;
  const int ntw = (int)max((int64_t)0, min((int64_t)2, (off1 - wp0 + 31) >> 5));
  auto path_of = [&](int u) { return wp0 + 32 * u + col; };
  double tv[2];
  float2 v1[2], v16[2], da[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int64_t p = path_of(u);
    tv[u] = p < off1 ? A.tau[p] : 0.0;
    v1[u] = expm2pi_f64_hw(A.df * tv[u]);
    v16[u] = expm2pi_f64_hw(16.0 * A.df * tv[u]);
    da[u] = make_float2(0.0f, 0.0f);
  }
  const int nblk = (Q + C::BLK - 1) / C::BLK;

  for (int mblk = 0; mblk < n_mblk; ++mblk) {
    // G~ = X - j Y accumulated directly:
    //   Re G~ += S_re Re u + D_im Im u,  Im G~ += S_im Re u - D_re Im u
    floatx16 gre[2], gim[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      gre[u] = floatx16{0};
      gim[u] = floatx16{0};
    }
    // The A operand (S and D) carries the workgroup's scale 2^sx: every
    // value seen so far is below lim = 2^(14 - sx), so scaled it stays below
    // 2^14 (FP16 holds up to 65504) and values down to 2^-28 of the largest
    // keep all their bits.  A block reaching lim lowers the scale and
    // multiplies the accumulators by the same power of two (exact); lim = 0
    // until the first nonzero block.
    int sx = 0;
    float lim = 0.0f;
    // the thread's staging item: row r = tid / QB of the element block,
    // pairs 4 (tid % QB) .. +3 of the pair block (QB = BLK / 4 quads per row;
    // consecutive threads read consecutive runs of a row)
    constexpr int QB = C::BLK / 4;
    const int srow = tid / QB, squad = tid % QB;
    float2 hv[4], lv[4];
    auto load_block = [&](int blk) {
      const int row = mblk * 32 + srow;
      const bool ok = row < M;
      adj_load4(dHl + (int64_t)(ok ? row : 0) * N, blk * C::BLK + 4 * squad, N, Q, vec, ok, hv,
                lv);
    };
    // the thread's largest |S|, |D| of the loaded block, published per wave
    // (the wave maximum only when some lane reaches the current limit)
    auto publish_max = [&](int slot) {
      float mx = 0.0f;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float2 s = cadd(hv[j], lv[j]), d = csub(hv[j], lv[j]);
        mx = fmaxf(mx, fmaxf(fmaxf(fabsf(s.x), fabsf(s.y)), fmaxf(fabsf(d.x), fabsf(d.y))));
      }
      if (__ballot(mx > 0.0f && mx >= lim)) mx = wave_max_f32(mx);
      else mx = 0.0f;
      if (lane == 0) smax[slot][wv] = mx;
    };
    // S, D of the loaded block times 2^sx, split into FP16 parts, to the
    // A-operand slots of buffer `buf`: chunk c = quad / 4, lane
    // r + 32 ((quad % 4) / 2), elements 4 (quad % 2) .. +3 of each part's
    // 8-vector
    auto store_block = [&](int buf, float sc) {
      {
        float sr[4], si[4], nd[4], di[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          sr[j] = (hv[j].x + lv[j].x) * sc;
          si[j] = (hv[j].y + lv[j].y) * sc;
          nd[j] = (lv[j].x - hv[j].x) * sc;
          di[j] = (hv[j].y - lv[j].y) * sc;
        }
        const int c = squad >> 2, qr = squad & 3;
        const int L = srow + 32 * (qr >> 1);
        unsigned* base = opnd[buf] + ((c * 8) * 64 + L) * 4 + 2 * (qr & 1);
        auto put = [&](int part, const float (&v)[4]) {
          const unsigned h0 = pack_f16(v[0], v[1]), h1 = pack_f16(v[2], v[3]);
          const unsigned l0 = pack_f16(sub_f16<true>(v[0], h0), sub_f16<false>(v[1], h0));
          const unsigned l1 = pack_f16(sub_f16<true>(v[2], h1), sub_f16<false>(v[3], h1));
          *reinterpret_cast<uint2*>(base + (2 * part) * 64 * 4) = make_uint2(h0, h1);
          *reinterpret_cast<uint2*>(base + (2 * part + 1) * 64 * 4) = make_uint2(l0, l1);
        };
        put(0, sr);
        put(1, si);
        put(2, nd);
        put(3, di);
      }
    };
    load_block(0);
    publish_max(0);
    __syncthreads();
    for (int blk = 0; blk < nblk; ++blk) {
      // the block's scale (the same on every lane)
      float mxb = smax[blk & 1][0];
#pragma unroll
      for (int w = 1; w < NWA; ++w) mxb = fmaxf(mxb, smax[blk & 1][w]);
      if (mxb > 0.0f && mxb >= lim) {
        int e = 0;
        frexpf(mxb, &e);  // mxb < 2^e
        e = min(max(e, -100), 100);
        if (lim > 0.0f) {
          const float f = ldexpf(1.0f, (14 - e) - sx);
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            gre[u] *= f;
            gim[u] *= f;
          }
        }
        sx = 14 - e;
        lim = ldexpf(1.0f, e);
      }
      store_block(blk & 1, ldexpf(1.0f, sx));
      if (blk + 1 < nblk) load_block(blk + 1);  // in flight during the products
      __syncthreads();
      if (ntw > 0) {
        const int g0 = blk * C::BLK;
        float2 uf[2];  // u_p(t) at the lane's first pair of the chunk
        const double t_first = (double)(g0 + 8 * half) + A.t_off;
#pragma unroll
        for (int u = 0; u < 2; ++u) uf[u] = expm2pi_f64_hw(t_first * A.df * tv[u]);
#pragma unroll
        for (int c = 0; c < C::NCH; ++c) {
          if (g0 + 16 * c >= Q) break;
          const u32x4* ob = reinterpret_cast<const u32x4*>(opnd[blk & 1]) + (c * 8) * 64 + lane;
          Split2 SR, SI, NDR, DI;
          SR.h = __builtin_bit_cast(halfx8, ob[0]);
          SR.l = __builtin_bit_cast(halfx8, ob[64]);
          SI.h = __builtin_bit_cast(halfx8, ob[128]);
          SI.l = __builtin_bit_cast(halfx8, ob[192]);
          NDR.h = __builtin_bit_cast(halfx8, ob[256]);
          NDR.l = __builtin_bit_cast(halfx8, ob[320]);
          DI.h = __builtin_bit_cast(halfx8, ob[384]);
          DI.l = __builtin_bit_cast(halfx8, ob[448]);
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            if (u < ntw) {
              if (c > 0) uf[u] = cmul(uf[u], v16[u]);
              float ur[8], ui[8];
              float2 e = uf[u];
#pragma unroll
              for (int j = 0; j < 8; ++j) {
                if (j > 0) e = cmul(e, v1[u]);
                ur[j] = e.x;
                ui[j] = e.y;
              }
              const Split2 UR = split2(ur), UI = split2(ui);
              gre[u] = mac3(SR, UR, gre[u]);
              gim[u] = mac3(SI, UR, gim[u]);
              gre[u] = mac3(DI, UI, gre[u]);
              gim[u] = mac3(NDR, UI, gim[u]);
            }
          }
        }
      }
      if (blk + 1 < nblk) publish_max((blk + 1) & 1);
      __syncthreads();
    }
    // epilogue: rows m = mblk*32 + 8(r/4) + 4 half + r%4, column = path
    const float unscale = ldexpf(1.0f, -sx);
    float gacc_re[16], gacc_im[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) gacc_re[r] = gacc_im[r] = 0.0f;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (u < ntw) {
        gre[u] *= unscale;
        gim[u] *= unscale;
        const int64_t p = path_of(u);
        const bool ok = p < off1;
        const float2 ai = ok ? A.a[p] : make_float2(0.0f, 0.0f);
        const double psi_cyc = (double)(ok ? A.psi[p] : 0.0f) * kInv2Pi;
        const float2 cc = cconj(expm2pi_f64_hw(A.fref * tv[u]));  // conj(c_p)
        const float2 step = expm2pi_f64_hw(psi_cyc);
#pragma unroll
        for (int g4 = 0; g4 < 4; ++g4) {
          const int mrow0 = mblk * 32 + 8 * g4 + 4 * half;
          float2 ph = expm2pi_f64_hw(psi_cyc * ((double)mrow0 - A.cm));  // exp(-j psi (m - c))
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = g4 * 4 + q;
            const int mrow = mrow0 + q;
            if (q > 0) ph = cmul(ph, step);
            const float2 G = cmul(cc, make_float2(gre[u][r], gim[u][r]));  // conj(c_p) G~
            const float2 gm = mrow < M ? A.g[mrow] : make_float2(0.0f, 0.0f);
            const float2 Gph = cmul(G, ph);
            da[u] = cadd(da[u], cmulc(gm, Gph));
            const float2 tg2 = cmulc(ai, Gph);
            gacc_re[r] += tg2.x;  // tiles in order
            gacc_im[r] += tg2.y;
          }
        }
      }
    }
    if (A.g_part) {
      // the wave's rows summed over its paths (each half's 32, fixed
      // butterfly), then the waves in order
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float vr = half_sum_f32(gacc_re[r]), vi = half_sum_f32(gacc_im[r]);
        if (col == 0) {
          const int rl = 8 * (r >> 2) + 4 * half + (r & 3);
          gsh[wv][rl][0] = (double)vr;
          gsh[wv][rl][1] = (double)vi;
        }
      }
      __syncthreads();
      if (tid < 64) {
        const int rl = tid & 31, k = tid >> 5;
        double s = gsh[0][rl][k];
#pragma unroll
        for (int w = 1; w < NWA; ++w) s += gsh[w][rl][k];
        const int mrow = mblk * 32 + rl;
        if (mrow < M) A.g_part[(unit * M + mrow) * 2 + k] = s;
      }
      __syncthreads();
    }
  }
  if (A.dLda) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      float2 d = da[u];
      d.x += __shfl_xor(d.x, 32, 64);
      d.y += __shfl_xor(d.y, 32, 64);
      const int64_t p = path_of(u);
      if (u < ntw && half == 0 && p < off1) A.dLda[p] = d;
    }
  }
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

// Eight dL/dH values of a row at subcarriers n_lo(q) = N - 1 - floor(N/2) - q
// for pairs q = q1 .. q1+7 (a descending run of the row; zero where q >= Q,
// for a padding row, and for the middle subcarrier of odd N, which pairs
// with itself and is counted on the n_hi side).
__device__ __forceinline__ void load8_lo(const float2* row, int q1, int N, int Q, bool vec,
                                         bool ok, float2 (&h)[8]) {
  const int n_top = N - 1 - N / 2 - q1;  // n_lo(q1), the highest address
  if (ok && vec && q1 + 7 < Q && q1 > 0) {
    const float4* p = reinterpret_cast<const float4*>(row + (n_top - 7));
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float4 x = p[k];
      h[7 - 2 * k] = make_float2(x.x, x.y);
      h[6 - 2 * k] = make_float2(x.z, x.w);
    }
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int q = q1 + j;
      const bool use = ok && q < Q && !((N & 1) && q == 0);
      h[j] = use ? row[n_top - j] : make_float2(0.0f, 0.0f);
    }
  }
}

// The adjoint for links of a few hundred paths: one wave per (link, group of
// kAdjTP 32-path tiles), found by binary search in a per-link exclusive scan
// of wave counts, each wave forming the S/D operand of its link itself (no
// workgroup-wide stage, so no tiles idle at the links' ends).  Contraction of
// one wave over NT (1 or 2) consecutive 32-path tiles of link l, starting at
// tile grp * kAdjTP; the caller picks NT = 1 for a link's last wave when it
// holds a single tile, so no MFMA runs on empty tiles.
//
// Conjugate pairs of subcarriers (as in the forward product): with c_p =
// exp(-j 2 pi f_ref tau_p) and u_p(t) = exp(-j 2 pi t df tau_p),
// conj(E[p, n_hi]) = conj(c_p) conj(u_p(t_q)) and conj(E[p, n_lo]) =
// conj(c_p) u_p(t_q), so
//     G[m, p] = conj(c_p) sum_q (S[m, q] Re u_p(t_q) - j D[m, q] Im u_p(t_q))
// with S = dH[., n_hi] + dH[., n_lo] and D = dH[., n_hi] - dH[., n_lo]: two
// complex-by-real products per 16 pairs (32 subcarriers), accumulated over
// the row in the matrix cores, and the path phase conj(c_p) applied once.
template <int NT>
__device__ __forceinline__ void adj_wave(const AdjArgs& A, int64_t w, int64_t l, int grp,
                                         int lane) {
  const int half = lane >> 5;
  const int col = lane & 31;
  const int64_t off0 = A.link_off[l];
  const int64_t off1 = A.link_off[l + 1];
  const int n_mblk = (A.M + 31) / 32;
  const int N = A.N, Q = A.Q, nh = A.N / 2;
  // 16-byte loads need aligned rows and runs starting at even subcarriers
  const bool vec = (N & 3) == 0 && (reinterpret_cast<uintptr_t>(A.dH) & 15) == 0;
  const float2* dHl = A.dH + l * (int64_t)A.M * N;

  // the lane's path in tile u (a, psi are read again in the epilogue)
  auto path_of = [&](int u) { return off0 + (int64_t)(grp * kAdjTP + u) * 32 + col; };
  double tv[NT];
  float2 v1[NT], v16[NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) {
    const int64_t p = path_of(u);
    tv[u] = p < off1 ? A.tau[p] : 0.0;
    v1[u] = expm2pi_f64_hw(A.df * tv[u]);
    v16[u] = expm2pi_f64_hw(16.0 * A.df * tv[u]);
  }
  float2 da[NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) da[u] = make_float2(0.0f, 0.0f);

  for (int mblk = 0; mblk < n_mblk; ++mblk) {
    const int row = mblk * 32 + col;
    const bool row_ok = row < A.M;
    const float2* rp = dHl + (int64_t)(row_ok ? row : 0) * N;
    // G~ = X - j Y accumulated directly:
    //   Re G~ += S_re Re u + D_im Im u,  Im G~ += S_im Re u - D_re Im u
    floatx16 gre[NT], gim[NT];
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      gre[u] = floatx16{0};
      gim[u] = floatx16{0};
    }
    // The A operand (sums and differences of dL/dH) carries the wave-wide
    // scale 2^sx: every value read so far is below lim = 2^(14 - sx), so
    // scaled it stays below 2^14 (FP16 holds up to 65504) and values down to
    // 2^-28 of the largest keep all their bits.  A chunk reaching lim lowers
    // the scale and multiplies the accumulators by the same power of two
    // (exact); lim = 0 until the first nonzero chunk.
    int sx = 0;
    float lim = 0.0f;
    // 16-pair chunks: lane l holds pairs q0 + 8(l/32) + j of its dL/dH row
    // (A operand); the next chunk's values are loaded while the current
    // chunk's MFMAs run.  u_p is anchored in FP64 at the start of every
    // 64-pair group and advanced by exp(-j 2 pi 16 df tau_p) per chunk.
    float2 hv[8], lv[8];
    // a chunk's runs: with aligned rows and a whole chunk (a condition the
    // same for every lane) eight 16-byte loads, lanes of rows past M reading
    // row 0 (their products are discarded); otherwise element loads with
    // the checks of load8 / load8_lo
    auto load_chunk = [&](int qs) {
      if (vec && qs + 16 <= Q) {
        const int q1 = qs + 8 * half;
        const float4* hi4 = reinterpret_cast<const float4*>(rp + nh + q1);
        const float4* lo4 = reinterpret_cast<const float4*>(rp + (N - 8 - nh - q1));
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float4 x = hi4[r], y = lo4[r];
          hv[2 * r] = make_float2(x.x, x.y);
          hv[2 * r + 1] = make_float2(x.z, x.w);
          lv[7 - 2 * r] = make_float2(y.x, y.y);
          lv[6 - 2 * r] = make_float2(y.z, y.w);
        }
      } else {
        load8(rp, nh + qs + 8 * half, N, false, row_ok, hv);
        load8_lo(rp, qs + 8 * half, N, Q, false, row_ok, lv);
      }
    };
    load_chunk(0);
    for (int g0 = 0; g0 < Q; g0 += 64) {
      float2 uf[NT];  // u_p(t) at the lane's first pair of the chunk
      const double t_first = (double)(g0 + 8 * half) + A.t_off;
#pragma unroll
      for (int u = 0; u < NT; ++u) uf[u] = expm2pi_f64_hw(t_first * A.df * tv[u]);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int q0 = g0 + 16 * k;
        if (q0 >= Q) break;
        float sr[8], si[8], ndr[8], di[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          sr[j] = hv[j].x + lv[j].x;
          si[j] = hv[j].y + lv[j].y;
          ndr[j] = lv[j].x - hv[j].x;
          di[j] = hv[j].y - lv[j].y;
        }
        if (q0 + 16 < Q) load_chunk(q0 + 16);
        float mx = 0.0f;
#pragma unroll
        for (int j = 0; j < 8; ++j)
          mx = fmaxf(mx, fmaxf(fmaxf(fabsf(sr[j]), fabsf(si[j])),
                               fmaxf(fabsf(ndr[j]), fabsf(di[j]))));
        // the wave-wide maximum only when some lane reaches the limit (a
        // ballot; rare once the scale has settled)
        if (__ballot(mx > 0.0f && mx >= lim)) mx = wave_max_f32(mx);
        if (mx > 0.0f && mx >= lim) {  // the same on every lane
          int e = 0;
          frexpf(mx, &e);  // mx < 2^e
          e = min(max(e, -100), 100);
          if (lim > 0.0f) {
            const float f = ldexpf(1.0f, (14 - e) - sx);
#pragma unroll
            for (int u = 0; u < NT; ++u) {
              gre[u] *= f;
              gim[u] *= f;
            }
          }
          sx = 14 - e;
          lim = ldexpf(1.0f, e);
        }
        const float sc = ldexpf(1.0f, sx);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          sr[j] *= sc;
          si[j] *= sc;
          ndr[j] *= sc;
          di[j] *= sc;
        }
        const Split2 SR = split2(sr), SI = split2(si);
        const Split2 NDR = split2(ndr), DI = split2(di);
#pragma unroll
        for (int u = 0; u < NT; ++u) {
          if (k > 0) uf[u] = cmul(uf[u], v16[u]);
          float ur[8], ui[8];
          float2 e = uf[u];
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            if (j > 0) e = cmul(e, v1[u]);
            ur[j] = e.x;
            ui[j] = e.y;
          }
          const Split2 UR = split2(ur), UI = split2(ui);
          gre[u] = mac3(SR, UR, gre[u]);
          gim[u] = mac3(SI, UR, gim[u]);
          gre[u] = mac3(DI, UI, gre[u]);
          gim[u] = mac3(NDR, UI, gim[u]);
        }
      }
    }
    // epilogue: rows m = mblk*32 + 8(r/4) + 4 half + r%4, column = path
    const float unscale = ldexpf(1.0f, -sx);
    // dL/dg: each lane sums its paths over the tiles, the half-wave's lanes
    // are added once after them (fixed butterfly)
    float gacc_re[16], gacc_im[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) gacc_re[r] = gacc_im[r] = 0.0f;
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      gre[u] *= unscale;
      gim[u] *= unscale;
      const int64_t p = path_of(u);
      const bool ok = p < off1;
      const float2 ai = ok ? A.a[p] : make_float2(0.0f, 0.0f);
      const double psi_cyc = (double)(ok ? A.psi[p] : 0.0f) * kInv2Pi;
      const float2 cc = cconj(expm2pi_f64_hw(A.fref * tv[u]));  // conj(c_p)
#pragma unroll
      for (int grp4 = 0; grp4 < 4; ++grp4) {
        const int mrow0 = mblk * 32 + 8 * grp4 + 4 * half;
        float2 ph = expm2pi_f64_hw(psi_cyc * ((double)mrow0 - A.cm));  // exp(-j psi (m - c))
        const float2 step = expm2pi_f64_hw(psi_cyc);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = grp4 * 4 + q;
          const int mrow = mrow0 + q;
          if (q > 0) ph = cmul(ph, step);
          const float2 G = cmul(cc, make_float2(gre[u][r], gim[u][r]));  // conj(c_p) G~
          float2 gm = mrow < A.M ? A.g[mrow] : make_float2(0.0f, 0.0f);
          float2 Gph = cmul(G, ph);
          da[u] = cadd(da[u], cmulc(gm, Gph));
          float2 tg2 = cmulc(ai, Gph);
          gacc_re[r] += tg2.x;  // tiles in order
          gacc_im[r] += tg2.y;
        }
      }
    }
    if (A.g_part) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float vr = half_sum_f32(gacc_re[r]), vi = half_sum_f32(gacc_im[r]);
        const int mrow = mblk * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
        if (col == 0 && mrow < A.M) {
          double* dst = A.g_part + (w * A.M + mrow) * 2;
          dst[0] = (double)vr;
          dst[1] = (double)vi;
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

__global__ void __launch_bounds__(kAdjWaves * 64, 2) cfr_adjoint_wave_kernel(AdjArgs A) {
  const int lane = threadIdx.x & 63;
  // XCD-aware order: workgroups go to the eight XCDs in turn, so the first
  // 8 nb workgroups (nb = the workgroups of real waves per XCD) give XCD
  // b % 8 the (b % 8)-th eighth of the real waves, in order; the waves of
  // one link then sit on one XCD and share its L2 for the link's dL/dH,
  // which they all read.  The surplus workgroups come after them (the grid
  // is a multiple of eight workgroups, sized for the most waves possible).
  const int64_t total = A.wave_off[A.n_links];
  const int64_t nb = ((total + kAdjWaves - 1) / kAdjWaves + 7) / 8;
  const int64_t b = blockIdx.x, x = b & 7, bs = b >> 3;
  const int64_t vb = bs < nb ? x * nb + bs : 8 * nb + (bs - nb) * 8 + x;
  const int64_t w = vb * kAdjWaves + (threadIdx.x >> 6);
  if (w >= A.max_waves) return;
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
  if constexpr (kAdjTP == 2) {
    if (grp * kAdjTP + 1 < n_tiles)
      adj_wave<2>(A, w, l, grp, lane);
    else
      adj_wave<1>(A, w, l, grp, lane);
  } else {
    (void)n_tiles;
    adj_wave<1>(A, w, l, grp, lane);
  }
}

// ------------------------------------------------- one array element (M = 1)
// With a single element there is no matrix product (a row of the product
// is all there is), so these kernels run on the vector units: the forward
// takes a thread per subcarrier pair and a link's paths from LDS (staged per
// 256 paths: A' = a g c_p and df tau_p); the adjoint takes a thread per path
// and the link's pair sums S, D of dL/dH from LDS.  Conjugate pairs as in
// the matrix-core kernels; the subcarrier phase of every (path, pair) is
// reduced in FP64 in the forward, and advanced by exp(-j 2 pi df tau) and
// re-anchored in FP64 every 64 pairs in the adjoint.
constexpr int kM1Block = 256;

__global__ void __launch_bounds__(kM1Block) cfr_m1_kernel(CfrArgs A, float2* __restrict__ H) {
  __shared__ float2 sa[kM1Block];   // A' = a g c_p
  __shared__ double sw[kM1Block];   // df tau_p
  const int64_t l = blockIdx.x / A.n_qchunk;
  const int q = (int)(blockIdx.x % A.n_qchunk) * kM1Block + threadIdx.x;
  const int64_t off0 = A.link_off[l], off1 = A.link_off[l + 1];
  const float2 g0 = A.g[0];
  const double t = (double)q + A.t_off;
  float2 X = make_float2(0.0f, 0.0f), Y = make_float2(0.0f, 0.0f);
  for (int64_t c0 = off0; c0 < off1; c0 += kM1Block) {
    const int n = (int)min((int64_t)kM1Block, off1 - c0);
    __syncthreads();
    if ((int)threadIdx.x < n) {
      const int64_t p = c0 + threadIdx.x;
      const double tau = A.tau[p];
      sa[threadIdx.x] = cmul(cmul(A.a[p], g0), expm2pi_f64_hw(A.fref * tau));
      sw[threadIdx.x] = A.df * tau;
    }
    __syncthreads();
    for (int i = 0; i < n; ++i) {
      const float2 u = expm2pi_f64_hw(t * sw[i]);  // u_p(t_q)
      const float2 ap = sa[i];
      X.x = fmaf(ap.x, u.x, X.x);
      X.y = fmaf(ap.y, u.x, X.y);
      Y.x = fmaf(ap.x, u.y, Y.x);
      Y.y = fmaf(ap.y, u.y, Y.y);
    }
  }
  if (q < A.Q) {
    float2* row = H + l * (int64_t)A.N;
    const int n_hi = A.N / 2 + q, n_lo = A.N - 1 - n_hi;
    row[n_hi] = make_float2(X.x - Y.y, X.y + Y.x);  // X + jY
    if (n_lo != n_hi) row[n_lo] = make_float2(X.x + Y.y, X.y - Y.x);  // X - jY
  }
}

__global__ void __launch_bounds__(kM1Block) cfr_adjoint_m1_kernel(AdjArgs A) {
  __shared__ float4 sd[kM1Block];   // (S, D) of kM1Block pairs
  __shared__ double red[kM1Block / 64];
  const int64_t w = blockIdx.x;
  const int64_t total = A.wave_off[A.n_links];
  if (w >= total) {
    // surplus workgroup: its dL/dg partial row is zero
    if (A.g_part && threadIdx.x < 2) A.g_part[w * 2 + threadIdx.x] = 0.0;
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
  const int64_t off1 = A.link_off[l + 1];
  const int64_t p = A.link_off[l] + (w - A.wave_off[l]) * kM1Block + threadIdx.x;
  const bool ok = p < off1;
  const double tau = ok ? A.tau[p] : 0.0;
  const float2 v1 = expm2pi_f64_hw(A.df * tau);
  const float2* row = A.dH + l * (int64_t)A.N;
  const int N = A.N, Q = A.Q, nh = N / 2;
  float gre = 0.0f, gim = 0.0f;  // G~ = X - jY, accumulated as in cfr_adjoint_kernel
  float2 u = make_float2(1.0f, 0.0f);
  for (int q0 = 0; q0 < Q; q0 += kM1Block) {
    const int nq = min(kM1Block, Q - q0);
    __syncthreads();
    if ((int)threadIdx.x < nq) {
      const int q = q0 + threadIdx.x;
      const float2 hv = row[nh + q];
      const bool mid = (N & 1) && q == 0;  // the middle subcarrier pairs with itself
      const float2 lv = mid ? make_float2(0.0f, 0.0f) : row[N - 1 - nh - q];
      sd[threadIdx.x] = make_float4(hv.x + lv.x, hv.y + lv.y, hv.x - lv.x, hv.y - lv.y);
    }
    __syncthreads();
    for (int j = 0; j < nq; ++j) {
      if ((j & 63) == 0) u = expm2pi_f64_hw(((double)(q0 + j) + A.t_off) * A.df * tau);
      const float4 v = sd[j];
      // Re G~ += S_re Re u + D_im Im u,  Im G~ += S_im Re u - D_re Im u
      gre = fmaf(v.x, u.x, fmaf(v.w, u.y, gre));
      gim = fmaf(v.y, u.x, fmaf(-v.z, u.y, gim));
      u = cmul(u, v1);
    }
  }
  float2 da = make_float2(0.0f, 0.0f), dg = make_float2(0.0f, 0.0f);
  if (ok) {
    const float2 G = cmul(cconj(expm2pi_f64_hw(A.fref * tau)), make_float2(gre, gim));
    da = cmulc(A.g[0], G);      // conj(g) G
    dg = cmulc(A.a[p], G);      // conj(a_p) G
    if (A.dLda) A.dLda[p] = da;
  }
  if (A.g_part) {
    const double sr = block_sum_f64((double)dg.x, red);
    const double si = block_sum_f64((double)dg.y, red);
    if (threadIdx.x == 0) {
      A.g_part[w * 2 + 0] = sr;
      A.g_part[w * 2 + 1] = si;
    }
  }
}

__global__ void to_c64_kernel(const double* v, int M, float2* out) {
  int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < M) out[m] = make_float2((float)v[2 * m], (float)v[2 * m + 1]);
}

static int64_t adj_max_waves(int32_t n_links, int32_t n_paths) {
  // sum over links of ceil(P_l / 64) <= n_paths / 64 + n_links: bounds the
  // work units (dL/dg partial rows) of any workgroup size
  return (int64_t)n_paths / kAdjPathsPerWave + n_links + 1;
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
  A.Q = (A.N + 1) / 2;
  // waves per workgroup: enough for the pairs, at most kCfrWaves, and even
  // (a stage of the shared path operand is 8 paths per wave, and the
  // products take 16 at a time)
  const int pw = 32 * kCfrPairTiles;
  const int nw = (int)std::min<int64_t>(kCfrWaves, ((A.Q + pw - 1) / pw + 1) / 2 * 2);
  A.n_qchunk = (A.Q + nw * pw - 1) / (nw * pw);
  A.link_off = paths->link_off;
  A.a = reinterpret_cast<const float2*>(a);
  A.psi = psi;
  A.tau = paths->tau;
  A.g = reinterpret_cast<const float2*>(g);
  A.fref = subcarrier0(radio) + 0.5 * (double)(A.N - 1) * radio->df_hz;
  A.t_off = (A.N % 2 == 0) ? 0.5 : 0.0;
  A.df = radio->df_hz;
  A.cm = 0.5 * (double)(radio->n_elem - 1);
  if (A.M == 1) {
    // one element: no matrix product to form; a thread per subcarrier pair
    A.n_qchunk = (A.Q + kM1Block - 1) / kM1Block;
    const int64_t blocks = (int64_t)A.n_links * A.n_qchunk;
    RTC_REQUIRE(blocks < (1ll << 31), RTC_ERR_RANGE, "%s: problem too large for one launch", fn);
    hipLaunchKernelGGL(cfr_m1_kernel, dim3((unsigned)blocks), dim3(kM1Block), 0,
                       as_stream(stream), A, reinterpret_cast<float2*>(H));
    return check_launch(fn);
  }
  const int64_t blocks = (int64_t)A.n_links * A.n_mblk * A.n_qchunk;
  // persistent workgroups for short links (their stores are a large part of
  // an item); long links of uneven length balance better one workgroup per
  // item, dispatched by the hardware as CUs free up
  const bool persistent = paths->n_paths < 512 * (int64_t)paths->n_links;
  const int64_t grid =
      persistent ? std::min<int64_t>(blocks, resident_workgroups((const void*)cfr_kernel, nw * 64))
                 : blocks;
  RTC_REQUIRE(grid < (1ll << 31), RTC_ERR_RANGE, "%s: problem too large for one launch", fn);
  hipLaunchKernelGGL(cfr_kernel, dim3((unsigned)grid), dim3(nw * 64), 0, as_stream(stream), A,
                     reinterpret_cast<float2*>(H), blocks);
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
    if (dLdg) return zero_floats(reinterpret_cast<float*>(dLdg), 2 * (int64_t)radio->n_elem, s, fn);
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
  A.Q = (A.N + 1) / 2;
  A.fref = subcarrier0(radio) + 0.5 * (double)(A.N - 1) * radio->df_hz;
  A.t_off = (A.N % 2 == 0) ? 0.5 : 0.0;
  A.df = radio->df_hz;
  A.cm = 0.5 * (double)(radio->n_elem - 1);
  const bool m1 = radio->n_elem == 1;
  // links of many paths (on average at least 512): workgroups of eight
  // waves sharing the S/D operand; otherwise one wave per 64 paths
  const bool wg = (int64_t)paths->n_paths >= 512 * (int64_t)std::max(1, paths->n_links);
  constexpr int nwa = 8;
  hipLaunchKernelGGL(adj_wave_scan_kernel, dim3(1), dim3(1024), 0, s, paths->link_off,
                     paths->n_links,
                     m1 ? kM1Block : (wg ? kAdjPathsPerWave * nwa : kAdjPathsPerWave), wave_off);
  if ((st = check_launch(fn)) != RTC_OK) return st;
  // partial dL/dg rows the launch writes (every one, surplus ones as zeros)
  int64_t part_rows = A.max_waves;
  if (m1) {
    // one workgroup per (link, kM1Block paths): at most n_paths / kM1Block +
    // n_links of them, within the max_waves partial rows
    const int64_t blocks = (int64_t)paths->n_paths / kM1Block + paths->n_links + 1;
    part_rows = blocks;
    RTC_REQUIRE(blocks <= A.max_waves && blocks < (1ll << 31), RTC_ERR_RANGE,
                "%s: problem too large for one launch", fn);
    hipLaunchKernelGGL(cfr_adjoint_m1_kernel, dim3((unsigned)blocks), dim3(kM1Block), 0, s, A);
  } else if (wg) {
    // work units: sum over links of ceil(P_l / (64 nwa)), at most this many
    A.max_waves = (int64_t)paths->n_paths / (kAdjPathsPerWave * nwa) + paths->n_links + 1;
    part_rows = A.max_waves;
    // a multiple of eight workgroups (the kernel's XCD-aware order)
    const int64_t blocks = (A.max_waves + 7) / 8 * 8;
    RTC_REQUIRE(blocks < (1ll << 31), RTC_ERR_RANGE, "%s: problem too large for one launch", fn);
    hipLaunchKernelGGL(cfr_adjoint_kernel<nwa>, dim3((unsigned)blocks), dim3(nwa * 64), 0, s, A);
  } else {
    // a multiple of eight workgroups (the kernel's XCD-aware order)
    const int64_t blocks = ((A.max_waves + kAdjWaves - 1) / kAdjWaves + 7) / 8 * 8;
    RTC_REQUIRE(blocks < (1ll << 31), RTC_ERR_RANGE, "%s: problem too large for one launch", fn);
    hipLaunchKernelGGL(cfr_adjoint_wave_kernel, dim3((unsigned)blocks), dim3(kAdjWaves * 64), 0,
                       s, A);
  }
  if ((st = check_launch(fn)) != RTC_OK) return st;
  if (dLdg) {
    // dL/dg_m = sum over waves (links in order) of the partials, fixed order, FP64
    const int K = 2 * A.M;
    double* tmp = A.g_part + A.max_waves * K;
    double* red = tmp + reduce_tmp_doubles(A.max_waves, K);
    if ((st = reduce_all(A.g_part, part_rows, K, tmp, red, s, fn)) != RTC_OK) return st;
    hipLaunchKernelGGL(to_c64_kernel, dim3((A.M + 63) / 64), dim3(64), 0, s, red, A.M,
                       reinterpret_cast<float2*>(dLdg));
    return check_launch(fn);
  }
  return RTC_OK;
}
