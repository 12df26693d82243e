// The calibration step's channel part fused per link: CFR synthesis, the
// workload loss with its gradient dL/dH, and the CFR adjoint, with H and
// dL/dH kept on chip (registers and LDS) from the product that forms them to
// the product that consumes them.
//
// One workgroup owns one link: NW = N/128 waves (eight at 1,024
// subcarriers, two per SIMD), wave w the 64 subcarrier pairs q in
// [64 w, 64 w + 64) of all M <= 32 elements (the conjugate pairs of cfr.hip:
// pair q joins n_hi = N/2 + q and n_lo = N/2 - 1 - q).  At two waves per
// SIMD one wave's vector work overlaps the other's matrix products and
// memory waits; a wave alone issues vector instructions at about two thirds
// of the SIMD's rate.
//
//  1. Forward product (Eq. cfr_cont at the discrete subcarriers of
//     Sec. II-A) with the MFMA operands swapped so the accumulators hold H
//     transposed: lane l%32 is the element m, the register is the pair.  This
//     is the layout the adjoint's product takes its dL/dH operand in, so no
//     transpose is needed between them.  The path operand A'[i, m] =
//     a_i g_m exp(j psi_i (m - c)) exp(-j 2 pi f_ref tau_i) is the same for
//     every wave: the workgroup forms it once per stage of 64 paths, split
//     into FP16 parts and stored in LDS in the MFMA's B-operand layout, and
//     each wave reads it back with four 16-byte loads per 16 paths.  Each wave
//     forms its own subcarrier operand exp(-j 2 pi t_q df tau_i) directly
//     from FP64-reduced phases (no recurrence).
//  2. Loss (coherent + power-delay-profile NMSE, normalised by the target
//     statistics of the batch), per group of 8 element rows: the lanes of
//     those rows write H in pair order to LDS, each wave takes rows of the
//     group through the one-wave FFT in place in the row's own slot (tap
//     domain, PDP, gradient, inverse FFT; targets H* and p* read from HBM,
//     H - H* parked in LDS), and writes dL/dH back to the slot; the owning
//     lanes read their pairs back as S = dH[n_hi] + dH[n_lo] and
//     D = dH[n_hi] - dH[n_lo], into the registers H occupied.
//  3. Adjoint product G[m, p] = sum_q (S Re u_p(t_q) - j D Im u_p(t_q)) for
//     each 32-path tile of the link, each wave over its own pairs: dL/dH is
//     split into FP16 parts once (one power-of-two scale for the link, from
//     its largest value), so per tile only the exponentials are generated;
//     the waves' partial G meet in LDS and each wave applies the path phase,
//     array phases and gains to four element rows: dL/da per path, dL/dg
//     summed over the link's tiles in order (FP64), one row per link.
// The loss sums {sum|H-H*|^2, sum(p-p*)^2} of each (link, wave) and the
// per-link dL/dg rows are reduced across the batch in a fixed order.
#include <cmath>

#include "api_common.h"
#include "cfr_common.h"
#include "dev_common.h"
#include "fft_wave.h"
#include "split_f16.h"

namespace rtc {

template <int LOGN>
struct Fz {
  static constexpr int N = 1 << LOGN;
  static constexpr int Q = N / 2;         // subcarrier pairs
  static constexpr int TPW = 2;           // 32-pair tiles per wave
  static constexpr int NW = Q / (32 * TPW);
  static constexpr int NCH = 2 * TPW;     // 16-pair chunks per wave
  static constexpr int GROUP = 8;         // element rows per loss group
  static constexpr int RPW = GROUP / NW;  // rows per wave per group
  static_assert(NW >= 1 && NW <= 8 && GROUP % NW == 0, "1 to 8 waves");
  // LDS in two arrays, so that the compiler can tell the direct-to-LDS
  // target loads (second array) from the row slots' traffic (first array)
  // and does not wait for those loads at every slot access.
  // loss: eight row slots of Q + Q/16 + 16 float4 (a slot is also its row's
  // FFT buffer, N + N/16 float2 with the bank shift of row_slot0) in the
  // first array; each wave's N targets (then H - H*) in the second
  static constexpr int LDQ = Q + Q / 16 + 16;
  static constexpr int ROW_BYTES = (GROUP * LDQ + 16) * 16;
  static constexpr int DIFF_BYTES = NW * N * 8;
  // adjoint: each wave's partial G of a tile, two tiles in flight (tile T
  // in array T % 2)
  static constexpr int GBUF_FLOATS = 64 * 32;
  static constexpr int GBUF_HALF = NW * GBUF_FLOATS * 4;
  // and after them the waves' shares of the tile's dL/da
  static constexpr int DA_BYTES = NW * 64 * 8;
  // forward: one stage of NW x 8 paths, the path operand in FP16 parts
  // and the delays (path_stage_store), in the first array
  static constexpr int ST_PATHS = path_stage_paths(NW * 64);
  static constexpr int ST_OPND_BYTES = path_stage_opnd_bytes(NW * 64);
  static constexpr int ST_BYTES = path_stage_bytes(NW * 64);
  static constexpr int cmax(int a, int b) { return a > b ? a : b; }
  static constexpr int SMEM_A = cmax(cmax(ROW_BYTES, GBUF_HALF + DA_BYTES), ST_BYTES);
  static constexpr int SMEM_B = cmax(DIFF_BYTES, GBUF_HALF + DA_BYTES);
  // with X* targets the loss takes 16 rows per group, eight slots in each
  // array (the second holds no targets then)
  static constexpr int SMEM_B16 = cmax(SMEM_B, ROW_BYTES);
};

struct FusedArgs {
  int n_links, M;
  const int64_t* link_off;
  const float2* a;
  const float* psi;
  const double* tau;
  const float2* g;
  const float2* Ht;  // targets c64 [L, M, N], or null with Xt
  const float* Pt;   // target PDP f32 [L, M, N] (natural tap order), or null with Xt
  const float2* Xt;  // or the targets' transforms X* c64 [L, M, N] (natural tap order)
  const double* Z;   // {sum |H*|^2, sum (p*)^2} over the batch
  float w_coh, w_pdp;
  double fref, t_off, df, cm;  // grid midpoint, t of pair 0, spacing, (M-1)/2
  double* row_out;  // [L*NW][2] loss sums per link and wave
  float2* dLda;     // [P] or null
  double* g_part;   // [L][M][2] per-link dL/dg, or null
};

// Start of element row rl's pair slots in the LDS row buffer: rows LDQ
// slots apart plus a shift that puts the 8 rows and the two lane halves of a
// register's writes on distinct banks.
RTC_DEV int row_slot0(int rl, int ldq) { return rl * ldq + (rl & 3) + 8 * (rl >> 2); }

// A row's target CFR H* straight from HBM into the wave's LDS buffer dbuf
// (natural order, dbuf[n] = H*[n]), without passing through registers: N/128
// direct-to-LDS loads of 16 bytes per lane, lane l of load i taking
// H*[128 i + 2 l] and H*[128 i + 2 l + 1].  Issued a row ahead; the row's
// first read of dbuf waits for them (the compiler counts the loads).
template <int LOGN>
__device__ __forceinline__ void prefetch_row_targets(const float2* Ht, int64_t ridx, float2* dbuf,
                                                     int lane) {
  constexpr int N = 1 << LOGN;
  const float2* src = Ht + ridx * N + 2 * lane;
#pragma unroll
  for (int i = 0; i < N / 128; ++i)
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(src + 128 * i),
                                     (__attribute__((address_space(3))) void*)(dbuf + 128 * i), 16,
                                     0, 0);
}

template <int LOGN>
struct RowTargets {
  static constexpr int NP = fft_npass(LOGN);
  static constexpr int RZ = fft_radix(LOGN, NP - 1);
  static constexpr int JZ = fft_bpl(1 << LOGN, RZ);
};

// The row's target PDP, loaded into registers when the row starts (it is
// needed only after the first transform)
template <int LOGN>
__device__ __forceinline__ void load_row_pdp(const float* Pt, int64_t ridx, int lane,
                                             float (&p)[RowTargets<LOGN>::JZ][RowTargets<LOGN>::RZ]) {
  constexpr int N = 1 << LOGN;
  constexpr int BZ = N / RowTargets<LOGN>::RZ;
  const float* ps = Pt + ridx * N;
#pragma unroll
  for (int i = 0; i < RowTargets<LOGN>::JZ; ++i) {
    const int jj = lane + 64 * i;
#pragma unroll
    for (int r = 0; r < RowTargets<LOGN>::RZ; ++r)
      p[i][r] = (BZ % 64 == 0 || jj < BZ) ? ps[jj + r * BZ] : 0.0f;
  }
}

// Loss of one CFR row whose pair accumulators sit in LDS, in place.  Slot q
// of `row` holds {Re X, Im X, Re Y, Im Y} of pair q (unscaled by `us`), so
// H[N/2 + q] = X + jY and H[N/2 - 1 - q] = X - jY.  One wave; the slot is
// also the FFT's buffer (each pass reads all its values before it writes,
// and LDS operations of one wave complete in order, so one buffer serves
// in place), `dbuf` (N values) comes in holding the row's H* (natural
// order, prefetch_row_targets) and holds H - H* across the transforms, `tw`
// is the twiddle table.  The
// row's two loss sums, sum |H - H*|^2 and sum (p - p*)^2, are added to
// `sums` (per lane, FP64; the normalisers come from the targets'
// statistics).  On return slot q holds {dL/dH[N/2 + q], dL/dH[N/2 - 1 - q]}
// (the lanes that own the pair form S and D from them).  The loss
// arithmetic is that of cfr_loss_wave_kernel with a precomputed target PDP
// (loss.hip).  Lanes j >= N/16 (N < 1,024) hold no
// elements and touch neither the slot nor dbuf.  Element n = j + BA r of the first FFT
// pass (lane j < BA) is pair j + BA (r - 8) (upper half, r >= 8) or
// BA - 1 - j + BA (7 - r) (lower half) -- the mirror n -> N - 1 - n is lane
// BA - 1 - j, register 15 - r.
template <int LOGN, bool CIR>
__device__ __forceinline__ void fused_loss_row(float4* row, const float* Pt, int64_t ridx,
                                               const float2* tgt, int64_t next_ridx, float us,
                                               float2* dbuf, const float2* tw, float gc,
                                               float gp, double (&sums)[2], int lane_in) {
  // the FFT twiddles depend on the lane and the pass only; an opaque lane
  // index keeps the compiler from holding them across rows (and the group
  // loop), where they would take registers the loop needs
  int lane = lane_in;
  asm volatile("" : "+v"(lane));
  constexpr int N = 1 << LOGN;
  constexpr int NP = fft_npass(LOGN);
  constexpr int RA = fft_radix(LOGN, 0), RZ = fft_radix(LOGN, NP - 1);
  constexpr int JA = fft_bpl(N, RA), JZ = fft_bpl(N, RZ);
  constexpr int BA = N / RA, BZ = N / RZ;
  static_assert(RA == 16 && JA == 1 && BA <= 64, "first pass: one radix-16 butterfly per lane");
  const float invN = 1.0f / (float)N;
  const int j = lane;
  const bool act = BA == 64 || j < BA;
  float2* fb = reinterpret_cast<float2*>(row);
  if constexpr (CIR) {
    // targets as X*: the coherent sum by Parseval, sum |H - H*|^2 =
    // sum |X - X*|^2 / N, and dL/dH = IDFT(gc/N (X - X*) + gp d X) (the
    // unnormalised inverse of the forward transform returns N H).  The
    // row's X* loads into registers now and is first used after the forward
    // transform; plain loads, unlike direct-to-LDS ones, pass the group
    // barriers without a wait.
    float2 xs[JZ][RZ];
    {
      const float2* xr = tgt + ridx * N;
#pragma unroll
      for (int i = 0; i < JZ; ++i) {
        const int jj = lane + 64 * i;
#pragma unroll
        for (int r = 0; r < RZ; ++r)
          xs[i][r] = (BZ % 64 == 0 || jj < BZ) ? xr[jj + r * BZ] : make_float2(0.0f, 0.0f);
      }
    }
    float2 vh[1][16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      float2 h = make_float2(0.0f, 0.0f);
      if (act) {
        if (r >= 8) {
          const float4 v = row[j + BA * (r - 8)];
          h = make_float2((v.x - v.w) * us, (v.y + v.z) * us);  // X + jY
        } else {
          const float4 v = row[BA - 1 - j + BA * (7 - r)];
          h = make_float2((v.x + v.w) * us, (v.y - v.z) * us);  // X - jY
        }
      }
      vh[0][r] = h;
    }
    float2 xh[JZ][RZ];
    WaveSync::sync();  // the row's reads are done before the transform writes
    fft_full<LOGN, +1, +1, WaveSync, 64, true>(vh, xh, fb, fb, lane, tw);
    const float gcn = gc * invN;
    float ec = 0.0f, ep = 0.0f;
#pragma unroll
    for (int i = 0; i < JZ; ++i) {
      const int jj = lane + 64 * i;
      if (BZ % 64 == 0 || jj < BZ) {
#pragma unroll
        for (int r = 0; r < RZ; ++r) {
          const float2 dx = csub(xh[i][r], xs[i][r]);
          ec += cabs2(dx);
          const float d = cabs2(xh[i][r]) * invN - cabs2(xs[i][r]) * invN;  // p - p*
          ep += d * d;
          xh[i][r] = cadd(cscale(dx, gcn), cscale(xh[i][r], gp * d));
        }
      }
    }
    sums[0] += (double)ec * (double)invN;
    sums[1] += (double)ep;
    float2 G[1][16];
    fft_full<LOGN, -1, -1, WaveSync, 64, true>(xh, G, fb, fb, lane, tw);
    if (act) {
      float2* half_slots = reinterpret_cast<float2*>(row);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        if (r >= 8)
          half_slots[2 * (j + BA * (r - 8))] = G[0][r];
        else
          half_slots[2 * (BA - 1 - j + BA * (7 - r)) + 1] = G[0][r];
      }
    }
    return;
  }
  float tp[JZ][RZ];
  load_row_pdp<LOGN>(Pt, ridx, lane, tp);
  float2 vh[1][16];
  float ec = 0.0f;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    float2 h = make_float2(0.0f, 0.0f);
    if (act) {
      if (r >= 8) {
        const float4 v = row[j + BA * (r - 8)];
        h = make_float2((v.x - v.w) * us, (v.y + v.z) * us);  // X + jY
      } else {
        const float4 v = row[BA - 1 - j + BA * (7 - r)];
        h = make_float2((v.x + v.w) * us, (v.y - v.z) * us);  // X - jY
      }
    }
    vh[0][r] = h;
    const float2 df = csub(h, act ? dbuf[r * BA + j] : make_float2(0.0f, 0.0f));
    ec += cabs2(df);
    if (act) dbuf[r * BA + j] = df;
  }
  float2 xh[JZ][RZ];
  WaveSync::sync();  // the row's reads are done before the transform writes
  fft_full<LOGN, +1, +1, WaveSync, 64, true>(vh, xh, fb, fb, lane, tw);
  float ep = 0.0f;
#pragma unroll
  for (int i = 0; i < JZ; ++i) {
    const int jj = lane + 64 * i;
    if (BZ % 64 == 0 || jj < BZ) {
#pragma unroll
      for (int r = 0; r < RZ; ++r) {
        const float p = cabs2(xh[i][r]) * invN;
        const float d = p - tp[i][r];
        ep += d * d;
        xh[i][r] = cscale(xh[i][r], gp * d);  // gradient source
      }
    }
  }
  sums[0] += (double)ec;
  sums[1] += (double)ep;
  float2 G[1][16];
  fft_full<LOGN, -1, -1, WaveSync, 64, true>(xh, G, fb, fb, lane, tw);
  // dL/dH = gc (H - H*) + G, each element into its pair's slot: the upper
  // one (register r >= 8, pair j + BA (r - 8)) as the slot's first two
  // floats, the lower one (r < 8, pair BA - 1 - j + BA (7 - r)) as its last
  // two; the owners form S and D when they read the slots back
  if (act) {
    float2* half_slots = reinterpret_cast<float2*>(row);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float2 dh = cadd(cscale(dbuf[r * BA + j], gc), G[0][r]);
      if (r >= 8)
        half_slots[2 * (j + BA * (r - 8))] = dh;
      else
        half_slots[2 * (BA - 1 - j + BA * (7 - r)) + 1] = dh;
    }
  }
  // the buffer's last reads are done: the next row's targets go in
  if (next_ridx >= 0) prefetch_row_targets<LOGN>(tgt, next_ridx, dbuf, lane);
}

template <int LOGN, bool CIR>
__global__ void __launch_bounds__(Fz<LOGN>::NW * 64) cfr_fused_kernel(FusedArgs A) {
  using F = Fz<LOGN>;
  constexpr int N = F::N, NW = F::NW, TPW = F::TPW, NCH = F::NCH;
  constexpr int NT = NW * 64;
  __shared__ __align__(16) char smem[F::SMEM_A];
  // rows per loss group: 16 (eight slots in each LDS array) with X* targets
  // (half the groups, so half the group barriers, and twice the lanes in
  // each slot write and read-back), else 8 (the second array holds the
  // rows' targets)
  constexpr int GRP = CIR ? 16 : F::GROUP;
  constexpr int RPW = GRP / NW;  // rows per wave per group
  __shared__ __align__(16) char smem_b[GRP == 16 ? F::SMEM_B16 : F::SMEM_B];
  __shared__ float wmax[NW];
  __shared__ float2 twtab[fft_tw_len<LOGN>()];  // FFT twiddle rows (fft_tw_fill)
  float4* rowbuf = reinterpret_cast<float4*>(smem);
  auto gbuf = [&](int b) { return reinterpret_cast<float*>(b ? smem_b : smem); };
  // the waves' shares of a tile's dL/da (adjoint), after the partial G of
  // the same array
  auto dabuf = [&](int b) {
    return reinterpret_cast<float2*>((b ? smem_b : smem) + F::GBUF_HALF);
  };

  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int half = lane >> 5;
  const int col = lane & 31;
  const int64_t l = blockIdx.x;
  const int M = A.M;
  const int64_t off0 = A.link_off[l];
  const int64_t off1 = A.link_off[l + 1];
  const int q_base = wv * 32 * TPW;
  fft_tw_fill<LOGN>(twtab, tw_rows<LOGN>(), threadIdx.x, NT);  // read after the barriers below
  // loss rows of this wave: k -> element row GRP (k / RPW) + wv + NW (k % RPW);
  // the rows that exist (< M) are a prefix.  The first one's targets load
  // into the wave's LDS buffer while the forward product runs (the buffer
  // lies outside the forward's stage area).
  auto row_of = [&](int k) { return GRP * (k / RPW) + wv + NW * (k % RPW); };
  // slot of row rl of a group: the first eight in the first array, the rest
  // in the second
  auto slot = [&](int rl) {
    return rl < 8 ? rowbuf + row_slot0(rl, F::LDQ)
                  : reinterpret_cast<float4*>(smem_b) + row_slot0(rl - 8, F::LDQ);
  };
  float2* dbuf = reinterpret_cast<float2*>(smem_b) + wv * N;
  const float2* tgt = CIR ? A.Xt : A.Ht;
  if (!CIR && row_of(0) < M) prefetch_row_targets<LOGN>(tgt, l * M + row_of(0), dbuf, lane);

  // ------------------------------------------------------------ 1. forward
  // lane: element m = col (B operand A'), pair column col of each tile (A
  // operand u); acc[t][*] register r holds pair q_base + 32 t + 8 (r/4) +
  // 4 half + r%4 of element col: X = (acc0, acc1), Y = (acc2, acc3)
  floatx16 acc[TPW][4];
  float unscale = 1.0f;  // the forward operand's link scale, removed in the loss
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[t][k] = floatx16{0};
  {
    // the path operand: formed by the workgroup per stage (path_stage_store)
    const int m = col;
    const float2 g_row = m < M ? A.g[m] : make_float2(0.0f, 0.0f);
    const double mc_cyc = ((double)m - A.cm) * kInv2Pi;
    const int sx = 14 - cfr_link_scale_exp(A.a, off0, off1, g_row, lane);
    const float2 gm = make_float2(ldexpf(g_row.x, sx), ldexpf(g_row.y, sx));
    unsigned* opnd = reinterpret_cast<unsigned*>(smem);
    double* tau_s = reinterpret_cast<double*>(smem + F::ST_OPND_BYTES);
    // the wave's subcarrier phase slope per tile: t_q df for its lane's pair
    double tq[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) tq[t] = ((double)(q_base + 32 * t + col) + A.t_off) * A.df;
    PathFetch pf;
    if (off0 < off1) path_fetch(A.a, A.psi, A.tau, off0, off1, NT, pf);
    for (int64_t s0 = off0; s0 < off1; s0 += F::ST_PATHS) {
      __syncthreads();  // the previous stage's operands are consumed
      path_stage_store(pf, s0, off1, NT, A.fref, mc_cyc, gm, col, opnd, tau_s);
      __syncthreads();
      // the next stage's path data load while this stage's products run
      if (s0 + F::ST_PATHS < off1) path_fetch(A.a, A.psi, A.tau, s0 + F::ST_PATHS, off1, NT, pf);
      const int nch = (int)min((int64_t)(F::ST_PATHS / 16), (off1 - s0 + 15) >> 4);
      for (int c = 0; c < nch; ++c) {
        Split2 AR, AI;
        path_stage_read(opnd, c, lane, AR, AI);
        const double* tp = tau_s + 16 * c + 8 * half;
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
          float ur[8], ui[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const float2 u = expm2pi_f64_hw(tq[t] * tp[j]);
            ur[j] = u.x;
            ui[j] = u.y;
          }
          const Split2 UR = split2(ur), UI = split2(ui);
          acc[t][0] = mac3(UR, AR, acc[t][0]);
          acc[t][1] = mac3(UR, AI, acc[t][1]);
          acc[t][2] = mac3(UI, AR, acc[t][2]);
          acc[t][3] = mac3(UI, AI, acc[t][3]);
        }
      }
    }
    unscale = ldexpf(1.0f, -sx);
  }

  // --------------------------------------------------------------- 2. loss
  const float gc = (float)(2.0 * (double)A.w_coh / A.Z[0]);
  const float gp = (float)(4.0 * (double)A.w_pdp / (A.Z[1] * (double)N));
  const int n_groups = (M + GRP - 1) / GRP;
  double sums[2] = {0.0, 0.0};
  for (int grp = 0; grp < n_groups; ++grp) {
    __syncthreads();  // the forward's stage buffer, or the previous group's read-back, is done
    if (col / GRP == grp) {
      float4* row = slot(col % GRP);
#pragma unroll
      for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int q = q_base + 32 * t + 8 * (r >> 2) + 4 * half + (r & 3);
          row[q] = make_float4(acc[t][0][r], acc[t][1][r], acc[t][2][r], acc[t][3][r]);
        }
    }
    __syncthreads();
#pragma unroll 1
    for (int i = 0; i < RPW; ++i) {
      const int k = grp * RPW + i;
      const int mrow = row_of(k);
      if (mrow < M) {
        const int mnext = row_of(k + 1);
        fused_loss_row<LOGN, CIR>(slot(mrow % GRP), A.Pt, l * M + mrow, tgt,
                                  mnext < M ? l * M + mnext : -1, unscale, dbuf, twtab, gc, gp,
                                  sums, lane);
      }
    }
    __syncthreads();
    if (col / GRP == grp) {
      // slot q: {dL/dH[N/2 + q], dL/dH[N/2 - 1 - q]} -> S = hi + lo,
      // D = hi - lo; rows m >= M hold X = Y = 0 (zero gains), read back as
      // zero operands
      const float4* row = slot(col % GRP);
#pragma unroll
      for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int q = q_base + 32 * t + 8 * (r >> 2) + 4 * half + (r & 3);
          const float4 v = row[q];
          acc[t][0][r] = v.x + v.z;  // Re S
          acc[t][1][r] = v.y + v.w;  // Im S
          acc[t][2][r] = v.z - v.x;  // -Re D
          acc[t][3][r] = v.y - v.w;  // Im D
        }
    }
  }
  // the wave's loss sums over its rows: lanes in a fixed butterfly order
#pragma unroll
  for (int k = 0; k < 2; ++k) sums[k] = wave_sum_f64(sums[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 2; ++k) A.row_out[(l * NW + wv) * 2 + k] = sums[k];
  }

  // ------------------------------------------------------------ 3. adjoint
  // one power-of-two scale for the link's dL/dH operand: its largest value
  // below 2^14 (exact both ways; values down to 2^-28 of it keep all bits)
  float mx = 0.0f;
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int r = 0; r < 16; ++r) mx = fmaxf(mx, fabsf(acc[t][k][r]));
  mx = wave_max_f32(mx);
  if (lane == 0) wmax[wv] = mx;
  __syncthreads();
  mx = wmax[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) mx = fmaxf(mx, wmax[w]);
  int sxa = 0;
  if (mx > 0.0f) {
    int e = 0;
    frexpf(mx, &e);
    sxa = 14 - min(max(e, -100), 100);
  }
  const float sca = ldexpf(1.0f, sxa);
  const float unsca = ldexpf(1.0f, -sxa);
  // chunk c (16 pairs): tile c/2, registers 8 (c%2) .. +7; k slot (half, j)
  // is pair q_base + 16 c + 8 (j/4) + 4 half + j%4
  Split2 SR[NCH], SI[NCH], NDR[NCH], DI[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
    float sr[8], si[8], nd[8], di[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int r = 8 * (c & 1) + j;
      sr[j] = acc[c >> 1][0][r] * sca;
      si[j] = acc[c >> 1][1][r] * sca;
      nd[j] = acc[c >> 1][2][r] * sca;
      di[j] = acc[c >> 1][3][r] * sca;
    }
    SR[c] = split2(sr);
    SI[c] = split2(si);
    NDR[c] = split2(nd);
    DI[c] = split2(di);
    // packed here: the FP32 values die before the adjoint loop starts
    asm volatile("" : "+v"(SR[c].h), "+v"(SR[c].l), "+v"(SI[c].h), "+v"(SI[c].l));
    asm volatile("" : "+v"(NDR[c].h), "+v"(NDR[c].l), "+v"(DI[c].h), "+v"(DI[c].l));
  }

  // The epilogue of a tile is split over the waves by element rows, RPL rows
  // per lane: with up to four waves, wave w takes the row groups g4 in
  // [G4W w, G4W (w + 1)) (rows 8 g4 + 4 half + 0..3, registers 4 g4 ..
  // 4 g4 + 3 of G, in the lane's own half); with eight, wave w takes rows
  // 8 (w/2) + 4 (w%2) + 0..3 (registers of the lanes of half w%2), two per
  // lane: rows 2 half, 2 half + 1 of the four.  Its dL/dg rows accumulate in
  // the lanes' registers (FP64, each lane its paths, tiles in order; the
  // half-wave's lanes are added at the end of the link); each half-wave's share of
  // dL/da goes to LDS and the wave that finishes the tile adds the shares in
  // order after the next barrier.
  constexpr int G4W = NW <= 4 ? 4 / NW : 1;
  constexpr int RPL = NW <= 4 ? 4 * G4W : 2;  // rows per lane
  auto ep_reg = [&](int i) {  // register of G (row within the 32-row block)
    return NW <= 4 ? 4 * (G4W * wv + i / 4) + i % 4 : 4 * (wv >> 1) + 2 * half + i;
  };
  auto ep_row = [&](int i) {  // element row
    return NW <= 4 ? 8 * (G4W * wv + i / 4) + 4 * half + i % 4
                   : 8 * (wv >> 1) + 4 * (wv & 1) + 2 * half + i;
  };
  const int ep_src = NW <= 4 ? lane : 32 * (wv & 1) + col;  // the lane holding the rows
  double dgw[RPL][2];
#pragma unroll
  for (int i = 0; i < RPL; ++i) dgw[i][0] = dgw[i][1] = 0.0;
  auto finish_da = [&](int T) {
    // dL/da of tile T: the shares of the waves' half-waves, in order
    const float2* db = dabuf(T & 1);
    const int64_t p = off0 + 32 * (int64_t)T + col;
    if (half == 0 && p < off1 && A.dLda) {
      float2 d = cadd(db[col], db[32 + col]);
#pragma unroll
      for (int w = 1; w < NW; ++w) d = cadd(d, cadd(db[w * 64 + col], db[w * 64 + 32 + col]));
      A.dLda[p] = d;
    }
  };
  // the gains of the lane's epilogue rows (zero for rows >= M), loaded once
  float2 gep[RPL];
#pragma unroll
  for (int i = 0; i < RPL; ++i)
    gep[i] = ep_row(i) < M ? A.g[ep_row(i)] : make_float2(0.0f, 0.0f);
  // One tile's products: the wave's partial G~ of the tile's 32 paths (tau:
  // the lane's path delay).  G~ = X - jY: Re G~ += S_re Re u + D_im Im u,
  // Im G~ += S_im Re u - D_re Im u
  auto tile_products = [&](double tau, floatx16& gre, floatx16& gim) {
    const float2 v1 = expm2pi_f64_hw(A.df * tau);
    const float2 v8 = expm2pi_f64_hw(8.0 * A.df * tau);
    const float2 v16 = expm2pi_f64_hw(16.0 * A.df * tau);
    gre = floatx16{0};
    gim = floatx16{0};
    float2 e0 = make_float2(1.0f, 0.0f);
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      // u_p at the lane's first pair of the chunk: FP64 anchor every 64 pairs
      if ((c & 3) == 0)
        e0 = expm2pi_f64_hw(((double)(q_base + 16 * c + 4 * half) + A.t_off) * A.df * tau);
      else
        e0 = cmul(e0, v16);
      float ur[8], ui[8];
      float2 e = e0, f = cmul(e0, v8);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (j > 0) {
          e = cmul(e, v1);
          f = cmul(f, v1);
        }
        ur[j] = e.x;
        ui[j] = e.y;
        ur[j + 4] = f.x;
        ui[j + 4] = f.y;
      }
      const Split2 UR = split2(ur), UI = split2(ui);
      gre = mac3(SR[c], UR, gre);
      gim = mac3(SI[c], UR, gim);
      gre = mac3(DI[c], UI, gre);
      gim = mac3(NDR[c], UI, gim);
    }
  };
  // the waves' partial sums over their pairs meet in LDS (two buffers,
  // alternating by tile; register r at float r*64 + lane, conflict-free)
  auto tile_store = [&](int T, const floatx16& gre, const floatx16& gim) {
    float* gb = gbuf(T & 1) + wv * F::GBUF_FLOATS;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      gb[r * 64 + lane] = gre[r];
      gb[(16 + r) * 64 + lane] = gim[r];
    }
  };
  // The epilogue of tile T, its G~ complete in gbuf(T & 1): this wave's rows
  // of the tile, its half-wave's share of dL/da into dabuf(T & 1) (added in
  // order by the wave that finishes the tile) and dL/dg into dgw.  ai,
  // psi_cyc, tau: the lane's path of the tile (zero past the link).
  auto tile_epilogue = [&](int T, float2 ai, double psi_cyc, double tau) {
    const float* g0 = gbuf(T & 1);
    const float2 cc = cconj(expm2pi_f64_hw(A.fref * tau));  // conj(c_p)
    const float2 step = expm2pi_f64_hw(psi_cyc);
    float2 da = make_float2(0.0f, 0.0f);
    float2 ph = make_float2(1.0f, 0.0f);
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int r = ep_reg(i);
      const int mrow = ep_row(i);
      // exp(-j psi (m - c)) at the first row of each run of four, then by step
      if (i % 4 == 0)
        ph = expm2pi_f64_hw(psi_cyc * ((double)mrow - A.cm));
      else
        ph = cmul(ph, step);
      float gr = 0.0f, gi = 0.0f;
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        gr += g0[w * F::GBUF_FLOATS + r * 64 + ep_src];
        gi += g0[w * F::GBUF_FLOATS + (16 + r) * 64 + ep_src];
      }
      const float2 G = cmul(cc, make_float2(gr * unsca, gi * unsca));
      const float2 Gph = cmul(G, ph);
      da = cadd(da, cmulc(gep[i], Gph));
      // dL/dg: the lane's path, summed over the tiles in the lane (FP64),
      // over the half's 32 lanes once at the end of the link
      const float2 tg = cmulc(ai, Gph);
      dgw[i][0] += (double)tg.x;
      dgw[i][1] += (double)tg.y;
    }
    dabuf(T & 1)[wv * 64 + lane] = da;
  };
  // the lane's path data of tile T, loaded without a branch (index clamped
  // to the link, values zeroed past it)
  auto tile_path = [&](int T, float2& ai, double& psi_cyc, double& tau) {
    const int64_t p = off0 + 32 * (int64_t)T + col;
    const bool ok = p < off1;
    const int64_t pc = ok ? p : off1 - 1;
    const float2 a = A.a[pc];
    const float ps = A.psi[pc];
    const double tv = A.tau[pc];
    ai = ok ? a : make_float2(0.0f, 0.0f);
    psi_cyc = (double)(ok ? ps : 0.0f) * kInv2Pi;
    tau = ok ? tv : 0.0;
  };
  // Software-pipelined by one tile: tile T's products are issued in the same
  // straight-line code as tile T - 1's epilogue (VALU and LDS work), so the
  // matrix cores and the vector units overlap; one barrier per tile.
  const int n_tiles = (int)((off1 - off0 + 31) >> 5);
  if (n_tiles > 0) {
    float2 ai_c;
    double psi_c, tau_c;
    tile_path(0, ai_c, psi_c, tau_c);
    {
      floatx16 gre, gim;
      tile_products(tau_c, gre, gim);
      tile_store(0, gre, gim);
    }
    __syncthreads();
    for (int T = 1; T < n_tiles; ++T) {
      float2 ai_t;
      double psi_t, tau_t;
      tile_path(T, ai_t, psi_t, tau_t);
      floatx16 gre, gim;
      tile_products(tau_t, gre, gim);
      tile_epilogue(T - 1, ai_c, psi_c, tau_c);
      tile_store(T, gre, gim);
      __syncthreads();
      if (wv == (T - 1) % NW) finish_da(T - 1);
      ai_c = ai_t;
      psi_c = psi_t;
      tau_c = tau_t;
    }
    tile_epilogue(n_tiles - 1, ai_c, psi_c, tau_c);
  }
  __syncthreads();  // the last tile's shares are in LDS; every epilogue is done
  if (n_tiles > 0 && wv == (n_tiles - 1) % NW) finish_da(n_tiles - 1);
  if (A.g_part) {
    // this wave's dL/dg rows of the link (disjoint across waves and halves):
    // the lanes' sums over their paths, added over the half (fixed butterfly)
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      dgw[i][0] = half_sum_f64(dgw[i][0]);
      dgw[i][1] = half_sum_f64(dgw[i][1]);
    }
    if (col == 0) {
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int mrow = ep_row(i);
        if (mrow < M) {
          A.g_part[(l * M + mrow) * 2 + 0] = dgw[i][0];
          A.g_part[(l * M + mrow) * 2 + 1] = dgw[i][1];
        }
      }
    }
  }
}

__global__ void fused_finish_kernel(const double* sums, const double* Z, float w_coh,
                                    float w_pdp, double* loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double coh = sums[0] / Z[0];
  const double pdp = sums[1] / Z[1];
  loss[0] = (double)w_coh * coh + (double)w_pdp * pdp;
  loss[1] = coh;
  loss[2] = pdp;
}

__global__ void fused_to_c64_kernel(const double* v, int M, float2* out) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < M) out[m] = make_float2((float)v[2 * m], (float)v[2 * m + 1]);
}

bool fused_supported(const rtc_radio* r) {
  return r->n_elem >= 1 && r->n_elem <= 32 &&
         (r->n_sc == 256 || r->n_sc == 512 || r->n_sc == 1024);
}

// waves per workgroup of the fused kernel for n_sc subcarriers
static int fused_waves(int n_sc) { return n_sc / 128; }

// Workspace: loss sums [L*NW][2] | their reduction tmp | sums [2] |
// per-link dL/dg [L][M][2] | its reduction tmp | reduced [M][2] (doubles).
size_t ws_cfr_loss_adjoint(const rtc_radio* r, int32_t n_links) {
  if (!fused_supported(r)) return 0;
  const int64_t L = n_links > 0 ? n_links : 1;
  const int64_t R = L * fused_waves(r->n_sc);
  const int K = 2 * r->n_elem;
  return (size_t)(R * 2 + reduce_tmp_doubles(R, 2) + 2 + L * K + reduce_tmp_doubles(L, K) + K) *
         sizeof(double);
}

}  // namespace rtc

using namespace rtc;

// The fused pass with the targets as H* and p* (Xt null) or as X* (Ht and
// Pt null); the arguments are checked by the entry points below.
static rtc_status fused_run(const char* fn, const rtc_radio* radio, const rtc_paths* paths,
                            const void* a, const float* psi, const void* g, const void* H_tgt,
                            const float* p_tgt, const void* X_tgt, const double* tgt_stats,
                            float w_coh, float w_pdp, double* loss, void* dLda, void* dLdg,
                            void* ws, size_t ws_bytes, void* stream) {
  rtc_status st;
  if ((st = check_radio(radio, fn)) != RTC_OK) return st;
  if ((st = check_paths(paths, fn, false)) != RTC_OK) return st;
  RTC_REQUIRE(fused_supported(radio), RTC_ERR_UNSUPPORTED,
              "%s: needs 1 <= n_elem <= 32 and n_sc of 256, 512 or 1024 (got %d, %d); use "
              "rtc_cfr, rtc_cfr_loss and rtc_cfr_adjoint",
              fn, radio->n_elem, radio->n_sc);
  RTC_REQUIRE(paths->n_links >= 1, RTC_ERR_SHAPE, "%s: n_links must be >= 1", fn);
  RTC_REQUIRE(g != nullptr, RTC_ERR_INVALID_ARG, "%s: g is NULL", fn);
  RTC_REQUIRE((a != nullptr && psi != nullptr) || paths->n_paths == 0, RTC_ERR_INVALID_ARG,
              "%s: a and psi are required", fn);
  RTC_REQUIRE(((H_tgt && p_tgt) || X_tgt) && tgt_stats && loss, RTC_ERR_INVALID_ARG,
              "%s: the targets, tgt_stats and loss are required", fn);
  const size_t need = ws_cfr_loss_adjoint(radio, paths->n_links);
  RTC_REQUIRE(ws != nullptr && ws_bytes >= need, RTC_ERR_WORKSPACE,
              "%s: workspace of %zu bytes required", fn, need);
  hipStream_t s = as_stream(stream);
  const int64_t L = paths->n_links;
  const int M = radio->n_elem, N = radio->n_sc;
  const int64_t R = L * fused_waves(N);
  const int K = 2 * M;
  double* rows = reinterpret_cast<double*>(ws);
  double* rtmp = rows + R * 2;
  double* sums = rtmp + reduce_tmp_doubles(R, 2);
  double* gpart = sums + 2;
  double* gtmp = gpart + L * K;
  double* gred = gtmp + reduce_tmp_doubles(L, K);

  FusedArgs A;
  A.n_links = paths->n_links;
  A.M = M;
  A.link_off = paths->link_off;
  A.a = reinterpret_cast<const float2*>(a);
  A.psi = psi;
  A.tau = paths->tau;
  A.g = reinterpret_cast<const float2*>(g);
  A.Ht = reinterpret_cast<const float2*>(H_tgt);
  A.Pt = p_tgt;
  A.Xt = reinterpret_cast<const float2*>(X_tgt);
  A.Z = tgt_stats;
  A.w_coh = w_coh;
  A.w_pdp = w_pdp;
  const double f0 = radio->fc_hz - (double)(N / 2) * radio->df_hz;
  A.fref = f0 + 0.5 * (double)(N - 1) * radio->df_hz;
  A.t_off = 0.5;  // N even
  A.df = radio->df_hz;
  A.cm = 0.5 * (double)(M - 1);
  A.row_out = rows;
  A.dLda = reinterpret_cast<float2*>(dLda);
  A.g_part = dLdg ? gpart : nullptr;
  const bool cir = X_tgt != nullptr;
#define RTC_FUSED(LG)                                                                         \
  if (cir)                                                                                    \
    hipLaunchKernelGGL((cfr_fused_kernel<LG, true>), dim3((unsigned)L), dim3(Fz<LG>::NW * 64), \
                       0, s, A);                                                              \
  else                                                                                        \
    hipLaunchKernelGGL((cfr_fused_kernel<LG, false>), dim3((unsigned)L),                      \
                       dim3(Fz<LG>::NW * 64), 0, s, A);
  switch (N) {
    case 256:
      RTC_FUSED(8)
      break;
    case 512:
      RTC_FUSED(9)
      break;
    default:
      RTC_FUSED(10)
  }
#undef RTC_FUSED
  if ((st = check_launch(fn)) != RTC_OK) return st;
  if ((st = reduce_all(rows, R, 2, rtmp, sums, s, fn)) != RTC_OK) return st;
  hipLaunchKernelGGL(fused_finish_kernel, dim3(1), dim3(64), 0, s, sums, tgt_stats, w_coh, w_pdp,
                     loss);
  if ((st = check_launch(fn)) != RTC_OK) return st;
  if (dLdg) {
    if ((st = reduce_all(gpart, L, K, gtmp, gred, s, fn)) != RTC_OK) return st;
    hipLaunchKernelGGL(fused_to_c64_kernel, dim3((M + 63) / 64), dim3(64), 0, s, gred, M,
                       reinterpret_cast<float2*>(dLdg));
    return check_launch(fn);
  }
  return RTC_OK;
}

extern "C" rtc_status rtc_cfr_loss_adjoint(const rtc_radio* radio, const rtc_paths* paths,
                                           const void* a, const float* psi, const void* g,
                                           const void* H_tgt, const double* tgt_stats,
                                           const float* p_tgt, float w_coh, float w_pdp,
                                           double* loss, void* dLda, void* dLdg, void* ws,
                                           size_t ws_bytes, void* stream) {
  const char* fn = "rtc_cfr_loss_adjoint";
  RTC_REQUIRE(H_tgt && p_tgt, RTC_ERR_INVALID_ARG, "%s: H_tgt and p_tgt are required", fn);
  return fused_run(fn, radio, paths, a, psi, g, H_tgt, p_tgt, nullptr, tgt_stats, w_coh, w_pdp,
                   loss, dLda, dLdg, ws, ws_bytes, stream);
}

extern "C" rtc_status rtc_cfr_loss_adjoint_cir(const rtc_radio* radio, const rtc_paths* paths,
                                               const void* a, const float* psi, const void* g,
                                               const void* X_tgt, const double* tgt_stats,
                                               float w_coh, float w_pdp, double* loss,
                                               void* dLda, void* dLdg, void* ws,
                                               size_t ws_bytes, void* stream) {
  const char* fn = "rtc_cfr_loss_adjoint_cir";
  RTC_REQUIRE(X_tgt, RTC_ERR_INVALID_ARG, "%s: X_tgt is required", fn);
  return fused_run(fn, radio, paths, a, psi, g, nullptr, nullptr, X_tgt, tgt_stats, w_coh, w_pdp,
                   loss, dLda, dLdg, ws, ws_bytes, stream);
}
