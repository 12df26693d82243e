// Register FFTs of length N = 2^LOGN (2..4096) for the CFR losses: one
// wave per transform up to N = 1024, T = N/16 threads (one radix-16
// butterfly each per pass) beyond.
//
// Stockham autosort formulation: pass p (radix R, Ns = product of the radices
// before it) takes butterfly j (0 <= j < N/R), reads x[j + r N/R], multiplies
// element r by exp(+-j 2 pi r (j mod Ns) / (Ns R)), applies an R-point DFT
// and writes element r to (j / Ns) Ns R + (j mod Ns) + r Ns.  After the last
// pass the output is in natural order.  Radices are 16 while possible, then
// the remaining 2, 4 or 8.  Butterfly j of every pass belongs to thread
// j mod T of the T threads that share the transform (T = 64: one wave).
//
// Two properties let the loss keep data in registers between transforms:
//  * the first pass (Ns = 1) reads x[j + r N/R0] and the last pass leaves
//    element r of butterfly j at index j + r N/R_last;
//  * running the radices in reverse order, the first pass of the reverse
//    transform reads exactly the indices the last pass of the forward
//    transform left in each lane, and vice versa.
#pragma once

#include <type_traits>

#include "dev_common.h"

namespace rtc {

constexpr int fft_npass(int logn) { return logn / 4 + (logn % 4 != 0 ? 1 : 0); }

// LDS rows are padded by one value per 16: the first pass writes each
// butterfly's R outputs contiguously (lane stride R values), which would put
// every lane of a wave on the same bank; the pad spreads them.
RTC_DEV constexpr int lds_pad(int i) { return i + (i >> 4); }
// lds_pad(i + k S) = lds_pad(i) + lds_off(k S) wherever the passes use it:
// for the reads i = j < B and S = B = N/R, for the writes i = d (below) and
// S = Ns; in both cases the low four bits of i plus those of k S never carry
// (S a multiple of 16, or S | 16 and i mod 16 + k S mod 16 < 16), so every
// element's LDS slot is a per-lane base plus a compile-time offset.
RTC_DEV constexpr int lds_off(int ks) { return ks + (ks >> 4); }
constexpr int fft_lds_len(int n) { return n + n / 16; }
// radix of pass p in the "inverse" order: 16, 16, ..., then the remainder
constexpr int fft_radix(int logn, int p) {
  return p < logn / 4 ? 16 : (1 << (logn % 4));
}

// R-point DFT in registers: X_k = sum_n v_n exp(SIGN j 2 pi n k / R).
template <int SIGN>
RTC_DEV void dft2(float2* v) {
  float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

// multiply by SIGN * j
template <int SIGN>
RTC_DEV float2 mulj(float2 a) {
  return SIGN > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <int SIGN>
RTC_DEV void dft4(float2& v0, float2& v1, float2& v2, float2& v3) {
  float2 t0 = cadd(v0, v2), t1 = csub(v0, v2);
  float2 t2 = cadd(v1, v3), t3 = mulj<SIGN>(csub(v1, v3));
  v0 = cadd(t0, t2);
  v2 = csub(t0, t2);
  v1 = cadd(t1, t3);
  v3 = csub(t1, t3);
}

template <int SIGN>
RTC_DEV void dft8(float2* v) {
  // n = 2 n1 + n2, k = k1 + 4 k2
  constexpr float h = 0.70710678118654752440f;
  float2 u0[4] = {v[0], v[2], v[4], v[6]};
  float2 u1[4] = {v[1], v[3], v[5], v[7]};
  dft4<SIGN>(u0[0], u0[1], u0[2], u0[3]);
  dft4<SIGN>(u1[0], u1[1], u1[2], u1[3]);
  // u1[k1] *= exp(SIGN j 2 pi k1 / 8)
  u1[1] = cmul(u1[1], make_float2(h, SIGN * h));
  u1[2] = mulj<SIGN>(u1[2]);
  u1[3] = cmul(u1[3], make_float2(-h, SIGN * h));
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    v[k1] = cadd(u0[k1], u1[k1]);
    v[k1 + 4] = csub(u0[k1], u1[k1]);
  }
}

template <int SIGN>
RTC_DEV void dft16(float2* v) {
  // n = 4 n1 + n2, k = k1 + 4 k2
  constexpr float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f;
  constexpr float h = 0.70710678118654752440f;
  float2 u[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    u[n2][0] = v[n2];
    u[n2][1] = v[4 + n2];
    u[n2][2] = v[8 + n2];
    u[n2][3] = v[12 + n2];
    dft4<SIGN>(u[n2][0], u[n2][1], u[n2][2], u[n2][3]);
  }
  // u[n2][k1] *= exp(SIGN j 2 pi n2 k1 / 16), n2 k1 in {1, 2, 3, 4, 6, 9}
  const float2 w1 = make_float2(c1, SIGN * s1);
  const float2 w2 = make_float2(h, SIGN * h);
  const float2 w3 = make_float2(s1, SIGN * c1);
  const float2 w6 = make_float2(-h, SIGN * h);
  const float2 w9 = make_float2(-c1, -SIGN * s1);
  u[1][1] = cmul(u[1][1], w1);
  u[1][2] = cmul(u[1][2], w2);
  u[1][3] = cmul(u[1][3], w3);
  u[2][1] = cmul(u[2][1], w2);
  u[2][2] = mulj<SIGN>(u[2][2]);
  u[2][3] = cmul(u[2][3], w6);
  u[3][1] = cmul(u[3][1], w3);
  u[3][2] = cmul(u[3][2], w6);
  u[3][3] = cmul(u[3][3], w9);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    float2 a = u[0][k1], b = u[1][k1], c = u[2][k1], d = u[3][k1];
    dft4<SIGN>(a, b, c, d);
    v[k1] = a;
    v[k1 + 4] = b;
    v[k1 + 8] = c;
    v[k1 + 12] = d;
  }
}

template <int R, int SIGN>
RTC_DEV void dft(float2* v) {
  if constexpr (R == 2) dft2<SIGN>(v);
  if constexpr (R == 4) dft4<SIGN>(v[0], v[1], v[2], v[3]);
  if constexpr (R == 8) dft8<SIGN>(v);
  if constexpr (R == 16) dft16<SIGN>(v);
}

// Threads that share a transform of length 2^logn in the loss kernels: one
// wave up to 1024 points, then one radix-16 butterfly per thread.
constexpr int fft_threads(int logn) { return logn <= 10 ? 64 : (1 << logn) / 16; }

// Butterflies per thread for a pass of radix R over N points, T threads.
constexpr int fft_bpl(int n, int r, int t = 64) { return (n / r + t - 1) / t; }

// Twiddle of pass (Ns, R) for butterfly j: element r times w^r,
// w = exp(SIGN j 2 pi (j mod Ns) / (Ns R)).  Up to 1024 points w comes from
// the transcendental unit and its powers by recurrence; beyond (ACC), where
// the longer recurrences of radix-8 and -16 passes would multiply w's error
// by up to 15 (and the losses of long rows are sensitive to it), w and w^4
// are evaluated by polynomial (sincos2pi) and w^(4a+b) = (w^4)^a w^b with
// a, b <= 3, so no power is more than a few products from an evaluated
// value.
template <int R, int SIGN, bool ACC = false>
RTC_DEV void fft_twiddle(float2* v, int j, int Ns) {
  if (Ns == 1) return;
  const int k = j % Ns;
  if constexpr (ACC) {
    constexpr int NB = R < 4 ? R : 4, NA = R < 4 ? 1 : R / 4;
    const float x = (float)k / (float)(Ns * R);  // exact, as is 4x
    float2 p[4], q[4];
    float s1, c1;
    sincos2pi(x, &s1, &c1);
    p[1] = make_float2(c1, SIGN * s1);
#pragma unroll
    for (int b = 2; b < NB; ++b) p[b] = cmul(p[b - 1], p[1]);
    if constexpr (NA > 1) {
      float s4, c4;
      sincos2pi(4.0f * x, &s4, &c4);
      q[1] = make_float2(c4, SIGN * s4);
#pragma unroll
      for (int a = 2; a < NA; ++a) q[a] = cmul(q[a - 1], q[1]);
    }
#pragma unroll
    for (int r = 1; r < R; ++r) {
      const int a = r / NB, b = r % NB;
      const float2 wr = a == 0 ? p[b] : (b == 0 ? q[a] : cmul(q[a], p[b]));
      v[r] = cmul(v[r], wr);
    }
    return;
  }
  // k / (Ns R) is an exact fraction in [0, 1) (powers of two); the
  // transcendental unit takes it in revolutions
  const float x = (float)k / (float)(Ns * R);
  const float2 w = make_float2(__builtin_amdgcn_cosf(x), SIGN * __builtin_amdgcn_sinf(x));
  float2 wr = w;
#pragma unroll
  for (int r = 1; r < R; ++r) {
    v[r] = cmul(v[r], wr);
    wr = cmul(wr, w);
  }
}

// The same twiddles read from LDS rows (filled once by fft_tw_fill): for a
// pass (R, Ns), row r - 1 holds w^r of every j mod Ns = 0 .. Ns - 1 side by
// side, conjugated on reading for SIGN < 0.  A lane reads its values at one
// base plus a constant offset per r, and the lanes of one read hit
// consecutive values.  (In a plain table exp(j 2 pi k / N) the lanes'
// indices for one r lie r N / (Ns R) apart, a power-of-two stride that puts
// them on one or a few LDS banks.)  No error growth: every value is
// evaluated, none is a product of others.
//
// Segments: one per (R, Ns) of the passes with Ns > 1 of the forward and
// then the reverse radix order, each pair once.
template <int LOGN>
struct TwSegs {
  static constexpr int NP = fft_npass(LOGN);
  // pass p of order o (0 forward, 1 reverse): radix and Ns
  static constexpr int rad(int o, int p) { return fft_radix(LOGN, o == 0 ? p : NP - 1 - p); }
  static constexpr int ns(int o, int p) {
    int v = 1;
    for (int q = 0; q < p; ++q) v *= rad(o, q);
    return v;
  }
  // offset of the segment of (R, Ns), or the total length for R = 0
  static constexpr int off(int R, int Ns) {
    int o_acc = 0;
    for (int o = 0; o < 2; ++o)
      for (int p = 1; p < NP; ++p) {
        const int r = rad(o, p), n = ns(o, p);
        bool seen = false;
        for (int o2 = 0; o2 <= o; ++o2)
          for (int p2 = 1; p2 < (o2 < o ? NP : p); ++p2)
            if (rad(o2, p2) == r && ns(o2, p2) == n) seen = true;
        if (seen) continue;
        if (r == R && n == Ns) return o_acc;
        o_acc += (r - 1) * n;
      }
    return o_acc;
  }
};
template <int LOGN>
constexpr int fft_tw_len() {
  return TwSegs<LOGN>::off(0, 0);
}

template <int N, int R, int SIGN>
RTC_DEV void fft_twiddle_tab(float2* v, int j, int Ns, const float2* tw) {
  if (Ns == 1) return;
  constexpr int LOGN = __builtin_ctz(N);
  const float2* row = tw + TwSegs<LOGN>::off(R, Ns) + (j % Ns);
#pragma unroll
  for (int r = 1; r < R; ++r) {
    const float2 w = row[(r - 1) * Ns];
    v[r] = SIGN > 0 ? cmul(v[r], w) : cmulc(w, v[r]);
  }
}

// The row values, computed at compile time: exp(j 2 pi k / N) in double
// (exact reduction of k / N to the first eighth of a turn by symmetry, then
// Taylor series whose remainder is far below FP32 rounding), rounded once to
// FP32.  Entry m of row r - 1 of segment (R, Ns) has k = r m N / (Ns R).
struct TwVal {
  float x, y;
};
template <int LOGN>
struct alignas(16) TwTable {
  TwVal v[fft_tw_len<LOGN>()];
};

// sin x (sine) or cos x by their Taylor series, |x| <= pi / 4
constexpr double cx_taylor(double x, bool sine) {
  double t = sine ? x : 1.0, s = t;
  for (int m = 2; m < 40; m += 2) {
    t *= -x * x / (double)(sine ? m * (m + 1) : m * (m - 1));
    s += t;
  }
  return s;
}
// cos and sin of 2 pi k / n (n a multiple of 8)
constexpr TwVal cx_expj2pi(int k, int n) {
  constexpr double kTwoPi = 6.283185307179586476925286766559;
  k %= n;
  const int q = 4 * k / n;           // quarter turns
  const int r = k - q * (n / 4);     // 0 <= r < n / 4
  const bool comp = 8 * r > n;       // beyond an eighth: use the complement
  const double x = kTwoPi * (double)(comp ? n / 4 - r : r) / (double)n;
  const double sx = cx_taylor(x, true), cxv = cx_taylor(x, false);
  double c = comp ? sx : cxv, s = comp ? cxv : sx;
  for (int i = 0; i < q; ++i) {  // rotate by a quarter turn
    const double t = c;
    c = -s;
    s = t;
  }
  return TwVal{(float)c, (float)s};
}

template <int LOGN>
constexpr TwTable<LOGN> make_tw_table() {
  using S = TwSegs<LOGN>;
  constexpr int N = 1 << LOGN;
  TwTable<LOGN> t{};
  for (int o = 0; o < 2; ++o)
    for (int p = 1; p < S::NP; ++p) {
      const int R = S::rad(o, p), n = S::ns(o, p), b = S::off(R, n);
      for (int r = 1; r < R; ++r)
        for (int m = 0; m < n; ++m) t.v[b + (r - 1) * n + m] = cx_expj2pi(r * m * (N / (n * R)), N);
    }
  return t;
}

// The rows of the lengths whose one-wave transforms read them from LDS
// (256 to 1,024 points), one copy per code object.
static __constant__ TwTable<8> kTwRows8 = make_tw_table<8>();
static __constant__ TwTable<9> kTwRows9 = make_tw_table<9>();
static __constant__ TwTable<10> kTwRows10 = make_tw_table<10>();
template <int LOGN>
RTC_DEV const TwTable<LOGN>* tw_rows() {
  static_assert(LOGN >= 8 && LOGN <= 10, "lengths with twiddle rows");
  if constexpr (LOGN == 8)
    return &kTwRows8;
  else if constexpr (LOGN == 9)
    return &kTwRows9;
  else
    return &kTwRows10;
}

// Row-parallel transforms (the loss kernels): up to 1,024 points a wave
// takes a row, four waves per workgroup, each transforming in place in its
// own LDS buffer and all reading the workgroup's twiddle rows (256 points
// and up); longer rows take a workgroup of N/16 threads and two buffers.
constexpr int fft_row_waves(int logn) { return logn <= 10 ? 4 : 1; }
constexpr bool fft_row_tab(int logn) { return logn >= 8 && logn <= 10; }
constexpr int fft_row_tab_logn(int logn) { return fft_row_tab(logn) ? logn : 8; }

// Declarations of a row-parallel transform kernel over rows of N = 2^LOGN
// points with T = fft_threads(LOGN) threads per row: W rows in flight, the
// exchange order SY, the row buffers b0, b1 of this thread's row (one buffer
// in place for one-wave rows), the twiddle rows twr (filled here, TAB), the
// reduction scratch red, the thread's row slot wv and index lane0 in its row.
#define RTC_FFT_ROWS_SETUP()                                                               \
  constexpr int W = fft_row_waves(LOGN);                                                   \
  constexpr bool TAB = fft_row_tab(LOGN);                                                  \
  using SY = typename std::conditional<W == 1, BlockSync, WaveSync>::type;                 \
  __shared__ float2 rowbufs[W == 1 ? 2 : W][fft_lds_len(N)];                               \
  __shared__ float2 twr[TAB ? fft_tw_len<fft_row_tab_logn(LOGN)>() : 2];                   \
  __shared__ double red[T / 64];                                                           \
  const int wv = W == 1 ? 0 : (int)(threadIdx.x >> 6);                                     \
  const int lane0 = W == 1 ? (int)threadIdx.x : (int)(threadIdx.x & 63);                   \
  float2* b0 = rowbufs[wv];                                                                \
  float2* b1 = rowbufs[W == 1 ? 1 : wv];                                                   \
  if constexpr (TAB) {                                                                     \
    fft_tw_fill<fft_row_tab_logn(LOGN)>(twr, tw_rows<fft_row_tab_logn(LOGN)>(),            \
                                        (int)threadIdx.x, (int)blockDim.x);                \
    __syncthreads();                                                                       \
  }

// Copies the rows from global memory (tab: make_tw_table<LOGN>()) into LDS.
template <int LOGN>
RTC_DEV void fft_tw_fill(float2* tw, const TwTable<LOGN>* tab, int tid, int nthreads) {
  constexpr int L4 = fft_tw_len<LOGN>() / 2;
  static_assert(fft_tw_len<LOGN>() % 2 == 0, "whole 16-byte pairs");
  const float4* src = reinterpret_cast<const float4*>(tab->v);
  float4* dst = reinterpret_cast<float4*>(tw);
  for (int i = tid; i < L4; i += nthreads) dst[i] = src[i];
}

template <int N, int R, int SIGN, bool TAB>
RTC_DEV void fft_twiddle_any(float2* v, int j, int Ns, const float2* tw) {
  if constexpr (TAB)
    fft_twiddle_tab<N, R, SIGN>(v, j, Ns, tw);
  else
    fft_twiddle<R, SIGN, (N > 1024)>(v, j, Ns);
}

// Pass from registers (v[i][r] of butterfly j = lane + T i) to LDS `out`.
template <int N, int R, int SIGN, int T = 64, bool TAB = false>
RTC_DEV void fft_pass_r2l(float2 (*v)[R], float2* out, int Ns, int lane,
                          const float2* tw = nullptr) {
  constexpr int B = N / R;
#pragma unroll
  for (int i = 0; i < fft_bpl(N, R, T); ++i) {
    const int j = lane + T * i;
    if (j < B) {
      fft_twiddle_any<N, R, SIGN, TAB>(v[i], j, Ns, tw);
      dft<R, SIGN>(v[i]);
      float2* o = out + lds_pad((j / Ns) * Ns * R + (j % Ns));
#pragma unroll
      for (int r = 0; r < R; ++r) o[lds_off(r * Ns)] = v[i][r];
    }
  }
}

// Pass from LDS `in` to registers v[i][r] (no store).
template <int N, int R, int SIGN, int T = 64, bool TAB = false>
RTC_DEV void fft_pass_l2r(const float2* in, float2 (*v)[R], int Ns, int lane,
                          const float2* tw = nullptr) {
  constexpr int B = N / R;
#pragma unroll
  for (int i = 0; i < fft_bpl(N, R, T); ++i) {
    const int j = lane + T * i;
    if (j < B) {
      const float2* src = in + lds_pad(j);
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = src[lds_off(r * B)];
      fft_twiddle_any<N, R, SIGN, TAB>(v[i], j, Ns, tw);
      dft<R, SIGN>(v[i]);
    }
  }
}

// Ordering of the LDS exchanges between passes.  BlockSync: a workgroup
// barrier (a one-wave workgroup, or every wave of the workgroup transforming
// at the same time).  WaveSync: the wave's own buffers only; LDS operations
// of one wave complete in issue order, so keeping the compiler from moving
// them across the exchange is all that is needed.
struct BlockSync {
  static RTC_DEV void sync() { __syncthreads(); }
};
struct WaveSync {
  static RTC_DEV void sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
};

// Radix and Ns of position P in a pass sequence: ORDER = +1 runs the radices
// as fft_radix lists them, ORDER = -1 in reverse.
template <int LOGN, int ORDER, int P>
constexpr int seq_radix() {
  return fft_radix(LOGN, ORDER > 0 ? P : fft_npass(LOGN) - 1 - P);
}
template <int LOGN, int ORDER, int P>
constexpr int seq_ns() {
  if constexpr (P == 0)
    return 1;
  else
    return seq_ns<LOGN, ORDER, P - 1>() * seq_radix<LOGN, ORDER, P - 1>();
}

// Pass P (1 <= P <= npass-2): LDS -> LDS, ping-ponging b0/b1 (pass 0
// writes b0), then the following middle passes.  b0 == b1 runs in place.
template <int LOGN, int SIGN, int ORDER, int P, class SY = BlockSync, int T = 64,
          bool TAB = false>
RTC_DEV void fft_mid(float2* b0, float2* b1, int lane, const float2* tw = nullptr) {
  constexpr int NP = fft_npass(LOGN);
  if constexpr (P <= NP - 2) {
    constexpr int N = 1 << LOGN;
    constexpr int R = seq_radix<LOGN, ORDER, P>();
    constexpr int NS = seq_ns<LOGN, ORDER, P>();
    const float2* in = ((P - 1) & 1) ? b1 : b0;
    float2* out = (P & 1) ? b1 : b0;
    SY::sync();
    float2 v[fft_bpl(N, R, T)][R];
    fft_pass_l2r<N, R, SIGN, T, TAB>(in, v, NS, lane, tw);
    if (in == out) SY::sync();  // one buffer: every read before any write
#pragma unroll
    for (int i = 0; i < fft_bpl(N, R, T); ++i) {
      const int j = lane + T * i;
      if (j < N / R) {
        float2* o = out + lds_pad((j / NS) * NS * R + (j % NS));
#pragma unroll
        for (int r = 0; r < R; ++r) o[lds_off(r * NS)] = v[i][r];
      }
    }
    fft_mid<LOGN, SIGN, ORDER, P + 1, SY, T, TAB>(b0, b1, lane, tw);
  }
}

// Whole transform: vin holds the first pass's inputs (butterfly j = lane +
// T i, element r = x[j + r N/R_first]); vout receives the last pass's
// outputs (element r of butterfly j = X[j + r N/R_last]).  b0, b1: two LDS
// buffers of fft_lds_len(N) values; lane = the thread's index among the T;
// with TAB the twiddles come from the table tw (fft_twiddle_tab).
template <int LOGN, int SIGN, int ORDER, class SY = BlockSync, int T = 64, bool TAB = false,
          int J0, int R0, int JL, int RL>
RTC_DEV void fft_full(float2 (&vin)[J0][R0], float2 (&vout)[JL][RL], float2* b0, float2* b1,
                      int lane, const float2* tw = nullptr) {
  constexpr int N = 1 << LOGN;
  constexpr int NP = fft_npass(LOGN);
  static_assert(R0 == seq_radix<LOGN, ORDER, 0>(), "first-pass layout");
  static_assert(RL == seq_radix<LOGN, ORDER, NP - 1>(), "last-pass layout");
  static_assert(J0 == fft_bpl(N, R0, T) && JL == fft_bpl(N, RL, T), "butterflies per thread");
  if constexpr (NP == 1) {
#pragma unroll
    for (int i = 0; i < fft_bpl(N, R0, T); ++i) {
      if (lane + T * i < N / R0) {
        dft<R0, SIGN>(vin[i]);
#pragma unroll
        for (int r = 0; r < R0; ++r) vout[i][r] = vin[i][r];
      }
    }
  } else {
    fft_pass_r2l<N, R0, SIGN, T, TAB>(vin, b0, 1, lane, tw);
    fft_mid<LOGN, SIGN, ORDER, 1, SY, T, TAB>(b0, b1, lane, tw);
    constexpr int PL = NP - 1;
    const float2* in = ((PL - 1) & 1) ? b1 : b0;
    SY::sync();
    fft_pass_l2r<N, RL, SIGN, T, TAB>(in, vout, seq_ns<LOGN, ORDER, PL>(), lane, tw);
    SY::sync();
  }
}

// Sum of a double over the T threads of a transform in a fixed order (wave
// butterflies, then the waves in index order); every thread gets the total.
// red: T/64 doubles of LDS (unused for T = 64).
template <int T>
RTC_DEV double group_sum_f64(double v, double* red) {
  v = wave_sum_f64(v);
  if constexpr (T == 64) {
    return v;
  } else {
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = red[0];
#pragma unroll
    for (int w = 1; w < T / 64; ++w) s += red[w];
    __syncthreads();
    return s;
  }
}

}  // namespace rtc
