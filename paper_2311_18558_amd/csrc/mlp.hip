// Neural materials (Sec. III-D): positional encoding + MLP 51 -> 128 x 4
// (ReLU) -> 3, outputs eps_r = 1 + softplus, sigma = softplus, S = logistic,
// on the BF16 matrix cores with FP32 accumulation.
//
// Forward: a wave per 32 points.  Activations are the B operand of
// v_mfma_f32_32x32x16_bf16 (rows = neurons, columns = points): lane l holds
// point l%32 and K slice 8(l/32)..+7.  The accumulator of a 32-neuron tile
// holds, in register r of lane l, neuron 8(r/4) + 4(l/32) + r%4 of point
// l%32, so registers 8e..8e+7 of a tile are directly the next layer's
// K-block (tile, e) when the K order inside that block is the permutation
// kperm(c, h, j) = 32(c/2) + 16(c%2) + 8(j/4) + 4h + j%4 -- the weights are
// packed in that order, so activations never leave the registers.  The
// layer inputs are saved for the backward exactly as they sit in the
// registers (one 16-byte vector per lane and K-block, a wave's block of 32
// points contiguous), so saving and reloading them are full-width accesses.
//
// Backward: one fused kernel.  A workgroup of four waves takes 128 points at
// a time; each wave reloads its 32 points' layer inputs and runs the deltas
// down through the transposed weights (the same register layout as the
// forward).  At every layer the four waves put that layer's output deltas
// and inputs, transposed to feature rows x point columns, into LDS; then the
// weight gradient is a product over the 128 points (the K dimension), and
// each wave owns a quarter of every layer's 32 x 32 gradient tiles, kept in
// registers for the whole run.  The workgroups' partial gradients are summed
// in a fixed order.
#include <cmath>

#include "api_common.h"
#include "dev_common.h"

namespace rtc {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kMlpIn = 51;     // 3 + 3 coords x 8 frequencies x (sin, cos)
constexpr int kMlpIn0 = 64;    // padded input width
constexpr int kMlpWidth = 128;
constexpr int kMlpOut = 3;
constexpr int kMlpFreq = 8;
constexpr int kMlpParams = 56579;

// parameter packing: W0 [128][51], b0, W1 [128][128], b1, W2, b2, W3, b3,
// W4 [3][128], b4
__host__ __device__ constexpr int mlp_off_w(int l) {
  return l == 0 ? 0 : l == 1 ? 6656 : l == 2 ? 23168 : l == 3 ? 39680 : 56192;
}
__host__ __device__ constexpr int mlp_off_b(int l) {
  return l == 0 ? 6528 : l == 1 ? 23040 : l == 2 ? 39552 : l == 3 ? 56064 : 56576;
}
__host__ __device__ constexpr int mlp_nout(int l) { return l == 4 ? kMlpOut : kMlpWidth; }
__host__ __device__ constexpr int mlp_nin(int l) { return l == 0 ? kMlpIn : kMlpWidth; }
// K-blocks (of 16) and output tiles (of 32) per layer
__host__ __device__ constexpr int mlp_kb(int l) { return l == 0 ? 4 : 8; }
__host__ __device__ constexpr int mlp_ot(int l) { return l == 4 ? 1 : 4; }
// packed forward operand offsets (in bf16 elements): [tile][kblock][64][8]
__host__ __device__ constexpr int fw_size(int l) { return mlp_ot(l) * mlp_kb(l) * 512; }
__host__ __device__ constexpr int fw_off(int l) {
  return l == 0 ? 0 : fw_off(l - 1) + fw_size(l - 1);
}
// packed backward operand (W^T), layers 1..4: [in tile 4][kblock over n_out][64][8]
__host__ __device__ constexpr int bw_kb(int l) { return l == 4 ? 1 : 8; }
__host__ __device__ constexpr int bw_size(int l) { return 4 * bw_kb(l) * 512; }
__host__ __device__ constexpr int bw_off(int l) {
  return l <= 1 ? fw_off(5) : bw_off(l - 1) + bw_size(l - 1);
}
constexpr int kPackedElems = bw_off(5);

RTC_DEV int kperm(int c, int h, int j) {
  return 32 * (c >> 1) + 16 * (c & 1) + 8 * (j >> 2) + 4 * h + (j & 3);
}

RTC_DEV uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (uint16_t)(u >> 16);
}
RTC_DEV float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// eight FP32 values rounded to BF16 (nearest even; v_cvt_pk_bf16_f32)
typedef float float8v __attribute__((ext_vector_type(8)));
RTC_DEV bf16x8 pack8(const float* v) {
  float8v f;
#pragma unroll
  for (int j = 0; j < 8; ++j) f[j] = v[j];
  return __builtin_convertvector(f, bf16x8);
}

RTC_DEV floatx16 mfma_bf16(bf16x8 a, bf16x8 b, floatx16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

RTC_DEV int drow(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }

// Pack FP32 master parameters into the BF16 operand layouts.
__global__ void mlp_pack_kernel(const float* __restrict__ prm, uint16_t* __restrict__ packed) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= kPackedElems) return;
  float v = 0.0f;
  if (idx < fw_off(5)) {
    int l = 0;
    while (l < 4 && idx >= fw_off(l + 1)) ++l;
    int r = idx - fw_off(l);
    int j = r & 7, lane = (r >> 3) & 63, c = (r >> 9) % mlp_kb(l), t = (r >> 9) / mlp_kb(l);
    int i = lane & 31, h = lane >> 5;
    int n = 32 * t + i;
    int k = l == 0 ? 16 * c + 8 * h + j : kperm(c, h, j);
    if (n < mlp_nout(l) && k < mlp_nin(l)) v = prm[mlp_off_w(l) + n * mlp_nin(l) + k];
  } else {
    int l = 1;
    while (l < 4 && idx >= bw_off(l + 1)) ++l;
    int r = idx - bw_off(l);
    int j = r & 7, lane = (r >> 3) & 63, c = (r >> 9) % bw_kb(l), t = (r >> 9) / bw_kb(l);
    int i = lane & 31, h = lane >> 5;
    int nin = 32 * t + i;
    int nout = kperm(c, h, j);
    if (nout < mlp_nout(l) && nin < mlp_nin(l)) v = prm[mlp_off_w(l) + nout * mlp_nin(l) + nin];
  }
  packed[idx] = f2bf(v);
}

struct MlpArgs {
  int64_t n_points;
  int64_t qpad;  // points rounded up to 256 (saved-buffer geometry)
  const float *px, *py, *pz;
  float cx, cy, cz, inv_ext;
  const float* prm;          // FP32 master parameters
  const uint16_t* packed;    // BF16 operands
  float* out;                // [3][n_points]
  // saved for the backward, or null: layer inputs in the register layout
  // ([block of 32 points][K-block][lane] x 8 BF16) and the FP32 outputs
  bf16x8* x0;                // [qpad/32][4][64]
  bf16x8* hs;                // [4][qpad/32][8][64]  h1..h4
  float* o;                  // [3][qpad] pre-transform outputs
};

RTC_DEV bf16x8 load_op(const uint16_t* base, int idx8) {
  return *reinterpret_cast<const bf16x8*>(base + 8 * (int64_t)idx8);
}

RTC_DEV float softplusf(float x) { return x > 20.0f ? x : log1pf(expf(x)); }
RTC_DEV float sigmoidf(float x) { return 1.0f / (1.0f + expf(-x)); }

// Positional-encoding feature f (0..63) of normalised coordinates pb.
RTC_DEV float pe_feature(int f, const float pb[3]) {
  if (f < 3) return pb[f];
  if (f >= kMlpIn) return 0.0f;
  int g = f - 3;
  int c = g >> 4;          // coordinate
  int k = (g >> 1) & 7;    // frequency index 0..7 -> 2^(k+1) pi
  float x = ldexpf(pb[c], k);  // 2^k p_bar, exact; sin(2 pi x) = sin(2^(k+1) pi p_bar)
  float fr = x - floorf(x);
  float s, co;
  sincos2pi(fr, &s, &co);
  return (g & 1) ? co : s;
}

// saved-buffer offsets (in 16-byte vectors) of a wave block's K-block c
RTC_DEV int64_t sv_x0(int64_t blk, int c, int lane) { return (blk * 4 + c) * 64 + lane; }
RTC_DEV int64_t sv_h(int64_t nblk, int l, int64_t blk, int c, int lane) {
  return (((int64_t)l * nblk + blk) * 8 + c) * 64 + lane;
}

// Forward: persistent workgroups of kFwdWaves waves, one per CU.  The
// packed weights (120 KB) and the biases go to LDS once; each wave then
// takes blocks of 32 points in turn, its weight operands from LDS.
constexpr int kFwdWaves = 8;
constexpr int kFwdOps = fw_off(5) / 8;  // 16-byte weight operands
constexpr int kFwdBias = 4 * kMlpWidth + kMlpOut;
constexpr int kFwdBlocks = 256;

__global__ void __launch_bounds__(kFwdWaves * 64, 1) mlp_forward_kernel(MlpArgs A) {
  __shared__ bf16x8 wl[kFwdOps];
  __shared__ float bl[kFwdBias];
  {
    const bf16x8* src = reinterpret_cast<const bf16x8*>(A.packed);
    for (int i = threadIdx.x; i < kFwdOps; i += kFwdWaves * 64) wl[i] = src[i];
    for (int i = threadIdx.x; i < kFwdBias; i += kFwdWaves * 64)
      bl[i] = A.prm[i < 4 * kMlpWidth ? mlp_off_b(i / kMlpWidth) + i % kMlpWidth
                                      : mlp_off_b(4) + i - 4 * kMlpWidth];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5;
  const int pt = lane & 31;
  const int64_t nblk = A.qpad / 32;
  const int64_t nreal = (A.n_points + 31) / 32;
  for (int64_t blk = (int64_t)blockIdx.x * kFwdWaves + (threadIdx.x >> 6); blk < nreal;
       blk += (int64_t)gridDim.x * kFwdWaves) {
    // an opaque zero keeps the weight and bias reads inside the loop
    // (hoisted, they would hold hundreds of registers)
    int z = 0;
    asm volatile("" : "+v"(z));
    const bf16x8* W0 = wl + z;
    const float* B0 = bl + z;
    const int64_t q0 = blk * 32;
    const int64_t q = q0 + pt;
    const bool valid = q < A.n_points;
    float pb[3] = {0.0f, 0.0f, 0.0f};
    if (valid) {
      pb[0] = (A.px[q] - A.cx) * A.inv_ext;
      pb[1] = (A.py[q] - A.cy) * A.inv_ext;
      pb[2] = (A.pz[q] - A.cz) * A.inv_ext;
    }
    // layer-0 input: K-block c holds features 16c + 8h + j
    bf16x8 xin[8];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      float v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = pe_feature(16 * c + 8 * h + j, pb);
      xin[c] = pack8(v);
      if (A.x0) A.x0[sv_x0(blk, c, lane)] = xin[c];
    }
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      floatx16 acc[4];
      const bf16x8* W = W0 + fw_off(l) / 8;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        acc[t] = floatx16{0};
#pragma unroll
        for (int c = 0; c < mlp_kb(l); ++c)
          acc[t] = mfma_bf16(W[(t * mlp_kb(l) + c) * 64 + lane], xin[c], acc[t]);
      }
      const float* b = B0 + l * kMlpWidth;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        float v[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = fmaxf(acc[t][r] + b[32 * t + drow(r, h)], 0.0f);
        xin[2 * t] = pack8(v);
        xin[2 * t + 1] = pack8(v + 8);
      }
      if (A.hs) {
#pragma unroll
        for (int c = 0; c < 8; ++c) A.hs[sv_h(nblk, l, blk, c, lane)] = xin[c];
      }
    }
    floatx16 acc = floatx16{0};
    const bf16x8* W4 = W0 + fw_off(4) / 8;
#pragma unroll
    for (int c = 0; c < 8; ++c) acc = mfma_bf16(W4[c * 64 + lane], xin[c], acc);
    if (h == 0 && valid) {
      const float* b4 = B0 + 4 * kMlpWidth;
      float o0 = acc[0] + b4[0], o1 = acc[1] + b4[1], o2 = acc[2] + b4[2];
      A.out[q] = 1.0f + softplusf(o0);
      A.out[A.n_points + q] = softplusf(o1);
      A.out[2 * A.n_points + q] = sigmoidf(o2);
      if (A.o) {
        A.o[q] = o0;
        A.o[A.qpad + q] = o1;
        A.o[2 * A.qpad + q] = o2;
      }
    }
  }
}

constexpr int kBwdWaves = 4;
constexpr int kBwdPts = 32 * kBwdWaves;  // points per workgroup step
constexpr int kBwdLd = kBwdPts + 8;      // LDS row stride (BF16): conflict-free 16-byte reads
constexpr int kBwdStage = 2 * 128 * kBwdLd;  // one layer: 128 delta rows, then 128 input rows
constexpr int kMlpBwdBlocks = 256;       // workgroups (their partials are summed in order)

struct MlpBwdArgs {
  int64_t n_points, qpad;
  const float* dout;        // [3][n_points] dL/d(eps_r, sigma, S)
  const uint16_t* packed;
  const bf16x8* x0;         // saved layer inputs (layout of MlpArgs)
  const bf16x8* hs;
  const float* o;           // [3][qpad]
  float* part;              // [gridDim.x][kMlpParams]
};

// Transposed store of a wave's K-blocks (register layout, feature order
// kperm or natural) into LDS rows = features, columns = the wave's 32
// points.  A word of the register layout holds features j, j + 1 (j even)
// of the lane's point; the lanes of points col, col ^ 1 swap that word (DPP
// within a quad), and the even lane stores feature j of both points, the odd
// lane feature j + 1, each as one 4-byte store (two 2-byte stores a lane
// otherwise, which bound the kernel).  Every lane of the wave must take part.
template <int NKB, bool KPERM>
RTC_DEV void put_rows(uint16_t* rows, const bf16x8* v, int col, int h) {
  const int odd = col & 1;
  const unsigned sel = odd ? 0x03020706u : 0x05040100u;  // {oth.hi, own.hi} : {own.lo, oth.lo}
  // feature j = 2 q + odd of K-block c is row fc(c, q) + the lane's part
  // (kperm: 4 h + odd; natural: 8 h + odd); the even column starts the word
  uint16_t* base = rows + (KPERM ? 4 * h : 8 * h) * kBwdLd + odd * kBwdLd + (col - odd);
#pragma unroll
  for (int c = 0; c < NKB; ++c) {
    const u32x4 w = __builtin_bit_cast(u32x4, v[c]);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const unsigned own = w[q];
      const unsigned oth = (unsigned)__builtin_amdgcn_mov_dpp((int)own, 0xB1, 0xF, 0xF, false);  // lane ^ 1
      const int fc = KPERM ? 32 * (c >> 1) + 16 * (c & 1) + 8 * (q >> 1) + 2 * (q & 1)
                           : 16 * c + 2 * q;
      *reinterpret_cast<uint32_t*>(base + fc * kBwdLd) = __builtin_amdgcn_perm(oth, own, sel);
    }
  }
}

RTC_DEV bf16x8 lds_op(const uint16_t* rows, int row, int k0) {
  return *reinterpret_cast<const bf16x8*>(rows + row * kBwdLd + k0);
}

RTC_DEV float bf_sum8(bf16x8 a) {
  const u32x4 w = __builtin_bit_cast(u32x4, a);
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < 4; ++j) s += __uint_as_float(w[j] << 16) + __uint_as_float(w[j] & 0xFFFF0000u);
  return s;
}

RTC_DEV bool bf_pos(bf16x8 v, int j) {
  const u32x4 w = __builtin_bit_cast(u32x4, v);
  const uint32_t b = (w[j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
  return b != 0u && (b & 0x8000u) == 0u;
}

// global-memory pointer (keeps the weight loads global, not flat, after the
// address has passed through an opaque copy)
typedef const __attribute__((address_space(1))) bf16x8* GPtr;

// d_in = W_l^T d_out * [h_l > 0] for one wave (register layout; blocks
// beyond the points carry zero inputs, hence zero deltas).
template <int L>
RTC_DEV void delta_down(GPtr packed, const bf16x8* din, const bf16x8* hv, int lane, bf16x8* nxt) {
  GPtr Wt = packed + bw_off(L) / 8;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    floatx16 acc = floatx16{0};
#pragma unroll
    for (int c = 0; c < bw_kb(L); ++c)
      acc = mfma_bf16(Wt[(t * bw_kb(L) + c) * 64 + lane], din[c], acc);
    float v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = bf_pos(hv[2 * t + (r >> 3)], r & 7) ? acc[r] : 0.0f;
    nxt[2 * t] = pack8(v);
    nxt[2 * t + 1] = pack8(v + 8);
  }
}

__global__ void __launch_bounds__(kBwdWaves * 64, 1) mlp_backward_kernel(MlpBwdArgs A) {
  __shared__ __align__(16) uint16_t lds[2 * kBwdStage];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5;
  const int i = lane & 31;
  const int col = 32 * wave + i;
  const int64_t nblk = A.qpad / 32;
  const int64_t nstep = (A.n_points + kBwdPts - 1) / kBwdPts;
  // this wave's gradient tiles: layers 1..3 (out tile = wave, in tiles 0..3),
  // layer 0 (out tile = wave, in tiles 0..1), layer 4 (in tile = wave)
  floatx16 g123[3][4], g0[2], g4;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) g123[a][b] = floatx16{0};
  g0[0] = g0[1] = g4 = floatx16{0};
  float gb[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};  // bias partial sums (rows of this lane)
  const bf16x8 zero8 = __builtin_bit_cast(bf16x8, u32x4{0u, 0u, 0u, 0u});
  int buf = 0;
  for (int64_t stp = blockIdx.x; stp < nstep; stp += gridDim.x) {
    // the packed weights are the same every step: an opaque copy of their
    // address keeps their loads inside the loop (hoisted, they would hold
    // hundreds of registers for the whole run)
    GPtr pk = (GPtr)A.packed;
    asm volatile("" : "+s"(pk));
    const int64_t blk = stp * kBwdWaves + wave;
    const bool live = blk * 32 < A.n_points;  // the forward saved this block
    const int64_t q = blk * 32 + i;
    const bool valid = q < A.n_points;
    // blocks beyond the points lie inside the saved buffer (it is padded to
    // 256 points) but were never written: their loads are replaced by zeros
    bf16x8 hv[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const bf16x8 v = A.hs[sv_h(nblk, 3, blk, c, lane)];
      hv[c] = live ? v : zero8;
    }
    // output deltas: rows 0..2 in lanes h = 0, registers 0..2 of K-block 0
    bf16x8 din[8];
    {
      const int64_t qc = valid ? q : A.n_points - 1;
      const float s0 = sigmoidf(A.o[qc]), s1 = sigmoidf(A.o[A.qpad + qc]);
      const float s2 = sigmoidf(A.o[2 * A.qpad + qc]);
      const bool on = h == 0 && valid;
      float dv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      dv[0] = on ? A.dout[qc] * s0 : 0.0f;                             // d eps/d o0
      dv[1] = on ? A.dout[A.n_points + qc] * s1 : 0.0f;                // d sigma/d o1
      dv[2] = on ? A.dout[2 * A.n_points + qc] * s2 * (1.0f - s2) : 0.0f;  // d S/d o2
      din[0] = pack8(dv);
#pragma unroll
      for (int c = 1; c < 8; ++c) din[c] = zero8;
    }
#pragma unroll
    for (int s = 4; s >= 0; --s) {
      uint16_t* Ds = lds + buf * kBwdStage;
      uint16_t* Xs = Ds + 128 * kBwdLd;
      // layer s: output deltas (rows) and inputs (rows) of this wave's points
      if (s == 4) {
        if (h == 0) {
          const u32x4 w = __builtin_bit_cast(u32x4, din[0]);
          Ds[0 * kBwdLd + col] = (uint16_t)(w[0] & 0xFFFFu);
          Ds[1 * kBwdLd + col] = (uint16_t)(w[0] >> 16);
          Ds[2 * kBwdLd + col] = (uint16_t)(w[1] & 0xFFFFu);
        }
      } else {
        put_rows<8, true>(Ds, din, col, h);
      }
      if (s == 0) put_rows<4, false>(Xs, hv, col, h);
      else put_rows<8, true>(Xs, hv, col, h);
      // deltas one layer down while the others write
      bf16x8 nxt[8];
      if (s == 4) delta_down<4>(pk, din, hv, lane, nxt);
      if (s == 3) delta_down<3>(pk, din, hv, lane, nxt);
      if (s == 2) delta_down<2>(pk, din, hv, lane, nxt);
      if (s == 1) delta_down<1>(pk, din, hv, lane, nxt);
      // inputs of the next layer down
      bf16x8 hn[8];
      if (s >= 2) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          const bf16x8 v = A.hs[sv_h(nblk, s - 2, blk, c, lane)];
          hn[c] = live ? v : zero8;
        }
      } else if (s == 1) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const bf16x8 v = A.x0[sv_x0(blk, c, lane)];
          hn[c] = live ? v : zero8;
        }
#pragma unroll
        for (int c = 4; c < 8; ++c) hn[c] = zero8;
      }
      __syncthreads();
      // weight gradient of layer s over the workgroup's 128 points
#pragma unroll
      for (int k = 0; k < kBwdPts / 16; ++k) {
        const int k0 = 16 * k + 8 * h;
        if (s == 4) {
          const bf16x8 a4 = lds_op(Ds, i < 3 ? i : 0, k0);
          const bf16x8 a = i < 3 ? a4 : zero8;
          g4 = mfma_bf16(a, lds_op(Xs, 32 * wave + i, k0), g4);
          if (wave == 0) gb[4] += bf_sum8(a);
        } else {
          const bf16x8 a = lds_op(Ds, 32 * wave + i, k0);
          gb[s] += bf_sum8(a);
          if (s == 0) {
#pragma unroll
            for (int ti = 0; ti < 2; ++ti) g0[ti] = mfma_bf16(a, lds_op(Xs, 32 * ti + i, k0), g0[ti]);
          } else {
#pragma unroll
            for (int ti = 0; ti < 4; ++ti)
              g123[s - 1][ti] = mfma_bf16(a, lds_op(Xs, 32 * ti + i, k0), g123[s - 1][ti]);
          }
        }
      }
      // no barrier here: the next layer writes the other buffer, and this
      // one is rewritten only after the next layer's barrier
      buf ^= 1;
      if (s >= 1) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          din[c] = nxt[c];
          hv[c] = hn[c];
        }
      }
    }
  }
  // this workgroup's partial gradient
  float* out = A.part + (int64_t)blockIdx.x * kMlpParams;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int no = 32 * wave + drow(r, h);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int ti = 0; ti < 4; ++ti)
        out[mlp_off_w(a + 1) + no * kMlpWidth + 32 * ti + i] = g123[a][ti][r];
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
      if (32 * ti + i < kMlpIn) out[mlp_off_w(0) + no * kMlpIn + 32 * ti + i] = g0[ti][r];
    const int n4 = drow(r, h);
    if (n4 < kMlpOut) out[mlp_off_w(4) + n4 * kMlpWidth + 32 * wave + i] = g4[r];
  }
#pragma unroll
  for (int l = 0; l < 5; ++l) gb[l] += __shfl_xor(gb[l], 32);
  if (h == 0) {
#pragma unroll
    for (int l = 0; l < 4; ++l) out[mlp_off_b(l) + 32 * wave + i] = gb[l];
    if (wave == 0 && i < kMlpOut) out[mlp_off_b(4) + i] = gb[4];
  }
}

// Sum the workgroup partials column-wise in workgroup order (FP64).
__global__ void reduce_cols_kernel(const float* part, int R, int K, float* out) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= K) return;
  double s = 0.0;
  for (int r = 0; r < R; ++r) s += (double)part[(int64_t)r * K + c];
  out[c] = (float)s;
}

static int64_t qpad_of(int64_t n) { return (n + 255) / 256 * 256; }

}  // namespace rtc

using namespace rtc;

extern "C" {

int32_t rtc_mlp_n_params(void) { return kMlpParams; }

size_t rtc_mlp_saved_size(int64_t n_points) {
  if (n_points < 0) return 0;
  int64_t qp = qpad_of(n_points);
  return (size_t)qp * (kMlpIn0 + 4 * kMlpWidth) * sizeof(uint16_t) + (size_t)qp * 3 * sizeof(float);
}

size_t rtc_mlp_workspace_size(int64_t n_points) {
  if (n_points < 0) return 0;
  return (size_t)kPackedElems * sizeof(uint16_t) + 256 +
         (size_t)kMlpBwdBlocks * kMlpParams * sizeof(float);
}

rtc_status rtc_mlp_forward(const rtc_mlp* net, int64_t n_points, const float* px, const float* py,
                           const float* pz, float* out, void* saved, size_t saved_bytes, void* ws,
                           size_t ws_bytes, void* stream) {
  const char* fn = "rtc_mlp_forward";
  RTC_REQUIRE(net && net->params, RTC_ERR_INVALID_ARG, "%s: net and net->params are required", fn);
  RTC_REQUIRE(net->n_freq == kMlpFreq && net->width == kMlpWidth && net->n_hidden == 4,
              RTC_ERR_UNSUPPORTED, "%s: this build implements n_freq 8, width 128, 4 hidden layers",
              fn);
  RTC_REQUIRE(net->inv_extent > 0.0f, RTC_ERR_INVALID_ARG, "%s: inv_extent must be > 0", fn);
  RTC_REQUIRE(n_points >= 0, RTC_ERR_SHAPE, "%s: n_points must be >= 0", fn);
  if (n_points == 0) return RTC_OK;
  RTC_REQUIRE(px && py && pz && out, RTC_ERR_INVALID_ARG, "%s: points and out are required", fn);
  RTC_REQUIRE(ws && ws_bytes >= (size_t)kPackedElems * 2, RTC_ERR_WORKSPACE,
              "%s: workspace of %zu bytes required", fn, (size_t)kPackedElems * 2);
  if (saved) {
    RTC_REQUIRE(saved_bytes >= rtc_mlp_saved_size(n_points), RTC_ERR_WORKSPACE,
                "%s: saved buffer of %zu bytes required", fn, rtc_mlp_saved_size(n_points));
  }
  hipStream_t s = as_stream(stream);
  uint16_t* packed = reinterpret_cast<uint16_t*>(ws);
  hipLaunchKernelGGL(mlp_pack_kernel, dim3((kPackedElems + 255) / 256), dim3(256), 0, s,
                     net->params, packed);
  rtc_status st;
  if ((st = check_launch(fn)) != RTC_OK) return st;
  MlpArgs A;
  A.n_points = n_points;
  A.qpad = qpad_of(n_points);
  A.px = px;
  A.py = py;
  A.pz = pz;
  A.cx = net->aabb_center[0];
  A.cy = net->aabb_center[1];
  A.cz = net->aabb_center[2];
  A.inv_ext = net->inv_extent;
  A.prm = net->params;
  A.packed = packed;
  A.out = out;
  uint16_t* sv = reinterpret_cast<uint16_t*>(saved);
  A.x0 = saved ? reinterpret_cast<bf16x8*>(sv) : nullptr;
  A.hs = saved ? reinterpret_cast<bf16x8*>(sv + (int64_t)kMlpIn0 * A.qpad) : nullptr;
  A.o = saved ? reinterpret_cast<float*>(sv + (int64_t)(kMlpIn0 + 4 * kMlpWidth) * A.qpad)
              : nullptr;
  const int64_t waves = (n_points + 31) / 32;
  const int64_t need = (waves + kFwdWaves - 1) / kFwdWaves;
  const int blocks = (int)(need < kFwdBlocks ? need : kFwdBlocks);
  hipLaunchKernelGGL(mlp_forward_kernel, dim3(blocks), dim3(kFwdWaves * 64), 0, s, A);
  return check_launch(fn);
}

rtc_status rtc_mlp_backward(const rtc_mlp* net, int64_t n_points, const float* dLdout,
                            const void* saved, float* dLdparams, void* ws, size_t ws_bytes,
                            void* stream) {
  const char* fn = "rtc_mlp_backward";
  RTC_REQUIRE(net && net->params, RTC_ERR_INVALID_ARG, "%s: net and net->params are required", fn);
  RTC_REQUIRE(net->n_freq == kMlpFreq && net->width == kMlpWidth && net->n_hidden == 4,
              RTC_ERR_UNSUPPORTED, "%s: this build implements n_freq 8, width 128, 4 hidden layers",
              fn);
  RTC_REQUIRE(n_points >= 0, RTC_ERR_SHAPE, "%s: n_points must be >= 0", fn);
  RTC_REQUIRE(dLdparams, RTC_ERR_INVALID_ARG, "%s: dLdparams is required", fn);
  hipStream_t s = as_stream(stream);
  if (n_points == 0) return zero_floats(dLdparams, kMlpParams, s, fn);
  RTC_REQUIRE(dLdout && saved, RTC_ERR_INVALID_ARG, "%s: dLdout and saved are required", fn);
  size_t need = rtc_mlp_workspace_size(n_points);
  RTC_REQUIRE(ws && ws_bytes >= need, RTC_ERR_WORKSPACE, "%s: workspace of %zu bytes required",
              fn, need);
  const int64_t qp = qpad_of(n_points);
  uint16_t* packed = reinterpret_cast<uint16_t*>(ws);
  float* part = reinterpret_cast<float*>(
      (reinterpret_cast<uintptr_t>(packed + kPackedElems) + 255) & ~(uintptr_t)255);
  hipLaunchKernelGGL(mlp_pack_kernel, dim3((kPackedElems + 255) / 256), dim3(256), 0, s,
                     net->params, packed);
  rtc_status st;
  if ((st = check_launch(fn)) != RTC_OK) return st;
  const uint16_t* sv = reinterpret_cast<const uint16_t*>(saved);
  MlpBwdArgs B;
  B.n_points = n_points;
  B.qpad = qp;
  B.dout = dLdout;
  B.packed = packed;
  B.x0 = reinterpret_cast<const bf16x8*>(sv);
  B.hs = reinterpret_cast<const bf16x8*>(sv + (int64_t)kMlpIn0 * qp);
  B.o = reinterpret_cast<const float*>(sv + (int64_t)(kMlpIn0 + 4 * kMlpWidth) * qp);
  B.part = part;
  const int64_t nstep = (n_points + kBwdPts - 1) / kBwdPts;
  const int nb = (int)(nstep < kMlpBwdBlocks ? nstep : kMlpBwdBlocks);
  hipLaunchKernelGGL(mlp_backward_kernel, dim3(nb), dim3(kBwdWaves * 64), 0, s, B);
  if ((st = check_launch(fn)) != RTC_OK) return st;
  hipLaunchKernelGGL(reduce_cols_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, part,
                     nb, kMlpParams, dLdparams);
  return check_launch(fn);
}

}  // extern "C"
