// Neural materials (Sec. III-D): positional encoding + MLP 51 -> 128 x 4
// (ReLU) -> 3, outputs eps_r = 1 + softplus, sigma = softplus, S = logistic,
// on the BF16 matrix cores with FP32 accumulation.
//
// Forward: one wave per 32 points.  Activations are the B operand of
// v_mfma_f32_32x32x16_bf16 (rows = neurons, columns = points): lane l holds
// point l%32 and K slice 8(l/32)..+7.  The accumulator of a 32-neuron tile
// holds, in register r of lane l, neuron 8(r/4) + 4(l/32) + r%4 of point
// l%32, so registers 8e..8e+7 of a tile are directly the next layer's
// K-block (tile, e) when the K order inside that block is the permutation
// kperm(c, h, j) = 32(c/2) + 16(c%2) + 8(j/4) + 4h + j%4 -- the weights are
// packed in that order, so activations never leave the registers.
//
// Backward: deltas run the same way through the transposed weights;
// weight gradients are a split-K product over points of feature-major BF16
// deltas and activations, reduced over slices in a fixed order.
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
constexpr int kMlpWaves = 4;
constexpr int kMlpSlices = 64;  // split-K slices for the weight gradients

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

RTC_DEV bf16x8 pack8(const float* v) {
  u32x4 w;
  w[0] = (uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
  w[1] = (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16);
  w[2] = (uint32_t)f2bf(v[4]) | ((uint32_t)f2bf(v[5]) << 16);
  w[3] = (uint32_t)f2bf(v[6]) | ((uint32_t)f2bf(v[7]) << 16);
  return __builtin_bit_cast(bf16x8, w);
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
  int64_t qpad;  // row stride of the feature-major saved arrays
  const float *px, *py, *pz;
  float cx, cy, cz, inv_ext;
  const float* prm;          // FP32 master parameters
  const uint16_t* packed;    // BF16 operands
  float* out;                // [3][n_points]
  // saved for the backward (feature-major, row stride qpad), or null
  uint16_t* x0;              // [64][qpad]
  uint16_t* hs;              // [4][128][qpad]  h1..h4
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

__global__ void __launch_bounds__(kMlpWaves * 64) mlp_forward_kernel(MlpArgs A) {
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5;
  const int pt = lane & 31;
  const int64_t q0 = ((int64_t)blockIdx.x * kMlpWaves + (threadIdx.x >> 6)) * 32;
  if (q0 >= A.n_points) return;
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
    if (A.x0 && valid) {
      const uint16_t* pv = reinterpret_cast<const uint16_t*>(&xin[c]);
#pragma unroll
      for (int j = 0; j < 8; ++j) A.x0[(int64_t)(16 * c + 8 * h + j) * A.qpad + q] = pv[j];
    }
  }
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    floatx16 acc[4];
    const uint16_t* W = A.packed + fw_off(l);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      acc[t] = floatx16{0};
#pragma unroll
      for (int c = 0; c < mlp_kb(l); ++c)
        acc[t] = mfma_bf16(load_op(W, (t * mlp_kb(l) + c) * 64 + lane), xin[c], acc[t]);
    }
    const float* b = A.prm + mlp_off_b(l);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      float v[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = fmaxf(acc[t][r] + b[32 * t + drow(r, h)], 0.0f);
      xin[2 * t] = pack8(v);
      xin[2 * t + 1] = pack8(v + 8);
      if (A.hs && valid) {
        const uint16_t* p0 = reinterpret_cast<const uint16_t*>(&xin[2 * t]);
        const uint16_t* p1 = reinterpret_cast<const uint16_t*>(&xin[2 * t + 1]);
        uint16_t* dst = A.hs + (int64_t)l * kMlpWidth * A.qpad;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          dst[(int64_t)(32 * t + drow(r, h)) * A.qpad + q] = p0[r];
          dst[(int64_t)(32 * t + drow(r + 8, h)) * A.qpad + q] = p1[r];
        }
      }
    }
  }
  floatx16 acc = floatx16{0};
  const uint16_t* W4 = A.packed + fw_off(4);
#pragma unroll
  for (int c = 0; c < 8; ++c) acc = mfma_bf16(load_op(W4, c * 64 + lane), xin[c], acc);
  if (h == 0 && valid) {
    const float* b4 = A.prm + mlp_off_b(4);
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

struct MlpBackArgs {
  int64_t n_points, qpad;
  const float* dout;        // [3][n_points] dL/d(eps_r, sigma, S)
  const uint16_t* packed;
  const uint16_t* hs;       // [4][128][qpad]
  const float* o;           // [3][qpad]
  uint16_t* dlt;            // [5][128][qpad]: delta of h1..h4 and (rows 0..2) of o
};

// Deltas: d_o = dL/do (output transforms), d_h4 = W4^T d_o * [h4 > 0], ...
__global__ void __launch_bounds__(kMlpWaves * 64) mlp_delta_kernel(MlpBackArgs A) {
  const int lane = threadIdx.x & 63;
  const int h = lane >> 5;
  const int pt = lane & 31;
  const int64_t q0 = ((int64_t)blockIdx.x * kMlpWaves + (threadIdx.x >> 6)) * 32;
  if (q0 >= A.qpad) return;
  const int64_t q = q0 + pt;
  const bool valid = q < A.n_points;
  // d_o in the accumulator layout of a 3-row tile: rows 0..2 live in lanes
  // h = 0, registers 0..2 (K-block 0, j = 0..2)
  float dv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (h == 0 && valid) {
    float o0 = A.o[q], o1 = A.o[A.qpad + q], o2 = A.o[2 * A.qpad + q];
    float s2 = sigmoidf(o2);
    dv[0] = A.dout[q] * sigmoidf(o0);                     // d eps/d o0
    dv[1] = A.dout[A.n_points + q] * sigmoidf(o1);        // d sigma/d o1
    dv[2] = A.dout[2 * A.n_points + q] * s2 * (1.0f - s2);  // d S/d o2
  }
  bf16x8 din[8];
  din[0] = pack8(dv);
  uint16_t* dst_o = A.dlt + 4 * (int64_t)kMlpWidth * A.qpad;
  {
    const uint16_t* p = reinterpret_cast<const uint16_t*>(&din[0]);
    if (h == 0) {
#pragma unroll
      for (int r = 0; r < 3; ++r) dst_o[(int64_t)r * A.qpad + q] = valid ? p[r] : 0;
    }
  }
#pragma unroll
  for (int l = 4; l >= 1; --l) {
    // d_h(l) = W_l^T d_(l+1) * relu'(h_l): rows = inputs of layer l
    const uint16_t* Wt = A.packed + bw_off(l);
    const uint16_t* hl = A.hs + (int64_t)(l - 1) * kMlpWidth * A.qpad;
    uint16_t* dst = A.dlt + (int64_t)(l - 1) * kMlpWidth * A.qpad;
    bf16x8 nxt[8];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      floatx16 acc = floatx16{0};
#pragma unroll
      for (int c = 0; c < bw_kb(l); ++c)
        acc = mfma_bf16(load_op(Wt, (t * bw_kb(l) + c) * 64 + lane), din[c], acc);
      float v[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int n = 32 * t + drow(r, h);
        uint16_t hb = valid ? hl[(int64_t)n * A.qpad + q] : 0;
        v[r] = (valid && bf2f(hb) > 0.0f) ? acc[r] : 0.0f;
      }
      nxt[2 * t] = pack8(v);
      nxt[2 * t + 1] = pack8(v + 8);
      const uint16_t* p0 = reinterpret_cast<const uint16_t*>(&nxt[2 * t]);
      const uint16_t* p1 = reinterpret_cast<const uint16_t*>(&nxt[2 * t + 1]);
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        dst[(int64_t)(32 * t + drow(r, h)) * A.qpad + q] = p0[r];
        dst[(int64_t)(32 * t + drow(r + 8, h)) * A.qpad + q] = p1[r];
      }
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) din[c] = nxt[c];
  }
}

struct MlpGradArgs {
  int64_t qpad;
  int64_t slice;  // points per slice (multiple of 16)
  const uint16_t* x0;   // [64][qpad]
  const uint16_t* hs;   // [4][128][qpad]
  const uint16_t* dlt;  // [5][128][qpad]
  float* part;          // [kMlpSlices][kMlpParams]
};

// One wave per (slice, layer, out tile, in tile): dW[n_out][n_in] =
// sum_points delta[n_out][q] x[n_in][q]; waves with in tile 0 also form
// db[n_out] = sum_points delta[n_out][q].
__global__ void __launch_bounds__(64) mlp_wgrad_kernel(MlpGradArgs A) {
  const int lane = threadIdx.x;
  const int h = lane >> 5;
  const int i = lane & 31;
  const int s = blockIdx.x;
  int pair = blockIdx.y;
  // enumerate (layer, out tile, in tile): layer 0: 4 x 2, layers 1-3: 4 x 4, layer 4: 1 x 4
  int l, to, ti;
  if (pair < 8) {
    l = 0;
    to = pair >> 1;
    ti = pair & 1;
  } else if (pair < 56) {
    l = 1 + (pair - 8) / 16;
    to = ((pair - 8) % 16) >> 2;
    ti = (pair - 8) & 3;
  } else {
    l = 4;
    to = 0;
    ti = pair - 56;
  }
  // delta of layer l's outputs: l = 0..3 -> d_h(l+1) rows 0..127, l = 4 -> d_o
  const uint16_t* D = A.dlt + (int64_t)(l == 4 ? 4 : l) * kMlpWidth * A.qpad;
  // inputs of layer l: x0 for l = 0, else h_l
  const uint16_t* X = l == 0 ? A.x0 : A.hs + (int64_t)(l - 1) * kMlpWidth * A.qpad;
  const int nrow = 32 * to + i;
  const int ncol = 32 * ti + i;
  const bool row_ok = nrow < mlp_nout(l);
  const int64_t p0 = (int64_t)s * A.slice;
  // the last slice is clipped at qpad (p0 and qpad are multiples of 16)
  const int64_t kend = p0 + A.slice <= A.qpad ? A.slice : A.qpad - p0;
  floatx16 acc = floatx16{0};
  floatx16 accb = floatx16{0};
  bf16x8 ones;
  {
    float o8[8] = {1, 1, 1, 1, 1, 1, 1, 1};
    ones = pack8(o8);
  }
  bf16x8 zero;
  {
    float z8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    zero = pack8(z8);
  }
  for (int64_t k = 0; k < kend; k += 16) {
    const int64_t pq = p0 + k + 8 * h;
    bf16x8 a = row_ok ? *reinterpret_cast<const bf16x8*>(D + (int64_t)nrow * A.qpad + pq) : zero;
    bf16x8 b = *reinterpret_cast<const bf16x8*>(X + (int64_t)ncol * A.qpad + pq);
    acc = mfma_bf16(a, b, acc);
    if (ti == 0) accb = mfma_bf16(a, ones, accb);
  }
  float* out = A.part + (int64_t)s * kMlpParams;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int no = 32 * to + drow(r, h);
    const int ni = 32 * ti + i;
    if (no < mlp_nout(l) && ni < mlp_nin(l)) out[mlp_off_w(l) + no * mlp_nin(l) + ni] = acc[r];
    if (ti == 0 && i == 0 && no < mlp_nout(l)) out[mlp_off_b(l) + no] = accb[r];
  }
}

// Zero the padded point columns [n, qpad) of the saved arrays (the split-K
// weight-gradient products read them).
__global__ void mlp_zero_tail_kernel(uint16_t* sv, int64_t n, int64_t qpad) {
  const int64_t tail = qpad - n;
  const int64_t rows16 = kMlpIn0 + 4 * kMlpWidth;
  const int64_t total = (rows16 + 6) * tail;  // 6 = the three FP32 rows as 16-bit halves
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / tail, c = n + i % tail;
    if (r < rows16) {
      sv[r * qpad + c] = 0;
    } else {
      float* o = reinterpret_cast<float*>(sv + rows16 * qpad);
      const int64_t fr = (r - rows16) >> 1;
      if (((r - rows16) & 1) == 0) o[fr * qpad + c] = 0.0f;
    }
  }
}

// Sum the slice partials column-wise in slice order (FP64).
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
  int64_t qp = qpad_of(n_points);
  return (size_t)kPackedElems * sizeof(uint16_t) + (size_t)5 * kMlpWidth * qp * sizeof(uint16_t) +
         (size_t)kMlpSlices * kMlpParams * sizeof(float) + 256;
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
  A.x0 = saved ? sv : nullptr;
  A.hs = saved ? sv + (int64_t)kMlpIn0 * A.qpad : nullptr;
  A.o = saved ? reinterpret_cast<float*>(sv + (int64_t)(kMlpIn0 + 4 * kMlpWidth) * A.qpad)
              : nullptr;
  if (saved && A.qpad > n_points) {
    // padded point columns must hold zeros for the split-K products
    hipLaunchKernelGGL(mlp_zero_tail_kernel, dim3(256), dim3(256), 0, s, sv, n_points, A.qpad);
    if ((st = check_launch(fn)) != RTC_OK) return st;
  }
  int64_t waves = (n_points + 31) / 32;
  int64_t blocks = (waves + kMlpWaves - 1) / kMlpWaves;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)blocks), dim3(kMlpWaves * 64), 0, s, A);
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
  uint16_t* dlt = packed + kPackedElems;
  float* part = reinterpret_cast<float*>(
      (reinterpret_cast<uintptr_t>(dlt + (int64_t)5 * kMlpWidth * qp) + 255) & ~(uintptr_t)255);
  hipLaunchKernelGGL(mlp_pack_kernel, dim3((kPackedElems + 255) / 256), dim3(256), 0, s,
                     net->params, packed);
  rtc_status st;
  if ((st = check_launch(fn)) != RTC_OK) return st;
  const uint16_t* sv = reinterpret_cast<const uint16_t*>(saved);
  MlpBackArgs B;
  B.n_points = n_points;
  B.qpad = qp;
  B.dout = dLdout;
  B.packed = packed;
  B.hs = sv + (int64_t)kMlpIn0 * qp;
  B.o = reinterpret_cast<const float*>(sv + (int64_t)(kMlpIn0 + 4 * kMlpWidth) * qp);
  B.dlt = dlt;
  int64_t waves = qp / 32;
  hipLaunchKernelGGL(mlp_delta_kernel, dim3((unsigned)((waves + kMlpWaves - 1) / kMlpWaves)),
                     dim3(kMlpWaves * 64), 0, s, B);
  if ((st = check_launch(fn)) != RTC_OK) return st;
  MlpGradArgs G;
  G.qpad = qp;
  G.slice = qp / kMlpSlices;  // qp is a multiple of 256, so slices are multiples of 4 ...
  G.slice = (G.slice + 15) / 16 * 16;
  G.x0 = sv;
  G.hs = B.hs;
  G.dlt = dlt;
  G.part = part;
  // slices must not run past qp: the last ones are clipped by construction
  int n_slices = (int)((qp + G.slice - 1) / G.slice);
  RTC_REQUIRE(n_slices <= kMlpSlices, RTC_ERR_RANGE, "%s: internal slicing error", fn);
  if (n_slices < kMlpSlices) {
    // unused slices contribute zero
    if ((st = zero_floats(part + (int64_t)n_slices * kMlpParams,
                          (int64_t)(kMlpSlices - n_slices) * kMlpParams, s, fn)) != RTC_OK)
      return st;
  }
  hipLaunchKernelGGL(mlp_wgrad_kernel, dim3(n_slices, 60), dim3(64), 0, s, G);
  if ((st = check_launch(fn)) != RTC_OK) return st;
  hipLaunchKernelGGL(reduce_cols_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, part,
                     kMlpSlices, kMlpParams, dLdparams);
  return check_launch(fn);
}

}  // extern "C"
