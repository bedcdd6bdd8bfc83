// The learned pose warm start: a BF16 convolutional network on the matrix cores.
//
// Every layer, forward and backward, is one GEMM C[M][N] = sum_k A(m, k) B(k, n)
// in a single kernel template: 256 threads (4 waves in a 2 x 2 grid), a BM x BN
// tile of C chosen per layer, K in steps of 32.  Convolutions are implicit GEMMs
// (no im2col buffer): activations are stored channels-last, [frame][y][x][c], and
// the weights have BF16 copies permuted so that the reduction index runs along
// channels, so every operand fetch is one aligned 16-byte load of 8 consecutive
// BF16 values -- 8 consecutive k of one row ("k-chunks"), or, for the weight
// gradients, whose reduction runs over pixels, 8 consecutive rows of one k
// ("row chunks", read back from LDS with the transposing LDS read).  Operands are
// fetched through buffer resources, whose range check supplies the zero padding.  The
// chunks of the step after next are loaded into registers while the matrix cores
// work on the current step from one of two LDS buffers (one barrier per step).  Each
// wave issues (BM/32) x (BN/32) v_mfma_f32_16x16x32_bf16 per step on its quarter of
// the tile, accumulating in FP32.  The layer's epilogue adds the bias, applies ReLU
// (or, in the backward, the ReLU mask of the layer's input), rounds to BF16 and
// stores 4 channels at once; weight gradients go to FP32 partial sums over split-K
// slices that one kernel per backward pass adds in a fixed order (deterministic) and
// maps back to the parameter layout, a constant-one column of B giving the bias
// gradient in the same GEMM.
//
//   layer              M        N              K
//   conv forward       Co       B OH OW        k k Ci    (the 4-channel input: 5 x 3 pairs x 8)
//   conv input grad    Ci       B H W / 4      taps Co   (one launch per output parity class:
//                                                         only the stride-2 taps that reach it)
//   conv weight grad   Co       k k Ci + 1     B OH OW   (split-K; the input layer 120 + 1)
//   fc forward         O        B              I
//   fc input grad      I        B              O
//   fc weight grad     O        I + 1          B         (split-K)
//
// In training, fc2 (256 -> 6) runs as one kernel of its own: forward, squared error,
// loss gradient, input and weight gradients.  In the proposal (batch 1) it runs in
// the closing launch, with the addition of fc1's split-K slices and T_0 = Exp(tau) T.
//
// MFMA operand layout used (16 x 16 x 32, wave64): lane l supplies row l % 16 of A
// and column l % 16 of B, each with the 8 consecutive k of group l / 16; the FP32
// result holds rows 4 (l / 16) + r, r < 4, of column l % 16.  (A and B only need
// the same k assignment, so the pairing of k groups with lanes cannot change a
// result.)
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>

#include "../../include/gs2d_warm.h"
#include "gs2d_internal.h"
#include "pose_step.h"

namespace gs2d {
namespace ws {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kBK = 32, kPad = 8, kThreads = 256, kStages = 2;
constexpr uint16_t kOne = 0x3F80;  // bfloat16 1.0
// The input layer's activations are stored with their 4 channels; its reduction index
// runs (ky, kx pair, kx within the pair, c), so 8 consecutive k are 2 horizontally
// adjacent pixels of one row (one 16-byte load), the 5 columns of a 5 x 5 kernel
// taking 3 pairs (the sixth column has zero weights).
constexpr int kInC = 4, kInPairs = 3, kInK = 5 * kInPairs * 2 * kInC;  // 120

// Round to the nearest bfloat16, ties to even (the hardware conversion,
// v_cvt_pk_bf16_f32, in the default round-to-nearest-even mode with FP32 denormals
// kept; NaN stays NaN).
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint16_t to_bf16(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ uint32_t to_bf16x2(float lo, float hi) {
  return __builtin_bit_cast(uint32_t, bf16x2{(__bf16)lo, (__bf16)hi});
}
// Post-ReLU activations are positive exactly when the sign bit is clear and they are not zero.
__device__ __forceinline__ bool positive(uint16_t h) { return h != 0 && !(h & 0x8000u); }
__device__ __forceinline__ float relu(float v) { return v > 0.f ? v : 0.f; }
// 4 consecutive BF16 values: y[0..3] = bf16(relu(v + bias)) (8-byte aligned destination).
__device__ __forceinline__ void store_relu4(uint16_t* y, const float* bias, f32x4 v) {
  const float4 b = *reinterpret_cast<const float4*>(bias);
  *reinterpret_cast<uint2*>(y) = uint2{to_bf16x2(relu(v[0] + b.x), relu(v[1] + b.y)),
                                       to_bf16x2(relu(v[2] + b.z), relu(v[3] + b.w))};
}
// 4 consecutive BF16 input gradients masked by the ReLU of the input x (8-byte aligned).
__device__ __forceinline__ void store_masked4(uint16_t* gx, const uint16_t* x, f32x4 v) {
  const uint2 xv = *reinterpret_cast<const uint2*>(x);
  const uint16_t x0 = (uint16_t)xv.x, x1 = (uint16_t)(xv.x >> 16), x2 = (uint16_t)xv.y, x3 = (uint16_t)(xv.y >> 16);
  *reinterpret_cast<uint2*>(gx) = uint2{to_bf16x2(positive(x0) ? v[0] : 0.f, positive(x1) ? v[1] : 0.f),
                                        to_bf16x2(positive(x2) ? v[2] : 0.f, positive(x3) ? v[3] : 0.f)};
}

// The workgroup's extent of a plain GEMM, blockIdx.z selecting a split-K slice of ks steps.
struct Dims {
  int M = 0, N = 0, K = 0, ks = 0;
  __device__ void dims(int& m, int& n, int& kb, int& ke) const {
    m = M;
    n = N;
    kb = blockIdx.z * ks;
    ke = min(K, kb + ks);
  }
};

// An operand op supplies, for its A and B, a per-chunk set-up and 16-byte chunks of 8
// BF16 values, zero unless `ok` (the chunk lies inside the matrix).  A k-chunk operand
// (kAk / kBk) gives the 8 consecutive k of one row: set-up a_prep(row), chunk
// a(prep, k, ok) (K % 8 == 0).  A row-chunk operand gives 8 consecutive rows at one
// k: set-up a_prep(first row), chunk a(prep, k, ok) (M % 8 == 0).
//
// k-chunks are stored in LDS row-major ([row][k]) and read as fragments with one
// 16-byte read.  Row chunks are stored as loaded ([k][row]) and read with two
// transposing reads (ds_read_b64_tr_b16): in each group of 16 lanes, lane q reads 8
// bytes (4 elements) of LDS row kb + q / 4 from column m0 + 4 (q % 4), so the group
// reads 16 columns of 4 rows, and lane i receives element i of each of the 4 rows --
// operand row m0 + i at k = kb .. kb + 3, the fragment's first or second 4 k.
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
#define GS2D_LDS __attribute__((address_space(3)))
__device__ __forceinline__ bf16x8 tr_fragment(const uint16_t* p0, const uint16_t* p1) {
  const s16x4 a = __builtin_amdgcn_ds_read_tr16_b64_v4i16((GS2D_LDS s16x4*)(p0));
  const s16x4 b = __builtin_amdgcn_ds_read_tr16_b64_v4i16((GS2D_LDS s16x4*)(p1));
  return __builtin_bit_cast(bf16x8, __builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7));
}

template <class Op, int BM, int BN>
__global__ __launch_bounds__(kThreads) void gemm_kernel(Op op) {
  constexpr int FM = BM / 32, FN = BN / 32;  // 16 x 16 blocks per wave
  constexpr int CA = BM * kBK / 8, CB = BN * kBK / 8;  // chunks per step
  constexpr int NA = (CA + kThreads - 1) / kThreads, NB = (CB + kThreads - 1) / kThreads;
  constexpr int RA = Op::kAk ? kBK / 8 : BM / 8, RB = Op::kBk ? kBK / 8 : BN / 8;
  // LDS: k-chunk operands [rows][kBK + 8], row-chunk operands [kBK][rows + 16] (the
  // row pitch puts the 4 rows of a transposing read in distinct banks)
  constexpr int LA = Op::kAk ? BM : kBK, PA = Op::kAk ? kBK + kPad : BM + 16;
  constexpr int LB = Op::kBk ? BN : kBK, PB = Op::kBk ? kBK + kPad : BN + 16;
  __shared__ __attribute__((aligned(16))) uint16_t As[2][LA][PA];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][LB][PB];
  int M, N, kb, ke;
  op.dims(M, N, kb, ke);
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  if (m0 >= M || n0 >= N) return;  // uniform over the workgroup
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * (BN / 2);
  const int li = lane & 15, g = lane >> 4;

  // chunk c of a step: a k-chunk c -> (row c / R, k 8 (c % R)); a row chunk c -> (rows
  // 8 (c % R) .., k c / R)
  typename Op::APrep ap[NA];
  typename Op::BPrep bp[NB];
  int ar[NA], ak[NA], br[NB], bk[NB];
  bool aon[NA], bon[NB];
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    const int c = t + i * kThreads;
    ar[i] = Op::kAk ? c / RA : (c % RA) * 8;
    ak[i] = Op::kAk ? (c % RA) * 8 : c / RA;
    aon[i] = c < CA && m0 + ar[i] < M;
    ap[i] = op.a_prep(aon[i] ? m0 + ar[i] : m0);
  }
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int c = t + i * kThreads;
    br[i] = Op::kBk ? c / RB : (c % RB) * 8;
    bk[i] = Op::kBk ? (c % RB) * 8 : c / RB;
    bon[i] = c < CB && n0 + br[i] < N;
    bp[i] = op.b_prep(bon[i] ? n0 + br[i] : n0);
  }
  // a ring of kStages register stages: the chunks of step s + kStages are requested
  // while step s is multiplied, so a step waits on memory only if kStages steps of
  // products took less than one round trip
  uint4 ra[kStages][NA], rb[kStages][NB];
  auto fetch = [&](uint4* xa, uint4* xb, int k0) {
#pragma unroll
    for (int i = 0; i < NA; ++i) xa[i] = op.a(ap[i], k0 + ak[i], aon[i] && k0 + ak[i] < ke);
#pragma unroll
    for (int i = 0; i < NB; ++i) xb[i] = op.b(bp[i], k0 + bk[i], bon[i] && k0 + bk[i] < ke);
  };
  auto stash = [&](const uint4* xa, const uint4* xb, int buf) {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      if (t + i * kThreads >= CA) continue;
      if constexpr (Op::kAk)
        *reinterpret_cast<uint4*>(&As[buf][ar[i]][ak[i]]) = xa[i];
      else
        *reinterpret_cast<uint4*>(&As[buf][ak[i]][ar[i]]) = xa[i];
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      if (t + i * kThreads >= CB) continue;
      if constexpr (Op::kBk)
        *reinterpret_cast<uint4*>(&Bs[buf][br[i]][bk[i]]) = xb[i];
      else
        *reinterpret_cast<uint4*>(&Bs[buf][bk[i]][br[i]]) = xb[i];
    }
  };

  f32x4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  auto multiply = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < kBK; kk += 32) {
      bf16x8 fa[FM], fb[FN];
      const int kq = kk + g * 8 + (li >> 2), mq = 4 * (li & 3);  // a transposing read's lane address
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        if constexpr (Op::kAk)
          fa[i] = *reinterpret_cast<const bf16x8*>(&As[buf][wm + i * 16 + li][kk + g * 8]);
        else
          fa[i] = tr_fragment(&As[buf][kq][wm + i * 16 + mq], &As[buf][kq + 4][wm + i * 16 + mq]);
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        if constexpr (Op::kBk)
          fb[j] = *reinterpret_cast<const bf16x8*>(&Bs[buf][wn + j * 16 + li][kk + g * 8]);
        else
          fb[j] = tr_fragment(&Bs[buf][kq][wn + j * 16 + mq], &Bs[buf][kq + 4][wn + j * 16 + mq]);
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
    }
  };
  const int steps = ke > kb ? (ke - kb + kBK - 1) / kBK : 0;
#pragma unroll
  for (int d = 0; d < kStages; ++d)
    if (d < steps) fetch(ra[d], rb[d], kb + d * kBK);
  for (int s0 = 0; s0 < steps; s0 += kStages) {
#pragma unroll
    for (int d = 0; d < kStages; ++d) {
      const int s = s0 + d;
      if (s >= steps) break;
      // LDS buffer s & 1 was last read at step s - 2, before the previous barrier
      stash(ra[d], rb[d], s & 1);
      __syncthreads();
      if (s + kStages < steps) fetch(ra[d], rb[d], kb + (s + kStages) * kBK);
      multiply(s & 1);
    }
  }
  // each lane holds rows mb .. mb + 3 of column n of every block: one 4-row store each
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int n = n0 + wn + j * 16 + li, mb = m0 + wm + i * 16 + g * 4;
      if (n < N && mb < M) op.store4(mb, n, acc[i][j], min(4, M - mb));
    }
}

// Operand sources are read through buffer resources with 32-bit byte offsets: a
// chunk outside the matrix or in the zero padding gets the offset kOOB, which the
// hardware's range check turns into zeros (no branch, no select).  Every source is
// smaller than 2 GiB (the largest, an activation array at the largest batch, is
// about 300 MiB).
typedef __amdgpu_buffer_rsrc_t Rsrc;
constexpr uint32_t kOOB = 0x80000000u;
__device__ __forceinline__ Rsrc rsrc(const void* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, 0x7FFFFFFF, 0x00020000);
}
__device__ __forceinline__ uint4 bload(Rsrc r, uint32_t off) {
  return __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}

struct OffPrep {
  uint32_t off;  // byte offset of the row (or of the first of 8 rows)
};

// n / d for 0 <= n < 2^23 by a multiply and a shift: m = floor(2^(32 + l) / d) + 1 with
// 2^l >= d, split as m = mh 2^32 + ml; n m / 2^(32 + l) exceeds n / d by less than
// n / 2^(32 + l) < 1 / d, so its floor is floor(n / d).
struct FastDiv {
  uint32_t ml, mh;
  int l;
  __device__ int div(int n) const {
    return (int)((__umulhi((uint32_t)n, ml) + (mh ? (uint32_t)n : 0u)) >> l);
  }
};

// y = bf16(relu(conv(x, w) + bias)), stride 2, zero padding KS / 2:
// M = co, N = B OH OW, K = KS KS cp (k = (ky, kx, c), c fastest).
template <int KS>
struct ConvFwd : Dims {
  static constexpr bool kAk = true, kBk = true;
  const uint16_t* w;  // [co][KS][KS][cp]
  const float* bias;
  const uint16_t* x;  // [B][H][W][cp]
  uint16_t* y;        // [B][OH][OW][co]
  int H, W, OH, OW, lc;  // lc = log2 ci
  FastDiv by_ohw, by_ow;
  using APrep = OffPrep;
  struct BPrep {
    uint32_t off;  // the frame
    int iy0, ix0;
  };
  __device__ APrep a_prep(int m) const { return {(uint32_t)m * (uint32_t)K * 2u}; }
  __device__ uint4 a(const APrep& q, int k, bool ok) const { return bload(rsrc(w), ok ? q.off + 2u * k : kOOB); }
  __device__ BPrep b_prep(int n) const {
    const int b = by_ohw.div(n), r = n - b * (OH * OW), oy = by_ow.div(r), ox = r - oy * OW;
    return {((uint32_t)(b * H * W) << lc) * 2u, 2 * oy - KS / 2, 2 * ox - KS / 2};
  }
  __device__ uint4 b(const BPrep& q, int k, bool ok) const {
    const int tap = k >> lc, c = k & ((1 << lc) - 1), ky = tap / KS, kx = tap - ky * KS;
    const int iy = q.iy0 + ky, ix = q.ix0 + kx;
    ok = ok && (unsigned)iy < (unsigned)H && (unsigned)ix < (unsigned)W;
    return bload(rsrc(x), ok ? q.off + 2u * (((uint32_t)(iy * W + ix) << lc) + c) : kOOB);
  }
  __device__ void store(int m, int n, float v) const { y[(size_t)n * M + m] = to_bf16(relu(v + bias[m])); }
  __device__ void store4(int m, int n, f32x4 v, int rows) const {  // co % 4 == 0: rows == 4
    store_relu4(y + (size_t)n * M + m, bias + m, v);
  }
};

// The input layer, 5 x 5, stride 2, zero padding 2, over the 4-channel input:
// y = bf16(relu(conv(x, w) + bias)); M = co, N = B OH OW, K = 120 (kInK).
struct ConvFwdIn : Dims {
  static constexpr bool kAk = true, kBk = true;
  const uint16_t* w;  // [co][5][3][2][4]
  const float* bias;
  const uint16_t* x;  // [B][H][W][4]
  uint16_t* y;        // [B][OH][OW][co]
  int H, W, OH, OW;
  FastDiv by_ohw, by_ow;
  using APrep = OffPrep;
  struct BPrep {
    uint32_t off;  // the frame
    int iy0, ix0;
  };
  __device__ APrep a_prep(int m) const { return {(uint32_t)m * (uint32_t)K * 2u}; }
  __device__ uint4 a(const APrep& q, int k, bool ok) const { return bload(rsrc(w), ok ? q.off + 2u * k : kOOB); }
  __device__ BPrep b_prep(int n) const {
    const int b = by_ohw.div(n), r = n - b * (OH * OW), oy = by_ow.div(r), ox = r - oy * OW;
    return {(uint32_t)(b * H * W * kInC) * 2u, 2 * oy - 2, 2 * ox - 2};
  }
  // k = 8 (3 ky + pair): pixels (iy0 + ky, ix0 + 2 pair + 0, 1); ix is even and W
  // even, so both lie inside or both outside
  __device__ uint4 b(const BPrep& q, int k, bool ok) const {
    const int r = k >> 3, ky = r / kInPairs, pr = r - ky * kInPairs;
    const int iy = q.iy0 + ky, ix = q.ix0 + 2 * pr;
    ok = ok && (unsigned)iy < (unsigned)H && (unsigned)ix < (unsigned)W;
    return bload(rsrc(x), ok ? q.off + 2u * (uint32_t)((iy * W + ix) * kInC) : kOOB);
  }
  __device__ void store(int m, int n, float v) const { y[(size_t)n * M + m] = to_bf16(relu(v + bias[m])); }
  __device__ void store4(int m, int n, f32x4 v, int rows) const {  // co % 4 == 0: rows == 4
    store_relu4(y + (size_t)n * M + m, bias + m, v);
  }
};

// Weight and bias gradient of the input layer, one split-K slice per blockIdx.z:
// part[z][co][120 + 1] = sum over pixels n of gy[n][co] [x pair patch | 1].
struct ConvBwdWeightIn : Dims {
  static constexpr bool kAk = false, kBk = false;
  const uint16_t* gy;  // [B][OH][OW][co]
  const uint16_t* x;   // [B][H][W][4]
  float* part;
  int H, W, OH, OW;
  FastDiv by_ohw, by_ow;
  using APrep = OffPrep;
  struct BPrep {
    int dy, dx;
    bool bias;
  };
  __device__ APrep a_prep(int m8) const { return {(uint32_t)m8 * 2u}; }
  __device__ uint4 a(const APrep& q, int k, bool ok) const {
    return bload(rsrc(gy), ok ? q.off + 2u * (uint32_t)(k * M) : kOOB);
  }
  __device__ BPrep b_prep(int n8) const {
    const int r = n8 >> 3, ky = r / kInPairs, pr = r - ky * kInPairs;
    return {ky - 2, 2 * pr - 2, n8 == N - 1};
  }
  __device__ uint4 b(const BPrep& q, int k, bool ok) const {
    if (q.bias) return ok ? uint4{kOne, 0u, 0u, 0u} : uint4{0u, 0u, 0u, 0u};
    const int b = by_ohw.div(k), r = k - b * (OH * OW), oy = by_ow.div(r), ox = r - oy * OW;
    const int iy = 2 * oy + q.dy, ix = 2 * ox + q.dx;
    ok = ok && (unsigned)iy < (unsigned)H && (unsigned)ix < (unsigned)W;
    return bload(rsrc(x), ok ? 2u * (uint32_t)(((b * H + iy) * W + ix) * kInC) : kOOB);
  }
  __device__ void store4(int m, int n, f32x4 v, int rows) const {
    float* p = part + ((size_t)blockIdx.z * M + m) * N + n;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (q < rows) p[(size_t)q * N] = v[q];
  }
};

// Input gradient of a 3 x 3 stride-2 convolution, masked by the ReLU of its input:
// gx = bf16(conv^T(gy, w) [x > 0]).  Workgroup z = the parity class (iy % 2, ix % 2)
// of the input pixels it computes: an even row is reached only by tap ky = 1 (from
// output row iy / 2), an odd one by ky = 0 and 2 (output rows (iy + 1) / 2 and
// (iy - 1) / 2), and likewise for columns.  M = ci, N = B Hc Wc (the class's pixels),
// K = (taps in y) (taps in x) co (k = (tap, o), o fastest).
struct ConvBwdData {
  static constexpr bool kAk = true, kBk = true;
  const uint16_t* wd;  // [ci][3][3][co]
  const uint16_t* gy;  // [B][OH][OW][co]
  const uint16_t* x;   // [B][H][W][ci], the layer's input (post-ReLU)
  uint16_t* gx;        // [B][H][W][ci]
  int Bn, ci, co, lco, H, W, OH, OW;
  FastDiv by_per[4], by_wc[4];  // per class: its pixels per frame, its columns
  using APrep = OffPrep;
  struct BPrep {
    uint32_t off;  // the frame
    int jy, jx;
  };
  __device__ int py() const { return blockIdx.z >> 1; }
  __device__ int px() const { return blockIdx.z & 1; }
  __device__ void dims(int& m, int& n, int& kb, int& ke) const {
    m = ci;
    n = Bn * ((H - py() + 1) >> 1) * ((W - px() + 1) >> 1);
    kb = 0;
    ke = ((1 + py()) * (1 + px())) << lco;
  }
  // tap t of the class -> (ty, tx); t = ty (taps in x) + tx
  __device__ void tap(int t, int& ty, int& tx) const {
    ty = px() ? t >> 1 : t;
    tx = px() ? t & 1 : 0;
  }
  __device__ APrep a_prep(int m) const { return {(uint32_t)m * 9u * (uint32_t)co * 2u}; }
  __device__ uint4 a(const APrep& q, int k, bool ok) const {
    int ty, tx;
    tap(k >> lco, ty, tx);
    const int ky = py() ? 2 * ty : 1, kx = px() ? 2 * tx : 1;
    return bload(rsrc(wd), ok ? q.off + 2u * (uint32_t)((ky * 3 + kx) * co + (k & (co - 1))) : kOOB);
  }
  // n -> (frame, class row, class column)
  __device__ void split(int n, int& b, int& jy, int& jx) const {
    const int Hc = (H - py() + 1) >> 1, Wc = (W - px() + 1) >> 1;
    b = by_per[blockIdx.z].div(n);
    const int r = n - b * (Hc * Wc);
    jy = by_wc[blockIdx.z].div(r);
    jx = r - jy * Wc;
  }
  __device__ BPrep b_prep(int n) const {
    int b, jy, jx;
    split(n, b, jy, jx);
    return {(uint32_t)(b * OH * OW * co) * 2u, jy, jx};
  }
  __device__ uint4 b(const BPrep& q, int k, bool ok) const {
    int ty, tx;
    tap(k >> lco, ty, tx);
    const int oy = py() ? q.jy + 1 - ty : q.jy, ox = px() ? q.jx + 1 - tx : q.jx;
    ok = ok && oy < OH && ox < OW;
    return bload(rsrc(gy), ok ? q.off + 2u * (uint32_t)((oy * OW + ox) * co + (k & (co - 1))) : kOOB);
  }
  __device__ void store4(int m, int n, f32x4 v, int rows) const {  // ci % 4 == 0: rows == 4
    int b, jy, jx;
    split(n, b, jy, jx);
    const size_t idx = (((size_t)b * H + 2 * jy + py()) * W + 2 * jx + px()) * ci + m;
    store_masked4(gx + idx, x + idx, v);
  }
};

// Weight and bias gradient of a convolution, one split-K slice per blockIdx.z:
// part[z][co][KS KS cp + 1] = sum over pixels n of gy[n][co] [x patch (ky, kx, c) | 1].
template <int KS>
struct ConvBwdWeight : Dims {
  static constexpr bool kAk = false, kBk = false;
  const uint16_t* gy;  // [B][OH][OW][co]
  const uint16_t* x;   // [B][H][W][cp]
  float* part;
  int H, W, OH, OW, lc;
  FastDiv by_ohw, by_ow;
  using APrep = OffPrep;
  struct BPrep {
    int dy, dx, c;
    bool bias;
  };
  __device__ APrep a_prep(int m8) const { return {(uint32_t)m8 * 2u}; }
  __device__ uint4 a(const APrep& q, int k, bool ok) const {
    return bload(rsrc(gy), ok ? q.off + 2u * (uint32_t)(k * M) : kOOB);
  }
  __device__ BPrep b_prep(int n8) const {
    const int tap = n8 >> lc, ky = tap / KS, kx = tap - ky * KS;
    return {ky - KS / 2, kx - KS / 2, n8 & ((1 << lc) - 1), n8 == N - 1};
  }
  // pixel k = (frame, oy, ox)
  __device__ uint4 b(const BPrep& q, int k, bool ok) const {
    if (q.bias) return ok ? uint4{kOne, 0u, 0u, 0u} : uint4{0u, 0u, 0u, 0u};
    const int b = by_ohw.div(k), r = k - b * (OH * OW), oy = by_ow.div(r), ox = r - oy * OW;
    const int iy = 2 * oy + q.dy, ix = 2 * ox + q.dx;
    ok = ok && (unsigned)iy < (unsigned)H && (unsigned)ix < (unsigned)W;
    return bload(rsrc(x), ok ? 2u * (((uint32_t)((b * H + iy) * W + ix) << lc) + q.c) : kOOB);
  }
  __device__ void store4(int m, int n, f32x4 v, int rows) const {
    float* p = part + ((size_t)blockIdx.z * M + m) * N + n;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (q < rows) p[(size_t)q * N] = v[q];
  }
};

// Fully connected forward: y[b][o] = sum_i w[o][i] x[b][i] + bias[o]; M = O, N = B, K = I.
struct FcFwd : Dims {
  static constexpr bool kAk = true, kBk = true;
  const uint16_t* w;  // [O][I]
  const float* bias;
  const uint16_t* x;  // [B][I]
  uint16_t* y;        // ReLU + bf16 (hidden layer), or
  float* yf;          // FP32, no ReLU (output layer)
  using APrep = OffPrep;
  using BPrep = OffPrep;
  __device__ APrep a_prep(int m) const { return {(uint32_t)m * (uint32_t)K * 2u}; }
  __device__ uint4 a(const APrep& q, int k, bool ok) const { return bload(rsrc(w), ok ? q.off + 2u * k : kOOB); }
  __device__ BPrep b_prep(int n) const { return {(uint32_t)n * (uint32_t)K * 2u}; }
  __device__ uint4 b(const BPrep& q, int k, bool ok) const { return bload(rsrc(x), ok ? q.off + 2u * k : kOOB); }
  __device__ void store(int m, int n, float v) const {
    v += bias[m];
    if (yf)
      yf[(size_t)n * M + m] = v;
    else
      y[(size_t)n * M + m] = to_bf16(relu(v));
  }
  __device__ void store4(int m, int n, f32x4 v, int rows) const {
    if (!yf && rows == 4) {
      store_relu4(y + (size_t)n * M + m, bias + m, v);
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q < rows) store(m + q, n, v[q]);
    }
  }
};

// Fully connected input gradient, masked by the ReLU of the input:
// gx[b][i] = bf16(sum_o w[o][i] gy[b][o] [x > 0]); M = I, N = B, K = O.
struct FcBwdData : Dims {
  static constexpr bool kAk = true, kBk = true;
  const uint16_t* wt;  // [I][O]
  const uint16_t* gy;  // [B][O]
  const uint16_t* x;   // [B][I]
  uint16_t* gx;
  using APrep = OffPrep;
  using BPrep = OffPrep;
  __device__ APrep a_prep(int m) const { return {(uint32_t)m * (uint32_t)K * 2u}; }
  __device__ uint4 a(const APrep& q, int k, bool ok) const { return bload(rsrc(wt), ok ? q.off + 2u * k : kOOB); }
  __device__ BPrep b_prep(int n) const { return {(uint32_t)n * (uint32_t)K * 2u}; }
  __device__ uint4 b(const BPrep& q, int k, bool ok) const { return bload(rsrc(gy), ok ? q.off + 2u * k : kOOB); }
  __device__ void store4(int m, int n, f32x4 v, int rows) const {  // I % 4 == 0: rows == 4
    const size_t idx = (size_t)n * M + m;
    store_masked4(gx + idx, x + idx, v);
  }
};

// Fully connected weight and bias gradient: part[z][o][I + 1] = sum_b gy[b][o] [x[b] | 1];
// M = O, N = I + 1, K = B.
struct FcBwdWeight : Dims {
  static constexpr bool kAk = false, kBk = false;
  const uint16_t* gy;  // [B][O]
  const uint16_t* x;   // [B][I]
  float* part;
  using APrep = OffPrep;
  struct BPrep {
    uint32_t off;
    bool bias;
  };
  __device__ APrep a_prep(int m8) const { return {(uint32_t)m8 * 2u}; }
  __device__ uint4 a(const APrep& q, int k, bool ok) const {
    return bload(rsrc(gy), ok ? q.off + 2u * (uint32_t)(k * M) : kOOB);
  }
  __device__ BPrep b_prep(int n8) const { return {(uint32_t)n8 * 2u, n8 == N - 1}; }
  __device__ uint4 b(const BPrep& q, int k, bool ok) const {
    if (q.bias) return ok ? uint4{kOne, 0u, 0u, 0u} : uint4{0u, 0u, 0u, 0u};
    return bload(rsrc(x), ok ? q.off + 2u * (uint32_t)(k * (N - 1)) : kOOB);
  }
  __device__ void store4(int m, int n, f32x4 v, int rows) const {
    float* p = part + ((size_t)blockIdx.z * M + m) * N + n;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (q < rows) p[(size_t)q * N] = v[q];
  }
};

// A forward layer with few output tiles (small batches) and a long reduction: each
// split-K slice writes FP32 partial sums, and a second kernel adds them in slice
// order and applies the layer's own epilogue (bias, ReLU, rounding) to the total.
// (Letting the last of a tile's workgroups add them instead needs device-scope fences,
// which write back the L2 and were measured several times slower.)
template <class Op>
struct SplitPart : Op {
  float* part;
  __device__ void store4(int m, int n, f32x4 v, int rows) const {
    float* p = part + ((size_t)blockIdx.z * this->M + m) * this->N + n;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (q < rows) p[(size_t)q * this->N] = v[q];
  }
};

// The slices are loaded 16 at a time, all 16 loads issued before the first addition
// (loads past the S M N floats of the partials return 0 and are not added).
template <class Op>
__global__ void split_finish_kernel(Op op, const float* __restrict__ part, int S) {
  const int M = op.M, N = op.N;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M * N) return;
  const Rsrc r = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(part), (short)0, 4 * S * M * N, 0x00020000);
  float v = 0.f;
  for (int z0 = 0; z0 < S; z0 += 16) {
    float q[16];
#pragma unroll
    for (int u = 0; u < 16; ++u)
      q[u] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, 4u * (uint32_t)((z0 + u) * M * N + i), 0, 0));
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (z0 + u < S) v += q[u];
  }
  op.store(i / N, i - (i / N) * N, v);
}

// How a weight-gradient column j (of ncol - 1) maps to the parameter layout: conv
// columns run (ky, kx, c) into [co][ci][ky][kx]; the input layer's run (ky, kx pair,
// kx within the pair, c), the sixth column of the pairs dropped; fc1 columns run
// (y, x, c) over the [128][4][5] feature map into the flattened (c, y, x) order; fc2
// columns map one to one.
struct GradMap {
  int kind;  // 0 conv, 1 fc1, 2 fc2, 3 the input layer's pairs
  int ks, lc, ci;
};

// The weight-gradient GEMMs of one backward pass, for the one kernel that adds their
// split-K partials: layer l's partials part[off + (z M + m) ncol + j], z < S, cover
// workgroups block0 .. of the reduction grid.
struct ReduceLayer {
  int64_t off, w_off, b_off;
  int S, M, ncol, block0, zl;  // zl: lanes adding one output's slices (S <= kReducePer zl, up to 64)
  GradMap map;
  float* dst;   // not NULL: the sums (times scale) go to dst[0 .. M ncol) instead
  float scale;
};
constexpr int kReducePer = 8;  // slices per lane of the split-K reduction
struct ReduceTable {
  ReduceLayer L[7];  // the five GEMM layers, fc2 (from the head) and the loss
  int n;
};

// grad[w][m][...] and grad[b][m] = the sum of the split-K partials: 256 / zl outputs per
// workgroup, lane group g < zl adding slices g, g + zl, g + 2 zl, ... in order, then the
// zl group sums in group order (a fixed order: deterministic).
__global__ __launch_bounds__(256) void reduce_parts_kernel(const float* __restrict__ part, float* __restrict__ grad,
                                                           ReduceTable tab) {
  __shared__ float red[256];
  int l = 0;
  while (l + 1 < tab.n && (int)blockIdx.x >= tab.L[l + 1].block0) ++l;
  const ReduceLayer& R = tab.L[l];
  const int opb = 256 / R.zl, ol = threadIdx.x % opb, zg = threadIdx.x / opb;
  const int64_t MN = (int64_t)R.M * R.ncol;
  const int64_t i = (int64_t)(blockIdx.x - R.block0) * opb + ol;
  float s = 0.f;
  if (i < MN) {
    // slices zg, zg + zl, ... (at most kReducePer when S <= kReducePer zl): every load
    // issued before the first addition; loads past the S slices return 0, unadded
    const int zl = R.zl;
    const Rsrc r = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(part + R.off), (short)0,
                                                     (int)(4 * R.S * MN), 0x00020000);
    for (int z0 = zg; z0 < R.S; z0 += kReducePer * zl) {
      float v[kReducePer];
#pragma unroll
      for (int u = 0; u < kReducePer; ++u)
        v[u] = __uint_as_float(
            __builtin_amdgcn_raw_buffer_load_b32(r, 4u * (uint32_t)((z0 + u * zl) * MN + i), 0, 0));
#pragma unroll
      for (int u = 0; u < kReducePer; ++u)
        if (z0 + u * zl < R.S) s += v[u];
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  if (zg != 0 || i >= MN) return;
  s = red[ol];
  for (int g = 1; g < R.zl; ++g) s += red[g * opb + ol];
  if (R.dst) {
    R.dst[i] = s * R.scale;
    return;
  }
  const int ncol = R.ncol, m = (int)(i / ncol), j = (int)(i - (int64_t)m * ncol);
  if (j == ncol - 1) {
    grad[R.b_off + m] = s;
    return;
  }
  float* gw = grad + R.w_off;
  const GradMap& map = R.map;
  if (map.kind == 0) {
    const int tap = j >> map.lc, c = j & ((1 << map.lc) - 1), ky = tap / map.ks, kx = tap - ky * map.ks;
    gw[(((size_t)m * map.ci + c) * map.ks + ky) * map.ks + kx] = s;
  } else if (map.kind == 3) {
    const int r = j >> 3, ky = r / kInPairs, kx = 2 * (r - ky * kInPairs) + ((j >> 2) & 1), c = j & 3;
    if (kx < 5) gw[(((size_t)m * kInC + c) * 5 + ky) * 5 + kx] = s;
  } else if (map.kind == 1) {
    const int yx = j >> 7, c = j & 127;
    gw[(size_t)m * (ncol - 1) + c * 20 + yx] = s;
  } else {
    gw[(size_t)m * (ncol - 1) + j] = s;
  }
}

// The BF16 copies of the weights, in the layouts the GEMMs read:
//   wf[l]: the input layer [co][5][3][2][4]; conv [co][k][k][ci]; fc1 [256][(y, x, c)];
//          fc2 [6][256]
//   wd[l]: conv [ci][k][k][co] (layers 1-3); fc1 [(y, x, c)][256]
// Entries no weight maps to (the input layer's sixth column) stay zero.
struct Packed {
  uint16_t* wf[6];
  uint16_t* wd[6];
  int64_t w_off[6], b_off[6];
};

__device__ void pack_weight(const Packed& pk, int64_t i, float v) {
  int li = 0;
  while (li < 5 && i >= pk.w_off[li + 1]) ++li;
  if (i >= pk.b_off[li]) return;  // a bias: read in FP32
  const int64_t r = i - pk.w_off[li];
  const uint16_t h = to_bf16(v);
  if (li == 0) {
    const int o = (int)(r / 100), rem = (int)(r - (int64_t)o * 100), c = rem / 25, tap = rem - c * 25;
    const int ky = tap / 5, kx = tap - ky * 5;
    pk.wf[0][(size_t)o * kInK + ((ky * kInPairs + (kx >> 1)) * 2 + (kx & 1)) * kInC + c] = h;
  } else if (li < 4) {
    const int ci = li == 1 ? 32 : (li == 2 ? 64 : 128), co = li == 1 ? 64 : 128;
    const int o = (int)(r / (ci * 9)), rem = (int)(r - (int64_t)o * ci * 9), c = rem / 9, tap = rem - c * 9;
    pk.wf[li][((size_t)o * 9 + tap) * ci + c] = h;
    pk.wd[li][((size_t)c * 9 + tap) * co + o] = h;
  } else if (li == 4) {
    const int o = (int)(r / 2560), in = (int)(r - (int64_t)o * 2560), c = in / 20, yx = in - c * 20;
    const int j = yx * 128 + c;
    pk.wf[4][(size_t)o * 2560 + j] = h;
    pk.wd[4][(size_t)j * 256 + o] = h;
  } else {
    const int o = (int)(r / 256), in = (int)(r - (int64_t)o * 256);
    pk.wf[5][(size_t)o * 256 + in] = h;
  }
}

__global__ void pack_kernel(const float* __restrict__ theta, Packed pk, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) pack_weight(pk, i, theta[i]);
}

// FP32 input [B][4][60][80] -> BF16 [B][60][80][4].
__global__ void load_input_kernel(const float* __restrict__ in, uint16_t* __restrict__ x, int64_t npix) {
  constexpr int hw = GS2D_WS_IN_H * GS2D_WS_IN_W;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npix) return;
  const int64_t b = i / hw, q = i - b * hw;
  const float* p = in + b * GS2D_WS_IN_C * hw + q;
  *reinterpret_cast<uint2*>(x + i * kInC) = uint2{to_bf16x2(p[0], p[hw]), to_bf16x2(p[2 * hw], p[3 * hw])};
}

// The network's output layer in training, for kHeadFrames frames per workgroup (two
// per wave; lane l holds inputs 4l .. 4l + 3 of the 256): fc2's forward, out = w2 h1 +
// b2; the squared error against the target; the loss gradient 2 d / n (n = 6 B)
// rounded to bfloat16; fc2's input gradient, bf16(w2^T g [h1 > 0]); and fc2's weight
// and bias gradient and the squared error summed over the workgroup's frames in a
// fixed order (partials part[blk][6][257] and loss_part[blk], added with the other
// layers' partials).
constexpr int kHeadFrames = 8;
__device__ __forceinline__ float bf16_at(uint32_t w, int hi) { return __uint_as_float(hi ? w & 0xFFFF0000u : w << 16); }

__global__ __launch_bounds__(256) void head_kernel(const uint16_t* __restrict__ h1, const uint16_t* __restrict__ w2,
                                                   const float* __restrict__ b2, const float* __restrict__ target,
                                                   int B, float* __restrict__ out, uint16_t* __restrict__ gh1,
                                                   float* __restrict__ part, float* __restrict__ loss_part) {
  __shared__ float red[4][6][256];
  __shared__ float redb[4][8];
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const float n = (float)(6 * B);
  float wv[6][4];
#pragma unroll
  for (int o = 0; o < 6; ++o) {
    const uint2 q = *reinterpret_cast<const uint2*>(w2 + o * 256 + 4 * l);
    wv[o][0] = bf16_at(q.x, 0);
    wv[o][1] = bf16_at(q.x, 1);
    wv[o][2] = bf16_at(q.y, 0);
    wv[o][3] = bf16_at(q.y, 1);
  }
  float acc[6][4] = {}, db[6] = {}, lsum = 0.f;
  for (int f = 0; f < 2; ++f) {
    const int b = blockIdx.x * kHeadFrames + w * 2 + f;
    if (b >= B) break;  // uniform over the wave
    const uint2 hq = *reinterpret_cast<const uint2*>(h1 + (size_t)b * 256 + 4 * l);
    const float h[4] = {bf16_at(hq.x, 0), bf16_at(hq.x, 1), bf16_at(hq.y, 0), bf16_at(hq.y, 1)};
    float g[6];
#pragma unroll
    for (int o = 0; o < 6; ++o) {
      float y = h[0] * wv[o][0];
      y = fmaf(h[1], wv[o][1], y);
      y = fmaf(h[2], wv[o][2], y);
      y = fmaf(h[3], wv[o][3], y);
#pragma unroll
      for (int m = 32; m > 0; m >>= 1) y += __shfl_xor(y, m, 64);
      const float v = y + b2[o];
      if (l == 0) out[(size_t)b * 6 + o] = v;
      const float d = v - target[(size_t)b * 6 + o];
      lsum = fmaf(d, d, lsum);
      g[o] = __uint_as_float((uint32_t)to_bf16(2.0f * d / n) << 16);
      db[o] += g[o];
    }
    float gi[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      float v = wv[0][e] * g[0];
#pragma unroll
      for (int o = 1; o < 6; ++o) v = fmaf(wv[o][e], g[o], v);
      gi[e] = h[e] > 0.f ? v : 0.f;
#pragma unroll
      for (int o = 0; o < 6; ++o) acc[o][e] = fmaf(g[o], h[e], acc[o][e]);
    }
    *reinterpret_cast<uint2*>(gh1 + (size_t)b * 256 + 4 * l) = uint2{to_bf16x2(gi[0], gi[1]), to_bf16x2(gi[2], gi[3])};
  }
#pragma unroll
  for (int o = 0; o < 6; ++o)
#pragma unroll
    for (int e = 0; e < 4; ++e) red[w][o][4 * l + e] = acc[o][e];
  if (l == 0) {
#pragma unroll
    for (int o = 0; o < 6; ++o) redb[w][o] = db[o];
    redb[w][6] = lsum;
  }
  __syncthreads();
  float* p = part + (size_t)blockIdx.x * 6 * 257;
#pragma unroll
  for (int o = 0; o < 6; ++o) p[o * 257 + t] = ((red[0][o][t] + red[1][o][t]) + red[2][o][t]) + red[3][o][t];
  if (t < 6) p[t * 257 + 256] = ((redb[0][t] + redb[1][t]) + redb[2][t]) + redb[3][t];
  if (t == 6) loss_part[blockIdx.x] = ((redb[0][6] + redb[1][6]) + redb[2][6]) + redb[3][6];
}

// AdamW on the FP32 master vector (bias corrections c1 = 1 - b1^t, c2 = 1 - b2^t from
// the host), then the BF16 copies.
__global__ void adamw_kernel(float* __restrict__ theta, float* __restrict__ m, float* __restrict__ v,
                             const float* __restrict__ g, Packed pk, int n, gs2d_ws_adamw o, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = o.beta1 * m[i] + (1.f - o.beta1) * gi;
  const float vi = o.beta2 * v[i] + (1.f - o.beta2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / c1, vh = vi / c2;
  const float th = theta[i] * (1.f - o.lr * o.weight_decay) - o.lr * mh / (sqrtf(vh) + o.eps);
  theta[i] = th;
  pack_weight(pk, i, th);
}

// input[b][c][Y][X] = mean over the f x f block of (img - tgt), c < 3 colour, c = 3 depth.
__global__ void residual_kernel(const float* __restrict__ rgb, const float* __restrict__ depth,
                                const float* __restrict__ trgb, const float* __restrict__ tdepth, int W, int H,
                                int f, int batch, float* __restrict__ input) {
  const int per = GS2D_WS_IN_C * GS2D_WS_IN_H * GS2D_WS_IN_W;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= batch * per) return;
  const int b = i / per, r = i - b * per;
  const int c = r / (GS2D_WS_IN_H * GS2D_WS_IN_W), q = r - c * (GS2D_WS_IN_H * GS2D_WS_IN_W);
  const int Y = q / GS2D_WS_IN_W, X = q - Y * GS2D_WS_IN_W;
  const size_t hw = (size_t)W * H;
  const float* img = c < 3 ? rgb + (size_t)b * 3 * hw + c * hw : depth + (size_t)b * hw;
  const float* tgt = c < 3 ? trgb + (size_t)b * 3 * hw + c * hw : tdepth + (size_t)b * hw;
  float s = 0.f;
  for (int dy = 0; dy < f; ++dy) {
    const size_t row = (size_t)(Y * f + dy) * W + (size_t)X * f;
    for (int dx = 0; dx < f; ++dx) s += img[row + dx] - tgt[row + dx];
  }
  input[i] = s / (float)(f * f);
}

// The proposal's two inputs from one rendered frame in one pass, one thread per f x f
// block: the network input x[Y][X][c] = bf16 of the block mean of (img - tgt)
// (channels as residual_kernel), and part[Y 80 + X] = the block's sum of |d r| +
// |d g| + |d b| + lambda_d |d depth|, the terms of the unmasked tracking loss.
__global__ __launch_bounds__(64) void residual_loss_kernel(const float* __restrict__ rgb,
                                                           const float* __restrict__ depth,
                                                           const float* __restrict__ trgb,
                                                           const float* __restrict__ tdepth, int W, int H, int f,
                                                           float lambda_d, uint16_t* __restrict__ x,
                                                           float* __restrict__ part) {
  constexpr int nb = GS2D_WS_IN_H * GS2D_WS_IN_W;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  const int Y = i / GS2D_WS_IN_W, X = i - Y * GS2D_WS_IN_W;
  const size_t hw = (size_t)W * H;
  float s[4] = {0.f, 0.f, 0.f, 0.f}, a = 0.f;
  for (int dy = 0; dy < f; ++dy) {
    const size_t row = (size_t)(Y * f + dy) * W + (size_t)X * f;
    for (int dx = 0; dx < f; ++dx) {
      float d[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float* img = c < 3 ? rgb + c * hw : depth;
        const float* tgt = c < 3 ? trgb + c * hw : tdepth;
        d[c] = img[row + dx] - tgt[row + dx];
      }
      a += fabsf(d[0]) + fabsf(d[1]) + fabsf(d[2]) + lambda_d * fabsf(d[3]);
#pragma unroll
      for (int c = 0; c < 4; ++c) s[c] += d[c];
    }
  }
  const float ff = (float)(f * f);
  *reinterpret_cast<uint2*>(x + (size_t)i * kInC) = uint2{to_bf16x2(s[0] / ff, s[1] / ff),
                                                          to_bf16x2(s[2] / ff, s[3] / ff)};
  part[i] = a;
}

// Keep T_0 unless its loss exceeds the start pose's.
__global__ void choose_pose_kernel(const float* __restrict__ loss, const float* __restrict__ p_start,
                                   const float* __restrict__ p0, float* __restrict__ out, float* __restrict__ info) {
  const int i = threadIdx.x;
  const bool keep = loss[1] <= loss[0];
  if (i < 12) out[i] = keep ? p0[i] : p_start[i];
  if (i == 0 && info) {
    info[0] = loss[0];
    info[1] = loss[1];
    info[2] = keep ? 1.f : 0.f;
    info[3] = 0.f;
  }
}

// The proposal's last launch, at batch 1 (one 256-thread workgroup).  Thread t forms
// fc1's output h[t] = bf16(ReLU(b1[t] + the sum of fc1's S split-K slices, added in
// slice order)), as the split finish does (S = 0: h1 holds it already).  The six
// outputs are b2[o] + sum_t w2[o][t] h[t], each wave adding its 64 products by a
// butterfly and the four wave sums in wave order, then scaled from the normalised
// twist to (rho in m, phi in rad): tau.  Wave 0 then forms T_0 = Exp(tau) T_start in
// FP64 and lane k < 12 writes entry k, rounded to FP32.  With loss_part, also
// *loss = scale x the sum of loss_part[0 .. n), n <= 256 kLossPer (thread t adding
// t, t + 256, ... in order, then a halving tree).  Every load is issued before the
// first sum: the kernel is one memory latency, then arithmetic.
constexpr int kLossPer = (GS2D_WS_IN_H * GS2D_WS_IN_W + 255) / 256;
constexpr int kCloseSlices = 24;  // slices loaded at once (a batch-1 fc1 has 20)
__global__ __launch_bounds__(256) void propose_close_kernel(
    const float* __restrict__ part, int S, const uint16_t* __restrict__ h1, const float* __restrict__ b1,
    const uint16_t* __restrict__ w2, const float* __restrict__ b2, const float* __restrict__ pin,
    float* __restrict__ pout, float* __restrict__ tau_out, const float* __restrict__ loss_part, int n, float scale,
    float* __restrict__ loss) {
  __shared__ float red[4][6];
  __shared__ float sh[256];
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  // buffer loads past a resource's range return 0 (a NULL loss_part: an empty range)
  const Rsrc rl = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(loss_part), (short)0,
                                                    loss_part ? 4 * n : 0, 0x00020000);
  const Rsrc rp = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(part), (short)0,
                                                    S > 0 ? 4 * 256 * min(S, kCloseSlices) : 0, 0x00020000);
  float lv[kLossPer], pv[kCloseSlices], wv[6];
#pragma unroll
  for (int j = 0; j < kLossPer; ++j)
    lv[j] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rl, 4u * (uint32_t)(t + 256 * j), 0, 0));
#pragma unroll
  for (int z = 0; z < kCloseSlices; ++z)
    pv[z] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rp, 4u * (uint32_t)(z * 256 + t), 0, 0));
#pragma unroll
  for (int o = 0; o < 6; ++o) wv[o] = __uint_as_float((uint32_t)w2[o * 256 + t] << 16);
  const float bias1 = b1[t];
  const uint16_t hq = S > 0 ? 0 : h1[t];
  float bo[6], col[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int o = 0; o < 6; ++o) bo[o] = b2[o];
  if (t < 12)
#pragma unroll
    for (int q = 0; q < 3; ++q) col[q] = pin[q * 4 + t % 4];
  float a = 0.f;
#pragma unroll
  for (int j = 0; j < kLossPer; ++j) a += lv[j];
  float h;
  if (S > 0) {
    float v = 0.f;
#pragma unroll
    for (int z = 0; z < kCloseSlices; ++z)
      if (z < S) v += pv[z];
    for (int z = kCloseSlices; z < S; ++z) v += part[(size_t)z * 256 + t];
    h = __uint_as_float((uint32_t)to_bf16(relu(v + bias1)) << 16);
  } else {
    h = __uint_as_float((uint32_t)hq << 16);
  }
#pragma unroll
  for (int o = 0; o < 6; ++o) {
    float y = wv[o] * h;
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) y += __shfl_xor(y, m, 64);
    if (l == 0) red[w][o] = y;
  }
  sh[t] = a;
  __syncthreads();
  if (loss_part) {
    for (int k = 128; k > 0; k >>= 1) {
      if (t < k) sh[t] += sh[t + k];
      __syncthreads();
    }
    if (t == 0) *loss = sh[0] * scale;
  }
  if (w != 0) return;
  double tau[6];
#pragma unroll
  for (int o = 0; o < 6; ++o) {
    const float v = (((red[0][o] + red[1][o]) + red[2][o]) + red[3][o]) + bo[o];
    const float f = v * (o < 3 ? 0.1f : (float)(8.0 * M_PI / 180.0));
    tau[o] = f;
    if (l == o) tau_out[o] = f;
  }
  double Re[9], te[3];
  se3_exp(tau, Re, te);
  if (l < 12) {
    const int r = l / 4, c = l % 4;
    double s = Re[r * 3 + 0] * (double)col[0] + Re[r * 3 + 1] * (double)col[1] + Re[r * 3 + 2] * (double)col[2];
    if (c == 3) s += te[r];
    pout[l] = (float)s;
  }
}

// ---- layer table -------------------------------------------------------------------

struct LayerDef {
  int ci, co, k, H, W;  // conv: input size H x W; fc: I = ci, O = co (H = W = k = 0)
};
constexpr LayerDef kLayers[6] = {{4, 32, 5, 60, 80}, {32, 64, 3, 30, 40}, {64, 128, 3, 15, 20},
                                 {128, 128, 3, 8, 10}, {2560, 256, 0, 0, 0}, {256, 6, 0, 0, 0}};

int out_size(int n, int k) { return (n + 2 * (k / 2) - k) / 2 + 1; }
int64_t layer_weights(const LayerDef& L) {
  return L.k ? (int64_t)L.co * L.ci * L.k * L.k : (int64_t)L.co * L.ci;
}
int log2i(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}
FastDiv fast_div(int d) {
  const int l = log2i(d);
  const uint64_t m = ((uint64_t)1 << (32 + l)) / (uint64_t)d + 1;
  return FastDiv{(uint32_t)m, (uint32_t)(m >> 32), l};
}
int64_t act_size(int li) {  // per frame, output of layer li (li = -1: the input as stored)
  if (li < 0) return (int64_t)kInC * GS2D_WS_IN_H * GS2D_WS_IN_W;
  const LayerDef& L = kLayers[li];
  if (L.k) return (int64_t)L.co * out_size(L.H, L.k) * out_size(L.W, L.k);
  return L.co;
}
// BF16 copies: forward and input-gradient layouts of each layer.
int64_t wf_size(int li) {
  const LayerDef& L = kLayers[li];
  if (li == 0) return (int64_t)L.co * kInK;
  return L.k ? (int64_t)L.co * L.k * L.k * L.ci : (int64_t)L.co * L.ci;
}
int64_t wd_size(int li) {
  const LayerDef& L = kLayers[li];
  if (L.k) return li == 0 ? 0 : (int64_t)L.ci * L.k * L.k * L.co;
  return li == 5 ? 0 : (int64_t)L.ci * L.co;
}

int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

template <int BM, int BN, class Op>
void run(const Op& op, int M, int N, int gz, hipStream_t s) {
  dim3 grid(cdiv(N, BN), cdiv(M, BM), gz);
  gemm_kernel<Op, BM, BN><<<grid, kThreads, 0, s>>>(op);
}

// Tile columns: 128 while that still makes 512 workgroups, else 64 while that makes
// 256, else 32 (groups: workgroups per tile, i.e. the parity classes).
int pick_bn(int M, int N, int BM, int groups) {
  if ((int64_t)cdiv(N, 128) * cdiv(M, BM) * groups >= 512) return 128;
  if ((int64_t)cdiv(N, 64) * cdiv(M, BM) * groups >= 256) return 64;
  return 32;
}

template <int BM, class Op>
void run_bn(const Op& op, int M, int N, int gz, int bn, hipStream_t s) {
  if (bn == 128)
    run<BM, 128>(op, M, N, gz, s);
  else if (bn == 64)
    run<BM, 64>(op, M, N, gz, s);
  else
    run<BM, 32>(op, M, N, gz, s);
}

// A forward layer: large outputs as one GEMM (tile columns by pick_bn); few output
// tiles with a long reduction split into slices whose sums a second kernel adds.
// Returns the number of split-K slices (0: one GEMM).  finish = false leaves a split
// layer's slices in part for the caller to add.
template <int BM, class Op>
int gemm_fwd(Op op, float* part, int64_t part_cap, hipStream_t s, bool finish = true) {
  const int M = op.M, N = op.N, K = op.K;
  const int tiles = cdiv(N, 64) * cdiv(M, BM);
  if (tiles < 64 && K >= 512) {  // (also splitting layers of 64-256 tiles was measured no faster)
    int S = K / 128;
    const int want = cdiv(128, tiles);  // about 128 workgroups
    S = S < want ? S : want;
    const int ks = cdiv(cdiv(K, S), kBK) * kBK;
    S = cdiv(K, ks);
    if (S > 1 && (int64_t)S * M * N <= part_cap && (int64_t)(S + 16) * M * N < (1 << 29)) {
      SplitPart<Op> sp;
      static_cast<Op&>(sp) = op;
      sp.ks = ks;
      sp.part = part;
      run<BM, 64>(sp, M, N, S, s);
      op.ks = ks;
      if (finish) split_finish_kernel<Op><<<cdiv((int64_t)M * N, 256), 256, 0, s>>>(op, part, S);
      return S;
    }
  }
  op.ks = cdiv(K, kBK) * kBK;
  run_bn<BM>(op, M, N, 1, pick_bn(M, N, BM, 1), s);
  return 0;
}

// Split-K slices of a weight-gradient GEMM: about 512 workgroups, at most 256 slices,
// at least 512 reduction indices each.
int wgrad_splits(int M, int N, int64_t K, int BM, int BN, int* ks_out) {
  const int tiles = cdiv(N, BN) * cdiv(M, BM);
  int64_t S = cdiv(512, tiles);
  if (S > 256) S = 256;
  const int64_t smax = K / 512 > 1 ? K / 512 : 1;
  if (S > smax) S = smax;
  if (S < 1) S = 1;
  const int ks = cdiv(cdiv(K, S), kBK) * kBK;
  if (ks_out) *ks_out = ks;
  return cdiv(K, ks);
}

}  // namespace
}  // namespace ws
}  // namespace gs2d

struct gs2d_ws {
  int device = 0;
  int max_batch = 0;
  float* theta = nullptr;   // FP32 master [P]
  float* m = nullptr;       // AdamW moments [P]
  float* v = nullptr;
  float* grad = nullptr;    // last gradient [P]
  uint16_t* wp = nullptr;   // BF16 copies (pk's layouts)
  int64_t wp_size = 0;
  gs2d::ws::Packed pk = {};
  uint16_t* act[6] = {};    // BF16 activations, channels last: input, conv1..4, fc1 ([max_batch] frames each)
  uint16_t* gact[6] = {};   // BF16 gradients of the same (masked by the ReLU: the pre-ReLU gradient)
  float* out = nullptr;     // FP32 [max_batch][6]
  float* part = nullptr;    // split-K partials
  int64_t part_cap = 0;
  float* lossbuf = nullptr; // [4]
  int64_t step = 0;         // AdamW step count
  // warm-start workspace (one frame)
  float* img = nullptr;     // rgb, depth, normal, alpha [8][hw]
  float* igrad = nullptr;   // d_rgb, d_depth [4][hw]
  int64_t img_cap = 0;
  float* wsf = nullptr;     // input [4][60][80], out [6], tau [6], pose0 [12], loss [2]
};

namespace {

using namespace gs2d::ws;

constexpr int64_t kInPlanar = (int64_t)GS2D_WS_IN_C * GS2D_WS_IN_H * GS2D_WS_IN_W;  // FP32 input per frame

int dev_alloc(void** p, size_t bytes) {
  if (hipMalloc(p, bytes) != hipSuccess) {
    *p = nullptr;
    return GS2D_ERR_OOM;
  }
  return GS2D_OK;
}

#define WS_TRY(x)                      \
  do {                                 \
    const int r_ = (x);                \
    if (r_ != GS2D_OK) return r_;      \
  } while (0)
#define WS_HIP(x)                                    \
  do {                                               \
    if ((x) != hipSuccess) return GS2D_ERR_HIP;      \
  } while (0)

int ensure_part(gs2d_ws* net, int64_t n) {
  if (n <= net->part_cap) return GS2D_OK;
  if (net->part) WS_HIP(hipFree(net->part));
  net->part = nullptr;
  net->part_cap = 0;
  WS_TRY(dev_alloc((void**)&net->part, (size_t)n * sizeof(float)));
  net->part_cap = n;
  return GS2D_OK;
}

// The tile of each layer's weight-gradient GEMM: rows (M = co or O) and columns (64:
// wider tiles at small M halve the workgroups and were measured slower).
int wgrad_bm(int li) { return kLayers[li].co >= 128 ? 128 : (kLayers[li].co >= 64 ? 64 : 32); }
int wgrad_bn(int) { return 64; }

// Weight-gradient GEMM of layer li over a batch of B: M, N (columns incl. bias), K.
void wgrad_shape(int li, int B, int* M, int* N, int64_t* K) {
  const LayerDef& L = kLayers[li];
  *M = L.co;
  if (L.k) {
    *N = (li == 0 ? kInK : L.k * L.k * L.ci) + 1;
    *K = (int64_t)B * out_size(L.H, L.k) * out_size(L.W, L.k);
  } else {
    *N = L.ci + 1;
    *K = B;
  }
}

// Partial-sum floats of the weight-gradient GEMMs of a batch, each layer in its own
// region (offsets into off[6]; they are added by one kernel after the backward pass);
// the split forward layers of small batches use the start of the buffer.
int64_t part_layout(int B, int64_t* off) {
  int64_t o = 0;
  for (int li = 0; li < 5; ++li) {
    int M, N;
    int64_t K;
    wgrad_shape(li, B, &M, &N, &K);
    if (off) off[li] = o;
    o += (int64_t)wgrad_splits(M, N, K, wgrad_bm(li), wgrad_bn(li), nullptr) * M * N;
  }
  const int64_t hb = cdiv(B, kHeadFrames);  // fc2 and the loss: one partial per head workgroup
  if (off) off[5] = o;
  o += hb * 6 * 257;
  if (off) off[6] = o;
  o += hb;
  return o > (1 << 20) ? o : (1 << 20);
}

// Forward of B frames whose BF16 input is in act[0] up to fc1, then (out not NULL)
// fc2: the normalised FP32 output to out [B][6].  With fc1_slices, fc1 stops at its
// split-K slices (their count in *fc1_slices; 0 if it ran as one GEMM into act[5])
// and fc2 is left to the caller.
void forward_layers(gs2d_ws* net, int B, float* out, hipStream_t s, int* fc1_slices = nullptr) {
  for (int li = 0; li < 4; ++li) {
    const LayerDef& L = kLayers[li];
    const int OH = out_size(L.H, L.k), OW = out_size(L.W, L.k);
    auto fill = [&](auto& op) {
      op.M = L.co;
      op.N = B * OH * OW;
      op.K = li == 0 ? kInK : L.k * L.k * L.ci;
      op.w = net->pk.wf[li];
      op.bias = net->theta + net->pk.b_off[li];
      op.x = net->act[li];
      op.y = net->act[li + 1];
      op.H = L.H;
      op.W = L.W;
      op.OH = OH;
      op.OW = OW;
      op.by_ohw = fast_div(OH * OW);
      op.by_ow = fast_div(OW);
    };
    if (li == 0) {
      ConvFwdIn op;
      fill(op);
      gemm_fwd<32>(op, net->part, net->part_cap, s);
    } else {
      ConvFwd<3> op;
      fill(op);
      op.lc = log2i(L.ci);
      if (li == 1)
        gemm_fwd<64>(op, net->part, net->part_cap, s);
      else
        gemm_fwd<128>(op, net->part, net->part_cap, s);
    }
  }
  {
    FcFwd op;
    op.M = 256;
    op.N = B;
    op.K = 2560;
    op.w = net->pk.wf[4];
    op.bias = net->theta + net->pk.b_off[4];
    op.x = net->act[4];
    op.y = net->act[5];
    op.yf = nullptr;
    const int S = gemm_fwd<128>(op, net->part, net->part_cap, s, fc1_slices == nullptr);
    if (fc1_slices) {
      *fc1_slices = S;
      return;
    }
  }
  if (out) {
    FcFwd op;
    op.M = 6;
    op.N = B;
    op.K = 256;
    op.w = net->pk.wf[5];
    op.bias = net->theta + net->pk.b_off[5];
    op.x = net->act[5];
    op.y = nullptr;
    op.yf = out;
    gemm_fwd<32>(op, net->part, net->part_cap, s);
  }
}

// Appends a GEMM's split-K partials (S slices of M x ncol at part + off) to the table.
void add_reduce(ReduceTable* tab, int64_t off, int64_t w_off, int64_t b_off, int S, int M, int ncol, GradMap map,
                float* dst, float scale) {
  ReduceLayer& R = tab->L[tab->n];
  R.off = off;
  R.w_off = w_off;
  R.b_off = b_off;
  R.S = S;
  R.M = M;
  R.ncol = ncol;
  R.zl = 1;
  while (R.zl < 64 && R.S > kReducePer * R.zl) R.zl *= 2;
  R.map = map;
  R.dst = dst;
  R.scale = scale;
  tab->n += 1;
}

// Orders the table's layers by slice count, most first (their lanes' chains are the
// longest: their workgroups start first), and assigns each its run of workgroups.
// Returns the grid size.
int finish_reduce(ReduceTable* tab) {
  for (int a = 1; a < tab->n; ++a)
    for (int b = a; b > 0 && tab->L[b].S > tab->L[b - 1].S; --b) {
      const ReduceLayer t = tab->L[b];
      tab->L[b] = tab->L[b - 1];
      tab->L[b - 1] = t;
    }
  int blocks = 0;
  for (int k = 0; k < tab->n; ++k) {
    tab->L[k].block0 = blocks;
    blocks += cdiv((int64_t)tab->L[k].M * tab->L[k].ncol, 256 / tab->L[k].zl);
  }
  return blocks;
}

template <int BM, class Op>
void wgrad_run(gs2d_ws* net, Op op, int li, int B, ReduceTable* tab, hipStream_t s) {
  int M, N;
  int64_t K;
  wgrad_shape(li, B, &M, &N, &K);
  int64_t off[7];
  part_layout(B, off);
  int ks = 0;
  const int bn = wgrad_bn(li);
  const int S = wgrad_splits(M, N, K, BM, bn, &ks);
  op.M = M;
  op.N = N;
  op.K = (int)K;
  op.ks = ks;
  op.part = net->part + off[li];
  if (bn == 128)
    run<BM, 128>(op, M, N, S, s);
  else
    run<BM, 64>(op, M, N, S, s);
  const LayerDef& L = kLayers[li];
  add_reduce(tab, off[li], net->pk.w_off[li], net->pk.b_off[li], S, M, N,
             GradMap{li == 0 ? 3 : (L.k ? 0 : 1), L.k, log2i(L.ci), L.ci}, nullptr, 1.f);
}

void weight_grad(gs2d_ws* net, int li, int B, ReduceTable* tab, hipStream_t s) {
  const LayerDef& L = kLayers[li];
  if (L.k) {
    auto fill = [&](auto& op) {
      op.gy = net->gact[li + 1];
      op.x = net->act[li];
      op.H = L.H;
      op.W = L.W;
      op.OH = out_size(L.H, L.k);
      op.OW = out_size(L.W, L.k);
      op.by_ohw = fast_div(op.OH * op.OW);
      op.by_ow = fast_div(op.OW);
    };
    if (li == 0) {
      ConvBwdWeightIn op;
      fill(op);
      wgrad_run<32>(net, op, li, B, tab, s);
    } else {
      ConvBwdWeight<3> op;
      fill(op);
      op.lc = log2i(L.ci);
      if (li == 1)
        wgrad_run<64>(net, op, li, B, tab, s);
      else
        wgrad_run<128>(net, op, li, B, tab, s);
    }
  } else {  // fc1 (fc2's comes from the head kernel)
    FcBwdWeight op;
    op.gy = net->gact[li + 1];
    op.x = net->act[li];
    wgrad_run<128>(net, op, li, B, tab, s);
  }
}

// Input gradient of conv layer li (1..3), masked by the ReLU of its input.
void conv_data_grad(gs2d_ws* net, int li, int B, hipStream_t s) {
  const LayerDef& L = kLayers[li];
  ConvBwdData op;
  op.wd = net->pk.wd[li];
  op.gy = net->gact[li + 1];
  op.x = net->act[li];
  op.gx = net->gact[li];
  op.Bn = B;
  op.ci = L.ci;
  op.co = L.co;
  op.lco = log2i(L.co);
  op.H = L.H;
  op.W = L.W;
  op.OH = out_size(L.H, 3);
  op.OW = out_size(L.W, 3);
  for (int z = 0; z < 4; ++z) {
    const int Hc = (L.H - (z >> 1) + 1) >> 1, Wc = (L.W - (z & 1) + 1) >> 1;
    op.by_per[z] = fast_div(Hc * Wc);
    op.by_wc[z] = fast_div(Wc);
  }
  const int N = B * ((L.H + 1) >> 1) * ((L.W + 1) >> 1);  // the largest class
  if (L.ci == 32)
    run_bn<32>(op, L.ci, N, 4, pick_bn(L.ci, N, 32, 4), s);
  else if (L.ci == 64)
    run_bn<64>(op, L.ci, N, 4, pick_bn(L.ci, N, 64, 4), s);
  else
    run_bn<128>(op, L.ci, N, 4, pick_bn(L.ci, N, 128, 4), s);
}

int check_net(gs2d_ws* net, int batch) {
  if (!net || batch < 1 || batch > net->max_batch) return GS2D_ERR_INVALID_ARG;
  WS_HIP(hipSetDevice(net->device));
  return GS2D_OK;
}

void load_input(gs2d_ws* net, const float* input, int B, hipStream_t s) {
  const int64_t npix = (int64_t)B * GS2D_WS_IN_H * GS2D_WS_IN_W;
  load_input_kernel<<<cdiv(npix, 256), 256, 0, s>>>(input, net->act[0], npix);
}

}  // namespace

extern "C" {

GS2D_API int64_t gs2d_ws_param_count(void) {
  int64_t p = 0;
  for (const auto& L : kLayers) p += layer_weights(L) + L.co;
  return p;
}

GS2D_API int gs2d_ws_create(gs2d_ws** out, int device, int32_t max_batch) {
  if (!out || max_batch < 1 || max_batch > 4096) return GS2D_ERR_INVALID_ARG;
  *out = nullptr;
  if (hipSetDevice(device) != hipSuccess) return GS2D_ERR_HIP;
  gs2d_ws* net = new (std::nothrow) gs2d_ws();
  if (!net) return GS2D_ERR_OOM;
  net->device = device;
  net->max_batch = max_batch;
  int64_t o = 0, wo = 0;
  int64_t wf_off[6], wd_off[6];
  for (int li = 0; li < 6; ++li) {
    net->pk.w_off[li] = o;
    o += layer_weights(kLayers[li]);
    net->pk.b_off[li] = o;
    o += kLayers[li].co;
    wf_off[li] = wo;
    wo += wf_size(li);
    wd_off[li] = wo;
    wo += wd_size(li);
  }
  const int64_t P = o;
  net->wp_size = wo;
  int r = GS2D_OK;
  if (r == GS2D_OK) r = dev_alloc((void**)&net->theta, P * sizeof(float));
  if (r == GS2D_OK) r = dev_alloc((void**)&net->m, P * sizeof(float));
  if (r == GS2D_OK) r = dev_alloc((void**)&net->v, P * sizeof(float));
  if (r == GS2D_OK) r = dev_alloc((void**)&net->grad, P * sizeof(float));
  if (r == GS2D_OK) r = dev_alloc((void**)&net->wp, wo * sizeof(uint16_t));
  if (r == GS2D_OK)
    for (int li = 0; li < 6; ++li) {
      net->pk.wf[li] = net->wp + wf_off[li];
      net->pk.wd[li] = wd_size(li) ? net->wp + wd_off[li] : nullptr;
    }
  for (int i = 0; i < 6 && r == GS2D_OK; ++i) {
    const size_t bytes = (size_t)max_batch * act_size(i - 1) * sizeof(uint16_t);
    r = dev_alloc((void**)&net->act[i], bytes);
    if (r == GS2D_OK) r = dev_alloc((void**)&net->gact[i], bytes);
  }
  if (r == GS2D_OK) r = dev_alloc((void**)&net->out, (size_t)max_batch * 6 * sizeof(float));
  if (r == GS2D_OK) r = dev_alloc((void**)&net->lossbuf, 4 * sizeof(float));
  // warm-start scratch: input [4][60][80], out [8], tau [8], pose0 [12], losses [2]
  if (r == GS2D_OK) r = dev_alloc((void**)&net->wsf, (kInPlanar + 64) * sizeof(float));
  if (r == GS2D_OK) r = ensure_part(net, part_layout(max_batch, nullptr));

  if (r == GS2D_OK && (hipMemset(net->theta, 0, P * sizeof(float)) != hipSuccess ||
                       hipMemset(net->m, 0, P * sizeof(float)) != hipSuccess ||
                       hipMemset(net->v, 0, P * sizeof(float)) != hipSuccess ||
                       hipMemset(net->wp, 0, wo * sizeof(uint16_t)) != hipSuccess))
    r = GS2D_ERR_HIP;
  if (r != GS2D_OK) {
    gs2d_ws_destroy(net);
    return r;
  }
  *out = net;
  return GS2D_OK;
}

GS2D_API int gs2d_ws_destroy(gs2d_ws* net) {
  if (!net) return GS2D_OK;
  (void)hipSetDevice(net->device);
  float* fl[] = {net->theta, net->m, net->v, net->grad, net->out, net->part, net->lossbuf, net->img, net->igrad,
                 net->wsf};
  for (float* p : fl)
    if (p) (void)hipFree(p);
  if (net->wp) (void)hipFree(net->wp);
  for (int i = 0; i < 6; ++i) {
    if (net->act[i]) (void)hipFree(net->act[i]);
    if (net->gact[i]) (void)hipFree(net->gact[i]);
  }
  delete net;
  return GS2D_OK;
}

GS2D_API int gs2d_ws_set_params(gs2d_ws* net, const float* theta, hipStream_t s) {
  if (!net || !theta) return GS2D_ERR_INVALID_ARG;
  WS_HIP(hipSetDevice(net->device));
  const int64_t P = GS2D_WS_PARAMS;
  WS_HIP(hipMemcpyAsync(net->theta, theta, P * sizeof(float), hipMemcpyDeviceToDevice, s));
  WS_HIP(hipMemsetAsync(net->m, 0, P * sizeof(float), s));
  WS_HIP(hipMemsetAsync(net->v, 0, P * sizeof(float), s));
  pack_kernel<<<cdiv(P, 256), 256, 0, s>>>(net->theta, net->pk, P);
  net->step = 0;
  WS_HIP(hipGetLastError());
  return GS2D_OK;
}

GS2D_API int gs2d_ws_get_params(gs2d_ws* net, float* theta, hipStream_t s) {
  if (!net || !theta) return GS2D_ERR_INVALID_ARG;
  WS_HIP(hipSetDevice(net->device));
  WS_HIP(hipMemcpyAsync(theta, net->theta, (size_t)GS2D_WS_PARAMS * sizeof(float), hipMemcpyDeviceToDevice, s));
  return GS2D_OK;
}

GS2D_API int gs2d_ws_residual(const float* rgb, const float* depth, const float* tgt_rgb, const float* tgt_depth,
                              int32_t width, int32_t height, int32_t batch, float* input, hipStream_t s) {
  if (!rgb || !depth || !tgt_rgb || !tgt_depth || !input || batch < 1 || width <= 0 || height <= 0)
    return GS2D_ERR_INVALID_ARG;
  if (width % GS2D_WS_IN_W || height % GS2D_WS_IN_H || width / GS2D_WS_IN_W != height / GS2D_WS_IN_H)
    return GS2D_ERR_UNSUPPORTED;
  const int f = width / GS2D_WS_IN_W;
  const int64_t n = (int64_t)batch * kInPlanar;
  residual_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(rgb, depth, tgt_rgb, tgt_depth, width, height, f,
                                                               batch, input);
  WS_HIP(hipGetLastError());
  return GS2D_OK;
}

GS2D_API int gs2d_ws_forward(gs2d_ws* net, const float* input, int32_t batch, float* out, hipStream_t s) {
  WS_TRY(check_net(net, batch));
  if (!input || !out) return GS2D_ERR_INVALID_ARG;
  load_input(net, input, batch, s);
  forward_layers(net, batch, out, s);
  WS_HIP(hipGetLastError());
  return GS2D_OK;
}

GS2D_API int gs2d_ws_gradient(gs2d_ws* net, const float* input, const float* target, int32_t batch, float* loss,
                              float* out, float* grad, hipStream_t s) {
  WS_TRY(check_net(net, batch));
  if (!input || !target) return GS2D_ERR_INVALID_ARG;
  const int B = batch;
  float* outp = out ? out : net->out;
  load_input(net, input, B, s);
  forward_layers(net, B, nullptr, s);  // up to fc1
  int64_t off[7];
  part_layout(B, off);
  const int hb = cdiv(B, kHeadFrames);
  head_kernel<<<hb, 256, 0, s>>>(net->act[5], net->pk.wf[5], net->theta + net->pk.b_off[5], target, B, outp,
                                 net->gact[5], net->part + off[5], net->part + off[6]);
  ReduceTable tab{};
  add_reduce(&tab, off[5], net->pk.w_off[5], net->pk.b_off[5], hb, 6, 257, GradMap{2, 0, 0, 256}, nullptr, 1.f);
  add_reduce(&tab, off[6], 0, 0, hb, 1, 1, GradMap{2, 0, 0, 0}, loss ? loss : net->lossbuf, 1.f / (float)(6 * B));
  weight_grad(net, 4, B, &tab, s);
  {  // the masked input gradient of the fc1 input (conv4's output)
    FcBwdData op;
    op.M = 2560;
    op.N = B;
    op.K = 256;
    op.ks = 256;
    op.wt = net->pk.wd[4];
    op.gy = net->gact[5];
    op.x = net->act[4];
    op.gx = net->gact[4];
    run_bn<128>(op, 2560, B, 1, pick_bn(2560, B, 128, 1), s);
  }
  for (int li = 3; li >= 0; --li) {
    weight_grad(net, li, B, &tab, s);
    // layers 1-3 (the input gradient of layer 0 is not needed) are all 3 x 3
    if (li > 0) conv_data_grad(net, li, B, s);
  }
  const int blocks = finish_reduce(&tab);
  reduce_parts_kernel<<<blocks, 256, 0, s>>>(net->part, net->grad, tab);
  if (grad)
    WS_HIP(hipMemcpyAsync(grad, net->grad, (size_t)GS2D_WS_PARAMS * sizeof(float), hipMemcpyDeviceToDevice, s));
  WS_HIP(hipGetLastError());
  return GS2D_OK;
}

GS2D_API int gs2d_ws_adamw_step(gs2d_ws* net, const gs2d_ws_adamw* o, hipStream_t s) {
  if (!net || !o) return GS2D_ERR_INVALID_ARG;
  if (!(o->lr >= 0.f) || !(o->beta1 >= 0.f && o->beta1 < 1.f) || !(o->beta2 >= 0.f && o->beta2 < 1.f) ||
      !(o->eps > 0.f) || !(o->weight_decay >= 0.f))
    return GS2D_ERR_INVALID_ARG;
  WS_HIP(hipSetDevice(net->device));
  net->step += 1;
  const float c1 = (float)(1.0 - std::pow((double)o->beta1, (double)net->step));
  const float c2 = (float)(1.0 - std::pow((double)o->beta2, (double)net->step));
  const int P = GS2D_WS_PARAMS;
  adamw_kernel<<<(P + 255) / 256, 256, 0, s>>>(net->theta, net->m, net->v, net->grad, net->pk, P, *o, c1, c2);
  WS_HIP(hipGetLastError());
  return GS2D_OK;
}

}  // extern "C"

namespace {

// The render at T_start, its tracking loss (into losses[0]), the residual, the network
// and T_0 = Exp(tau_hat) T_start (into pose0).  rgb .. alpha: the network's image
// workspace, sized here.
int propose(gs2d_ctx* ctx, gs2d_ws* net, const float* params, int64_t n, const gs2d_camera* camera,
            const float* pose_start, const float* tgt_rgb, const float* tgt_depth, float lambda_d, int32_t use_masks,
            float* pose0, float* losses, hipStream_t s) {
  if (!ctx || !net || !camera || !pose_start || !tgt_rgb || !tgt_depth || !pose0 || !losses || (n > 0 && !params))
    return GS2D_ERR_INVALID_ARG;
  const int W = camera->width, H = camera->height;
  if (W <= 0 || H <= 0) return GS2D_ERR_INVALID_ARG;
  if (W % GS2D_WS_IN_W || H % GS2D_WS_IN_H || W / GS2D_WS_IN_W != H / GS2D_WS_IN_H) return GS2D_ERR_UNSUPPORTED;
  WS_HIP(hipSetDevice(net->device));
  const int64_t hw = (int64_t)W * H;
  if (hw > net->img_cap) {
    if (net->img) WS_HIP(hipFree(net->img));
    if (net->igrad) WS_HIP(hipFree(net->igrad));
    net->img = net->igrad = nullptr;
    net->img_cap = 0;
    WS_TRY(dev_alloc((void**)&net->img, (size_t)8 * hw * sizeof(float)));
    WS_TRY(dev_alloc((void**)&net->igrad, (size_t)4 * hw * sizeof(float)));
    net->img_cap = hw;
  }
  float* rgb = net->img;
  float* depth = rgb + 3 * hw;
  float* normal = rgb + 4 * hw;
  float* alpha = rgb + 7 * hw;
  float* input = net->wsf;
  float* tau = input + kInPlanar + 8;
  uint32_t gen = 0;
  const int f = W / GS2D_WS_IN_W, nb = GS2D_WS_IN_H * GS2D_WS_IN_W;
  float* part = net->igrad;  // per-block loss terms (the image-gradient workspace is free here)
  // loss at the start pose and the network's input
  if (use_masks) {
    WS_TRY(gs2d_render(ctx, params, n, camera, pose_start, rgb, depth, normal, alpha, &gen, s));
    WS_TRY(gs2d_tracking_loss(ctx, camera, rgb, depth, normal, alpha, tgt_rgb, tgt_depth, lambda_d, use_masks,
                              losses, net->igrad, net->igrad + 3 * hw, s));
    WS_TRY(gs2d_ws_residual(rgb, depth, tgt_rgb, tgt_depth, W, H, 1, input, s));
    load_input(net, input, 1, s);
  } else if (f == 8 && n > 0) {
    // the unmasked loss's block terms and the network's BF16 input from the forward
    // blend itself, each wave's 8 x 8 pixels being one block
    WS_TRY(gs2d::render_residual(ctx, params, n, camera, pose_start, tgt_rgb, tgt_depth, lambda_d, net->act[0],
                                 part, s));
  } else {  // the same from the rendered frames, in one pass over them
    WS_TRY(gs2d_render(ctx, params, n, camera, pose_start, rgb, depth, normal, alpha, &gen, s));
    residual_loss_kernel<<<cdiv(nb, 64), 64, 0, s>>>(rgb, depth, tgt_rgb, tgt_depth, W, H, f, lambda_d, net->act[0],
                                                     part);
  }
  // up to fc1's split-K slices; then its sum, fc2, the twist, T_0 = Exp(tau) T_start
  // and (unmasked) the start loss from the residual pass's block sums in one launch
  int S = 0;
  forward_layers(net, 1, nullptr, s, &S);
  propose_close_kernel<<<1, 256, 0, s>>>(net->part, S, net->act[5], net->theta + net->pk.b_off[4], net->pk.wf[5],
                                         net->theta + net->pk.b_off[5], pose_start, pose0, tau,
                                         use_masks ? nullptr : net->igrad, GS2D_WS_IN_H * GS2D_WS_IN_W,
                                         1.f / (float)hw, losses);
  WS_HIP(hipGetLastError());
  return GS2D_OK;
}

}  // namespace

extern "C" {

GS2D_API int gs2d_warm_start_propose(gs2d_ctx* ctx, gs2d_ws* net, const float* params, int64_t n,
                                     const gs2d_camera* camera, const float* pose_start, const float* tgt_rgb,
                                     const float* tgt_depth, float lambda_d, float* pose_out, float* start_loss,
                                     hipStream_t s) {
  if (!start_loss) return GS2D_ERR_INVALID_ARG;
  WS_TRY(propose(ctx, net, params, n, camera, pose_start, tgt_rgb, tgt_depth, lambda_d, 0, pose_out, start_loss,
                 s));
  WS_HIP(hipGetLastError());
  return GS2D_OK;
}

GS2D_API int gs2d_warm_start(gs2d_ctx* ctx, gs2d_ws* net, const float* params, int64_t n, const gs2d_camera* camera,
                             const float* pose_start, const float* tgt_rgb, const float* tgt_depth, float lambda_d,
                             int32_t use_masks, float* pose_out, float* info, hipStream_t s) {
  if (!net || !pose_out) return GS2D_ERR_INVALID_ARG;
  float* pose0 = net->wsf + kInPlanar + 16;
  float* losses = pose0 + 12;
  WS_TRY(propose(ctx, net, params, n, camera, pose_start, tgt_rgb, tgt_depth, lambda_d, use_masks, pose0, losses,
                 s));
  const int W = camera->width, H = camera->height;
  const int64_t hw = (int64_t)W * H;
  float* rgb = net->img;
  float* depth = rgb + 3 * hw;
  float* normal = rgb + 4 * hw;
  float* alpha = rgb + 7 * hw;
  uint32_t gen = 0;
  // loss at T_0, then the choice
  WS_TRY(gs2d_render(ctx, params, n, camera, pose0, rgb, depth, normal, alpha, &gen, s));
  WS_TRY(gs2d_tracking_loss(ctx, camera, rgb, depth, normal, alpha, tgt_rgb, tgt_depth, lambda_d, use_masks,
                            losses + 1, net->igrad, net->igrad + 3 * hw, s));
  choose_pose_kernel<<<1, 64, 0, s>>>(losses, pose_start, pose0, pose_out, info);
  WS_HIP(hipGetLastError());
  return GS2D_OK;
}

}  // extern "C"
