// The learned pose warm start: a BF16 convolutional network on the matrix cores.
//
// Every layer, forward and backward, is one GEMM C[M][N] = sum_k A(m, k) B(k, n)
// in a single kernel template: 256 threads, a 64 x 64 tile of C, K in steps of
// 32.  Each step gathers the A and B sub-tiles (64 x 32 BF16 each) through the
// layer's own index functions -- convolutions as implicit GEMMs, no im2col buffer
// -- into LDS; each of the 4 waves then issues 2 x 2 v_mfma_f32_16x16x32_bf16 on
// its 32 x 32 quarter, accumulating in FP32.  The layer's epilogue adds the bias,
// applies ReLU (or, in the backward, the ReLU mask of the layer's input), rounds to
// BF16 and stores; weight gradients go to FP32 partial sums over split-K slices
// that a second kernel adds in a fixed order (deterministic), a constant-one
// column of B giving the bias gradient in the same GEMM.
//
//   layer              M        N              K
//   conv forward       Co       B OH OW        Ci k k
//   conv input grad    Ci       B H W          Co k k   (stride-2 taps only)
//   conv weight grad   Co       Ci k k + 1     B OH OW  (split-K)
//   fc forward         O        B              I
//   fc input grad      I        B              O
//   fc weight grad     O        I + 1          B
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

namespace gs2d {
namespace ws {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kBM = 64, kBN = 64, kBK = 32, kPad = 8, kThreads = 256;
constexpr uint16_t kOne = 0x3F80;  // bfloat16 1.0

// Round to the nearest bfloat16, ties to even (finite inputs; NaN stays NaN).
__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// Post-ReLU activations are positive exactly when the sign bit is clear and they are not zero.
__device__ __forceinline__ bool positive(uint16_t h) { return h != 0 && !(h & 0x8000u); }

template <class Op>
__global__ __launch_bounds__(kThreads) void gemm_kernel(Op op, int M, int N, int K, int k_split) {
  __shared__ __attribute__((aligned(16))) uint16_t As[kBM][kBK + kPad];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[kBN][kBK + kPad];
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
  const int kb = blockIdx.z * k_split, ke = min(K, kb + k_split);
  const int r = t >> 2, kc = (t & 3) * 8;  // this thread's row (of A and of B^T) and k chunk
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int li = lane & 15, g = lane >> 4;
  const int m = m0 + r, n = n0 + r;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kb; k0 < ke; k0 += kBK) {
    // each op gathers 8 consecutive k of one row (zero past ke): the index is
    // decomposed once per chunk and stepped across the 8
    uint16_t va[8], vb[8];
    if (m < M)
      op.a8(m, k0 + kc, ke, va);
    else
#pragma unroll
      for (int i = 0; i < 8; ++i) va[i] = 0;
    if (n < N)
      op.b8(k0 + kc, n, ke, vb);
    else
#pragma unroll
      for (int i = 0; i < 8; ++i) vb[i] = 0;
    __syncthreads();  // the previous step's fragments have been read
    uint4 pa, pb;
    pa.x = va[0] | ((uint32_t)va[1] << 16);
    pa.y = va[2] | ((uint32_t)va[3] << 16);
    pa.z = va[4] | ((uint32_t)va[5] << 16);
    pa.w = va[6] | ((uint32_t)va[7] << 16);
    pb.x = vb[0] | ((uint32_t)vb[1] << 16);
    pb.y = vb[2] | ((uint32_t)vb[3] << 16);
    pb.z = vb[4] | ((uint32_t)vb[5] << 16);
    pb.w = vb[6] | ((uint32_t)vb[7] << 16);
    *reinterpret_cast<uint4*>(&As[r][kc]) = pa;
    *reinterpret_cast<uint4*>(&Bs[r][kc]) = pb;
    __syncthreads();
    bf16x8 fa[2], fb[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      fa[i] = *reinterpret_cast<const bf16x8*>(&As[wm + i * 16 + li][g * 8]);
      fb[i] = *reinterpret_cast<const bf16x8*>(&Bs[wn + i * 16 + li][g * 8]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int mm = m0 + wm + i * 16 + g * 4 + q, nn = n0 + wn + j * 16 + li;
        if (mm < M && nn < N) op.store(mm, nn, acc[i][j][q]);
      }
}

// Shapes of one stride-2 convolution over a batch (kernel side KS fixed by the op).
struct ConvShape {
  int B, ci, co, k, H, W, OH, OW;
};

// 8 consecutive values of a contiguous row, zero past `end`.
__device__ __forceinline__ void row8(const uint16_t* __restrict__ p, int k, int end, uint16_t* out) {
#pragma unroll
  for (int i = 0; i < 8; ++i) out[i] = k + i < end ? p[k + i] : (uint16_t)0;
}

// y = bf16(relu(conv(x, w) + bias)): M = co, N = B OH OW, K = ci KS KS.
template <int KS>
struct ConvFwd {
  ConvShape s;
  const uint16_t* w;
  const float* bias;
  const uint16_t* x;
  uint16_t* y;
  __device__ void a8(int m, int k, int ke, uint16_t* out) const {
    row8(w + (size_t)m * (s.ci * KS * KS), k, ke, out);
  }
  __device__ void b8(int k, int n, int ke, uint16_t* out) const {
    const int ohw = s.OH * s.OW;
    const int bi = n / ohw, rr = n - bi * ohw, oy = rr / s.OW, ox = rr - oy * s.OW;
    const int iy0 = 2 * oy - KS / 2, ix0 = 2 * ox - KS / 2;
    const uint16_t* __restrict__ xb = x + (size_t)bi * s.ci * s.H * s.W;
    int c = k / (KS * KS), t = k - c * (KS * KS), ky = t / KS, kx = t - ky * KS;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int iy = iy0 + ky, ix = ix0 + kx;
      out[i] = (k + i < ke && iy >= 0 && iy < s.H && ix >= 0 && ix < s.W) ? xb[((size_t)c * s.H + iy) * s.W + ix]
                                                                           : (uint16_t)0;
      if (++kx == KS) {
        kx = 0;
        if (++ky == KS) {
          ky = 0;
          ++c;
        }
      }
    }
  }
  __device__ void store(int m, int n, float v) const {
    const int ohw = s.OH * s.OW, bi = n / ohw, rr = n - bi * ohw;
    v += bias[m];
    y[((size_t)bi * s.co + m) * ohw + rr] = to_bf16(v > 0.f ? v : 0.f);
  }
};

// Input gradient of a convolution, masked by the ReLU of its input:
// gx = bf16(conv^T(gy, w) [x > 0]): M = ci, N = B H W, K = co KS KS.
template <int KS>
struct ConvBwdData {
  ConvShape s;
  const uint16_t* w;
  const uint16_t* gy;  // [B][co][OH][OW]
  const uint16_t* x;   // the layer's input (post-ReLU)
  uint16_t* gx;        // [B][ci][H][W]
  __device__ void a8(int m, int k, int ke, uint16_t* out) const {
    constexpr int KK = KS * KS;
    int o = k / KK, t = k - o * KK;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      out[i] = k + i < ke ? w[((size_t)o * s.ci + m) * KK + t] : (uint16_t)0;
      if (++t == KK) {
        t = 0;
        ++o;
      }
    }
  }
  __device__ void b8(int k, int n, int ke, uint16_t* out) const {
    const int hw = s.H * s.W;
    const int bi = n / hw, rr = n - bi * hw, iy = rr / s.W, ix = rr - iy * s.W;
    const uint16_t* __restrict__ gb = gy + (size_t)bi * s.co * s.OH * s.OW;
    int o = k / (KS * KS), t = k - o * (KS * KS), ky = t / KS, kx = t - ky * KS;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int ty = iy + KS / 2 - ky, tx = ix + KS / 2 - kx;  // = 2 oy, 2 ox
      const int oy = ty >> 1, ox = tx >> 1;
      const bool ok = k + i < ke && ty >= 0 && tx >= 0 && !(ty & 1) && !(tx & 1) && oy < s.OH && ox < s.OW;
      out[i] = ok ? gb[((size_t)o * s.OH + oy) * s.OW + ox] : (uint16_t)0;
      if (++kx == KS) {
        kx = 0;
        if (++ky == KS) {
          ky = 0;
          ++o;
        }
      }
    }
  }
  __device__ void store(int m, int n, float v) const {
    const int hw = s.H * s.W, bi = n / hw, rr = n - bi * hw;
    const size_t idx = ((size_t)bi * s.ci + m) * hw + rr;
    gx[idx] = to_bf16(positive(x[idx]) ? v : 0.f);
  }
};

// Weight and bias gradient of a convolution, one split-K slice per blockIdx.z:
// part[z][co][ci KS KS + 1] = sum_n gy[co][n] [x patch | 1][n].
template <int KS>
struct ConvBwdWeight {
  ConvShape s;
  const uint16_t* gy;
  const uint16_t* x;
  float* part;
  int ncol;  // ci KS KS + 1
  int M;
  __device__ void a8(int m, int k, int ke, uint16_t* out) const {
    const int ohw = s.OH * s.OW;
    int bi = k / ohw, rr = k - bi * ohw;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      out[i] = k + i < ke ? gy[((size_t)bi * s.co + m) * ohw + rr] : (uint16_t)0;
      if (++rr == ohw) {
        rr = 0;
        ++bi;
      }
    }
  }
  __device__ void b8(int k, int n, int ke, uint16_t* out) const {
    if (n == ncol - 1) {
#pragma unroll
      for (int i = 0; i < 8; ++i) out[i] = k + i < ke ? kOne : (uint16_t)0;
      return;
    }
    const int c = n / (KS * KS), t = n - c * (KS * KS), ky = t / KS, kx = t - ky * KS;
    const int ohw = s.OH * s.OW;
    int bi = k / ohw, rr = k - bi * ohw, oy = rr / s.OW, ox = rr - oy * s.OW;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int iy = 2 * oy + ky - KS / 2, ix = 2 * ox + kx - KS / 2;
      const bool ok = k + i < ke && iy >= 0 && iy < s.H && ix >= 0 && ix < s.W;
      out[i] = ok ? x[(((size_t)bi * s.ci + c) * s.H + iy) * s.W + ix] : (uint16_t)0;
      if (++ox == s.OW) {
        ox = 0;
        if (++oy == s.OH) {
          oy = 0;
          ++bi;
        }
      }
    }
  }
  __device__ void store(int m, int n, float v) const { part[((size_t)blockIdx.z * M + m) * ncol + n] = v; }
};

// Fully connected forward: y[b][o] = sum_i w[o][i] x[b][i] + bias[o]; M = O, N = B, K = I.
struct FcFwd {
  int I, O;
  const uint16_t* w;
  const float* bias;
  const uint16_t* x;
  uint16_t* y;   // ReLU + bf16 (hidden layer), or
  float* yf;     // FP32, no ReLU (output layer)
  __device__ void a8(int m, int k, int ke, uint16_t* out) const { row8(w + (size_t)m * I, k, ke, out); }
  __device__ void b8(int k, int n, int ke, uint16_t* out) const { row8(x + (size_t)n * I, k, ke, out); }
  __device__ void store(int m, int n, float v) const {
    v += bias[m];
    if (yf)
      yf[(size_t)n * O + m] = v;
    else
      y[(size_t)n * O + m] = to_bf16(v > 0.f ? v : 0.f);
  }
};

// Fully connected input gradient, masked by the ReLU of the input:
// gx[b][i] = bf16(sum_o w[o][i] gy[b][o] [x > 0]); M = I, N = B, K = O.
struct FcBwdData {
  int I, O;
  const uint16_t* w;
  const uint16_t* gy;
  const uint16_t* x;
  uint16_t* gx;
  __device__ void a8(int m, int k, int ke, uint16_t* out) const {
#pragma unroll
    for (int i = 0; i < 8; ++i) out[i] = k + i < ke ? w[(size_t)(k + i) * I + m] : (uint16_t)0;
  }
  __device__ void b8(int k, int n, int ke, uint16_t* out) const { row8(gy + (size_t)n * O, k, ke, out); }
  __device__ void store(int m, int n, float v) const {
    const size_t idx = (size_t)n * I + m;
    gx[idx] = to_bf16(positive(x[idx]) ? v : 0.f);
  }
};

// Fully connected weight and bias gradient: part[z][o][I + 1] = sum_b gy[b][o] [x[b] | 1].
struct FcBwdWeight {
  int I, O;
  const uint16_t* gy;
  const uint16_t* x;
  float* part;
  __device__ void a8(int m, int k, int ke, uint16_t* out) const {
#pragma unroll
    for (int i = 0; i < 8; ++i) out[i] = k + i < ke ? gy[(size_t)(k + i) * O + m] : (uint16_t)0;
  }
  __device__ void b8(int k, int n, int ke, uint16_t* out) const {
#pragma unroll
    for (int i = 0; i < 8; ++i) out[i] = k + i < ke ? (n == I ? kOne : x[(size_t)(k + i) * I + n]) : (uint16_t)0;
  }
  __device__ void store(int m, int n, float v) const { part[((size_t)blockIdx.z * O + m) * (I + 1) + n] = v; }
};

// grad[w_off + m ncol' + j] (j < ncol - 1) and grad[b_off + m] (j = ncol - 1) = the sum
// of the split-K partials in slice order.
__global__ void reduce_parts_kernel(const float* __restrict__ part, int splits, int M, int ncol,
                                    float* __restrict__ gw, float* __restrict__ gb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M * ncol) return;
  float s = 0.f;
  for (int z = 0; z < splits; ++z) s += part[(size_t)z * M * ncol + i];
  const int m = i / ncol, j = i - m * ncol;
  if (j == ncol - 1)
    gb[m] = s;
  else
    gw[(size_t)m * (ncol - 1) + j] = s;
}

__global__ void to_bf16_kernel(const float* __restrict__ x, uint16_t* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = to_bf16(x[i]);
}

// Mean squared error over n = B x 6 values (one workgroup, fixed-order sums), its
// gradient 2 d / n rounded to bfloat16, and the FP32 loss.
__global__ __launch_bounds__(256) void mse_kernel(const float* __restrict__ out, const float* __restrict__ target,
                                                  int n, uint16_t* __restrict__ gout, float* __restrict__ loss) {
  __shared__ float sh[256];
  float s = 0.f;
  for (int i = threadIdx.x; i < n; i += 256) {
    const float d = out[i] - target[i];
    s = fmaf(d, d, s);
    gout[i] = to_bf16(2.0f * d / (float)n);
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) *loss = sh[0] / (float)n;
}

// AdamW on the FP32 master vector (bias corrections c1 = 1 - b1^t, c2 = 1 - b2^t from
// the host), then the BF16 copy.
__global__ void adamw_kernel(float* __restrict__ theta, float* __restrict__ m, float* __restrict__ v,
                             const float* __restrict__ g, uint16_t* __restrict__ wb, int n, gs2d_ws_adamw o,
                             float c1, float c2) {
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
  wb[i] = to_bf16(th);
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

// tau = denormalised network output (rho x 0.1 m, phi x 8 deg).
__global__ void denormalise_kernel(const float* __restrict__ out, float* __restrict__ tau) {
  const int i = threadIdx.x;
  if (i < 6) tau[i] = out[i] * (i < 3 ? 0.1f : (float)(8.0 * M_PI / 180.0));
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
int64_t act_size(int li) {  // per frame, output of layer li (li = -1: the input)
  if (li < 0) return (int64_t)GS2D_WS_IN_C * GS2D_WS_IN_H * GS2D_WS_IN_W;
  const LayerDef& L = kLayers[li];
  if (L.k) return (int64_t)L.co * out_size(L.H, L.k) * out_size(L.W, L.k);
  return L.co;
}

template <class Op>
void gemm(const Op& op, int M, int N, int K, int splits, hipStream_t s) {
  const int ks = ((K + splits - 1) / splits + kBK - 1) / kBK * kBK;
  dim3 grid((N + kBN - 1) / kBN, (M + kBM - 1) / kBM, splits);
  gemm_kernel<Op><<<grid, kThreads, 0, s>>>(op, M, N, K, ks);
}

// A forward layer with few output tiles (small batches) and a long reduction: each
// split-K slice writes FP32 partial sums, and a second kernel adds them in slice
// order and applies the layer's own epilogue (bias, ReLU, rounding) to the total.
template <class Op>
struct SplitPart {
  Op op;
  float* part;
  int M, N;
  __device__ void a8(int m, int k, int ke, uint16_t* o) const { op.a8(m, k, ke, o); }
  __device__ void b8(int k, int n, int ke, uint16_t* o) const { op.b8(k, n, ke, o); }
  __device__ void store(int m, int n, float v) const { part[((size_t)blockIdx.z * M + m) * N + n] = v; }
};

template <class Op>
__global__ void split_finish_kernel(Op op, const float* __restrict__ part, int S, int M, int N) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M * N) return;
  float v = 0.f;
  for (int z = 0; z < S; ++z) v += part[(size_t)z * M * N + i];
  op.store(i / N, i - (i / N) * N, v);
}

template <class Op>
void gemm_fwd(const Op& op, int M, int N, int K, float* part, int64_t part_cap, hipStream_t s) {
  const int tiles = ((N + kBN - 1) / kBN) * ((M + kBM - 1) / kBM);
  int S = 1;
  if (tiles < 64 && K >= 256) {
    S = K / 128;
    const int want = (128 + tiles - 1) / tiles;  // about 128 workgroups in all
    S = S < want ? S : want;
  }
  if (S > 1 && (int64_t)S * M * N <= part_cap) {
    gemm(SplitPart<Op>{op, part, M, N}, M, N, K, S, s);
    split_finish_kernel<Op><<<(M * N + 255) / 256, 256, 0, s>>>(op, part, S, M, N);
  } else {
    gemm(op, M, N, K, 1, s);
  }
}

int splits_for(int64_t K) {  // split-K slices of about 2048 reduction steps
  int64_t s = (K + 2047) / 2048;
  return (int)(s < 1 ? 1 : (s > 512 ? 512 : s));
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
  uint16_t* wb = nullptr;   // BF16 copy [P]
  uint16_t* act[7] = {};    // BF16 activations: input, conv1..4, fc1 ([max_batch] frames each)
  uint16_t* gact[7] = {};   // BF16 gradients of the same (pre-ReLU for layer outputs)
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
  int64_t w_off[6] = {}, b_off[6] = {};
};

namespace {

using namespace gs2d::ws;

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

// Partial-sum floats of every weight-gradient GEMM of a batch (the largest one).
int64_t part_need(int B) {
  int64_t need = 0;
  for (int li = 0; li < 6; ++li) {
    const LayerDef& L = kLayers[li];
    int64_t M, ncol, K;
    if (L.k) {
      M = L.co;
      ncol = (int64_t)L.ci * L.k * L.k + 1;
      K = (int64_t)B * out_size(L.H, L.k) * out_size(L.W, L.k);
    } else {
      M = L.co;
      ncol = L.ci + 1;
      K = B;
    }
    const int64_t sz = (int64_t)splits_for(K) * M * ncol;
    need = sz > need ? sz : need;
  }
  return need;
}

ConvShape conv_shape(int li, int B) {
  const LayerDef& L = kLayers[li];
  return ConvShape{B, L.ci, L.co, L.k, L.H, L.W, out_size(L.H, L.k), out_size(L.W, L.k)};
}

// Forward of `batch` frames whose BF16 input is in act[0]; FP32 output to net->out.
void forward_layers(gs2d_ws* net, int B, hipStream_t s) {
  for (int li = 0; li < 4; ++li) {
    const ConvShape cs = conv_shape(li, B);
    const uint16_t* w = net->wb + net->w_off[li];
    const float* b = net->theta + net->b_off[li];
    if (cs.k == 5)
      gemm_fwd(ConvFwd<5>{cs, w, b, net->act[li], net->act[li + 1]}, cs.co, B * cs.OH * cs.OW, cs.ci * 25,
               net->part, net->part_cap, s);
    else
      gemm_fwd(ConvFwd<3>{cs, w, b, net->act[li], net->act[li + 1]}, cs.co, B * cs.OH * cs.OW, cs.ci * 9,
               net->part, net->part_cap, s);
  }
  {
    FcFwd op{2560, 256, net->wb + net->w_off[4], net->theta + net->b_off[4], net->act[4], net->act[5], nullptr};
    gemm_fwd(op, 256, B, 2560, net->part, net->part_cap, s);
  }
  {
    FcFwd op{256, 6, net->wb + net->w_off[5], net->theta + net->b_off[5], net->act[5], nullptr, net->out};
    gemm_fwd(op, 6, B, 256, net->part, net->part_cap, s);
  }
}

int weight_grad(gs2d_ws* net, int li, int B, hipStream_t s) {
  const LayerDef& L = kLayers[li];
  float* gw = net->grad + net->w_off[li];
  float* gb = net->grad + net->b_off[li];
  if (L.k) {
    const ConvShape cs = conv_shape(li, B);
    const int ncol = cs.ci * cs.k * cs.k + 1, K = B * cs.OH * cs.OW, sp = splits_for(K);
    if (cs.k == 5)
      gemm(ConvBwdWeight<5>{cs, net->gact[li + 1], net->act[li], net->part, ncol, cs.co}, cs.co, ncol, K, sp, s);
    else
      gemm(ConvBwdWeight<3>{cs, net->gact[li + 1], net->act[li], net->part, ncol, cs.co}, cs.co, ncol, K, sp, s);
    reduce_parts_kernel<<<(cs.co * ncol + 255) / 256, 256, 0, s>>>(net->part, sp, cs.co, ncol, gw, gb);
  } else {
    const int sp = splits_for(B);
    FcBwdWeight op{L.ci, L.co, net->gact[li + 1], net->act[li], net->part};
    gemm(op, L.co, L.ci + 1, B, sp, s);
    reduce_parts_kernel<<<(L.co * (L.ci + 1) + 255) / 256, 256, 0, s>>>(net->part, sp, L.co, L.ci + 1, gw, gb);
  }
  return GS2D_OK;
}

int check_net(gs2d_ws* net, int batch) {
  if (!net || batch < 1 || batch > net->max_batch) return GS2D_ERR_INVALID_ARG;
  WS_HIP(hipSetDevice(net->device));
  return GS2D_OK;
}

void load_input(gs2d_ws* net, const float* input, int B, hipStream_t s) {
  const int64_t n = (int64_t)B * act_size(-1);
  to_bf16_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(input, net->act[0], n);
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
  int64_t o = 0;
  for (int li = 0; li < 6; ++li) {
    net->w_off[li] = o;
    o += layer_weights(kLayers[li]);
    net->b_off[li] = o;
    o += kLayers[li].co;
  }
  const int64_t P = o;
  int r = GS2D_OK;
  if (r == GS2D_OK) r = dev_alloc((void**)&net->theta, P * sizeof(float));
  if (r == GS2D_OK) r = dev_alloc((void**)&net->m, P * sizeof(float));
  if (r == GS2D_OK) r = dev_alloc((void**)&net->v, P * sizeof(float));
  if (r == GS2D_OK) r = dev_alloc((void**)&net->grad, P * sizeof(float));
  if (r == GS2D_OK) r = dev_alloc((void**)&net->wb, P * sizeof(uint16_t));
  for (int i = 0; i < 6 && r == GS2D_OK; ++i) {
    const size_t bytes = (size_t)max_batch * act_size(i - 1) * sizeof(uint16_t);
    r = dev_alloc((void**)&net->act[i], bytes);
    if (r == GS2D_OK) r = dev_alloc((void**)&net->gact[i], bytes);
  }
  if (r == GS2D_OK) r = dev_alloc((void**)&net->gact[6], (size_t)max_batch * 6 * sizeof(uint16_t));
  if (r == GS2D_OK) r = dev_alloc((void**)&net->out, (size_t)max_batch * 6 * sizeof(float));
  if (r == GS2D_OK) r = dev_alloc((void**)&net->lossbuf, 4 * sizeof(float));
  // warm-start scratch: input [4][60][80], out [8], tau [8], pose0 [12], losses [2]
  if (r == GS2D_OK) r = dev_alloc((void**)&net->wsf, (act_size(-1) + 64) * sizeof(float));
  if (r == GS2D_OK) r = ensure_part(net, part_need(max_batch));
  if (r == GS2D_OK && (hipMemset(net->theta, 0, P * sizeof(float)) != hipSuccess ||
                       hipMemset(net->m, 0, P * sizeof(float)) != hipSuccess ||
                       hipMemset(net->v, 0, P * sizeof(float)) != hipSuccess ||
                       hipMemset(net->wb, 0, P * sizeof(uint16_t)) != hipSuccess))
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
  if (net->wb) (void)hipFree(net->wb);
  for (int i = 0; i < 7; ++i) {
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
  to_bf16_kernel<<<(unsigned)((P + 255) / 256), 256, 0, s>>>(net->theta, net->wb, P);
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
  const int64_t n = (int64_t)batch * act_size(-1);
  residual_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(rgb, depth, tgt_rgb, tgt_depth, width, height, f,
                                                               batch, input);
  WS_HIP(hipGetLastError());
  return GS2D_OK;
}

GS2D_API int gs2d_ws_forward(gs2d_ws* net, const float* input, int32_t batch, float* out, hipStream_t s) {
  WS_TRY(check_net(net, batch));
  if (!input || !out) return GS2D_ERR_INVALID_ARG;
  load_input(net, input, batch, s);
  forward_layers(net, batch, s);
  WS_HIP(hipMemcpyAsync(out, net->out, (size_t)batch * 6 * sizeof(float), hipMemcpyDeviceToDevice, s));
  WS_HIP(hipGetLastError());
  return GS2D_OK;
}

GS2D_API int gs2d_ws_gradient(gs2d_ws* net, const float* input, const float* target, int32_t batch, float* loss,
                              float* out, float* grad, hipStream_t s) {
  WS_TRY(check_net(net, batch));
  if (!input || !target) return GS2D_ERR_INVALID_ARG;
  const int B = batch;
  load_input(net, input, B, s);
  forward_layers(net, B, s);
  mse_kernel<<<1, 256, 0, s>>>(net->out, target, B * 6, net->gact[6], net->lossbuf);
  // fc2: weights, then the masked input gradient of h1
  WS_TRY(weight_grad(net, 5, B, s));
  {
    FcBwdData op{256, 6, net->wb + net->w_off[5], net->gact[6], net->act[5], net->gact[5]};
    gemm(op, 256, B, 6, 1, s);
  }
  WS_TRY(weight_grad(net, 4, B, s));
  {
    FcBwdData op{2560, 256, net->wb + net->w_off[4], net->gact[5], net->act[4], net->gact[4]};
    gemm(op, 2560, B, 256, 1, s);
  }
  for (int li = 3; li >= 0; --li) {
    WS_TRY(weight_grad(net, li, B, s));
    if (li > 0) {
      const ConvShape cs = conv_shape(li, B);
      // layers 1-3 (the input gradient of layer 0 is not needed) are all 3 x 3
      ConvBwdData<3> op{cs, net->wb + net->w_off[li], net->gact[li + 1], net->act[li], net->gact[li]};
      gemm(op, cs.ci, B * cs.H * cs.W, cs.co * 9, 1, s);
    }
  }
  if (loss) WS_HIP(hipMemcpyAsync(loss, net->lossbuf, sizeof(float), hipMemcpyDeviceToDevice, s));
  if (out) WS_HIP(hipMemcpyAsync(out, net->out, (size_t)B * 6 * sizeof(float), hipMemcpyDeviceToDevice, s));
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
  adamw_kernel<<<(P + 255) / 256, 256, 0, s>>>(net->theta, net->m, net->v, net->grad, net->wb, P, *o, c1, c2);
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
  float* out = input + act_size(-1);
  float* tau = out + 8;
  uint32_t gen = 0;
  // loss at the start pose and the network's input
  WS_TRY(gs2d_render(ctx, params, n, camera, pose_start, rgb, depth, normal, alpha, &gen, s));
  WS_TRY(gs2d_tracking_loss(ctx, camera, rgb, depth, normal, alpha, tgt_rgb, tgt_depth, lambda_d, use_masks, losses,
                            net->igrad, net->igrad + 3 * hw, s));
  WS_TRY(gs2d_ws_residual(rgb, depth, tgt_rgb, tgt_depth, W, H, 1, input, s));
  WS_TRY(gs2d_ws_forward(net, input, 1, out, s));
  denormalise_kernel<<<1, 64, 0, s>>>(out, tau);
  WS_TRY(gs2d_pose_exp(ctx, tau, pose_start, pose0, s));
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
  float* pose0 = net->wsf + act_size(-1) + 16;
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
