// Mapping loss (Sec. "Mapping") with its gradients to the rendered images:
//   L_m = (1/HW) sum_p [ w_l1 |I_r - I|_1 + w_ssim (1 - SSIM(p)) + w_d |D_r - D|
//                        + w_n (1 - N_D(p) . N_r(p)) ],
// SSIM(p) the mean over RGB of the SSIM map (11 x 11 Gaussian window, sigma 1.5, zero
// outside the image, C1 = 0.01^2, C2 = 0.03^2), N_D the normals of the rendered depth
// (eq:normal_fromD): normalised cross product of the central differences of the
// back-projected pixels, 0 on the image border and where the cross product vanishes.
//
// Two kernels over 16 x 16 pixel tiles with a 5-pixel halo staged in LDS, one colour
// channel at a time:
//  * forward: the 15 windowed statistics of each pixel by a horizontal then a
//    vertical pass, in FP64: the variances E[x^2] - mu^2 cancel in flat regions,
//    and the gradient that follows cancels again, so FP32 statistics leave it only a
//    few bits; SSIM and its per-pixel adjoint coefficients A, B, C (so that
//    dL/dI_r = W*A + 2 I_r (W*B) + I (W*C)); the depth normal, d_normal, and the
//    gradients to the two neighbour differences; one partial of each loss term per
//    workgroup.
//  * backward: the window filter of A, B, C (the Gaussian is symmetric, so the adjoint
//    of the zero-padded filter is the same filter), d_rgb and, gathering the
//    neighbour-difference gradients of the 4 neighbours, d_depth.  Workgroup 0 also
//    adds the forward's partials in a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/gs2d_map.h"

namespace gs2d {
namespace maploss {
namespace {

constexpr int kT = 16;              // output tile side
constexpr int kR = 5;               // window radius
constexpr int kS = kT + 2 * kR;     // staged side, 26
constexpr int kThreads = kT * kT;   // one thread per output pixel
constexpr double kC1 = 0.01 * 0.01;
constexpr double kC2 = 0.03 * 0.03;

struct Win {
  float g[2 * kR + 1];
  double gd[2 * kR + 1];
};

struct Args {
  const float* rgb;
  const float* depth;
  const float* normal;
  const float* trgb;
  const float* tdepth;
  float* d_rgb;
  float* d_depth;
  float* d_normal;
  float* coef;   // 9 planes: A (3 channels), B (3), C (3)
  float* gdiff;  // 6 planes: dL/d(dx) (3), dL/d(dy) (3)
  float* part;   // [tiles][4] partial sums of the four loss terms
  float* loss;   // [5]
  int W, H, tiles_x, n_tiles;
  float fx, fy, cx, cy;
  float w_l1, w_ssim, w_d, w_n;
  Win win;
};

__device__ __forceinline__ float sgn(float v) { return v > 0.f ? 1.f : (v < 0.f ? -1.f : 0.f); }

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

__device__ __forceinline__ float3 cross3(float3 a, float3 b) {
  return make_float3(fmaf(a.y, b.z, -a.z * b.y), fmaf(a.z, b.x, -a.x * b.z), fmaf(a.x, b.y, -a.y * b.x));
}

__global__ __launch_bounds__(kThreads) void maploss_fwd_kernel(Args a) {
  __shared__ float sx[kS][kS], sy[kS][kS];
  __shared__ double hs[5][kS][kT];
  __shared__ float red[4][kThreads / 64];
  const int t = threadIdx.x;
  const int tx0 = (blockIdx.x % a.tiles_x) * kT, ty0 = (blockIdx.x / a.tiles_x) * kT;
  const int HW = a.W * a.H;
  const int ly = t / kT, lx = t - ly * kT;
  const int gx = tx0 + lx, gy = ty0 + ly;
  const bool inside = gx < a.W && gy < a.H;
  const int p = gy * a.W + gx;
  const float inv = 1.0f / (float)HW;
  const double gs = -(double)a.w_ssim / (3.0 * (double)HW);  // dL/dSSIM_ch(p)
  float l1 = 0.f, dssim = 0.f, ld = 0.f, ln = 0.f;
  double ssum = 0.0;
  // one colour channel at a time, so that the staging stays small enough for several
  // workgroups per compute unit
  for (int ch = 0; ch < 3; ++ch) {
    if (ch) __syncthreads();
    for (int k = t; k < kS * kS; k += kThreads) {
      const int r = k / kS, c = k - r * kS;
      const int yy = ty0 - kR + r, xx = tx0 - kR + c;
      const bool in = xx >= 0 && xx < a.W && yy >= 0 && yy < a.H;
      const int q = ch * HW + yy * a.W + xx;
      sx[r][c] = in ? a.rgb[q] : 0.f;
      sy[r][c] = in ? a.trgb[q] : 0.f;
    }
    __syncthreads();
    // horizontal pass: x, y, x^2, y^2, xy along every staged row (FP64; the products of
    // two floats are exact)
    for (int k = t; k < kS * kT; k += kThreads) {
      const int r = k / kT, c = k - r * kT;
      double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0, m4 = 0.0;
#pragma unroll
      for (int j = 0; j < 2 * kR + 1; ++j) {
        const double x = sx[r][c + j], y = sy[r][c + j], g = a.win.gd[j];
        m0 = fma(g, x, m0);
        m1 = fma(g, y, m1);
        m2 = fma(g, x * x, m2);
        m3 = fma(g, y * y, m3);
        m4 = fma(g, x * y, m4);
      }
      hs[0][r][c] = m0;
      hs[1][r][c] = m1;
      hs[2][r][c] = m2;
      hs[3][r][c] = m3;
      hs[4][r][c] = m4;
    }
    __syncthreads();
    if (inside) {
      // vertical pass, SSIM and its adjoint coefficients
      double mx = 0.0, my = 0.0, exx = 0.0, eyy = 0.0, exy = 0.0;
#pragma unroll
      for (int i = 0; i < 2 * kR + 1; ++i) {
        const double g = a.win.gd[i];
        mx = fma(g, hs[0][ly + i][lx], mx);
        my = fma(g, hs[1][ly + i][lx], my);
        exx = fma(g, hs[2][ly + i][lx], exx);
        eyy = fma(g, hs[3][ly + i][lx], eyy);
        exy = fma(g, hs[4][ly + i][lx], exy);
      }
      const double vx = fma(-mx, mx, exx), vy = fma(-my, my, eyy), cxy = fma(-mx, my, exy);
      const double n1 = fma(2.0 * mx, my, kC1), n2 = fma(2.0, cxy, kC2);
      const double d1 = fma(mx, mx, fma(my, my, kC1)), d2 = vx + vy + kC2;
      const double rd = 1.0 / (d1 * d2);
      const double s = n1 * n2 * rd;
      ssum += s;
      // ds/dmu_x (through mu_x, var_x and cov), ds/dE[x^2], ds/dE[xy]
      const double ds_dm = fma(2.0 * my * (n2 - n1), rd, 2.0 * mx * s * (1.0 / d2 - 1.0 / d1));
      const double ds_dxx = -s / d2;
      const double ds_dxy = 2.0 * n1 * rd;
      a.coef[(0 + ch) * HW + p] = (float)(gs * ds_dm);
      a.coef[(3 + ch) * HW + p] = (float)(gs * ds_dxx);
      a.coef[(6 + ch) * HW + p] = (float)(gs * ds_dxy);
      l1 += fabsf(sx[ly + kR][lx + kR] - sy[ly + kR][lx + kR]);
    }
  }
  if (inside) {
    dssim = (float)(1.0 - ssum * (1.0 / 3.0));
    ld = fabsf(a.depth[p] - a.tdepth[p]);
    // depth normal from the central differences of the back-projected neighbours,
    // in the cancellation-free form D(x+1)(x+1-cx) - D(x-1)(x-1-cx) = dD (x-cx) + sD
    float3 nd = make_float3(0.f, 0.f, 0.f), gdx = nd, gdy = nd;
    if (gx >= 1 && gx <= a.W - 2 && gy >= 1 && gy <= a.H - 2) {
      const float xh = ((float)gx - a.cx) / a.fx, yh = ((float)gy - a.cy) / a.fy;
      const float dl = a.depth[p - 1], dr = a.depth[p + 1], du = a.depth[p - a.W], dd = a.depth[p + a.W];
      const float ddx = dr - dl, sdx = dr + dl, ddy = dd - du, sdy = dd + du;
      const float3 vx = make_float3(fmaf(ddx, (float)gx - a.cx, sdx) / a.fx, ddx * yh, ddx);
      const float3 vy = make_float3(ddy * xh, fmaf(ddy, (float)gy - a.cy, sdy) / a.fy, ddy);
      const float3 c = cross3(vx, vy);
      const float c2 = fmaf(c.x, c.x, fmaf(c.y, c.y, c.z * c.z));
      if (c2 > 0.f) {
        const float nc = sqrtf(c2), rn = 1.0f / nc;
        nd = make_float3(c.x * rn, c.y * rn, c.z * rn);
        const float N0 = a.normal[p], N1 = a.normal[HW + p], N2 = a.normal[2 * HW + p];
        const float dot = fmaf(nd.x, N0, fmaf(nd.y, N1, nd.z * N2));
        // dL/dc = -w_n/HW (N - (N_D . N) N_D) / |c|
        const float k = -a.w_n * inv * rn;
        const float3 G = make_float3(k * fmaf(-dot, nd.x, N0), k * fmaf(-dot, nd.y, N1), k * fmaf(-dot, nd.z, N2));
        gdx = cross3(vy, G);  // dL/d(dx) = dy x G
        gdy = cross3(G, vx);  // dL/d(dy) = G x dx
      }
    }
    const float N0 = a.normal[p], N1 = a.normal[HW + p], N2 = a.normal[2 * HW + p];
    ln = 1.0f - fmaf(nd.x, N0, fmaf(nd.y, N1, nd.z * N2));
    const float kn = -a.w_n * inv;
    a.d_normal[p] = kn * nd.x;
    a.d_normal[HW + p] = kn * nd.y;
    a.d_normal[2 * HW + p] = kn * nd.z;
    a.gdiff[0 * HW + p] = gdx.x;
    a.gdiff[1 * HW + p] = gdx.y;
    a.gdiff[2 * HW + p] = gdx.z;
    a.gdiff[3 * HW + p] = gdy.x;
    a.gdiff[4 * HW + p] = gdy.y;
    a.gdiff[5 * HW + p] = gdy.z;
  }
  const float v[4] = {wave_sum(l1), wave_sum(dssim), wave_sum(ld), wave_sum(ln)};
  if ((t & 63) == 0)
#pragma unroll
    for (int q = 0; q < 4; ++q) red[q][t >> 6] = v[q];
  __syncthreads();
  if (t < 4) {
    float s = 0.f;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) s += red[t][w];
    a.part[blockIdx.x * 4 + t] = s;
  }
}

__global__ __launch_bounds__(kThreads) void maploss_bwd_kernel(Args a) {
  __shared__ float sc[3][kS][kS];
  __shared__ float hc[3][kS][kT];
  __shared__ float red[4][kThreads / 64];
  const int t = threadIdx.x;
  const int tx0 = (blockIdx.x % a.tiles_x) * kT, ty0 = (blockIdx.x / a.tiles_x) * kT;
  const int HW = a.W * a.H;
  const int ly = t / kT, lx = t - ly * kT;
  const int gx = tx0 + lx, gy = ty0 + ly;
  const bool inside = gx < a.W && gy < a.H;
  const int p = gy * a.W + gx;
  const float inv = 1.0f / (float)HW;
  // one colour channel at a time: its A, B, C planes filtered, then its d_rgb
  for (int ch = 0; ch < 3; ++ch) {
    if (ch) __syncthreads();
    for (int k = t; k < kS * kS; k += kThreads) {
      const int r = k / kS, c = k - r * kS;
      const int yy = ty0 - kR + r, xx = tx0 - kR + c;
      const bool in = xx >= 0 && xx < a.W && yy >= 0 && yy < a.H;
      const int q = yy * a.W + xx;
#pragma unroll
      for (int m = 0; m < 3; ++m) sc[m][r][c] = in ? a.coef[(3 * m + ch) * HW + q] : 0.f;
    }
    __syncthreads();
    for (int k = t; k < 3 * kS * kT; k += kThreads) {
      const int m = k / (kS * kT), rem = k - m * (kS * kT), r = rem / kT, c = rem - r * kT;
      float acc = 0.f;
#pragma unroll
      for (int j = 0; j < 2 * kR + 1; ++j) acc = fmaf(a.win.g[j], sc[m][r][c + j], acc);
      hc[m][r][c] = acc;
    }
    __syncthreads();
    if (inside) {
      float f[3];
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        float acc = 0.f;
#pragma unroll
        for (int i = 0; i < 2 * kR + 1; ++i) acc = fmaf(a.win.g[i], hc[m][ly + i][lx], acc);
        f[m] = acc;
      }
      const float x = a.rgb[ch * HW + p], y = a.trgb[ch * HW + p];
      a.d_rgb[ch * HW + p] = fmaf(a.w_l1 * inv, sgn(x - y), fmaf(2.f * x, f[1], fmaf(y, f[2], f[0])));
    }
  }
  if (inside) {
    // d_depth: the depth L1 term, and the gradients of the neighbour differences that
    // contain this pixel: +dx of the left neighbour, -dx of the right one, +dy of the one
    // above, -dy of the one below (zero outside the image)
    float3 acc = make_float3(0.f, 0.f, 0.f);
    if (gx >= 1) {
      const int o = p - 1;
      acc.x += a.gdiff[o], acc.y += a.gdiff[HW + o], acc.z += a.gdiff[2 * HW + o];
    }
    if (gx <= a.W - 2) {
      const int o = p + 1;
      acc.x -= a.gdiff[o], acc.y -= a.gdiff[HW + o], acc.z -= a.gdiff[2 * HW + o];
    }
    if (gy >= 1) {
      const int o = p - a.W;
      acc.x += a.gdiff[3 * HW + o], acc.y += a.gdiff[4 * HW + o], acc.z += a.gdiff[5 * HW + o];
    }
    if (gy <= a.H - 2) {
      const int o = p + a.W;
      acc.x -= a.gdiff[3 * HW + o], acc.y -= a.gdiff[4 * HW + o], acc.z -= a.gdiff[5 * HW + o];
    }
    const float xh = ((float)gx - a.cx) / a.fx, yh = ((float)gy - a.cy) / a.fy;
    const float dr = fmaf(acc.x, xh, fmaf(acc.y, yh, acc.z));
    a.d_depth[p] = fmaf(a.w_d * inv, sgn(a.depth[p] - a.tdepth[p]), dr);
  }
  if (blockIdx.x == 0) {
    // the loss: wave q adds term q's partials in a fixed order
    const int wave = t >> 6, lane = t & 63;
    float s = 0.f;
    for (int b = lane; b < a.n_tiles; b += 64) s += a.part[b * 4 + wave];
    s = wave_sum(s);
    if (lane == 0) red[wave][0] = s;
    __syncthreads();
    if (t == 0) {
      const float inv = 1.0f / (float)HW;
      const float m1 = red[0][0] * inv, m2 = red[1][0] * inv, m3 = red[2][0] * inv, m4 = red[3][0] * inv;
      a.loss[1] = m1;
      a.loss[2] = m2;
      a.loss[3] = m3;
      a.loss[4] = m4;
      a.loss[0] = fmaf(a.w_l1, m1, fmaf(a.w_ssim, m2, fmaf(a.w_d, m3, a.w_n * m4)));
    }
  }
}

Win make_window() {
  double g[2 * kR + 1], s = 0.0;
  for (int i = -kR; i <= kR; ++i) s += g[i + kR] = std::exp(-(double)(i * i) / (2.0 * 1.5 * 1.5));
  Win w;
  for (int i = 0; i < 2 * kR + 1; ++i) {
    w.gd[i] = g[i] / s;
    w.g[i] = (float)w.gd[i];
  }
  return w;
}

}  // namespace
}  // namespace maploss
}  // namespace gs2d

using namespace gs2d::maploss;

GS2D_API int64_t gs2d_mapping_loss_workspace(int32_t width, int32_t height) {
  if (width <= 0 || height <= 0) return 0;
  const int64_t tiles = (int64_t)((width + kT - 1) / kT) * ((height + kT - 1) / kT);
  return 15 * (int64_t)width * height + 4 * tiles;
}

GS2D_API int gs2d_mapping_loss(const gs2d_camera* camera, const float* rgb, const float* depth, const float* normal,
                               const float* tgt_rgb, const float* tgt_depth, const gs2d_mapping_weights* weights,
                               float* loss, float* d_rgb, float* d_depth, float* d_normal, float* work,
                               hipStream_t stream) {
  if (!camera || camera->width <= 0 || camera->height <= 0 || !rgb || !depth || !normal || !tgt_rgb || !tgt_depth ||
      !loss || !d_rgb || !d_depth || !d_normal || !work || !(camera->fx != 0.f) || !(camera->fy != 0.f) ||
      (int64_t)camera->width * camera->height > (1ll << 30))
    return GS2D_ERR_INVALID_ARG;
  Args a{};
  a.rgb = rgb;
  a.depth = depth;
  a.normal = normal;
  a.trgb = tgt_rgb;
  a.tdepth = tgt_depth;
  a.d_rgb = d_rgb;
  a.d_depth = d_depth;
  a.d_normal = d_normal;
  a.W = camera->width;
  a.H = camera->height;
  const int64_t HW = (int64_t)a.W * a.H;
  a.coef = work;
  a.gdiff = work + 9 * HW;
  a.part = work + 15 * HW;
  a.loss = loss;
  a.tiles_x = (a.W + kT - 1) / kT;
  a.n_tiles = a.tiles_x * ((a.H + kT - 1) / kT);
  a.fx = camera->fx;
  a.fy = camera->fy;
  a.cx = camera->cx;
  a.cy = camera->cy;
  const gs2d_mapping_weights w = weights ? *weights : gs2d_mapping_weights{0.875f, 0.125f, 0.5f, 0.02f};
  a.w_l1 = w.w_l1;
  a.w_ssim = w.w_ssim;
  a.w_d = w.w_d;
  a.w_n = w.w_n;
  a.win = make_window();
  maploss_fwd_kernel<<<a.n_tiles, kThreads, 0, stream>>>(a);
  maploss_bwd_kernel<<<a.n_tiles, kThreads, 0, stream>>>(a);
  return hipGetLastError() == hipSuccess ? GS2D_OK : GS2D_ERR_HIP;
}
