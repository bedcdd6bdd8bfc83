// Per-surfel preprocessing (forward) and its reverse mode with the pose reduction.
//
// Forward, one thread per surfel (Sec. "2D Gaussian Splatting", eq:hc and eq:wth):
// camera-frame centre and tangents, the homography M = K [s_u t_uc | s_v t_vc | mu_c],
// culling, the screen box of the 3-sigma ellipse (dual conic M diag(9,9,-1) M^T)
// united with the low-pass disc, its tile rectangle, the float32 depth key, and the
// blend record.  The kernel is bound by HBM traffic (60 B in, about 110 B
// out per surfel), so it computes in FP64 at no cost and rounds once at the end:
// the depth keys then agree bit for bit with a double-precision reference.
//
// Reverse, one thread per surfel (Sec. "Camera Pose Optimization"): the blend
// backward leaves per surfel the camera-frame gradients g_mu_c, g_a, g_b
// (a = s_u t_uc, b = s_v t_vc), g_n (normal), g_rgb and g_o.  From them:
// dL/dt_uc = s_u g_a + t_vc x g_n, dL/dt_vc = s_v g_b + g_n x t_uc,
// dL/ds_u = t_uc . g_a, dL/ds_v = t_vc . g_b; world-frame gradients are R^T of the
// camera-frame ones.  The pose gradient is eq:derivatives:
// rho += g_mu_c, phi += mu_c x g_mu_c + t_uc x (s_u g_a) + t_vc x (s_v g_b) + n x g_n,
// reduced per block into partial sums.
#include "gs2d_internal.h"

namespace gs2d {
namespace {

// Copies up to 8 view descriptors (kernel arguments) into the device view table, so
// that the table is part of the launch sequence (and of a captured graph).
struct ViewChunk {
  ViewDesc v[8];
  int first, count;
};

__global__ void upload_views_kernel(ViewChunk c, ViewDesc* __restrict__ dst, Ctrl* __restrict__ ctrl) {
  const int i = threadIdx.x;
  if (i < c.count) dst[c.first + i] = c.v[i];
  if (ctrl && i == 0) ctrl->nonfinite = 0u;
}

// One item (view, surfel); returns its tile count.
template <bool ONE_VIEW>
__device__ inline uint32_t preprocess_item(const ViewDesc* __restrict__ views, int n_views, int item, float z_near,
                                           int filter, int tile_w, int tile_h, float4* __restrict__ rec,
                                           uint2* __restrict__ rect, uint32_t* __restrict__ count,
                                           uint32_t* __restrict__ dkey, float* __restrict__ saved_pose,
                                           Ctrl* __restrict__ ctrl) {
  // one view (tracking, single renders): a constant view index, so that its fields come
  // in through scalar loads rather than a round trip of vector loads
  const int v = ONE_VIEW ? 0 : view_of_item(views, n_views, item);
  const ViewDesc& V = views[v];
  const float* __restrict__ P = V.params;
  const float* __restrict__ pose = V.pose;
  const CamF cam = V.cam;
  const int n = V.n;
  const int i = item - V.item_base;  // surfel index within the view
  if (i < 12 && saved_pose) saved_pose[v * 12 + i] = pose[i];
  double R[9], t[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    R[r * 3 + 0] = pose[r * 4 + 0];
    R[r * 3 + 1] = pose[r * 4 + 1];
    R[r * 3 + 2] = pose[r * 4 + 2];
    t[r] = pose[r * 4 + 3];
  }
  double mu[3], tu[3], tv[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    mu[c] = P[(size_t)(0 + c) * n + i];
    tu[c] = P[(size_t)(3 + c) * n + i];
    tv[c] = P[(size_t)(6 + c) * n + i];
  }
  const double su = P[(size_t)9 * n + i], sv = P[(size_t)10 * n + i];
  double mc[3], uc[3], vc[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    mc[r] = R[r * 3 + 0] * mu[0] + R[r * 3 + 1] * mu[1] + R[r * 3 + 2] * mu[2] + t[r];
    uc[r] = R[r * 3 + 0] * tu[0] + R[r * 3 + 1] * tu[1] + R[r * 3 + 2] * tu[2];
    vc[r] = R[r * 3 + 0] * tv[0] + R[r * 3 + 1] * tv[1] + R[r * 3 + 2] * tv[2];
  }
  const double a[3] = {su * uc[0], su * uc[1], su * uc[2]};
  const double b[3] = {sv * vc[0], sv * vc[1], sv * vc[2]};
  // homography rows: M0 = fx col.x + cx col.z, M1 = fy col.y + cy col.z, M2 = col.z
  const double* col[3] = {a, b, mc};
  double M0[3], M1[3], m[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    M0[j] = (double)cam.fx * col[j][0] + (double)cam.cx * col[j][2];
    M1[j] = (double)cam.fy * col[j][1] + (double)cam.cy * col[j][2];
    m[j] = col[j][2];
  }
  // an item whose geometry or pose is not finite is culled and flagged (NaN or an
  // infinity in any input reaches one of these sums)
  const double chk = mc[0] + mc[1] + mc[2] + uc[0] + uc[1] + uc[2] + vc[0] + vc[1] + vc[2] + su + sv;
  bool finite = isfinite(chk);
  bool vis = finite && mc[2] > (double)z_near;
  // C*_22 = 9 (m0^2 + m1^2) - m2^2 < 0  <=>  the 3-sigma disk is wholly in front of z = 0
  const double c22 = 9.0 * (m[0] * m[0] + m[1] * m[1]) - m[2] * m[2];
  vis = vis && (c22 < 0.0);
  uint32_t cnt = 0;
  uint2 rc = make_uint2(1u, 0u);
  double bx0 = 0, bx1 = -1, by0 = 0, by1 = -1, ux0 = 0, ux1 = -1, uy0 = 0, uy1 = -1;
  double ecx = 0, ecy = 0, sxx = 0, sxy = 0, syy = 0;  // the 3-sigma ellipse: centre, support matrix
  float4 col4 = make_float4(0.f, 0.f, 0.f, 0.f);  // opacity and colour
  if (vis) {
    col4 = make_float4(P[(size_t)11 * n + i], P[(size_t)12 * n + i], P[(size_t)13 * n + i], P[(size_t)14 * n + i]);
    if (!isfinite(col4.x + col4.y + col4.z + col4.w)) {
      finite = false;
      vis = false;
    }
  }
  if (!finite) atomicOr(&ctrl->nonfinite, 1u);
  if (vis) {
    // dual conic entries needed for the box: C00, C11, C02, C12 (and C22)
    const double c00 = 9.0 * (M0[0] * M0[0] + M0[1] * M0[1]) - M0[2] * M0[2];
    const double c11 = 9.0 * (M1[0] * M1[0] + M1[1] * M1[1]) - M1[2] * M1[2];
    const double c02 = 9.0 * (M0[0] * m[0] + M0[1] * m[1]) - M0[2] * m[2];
    const double c12 = 9.0 * (M1[0] * m[0] + M1[1] * m[1]) - M1[2] * m[2];
    const double c01 = 9.0 * (M0[0] * M1[0] + M0[1] * M1[1]) - M0[2] * M1[2];
    const double ex = c02 / c22, ey = c12 / c22;
    // the ellipse's extent along a unit direction d is sqrt(d^T S d) about its centre,
    // S = e e^T - C*[0:2, 0:2] / C*22 (its tangent lines l satisfy l^T C* l = 0)
    ecx = ex;
    ecy = ey;
    sxx = ex * ex - c00 / c22;
    sxy = ex * ey - c01 / c22;
    syy = ey * ey - c11 / c22;
    const double hx = sqrt(fmax(0.0, sxx));
    const double hy = sqrt(fmax(0.0, syy));
    double x0 = ex - hx, x1 = ex + hx, y0 = ey - hy, y1 = ey + hy;
    if (filter) {
      const double pcx = M0[2] / m[2], pcy = M1[2] / m[2];
      const double rr = sqrt((double)kRhoCutoff / (double)kFilterScale);
      x0 = fmin(x0, pcx - rr);
      x1 = fmax(x1, pcx + rr);
      y0 = fmin(y0, pcy - rr);
      y1 = fmax(y1, pcy + rr);
    }
    // one pixel of slack; the record keeps the unclipped box (integer-valued, within
    // +-2^23 so that it is exact in float32), the tile rectangle the clipped one
    ux0 = fmin(fmax(floor(x0 - 1.0), -8388608.0), 8388608.0);
    ux1 = fmin(fmax(ceil(x1 + 1.0), -8388608.0), 8388608.0);
    uy0 = fmin(fmax(floor(y0 - 1.0), -8388608.0), 8388608.0);
    uy1 = fmin(fmax(ceil(y1 + 1.0), -8388608.0), 8388608.0);
    bx0 = fmax(ux0, 0.0);
    bx1 = fmin(ux1, (double)(cam.width - 1));
    by0 = fmax(uy0, 0.0);
    by1 = fmin(uy1, (double)(cam.height - 1));
    if (bx0 <= bx1 && by0 <= by1) {
      const int tx0 = (int)bx0 / tile_w, tx1 = (int)bx1 / tile_w;
      const int ty0 = (int)by0 / tile_h, ty1 = (int)by1 / tile_h;
      cnt = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
      rc = make_uint2((uint32_t)tx0 | ((uint32_t)tx1 << 16), (uint32_t)ty0 | ((uint32_t)ty1 << 16));
      GS2D_DCHECK(&ctrl->check_bits, 0 <= tx0 && tx0 <= tx1 && tx1 < V.tiles_x && 0 <= ty0 && ty0 <= ty1 &&
                  ty1 < V.tiles_y, kCheckRect);
    }
  }
  count[item] = cnt;
  if (cnt == 0) {
    rect[item] = make_uint2(1u, 0u);  // x0 = 1 > x1 = 0: empty
    dkey[item] = 0xFFFFFFFFu;
    return 0u;
  }
  rect[item] = rc;
  dkey[item] = __float_as_uint((float)mc[2]);
  // centre-relative homography rows (see gs2d_internal.h)
  const double pcx = M0[2] / m[2], pcy = M1[2] / m[2];
  const double P0 = M0[0] - pcx * m[0], P1 = M0[1] - pcx * m[1];
  const double Q0 = M1[0] - pcy * m[0], Q1 = M1[1] - pcy * m[1];
  const double Dt = P0 * Q1 - P1 * Q0;
  const double k0 = m[0] * Q1 - m[1] * Q0;
  const double k1 = P0 * m[1] - P1 * m[0];
  const double nn[3] = {uc[1] * vc[2] - uc[2] * vc[1], uc[2] * vc[0] - uc[0] * vc[2],
                        uc[0] * vc[1] - uc[1] * vc[0]};
  float4* r = rec + (size_t)item * kRecF4;
  // the projected centre is stored relative to the box corner (ux0, uy0), so that a
  // pixel's offset (x - ux0) - (cx - ux0) loses no precision at large x
  r[0] = make_float4((float)ux0, (float)ux1, (float)uy0, (float)uy1);
  r[1] = make_float4((float)(pcx - ux0), (float)(pcy - uy0), (float)Dt, (float)k0);
  r[2] = make_float4((float)k1, (float)P0, (float)P1, (float)Q0);
  r[3] = make_float4((float)Q1, (float)m[0], (float)m[1], (float)m[2]);
  r[4] = col4;
  r[5] = make_float4((float)nn[0], (float)nn[1], (float)nn[2], (float)syy);
  r[6] = make_float4((float)(ecx - ux0), (float)(ecy - uy0), (float)sxx, (float)sxy);
  return cnt;
}

__device__ inline uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += (uint32_t)__shfl_xor((int)v, m, 64);
  return v;
}

// One thread per item, kPartItems items per block; each block also stores its pair
// count and visible-item count (the pair duplication places pairs from them).
template <bool ONE_VIEW>
__global__ __launch_bounds__(kPartItems) void preprocess_kernel(
    const ViewDesc* __restrict__ views, int n_views, int64_t items, float z_near, int filter, int tile_w,
    int tile_h, float4* __restrict__ rec, uint2* __restrict__ rect, uint32_t* __restrict__ count,
    uint32_t* __restrict__ dkey, float* __restrict__ saved_pose, uint32_t* __restrict__ part_pairs,
    uint32_t* __restrict__ part_vis, Ctrl* __restrict__ ctrl, int clear_overflow) {
  const int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t cnt = gi < items ? preprocess_item<ONE_VIEW>(views, n_views, (int)gi, z_near, filter, tile_w,
                                                              tile_h, rec, rect, count, dkey, saved_pose, ctrl)
                                  : 0u;
  __shared__ uint32_t sp[kPartItems / 64], sv[kPartItems / 64];
  const uint32_t wp = wave_sum_u32(cnt), wv = wave_sum_u32(cnt != 0u ? 1u : 0u);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sp[wave] = wp;
    sv[wave] = wv;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t bp = 0, bv = 0;
#pragma unroll
    for (int w = 0; w < kPartItems / 64; ++w) {
      bp += sp[w];
      bv += sv[w];
    }
    part_pairs[blockIdx.x] = bp;
    part_vis[blockIdx.x] = bv;
    if (blockIdx.x == 0 && clear_overflow) ctrl->overflow = 0u;
  }
}

__device__ inline void cross3(const float* a, const float* b, float* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

// Zero the accumulator rows (16 floats) of the items that touch a tile: the only rows
// the backward blend adds into.  Four threads per row, one float4 each.
__global__ __launch_bounds__(256) void clear_rows_kernel(const uint32_t* __restrict__ count,
                                                          float4* __restrict__ gacc, int64_t items) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < items * 4 && count[q >> 2] != 0u) gacc[q] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// One item's parameter gradient o[15] (world frame) and pose terms pr[6] from its
// accumulator row g, for the view pose (3x4, world to camera).
__device__ __forceinline__ void item_grad(const float* __restrict__ P, int n, int i, const float* __restrict__ pose,
                                          const float* __restrict__ gacc_row, float o[15], float pr[6]) {
  float R[9], t[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    R[r * 3 + 0] = pose[r * 4 + 0];
    R[r * 3 + 1] = pose[r * 4 + 1];
    R[r * 3 + 2] = pose[r * 4 + 2];
    t[r] = pose[r * 4 + 3];
  }
  float mu[3], tu[3], tv[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    mu[c] = P[(size_t)(0 + c) * n + i];
    tu[c] = P[(size_t)(3 + c) * n + i];
    tv[c] = P[(size_t)(6 + c) * n + i];
  }
  const float su = P[(size_t)9 * n + i], sv = P[(size_t)10 * n + i];
  float mc[3], uc[3], vc[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    mc[r] = R[r * 3 + 0] * mu[0] + R[r * 3 + 1] * mu[1] + R[r * 3 + 2] * mu[2] + t[r];
    uc[r] = R[r * 3 + 0] * tu[0] + R[r * 3 + 1] * tu[1] + R[r * 3 + 2] * tu[2];
    vc[r] = R[r * 3 + 0] * tv[0] + R[r * 3 + 1] * tv[1] + R[r * 3 + 2] * tv[2];
  }
  const float4* g4 = reinterpret_cast<const float4*>(gacc_row);
  const float4 A = g4[0], B = g4[1], C = g4[2], D = g4[3];
  const float gmu[3] = {A.x, A.y, A.z};
  const float ga[3] = {A.w, B.x, B.y};
  const float gb[3] = {B.z, B.w, C.x};
  const float gn[3] = {C.y, C.z, C.w};
  const float grgb[3] = {D.x, D.y, D.z};
  const float go = D.w;
  float tmp[3], gtu[3], gtv[3];
  cross3(vc, gn, tmp);
  for (int c = 0; c < 3; ++c) gtu[c] = su * ga[c] + tmp[c];
  cross3(gn, uc, tmp);
  for (int c = 0; c < 3; ++c) gtv[c] = sv * gb[c] + tmp[c];
  const float gsu = uc[0] * ga[0] + uc[1] * ga[1] + uc[2] * ga[2];
  const float gsv = vc[0] * gb[0] + vc[1] * gb[1] + vc[2] * gb[2];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    o[0 + c] = R[0 * 3 + c] * gmu[0] + R[1 * 3 + c] * gmu[1] + R[2 * 3 + c] * gmu[2];
    o[3 + c] = R[0 * 3 + c] * gtu[0] + R[1 * 3 + c] * gtu[1] + R[2 * 3 + c] * gtu[2];
    o[6 + c] = R[0 * 3 + c] * gtv[0] + R[1 * 3 + c] * gtv[1] + R[2 * 3 + c] * gtv[2];
    o[12 + c] = grgb[c];
  }
  o[9] = gsu;
  o[10] = gsv;
  o[11] = go;
  // eq:derivatives, left perturbation: [I, -mu_c^x] and [0, -R_c[:,k]^x]
  float gcu[3], gcv[3], c1[3], c2[3], c3[3], c4[3];
  for (int c = 0; c < 3; ++c) {
    gcu[c] = su * ga[c];
    gcv[c] = sv * gb[c];
  }
  const float nn[3] = {uc[1] * vc[2] - uc[2] * vc[1], uc[2] * vc[0] - uc[0] * vc[2],
                       uc[0] * vc[1] - uc[1] * vc[0]};
  cross3(mc, gmu, c1);
  cross3(uc, gcu, c2);
  cross3(vc, gcv, c3);
  cross3(nn, gn, c4);
  for (int c = 0; c < 3; ++c) {
    pr[c] = gmu[c];
    pr[3 + c] = c1[c] + c2[c] + c3[c] + c4[c];
  }
}

// Per item the parameter gradient from its accumulator row, and the block sums of the
// pose terms.  An item that touches no tile has a zero gradient and no row to read.
__global__ __launch_bounds__(256) void preprocess_bwd_kernel(
    const float* __restrict__ P, int n, const float* __restrict__ pose, const uint32_t* __restrict__ count,
    const float* __restrict__ gacc, float* __restrict__ d_params, int accumulate,
    float* __restrict__ part) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  float pr[6] = {0, 0, 0, 0, 0, 0};
  const bool hit = i < n && count[i] != 0u;
  if (i < n && !hit && d_params && !accumulate) {
#pragma unroll
    for (int k = 0; k < 15; ++k) d_params[(size_t)k * n + i] = 0.f;
  }
  if (hit) {
    float o[15];
    item_grad(P, n, i, pose, gacc + (size_t)i * 16, o, pr);
    if (d_params) {
#pragma unroll
      for (int k = 0; k < 15; ++k) {
        float* dst = d_params + (size_t)k * n + i;
        *dst = accumulate ? *dst + o[k] : o[k];
      }
    }
  }
  // block reduction of the six pose terms (fixed order: deterministic)
  __shared__ float red[256][6];
#pragma unroll
  for (int k = 0; k < 6; ++k) red[threadIdx.x][k] = pr[k];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
#pragma unroll
      for (int k = 0; k < 6; ++k) red[threadIdx.x][k] += red[threadIdx.x + s][k];
    }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[(size_t)blockIdx.x * 8 + threadIdx.x] = red[0][threadIdx.x];
  if (threadIdx.x == 6 || threadIdx.x == 7) part[(size_t)blockIdx.x * 8 + threadIdx.x] = 0.0f;
}


// The parameter backward of up to kMaxGroup views that share one surfel set and one
// d_params buffer, in one pass over the surfels: each thread adds its surfel's
// gradients of the views in view order in registers and writes d_params once.  The
// pose terms of view g are summed per wave (no barrier) into rows
// [g * 4 * gridDim.x, (g + 1) * 4 * gridDim.x) of `part`, one per wave.
constexpr int kMaxGroup = 32;
struct BwdGroup {
  int n_views;
  const float* pose[kMaxGroup];
  const uint32_t* count[kMaxGroup];
  const float* gacc[kMaxGroup];
};
__global__ __launch_bounds__(256) void preprocess_bwd_group_kernel(const float* __restrict__ P, int n, BwdGroup grp,
                                                                   float* __restrict__ d_params, int accumulate,
                                                                   float* __restrict__ part) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // the running sum starts from d_params when accumulating, so the additions happen in
  // the order the one-view kernel makes them through memory
  float sum[15];
  const bool live = i < n && d_params != nullptr;
  bool have = live && accumulate, any = false;
#pragma unroll
  for (int k = 0; k < 15; ++k) sum[k] = have ? d_params[(size_t)k * n + i] : 0.f;
  for (int g = 0; g < grp.n_views; ++g) {
    float pr[6] = {0, 0, 0, 0, 0, 0};
    if (i < n && grp.count[g][i] != 0u) {
      float o[15];
      item_grad(P, n, i, grp.pose[g], grp.gacc[g] + (size_t)i * 16, o, pr);
#pragma unroll
      for (int k = 0; k < 15; ++k) sum[k] = have ? sum[k] + o[k] : o[k];
      have = true;
      any = true;
    }
    // the wave's sums of the pose terms (fixed order), lane k < 6 writing term k
    float mine = 0.f;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      float v = pr[k];
#pragma unroll
      for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
      mine = lane == k ? v : mine;
    }
    if (lane < 8) part[(((size_t)g * gridDim.x + blockIdx.x) * kGroupRowsPerBlock + wave) * 8 + lane] = mine;
  }
  if (live && (any || !accumulate)) {
#pragma unroll
    for (int k = 0; k < 15; ++k) d_params[(size_t)k * n + i] = sum[k];
  }
}
}  // namespace

void launch_upload_views(const ViewSet& vs, ViewDesc* dst, hipStream_t s, Ctrl* ctrl) {
  for (int f = 0; f < vs.n_views; f += 8) {
    ViewChunk c;
    c.first = f;
    c.count = vs.n_views - f < 8 ? vs.n_views - f : 8;
    for (int k = 0; k < c.count; ++k) c.v[k] = vs.v[f + k];
    upload_views_kernel<<<1, 64, 0, s>>>(c, dst, f == 0 ? ctrl : nullptr);
  }
}

void launch_preprocess(const ViewDesc* views, int n_views, int64_t items, float z_near, int filter, int tile_w,
                       int tile_h, float4* rec, uint2* rect, uint32_t* count, uint32_t* dkey, float* saved_pose,
                       uint32_t* part_pairs, uint32_t* part_vis, Ctrl* ctrl, hipStream_t s, bool clear_overflow) {
  const int grid = items > 0 ? (int)((items + kPartItems - 1) / kPartItems) : 1;
  const int co = clear_overflow ? 1 : 0;
  if (n_views == 1)
    preprocess_kernel<true><<<grid, kPartItems, 0, s>>>(views, n_views, items, z_near, filter, tile_w, tile_h, rec,
                                                        rect, count, dkey, saved_pose, part_pairs, part_vis, ctrl, co);
  else
    preprocess_kernel<false><<<grid, kPartItems, 0, s>>>(views, n_views, items, z_near, filter, tile_w, tile_h, rec,
                                                         rect, count, dkey, saved_pose, part_pairs, part_vis, ctrl, co);
}

void launch_clear_rows(const uint32_t* count, float* gacc, int64_t items, hipStream_t s) {
  if (items <= 0) return;
  const int64_t grid = (items * 4 + 255) / 256;
  clear_rows_kernel<<<(unsigned)grid, 256, 0, s>>>(count, reinterpret_cast<float4*>(gacc), items);
}

int launch_preprocess_bwd_group(const float* params, int n, int n_views, const float* const* poses,
                                const uint32_t* const* counts, const float* const* gaccs, float* d_params,
                                int accumulate, float* part, hipStream_t s) {
  if (n_views < 1 || n_views > kMaxGroup) return -1;
  BwdGroup grp;
  grp.n_views = n_views;
  for (int g = 0; g < n_views; ++g) {
    grp.pose[g] = poses[g];
    grp.count[g] = counts[g];
    grp.gacc[g] = gaccs[g];
  }
  const int grid = (n + 255) / 256 > 0 ? (n + 255) / 256 : 1;
  preprocess_bwd_group_kernel<<<grid, 256, 0, s>>>(params, n, grp, d_params, accumulate, part);
  return 0;
}

void launch_preprocess_bwd(const float* params, int n, const float* pose, const uint32_t* count, const float* gacc,
                           float* d_params, int accumulate, float* part, hipStream_t s) {
  const int grid = (n + 255) / 256 > 0 ? (n + 255) / 256 : 1;
  preprocess_bwd_kernel<<<grid, 256, 0, s>>>(params, n, pose, count, gacc, d_params, accumulate, part);
}

}  // namespace gs2d
