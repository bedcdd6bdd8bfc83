// Image losses with their image gradients, partial-sum reductions, and the pose step.
//
// The masked L1 image loss, one lane per pixel:
//   L = (1/HW) sum_p M (w_rgb |rgb - I|_1 + w_d |D - D_obs| + w_n |N - N_obs|_1),
// M the product of the selected masks.  The tracking loss (Sec. "Tracking and Keyframe
// Selection", eq:LD, eq:normal_mask, eq:opacity_mask, eq:tracking_loss) is w = (1,
// lambda_d, 0) with both masks, the relocalisation error e_t (eq:tracking_error) its
// depth term:
//   M_n = [N . r > 0] (the sign does not depend on normalising the ray, so the
//   ray (x - cx)/fx, (y - cy)/fy, 1 is used), M_o = [O > 0.95].
// Gradients hold the masks fixed and take d|x|/dx = sign(x) (0 at 0).  Each
// workgroup writes one partial sum; a single workgroup adds them in a fixed order.
// The pose step itself (AdamW and Exp) is in pose_step.h.
#include "pose_step.h"

namespace gs2d {
namespace {

__global__ __launch_bounds__(kLossThreads) void image_loss_kernel(const ViewDesc* __restrict__ views, LossW w,
                                                                  float* __restrict__ part, int part_stride) {
  const ViewDesc& V = views[blockIdx.y];
  const CamF cam = V.cam;
  const int HW = cam.width * cam.height;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.f;
  if (p < HW) {
    const float* rgb = V.rgb;
    const float* tgt_rgb = V.tgt_rgb;
    const float* normal = V.normal;
    const int y = p / cam.width, x = p - y * cam.width;
    bool m = true;
    if (w.normal_mask) {
      const float xh = ((float)x - cam.cx) / cam.fx, yh = ((float)y - cam.cy) / cam.fy;
      const float ndr = fmaf(normal[p], xh, fmaf(normal[HW + p], yh, normal[2 * HW + p]));
      m = ndr > 0.0f;
    }
    if (w.opacity_mask) m = m && (V.alpha[p] > kOpacityMask);
    const float inv = 1.0f / (float)HW;
    // no colour images: no colour term (the relocalisation error e_t is the depth term)
    const float d0 = rgb ? rgb[p] - tgt_rgb[p] : 0.f;
    const float d1 = rgb ? rgb[HW + p] - tgt_rgb[HW + p] : 0.f;
    const float d2 = rgb ? rgb[2 * HW + p] - tgt_rgb[2 * HW + p] : 0.f;
    const float dd = V.depth[p] - V.tgt_depth[p];
    const bool has_n = V.tgt_normal != nullptr;
    const float n0 = has_n ? normal[p] - V.tgt_normal[p] : 0.f;
    const float n1 = has_n ? normal[HW + p] - V.tgt_normal[HW + p] : 0.f;
    const float n2 = has_n ? normal[2 * HW + p] - V.tgt_normal[2 * HW + p] : 0.f;
    auto sgn = [](float v) { return v > 0.f ? 1.f : (v < 0.f ? -1.f : 0.f); };
    if (m) {
      l = w.w_rgb * (fabsf(d0) + fabsf(d1) + fabsf(d2)) + w.w_d * fabsf(dd);
      if (has_n) l += w.w_n * (fabsf(n0) + fabsf(n1) + fabsf(n2));
    }
    if (float* d_rgb = V.g_rgb) {
      d_rgb[p] = m ? w.w_rgb * sgn(d0) * inv : 0.f;
      d_rgb[HW + p] = m ? w.w_rgb * sgn(d1) * inv : 0.f;
      d_rgb[2 * HW + p] = m ? w.w_rgb * sgn(d2) * inv : 0.f;
    }
    if (float* d_depth = V.g_depth) d_depth[p] = m ? w.w_d * sgn(dd) * inv : 0.f;
    if (float* d_normal = V.g_normal) {
      d_normal[p] = m ? w.w_n * sgn(n0) * inv : 0.f;
      d_normal[HW + p] = m ? w.w_n * sgn(n1) * inv : 0.f;
      d_normal[2 * HW + p] = m ? w.w_n * sgn(n2) * inv : 0.f;
    }
  }
  __shared__ float red[kLossThreads];
  red[threadIdx.x] = l;
  __syncthreads();
  for (int s = kLossThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t)blockIdx.y * part_stride + blockIdx.x] = red[0];
}

// Sum n rows of `stride` floats, column k, in a fixed order (64 lanes, then a
// butterfly): deterministic for a given n.
__device__ inline double sum_parts(const float* part, int n, int stride, int k) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 64) s += (double)part[(size_t)i * stride + k];
  return wave_sum_d(s);
}
__device__ inline int loss_blocks_dev(int hw) { return (hw + kLossThreads - 1) / kLossThreads; }

__global__ void reduce_loss_kernel(const float* __restrict__ part, int n, float inv_hw, float* __restrict__ loss) {
  const double s = sum_parts(part, n, 1, 0) * (double)inv_hw;
  if (threadIdx.x == 0) *loss = (float)s;
}

// one wave per view: losses[v] = (sum of view v's partials) / HW_v
__global__ void reduce_loss_views_kernel(const ViewDesc* __restrict__ views, const float* __restrict__ part,
                                         int part_stride, float* __restrict__ losses) {
  const CamF cam = views[blockIdx.x].cam;
  const int hw = cam.width * cam.height;
  // the same scaling as the one-view reduction: a float reciprocal of HW
  const double s = sum_parts(part + (size_t)blockIdx.x * part_stride, loss_blocks_dev(hw), 1, 0) *
                   (double)(1.0f / (float)hw);
  if (threadIdx.x == 0) losses[blockIdx.x] = (float)s;
}

constexpr int kReduceThreads = 256;

// The six pose partials (the first six of each 8-float row) summed over `rows` rows in
// FP64 by one workgroup: every thread adds its rows' six values in one pass, then the
// waves and the workgroup in a fixed order.  d_pose (=, or += with accumulate).
__device__ void reduce_pose_rows(const float* __restrict__ part, int rows, float* __restrict__ d_pose,
                                 int accumulate) {
  __shared__ double sh[kReduceThreads / 64][6];
  // up to 8 rows per thread in flight before the first add; each thread adds its rows
  // in ascending order
  constexpr int kRowsInFlight = 8;
  double g[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i0 = threadIdx.x; i0 < rows; i0 += kReduceThreads * kRowsInFlight) {
    float4 a[kRowsInFlight];
    float2 b[kRowsInFlight];
#pragma unroll
    for (int u = 0; u < kRowsInFlight; ++u) {
      const int i = i0 + u * kReduceThreads;
      a[u] = i < rows ? reinterpret_cast<const float4*>(part + (size_t)i * 8)[0] : make_float4(0.f, 0.f, 0.f, 0.f);
      b[u] = i < rows ? reinterpret_cast<const float2*>(part + (size_t)i * 8)[2] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < kRowsInFlight; ++u) {
      if (i0 + u * kReduceThreads >= rows) break;
      g[0] += a[u].x, g[1] += a[u].y, g[2] += a[u].z, g[3] += a[u].w, g[4] += b[u].x, g[5] += b[u].y;
    }
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) g[k] = wave_sum_d(g[k]);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < 6; ++k) sh[threadIdx.x >> 6][k] = g[k];
  __syncthreads();
  if (threadIdx.x < 6) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kReduceThreads / 64; ++w) t += sh[w][threadIdx.x];
    d_pose[threadIdx.x] = accumulate ? d_pose[threadIdx.x] + (float)t : (float)t;
  }
}

__global__ __launch_bounds__(kReduceThreads) void reduce_pose_kernel(const float* __restrict__ part, int row0,
                                                                     int rows, float* __restrict__ d_pose,
                                                                     int accumulate) {
  reduce_pose_rows(part + (size_t)row0 * 8, rows, d_pose, accumulate);
}

struct PoseOuts {
  float* d_pose[kMaxViews];
};
// one workgroup per view of a group: d_pose[g] = sum of rows [g * rows, (g + 1) * rows)
__global__ __launch_bounds__(kReduceThreads) void reduce_pose_group_kernel(const float* __restrict__ part, int rows,
                                                                           PoseOuts out, int accumulate) {
  float* d_pose = out.d_pose[blockIdx.x];
  if (!d_pose) return;
  reduce_pose_rows(part + (size_t)blockIdx.x * rows * 8, rows, d_pose, accumulate);
}

// one workgroup per view: d_pose of view blockIdx.x = sum of the rows of its tiles
__global__ __launch_bounds__(kReduceThreads) void reduce_pose_views_kernel(const ViewDesc* __restrict__ views,
                                                                           const float* __restrict__ part,
                                                                           int accumulate) {
  const ViewDesc& V = views[blockIdx.x];
  float* d_pose = V.d_pose;
  if (!d_pose) return;
  reduce_pose_rows(part + (size_t)V.tile_base * 8, V.tiles_x * V.tiles_y, d_pose, accumulate);
}

__global__ void track_init_kernel(const ViewDesc* __restrict__ views, int n_views, Ctrl* __restrict__ ctrl,
                                  float* pose_history, float* loss_history, double* grad_history,
                                  int max_hist, Fallbacks fb) {
  const int t = threadIdx.x;
  for (int k = t; k < n_views; k += blockDim.x) {
    const bool armed = fb.pose[k] != nullptr && fb.loss[k] != nullptr;
    ctrl->fb_armed[k] = armed ? 1 : 0;
    ctrl->fb_used[k] = 0;
    ctrl->fb_loss[k] = armed ? (double)fb.loss[k][0] : 0.0;
  }
  for (int k = t; k < n_views * 12; k += blockDim.x) {
    const float* fp = fb.pose[k / 12];
    ctrl->fb_pose[k / 12][k % 12] = fp ? (double)fp[k % 12] : 0.0;
  }
  for (int k = t; k < n_views * 12; k += blockDim.x)
    ctrl->master_pose[k / 12][k % 12] = (double)views[k / 12].pose[k % 12];
  for (int k = t; k < n_views * 6; k += blockDim.x) {
    ctrl->adam_m[k / 6][k % 6] = 0.0;
    ctrl->adam_v[k / 6][k % 6] = 0.0;
  }
  for (int k = t; k < n_views; k += blockDim.x) {
    ctrl->loss[k] = 0.0;
    ctrl->iter_v[k] = 0;
    ctrl->adam_b1t[k] = 1.0;
    ctrl->adam_b2t[k] = 1.0;
    ctrl->status[k] = kTrackRan;
    ctrl->rising[k] = 0;
    ctrl->best_loss[k] = __builtin_inf();
  }
  for (int k = t; k < n_views * 12; k += blockDim.x) ctrl->best_pose[k / 12][k % 12] = (double)views[k / 12].pose[k % 12];
  if (t == 0) {
    ctrl->iter = 0;
    ctrl->overflow = 0u;  // kept for the whole call by the loop's renders
    ctrl->pose_history = pose_history;
    ctrl->loss_history = loss_history;
    ctrl->grad_history = grad_history;
    ctrl->max_hist = max_hist;
    ctrl->n_views = n_views;
  }
}

// One workgroup of 256 threads per view.
__global__ __launch_bounds__(256) void pose_step_kernel(const ViewDesc* __restrict__ views,
                                                        const float* __restrict__ pose_part, int loss_in_part,
                                                        const float* __restrict__ loss_part, int part_stride,
                                                        AdamArgs adam, Ctrl* __restrict__ ctrl) {
  pose_step_view(blockIdx.x, gridDim.x, views, pose_part, loss_in_part, loss_part, part_stride, adam, ctrl);
}

// Left Jacobian of SE(3) for tau = (rho, phi) (Barfoot, "State Estimation for
// Robotics", Sec. 7.1.5): J = [[J_so3, Q], [0, J_so3]] with
// Q = 1/2 R + c2 (F R + R F + F R F) + c3 (F F R + R F F - 3 F R F)
//     + c4 (F R F F + F F R F),  F = phi^, R = rho^,
// c2 = (th - sin th)/th^3, c3 = (th^2 + 2 cos th - 2)/(2 th^4),
// c4 = (2 th - 3 sin th + th cos th)/(2 th^5)  (series below 1e-3 rad).
__device__ void mat3_mul(const double* A, const double* B, double* C) {
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      C[r * 3 + c] = A[r * 3 + 0] * B[0 * 3 + c] + A[r * 3 + 1] * B[1 * 3 + c] + A[r * 3 + 2] * B[2 * 3 + c];
}

__device__ void se3_left_jacobian(const double tau[6], double Jl[36]) {
  const double px = tau[3], py = tau[4], pz = tau[5];
  const double th2 = px * px + py * py + pz * pz, th = sqrt(th2);
  double b, c, c2, c3, c4;  // J_so3 = I + b F + c F^2
  if (th < 1e-3) {
    b = 0.5 - th2 / 24.0;
    c = 1.0 / 6.0 - th2 / 120.0;
    c2 = 1.0 / 6.0 - th2 / 120.0;
    c3 = 1.0 / 24.0 - th2 / 720.0;
    c4 = 1.0 / 120.0 - th2 / 2520.0;
  } else {
    const double s = sin(th), co = cos(th);
    b = (1.0 - co) / th2;
    c = (th - s) / (th2 * th);
    c2 = c;
    c3 = (th2 + 2.0 * co - 2.0) / (2.0 * th2 * th2);
    c4 = (2.0 * th - 3.0 * s + th * co) / (2.0 * th2 * th2 * th);
  }
  const double F[9] = {0.0, -pz, py, pz, 0.0, -px, -py, px, 0.0};
  const double R[9] = {0.0, -tau[2], tau[1], tau[2], 0.0, -tau[0], -tau[1], tau[0], 0.0};
  double FF[9], FR[9], RF[9], FRF[9], FFR[9], RFF[9], FRFF[9], FFRF[9];
  mat3_mul(F, F, FF);
  mat3_mul(F, R, FR);
  mat3_mul(R, F, RF);
  mat3_mul(FR, F, FRF);
  mat3_mul(FF, R, FFR);
  mat3_mul(RF, F, RFF);
  mat3_mul(FRF, F, FRFF);
  mat3_mul(FF, RF, FFRF);
  double J3[9], Q[9];
  for (int k = 0; k < 9; ++k) {
    J3[k] = ((k % 4 == 0) ? 1.0 : 0.0) + b * F[k] + c * FF[k];
    Q[k] = 0.5 * R[k] + c2 * (FR[k] + RF[k] + FRF[k]) + c3 * (FFR[k] + RFF[k] - 3.0 * FRF[k]) +
           c4 * (FRFF[k] + FFRF[k]);
  }
  for (int k = 0; k < 36; ++k) Jl[k] = 0.0;
  for (int r = 0; r < 3; ++r)
    for (int cc = 0; cc < 3; ++cc) {
      Jl[r * 6 + cc] = J3[r * 3 + cc];
      Jl[r * 6 + 3 + cc] = Q[r * 3 + cc];
      Jl[(r + 3) * 6 + 3 + cc] = J3[r * 3 + cc];
    }
}

__global__ void pose_exp_kernel(const float* __restrict__ tau, const float* __restrict__ pin,
                                float* __restrict__ pout) {
  if (threadIdx.x != 0) return;
  double t[6], Re[9], te[3];
  for (int k = 0; k < 6; ++k) t[k] = tau[k];
  se3_exp(t, Re, te);
  double T[12];
  for (int k = 0; k < 12; ++k) T[k] = pin[k];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 4; ++c) {
      double s = Re[r * 3 + 0] * T[0 * 4 + c] + Re[r * 3 + 1] * T[1 * 4 + c] + Re[r * 3 + 2] * T[2 * 4 + c];
      if (c == 3) s += te[r];
      pout[r * 4 + c] = (float)s;
    }
}

__global__ void pose_tau_grad_kernel(const float* __restrict__ tau, const float* __restrict__ g,
                                     float* __restrict__ d_tau) {
  if (threadIdx.x != 0) return;
  double t[6], J[36];
  for (int k = 0; k < 6; ++k) t[k] = tau[k];
  se3_left_jacobian(t, J);
  for (int c = 0; c < 6; ++c) {
    double s = 0.0;
    for (int r = 0; r < 6; ++r) s += J[r * 6 + c] * (double)g[r];
    d_tau[c] = (float)s;
  }
}

}  // namespace

void launch_pose_exp(const float* tau, const float* pose_in, float* pose_out, hipStream_t s) {
  pose_exp_kernel<<<1, 64, 0, s>>>(tau, pose_in, pose_out);
}

void launch_pose_tau_grad(const float* tau, const float* d_pose, float* d_tau, hipStream_t s) {
  pose_tau_grad_kernel<<<1, 64, 0, s>>>(tau, d_pose, d_tau);
}

int loss_blocks(int hw) { return (hw + kLossThreads - 1) / kLossThreads; }

void launch_image_loss(const ViewDesc* views, int n_views, int max_hw, LossW w, float* part, int part_stride,
                       hipStream_t s) {
  const dim3 grid(loss_blocks(max_hw), n_views);
  image_loss_kernel<<<grid, kLossThreads, 0, s>>>(views, w, part, part_stride);
}

void launch_reduce_loss_views(const ViewDesc* views, int n_views, const float* part, int part_stride, float* losses,
                              hipStream_t s) {
  reduce_loss_views_kernel<<<n_views, 64, 0, s>>>(views, part, part_stride, losses);
}

void launch_reduce_loss(const float* part, int n_parts, float inv_hw, float* loss, hipStream_t s) {
  reduce_loss_kernel<<<1, 64, 0, s>>>(part, n_parts, inv_hw, loss);
}

void launch_reduce_pose(const float* part, int row0, int rows, float* d_pose, int accumulate, hipStream_t s) {
  reduce_pose_kernel<<<1, kReduceThreads, 0, s>>>(part, row0, rows, d_pose, accumulate);
}

void launch_reduce_pose_group(const float* part, int rows, int n_views, float* const* d_pose, int accumulate,
                              hipStream_t s) {
  if (n_views < 1 || n_views > kMaxViews) return;
  PoseOuts out;
  for (int g = 0; g < kMaxViews; ++g) out.d_pose[g] = g < n_views ? d_pose[g] : nullptr;
  reduce_pose_group_kernel<<<n_views, kReduceThreads, 0, s>>>(part, rows, out, accumulate);
}

void launch_reduce_pose_views(const ViewDesc* views, int n_views, const float* part, int accumulate,
                              hipStream_t s) {
  reduce_pose_views_kernel<<<n_views, kReduceThreads, 0, s>>>(views, part, accumulate);
}

void launch_track_init(const ViewDesc* views, int n_views, Ctrl* ctrl, float* pose_history, float* loss_history,
                       double* grad_history, int max_hist, hipStream_t s, const Fallbacks* fallback) {
  Fallbacks fb{};
  if (fallback) fb = *fallback;
  track_init_kernel<<<1, 256, 0, s>>>(views, n_views, ctrl, pose_history, loss_history, grad_history, max_hist, fb);
}

void launch_pose_step(const ViewDesc* views, int n_views, const float* pose_part, bool loss_in_part,
                      const float* loss_part, int part_stride, AdamArgs adam, Ctrl* ctrl, hipStream_t s) {
  pose_step_kernel<<<n_views, 256, 0, s>>>(views, pose_part, loss_in_part ? 1 : 0, loss_part, part_stride, adam,
                                           ctrl);
}

}  // namespace gs2d
