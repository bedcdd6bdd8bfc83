// The pose step of tracking: the device side of the AdamW + Exp update of each view.
//
// Pose step (Sec. "Tracking and Keyframe Selection": AdamW on the camera pose with
// the surfels frozen).  The step variable is the left-perturbation twist tau,
// which is zero before every step, so decoupled weight decay has no effect:
//   m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
//   tau = -lr m/(1-b1^t) / (sqrt(v/(1-b2^t)) + eps),  T <- Exp(tau) T.
// Exp on SE(3) is the closed form R = I + sin(th)/th K + (1-cos th)/th^2 K^2,
// t = J rho with J = I + (1-cos th)/th^2 K + (th - sin th)/th^3 K^2 (Barfoot,
// "State Estimation for Robotics", Sec. 7.1), evaluated in FP64 on a master copy
// of the pose so that repeated steps do not drift off SO(3).
#ifndef GS2D_POSE_STEP_H
#define GS2D_POSE_STEP_H

#include "gs2d_internal.h"

namespace gs2d {

constexpr int kLossThreads = 256;  // pixels per partial sum of the tracking loss kernel

__device__ inline double wave_sum_d(double v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

__device__ inline void se3_exp(const double tau[6], double R[9], double tt[3]) {
  const double px = tau[3], py = tau[4], pz = tau[5];
  const double th2 = px * px + py * py + pz * pz;
  const double th = sqrt(th2);
  double A, B, C;  // R = I + A K + B K^2,  J = I + B K + C K^2
  if (th < 1e-6) {
    A = 1.0 - th2 / 6.0;
    B = 0.5 - th2 / 24.0;
    C = 1.0 / 6.0 - th2 / 120.0;
  } else {
    A = sin(th) / th;
    B = (1.0 - cos(th)) / th2;
    C = (th - sin(th)) / (th2 * th);
  }
  const double K[9] = {0.0, -pz, py, pz, 0.0, -px, -py, px, 0.0};
  double K2[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      K2[r * 3 + c] = K[r * 3 + 0] * K[0 * 3 + c] + K[r * 3 + 1] * K[1 * 3 + c] + K[r * 3 + 2] * K[2 * 3 + c];
  double J[9];
  for (int k = 0; k < 9; ++k) {
    const double I = (k % 4 == 0) ? 1.0 : 0.0;
    R[k] = I + A * K[k] + B * K2[k];
    J[k] = I + B * K[k] + C * K2[k];
  }
  for (int r = 0; r < 3; ++r) tt[r] = J[r * 3 + 0] * tau[0] + J[r * 3 + 1] * tau[1] + J[r * 3 + 2] * tau[2];
}

// The AdamW + Exp step of view v, run by the 256 threads of one workgroup: a
// fixed-order (deterministic) reduction of the view's pose and loss partials, then
// the step on the first wave: lane k < 6 updates the moments of component k, every
// lane forms the same Exp, and lane k < 12 writes pose entry k.
__device__ inline void pose_step_view(int v, int n_views, const ViewDesc* __restrict__ views,
                                      const float* __restrict__ pose_part, int loss_in_part,
                                      const float* __restrict__ loss_part, int part_stride, const AdamArgs& adam,
                                      Ctrl* __restrict__ ctrl) {
  __shared__ double sh[8][4];
  const ViewDesc& V = views[v];
  const int HW = V.cam.width * V.cam.height;
  const int rows = V.tiles_x * V.tiles_y;
  const float* pp = pose_part + (size_t)V.tile_base * 8;
  const int l = threadIdx.x;
  // the step's state, loaded before the reduction so that its latency overlaps it
  double m_old = 0.0, v_old = 0.0, T_old = 0.0;
  if (l < 6) {
    m_old = ctrl->adam_m[v][l];
    v_old = ctrl->adam_v[v][l];
  }
  if (l < 12) T_old = ctrl->master_pose[v][l];
  const double b1t_old = ctrl->adam_b1t[v], b2t_old = ctrl->adam_b2t[v];
  const uint32_t it = ctrl->iter_v[v];
  float* const pose_out = V.pose;
  // the six pose sums, the loss and the unmasked loss in one pass and one block
  // reduction (fixed order)
  // Rows are read kRowsInFlight per thread at a time (two 16-byte loads each), all
  // issued before the first add; each thread adds its rows in ascending order.  The
  // loads go through a buffer resource over the view's rows: past its last row they
  // return zeros, so no branch (and no wait) sits between them.
  constexpr int kRowsInFlight = 8;
  double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const __amdgpu_buffer_rsrc_t prs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(pp), (short)0, rows * 32, 0x00020000);
  for (int i0 = l; i0 < rows; i0 += (int)blockDim.x * kRowsInFlight) {
    float4 lo[kRowsInFlight], hi[kRowsInFlight];
#pragma unroll
    for (int u = 0; u < kRowsInFlight; ++u) {
      const uint32_t off = 32u * (uint32_t)(i0 + u * (int)blockDim.x);
      lo[u] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(prs, off, 0, 0));
      hi[u] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(prs, off + 16u, 0, 0));
    }
    // (rows past the last read as zeros: adding them changes no sum)
#pragma unroll
    for (int u = 0; u < kRowsInFlight; ++u) {
      acc[0] += (double)lo[u].x;
      acc[1] += (double)lo[u].y;
      acc[2] += (double)lo[u].z;
      acc[3] += (double)lo[u].w;
      acc[4] += (double)hi[u].x;
      acc[5] += (double)hi[u].y;
      if (loss_in_part) {
        acc[6] += (double)hi[u].z;
        acc[7] += (double)hi[u].w;
      }
    }
  }
  if (!loss_in_part) {
    const int nl = (HW + kLossThreads - 1) / kLossThreads;
    for (int i = l; i < nl; i += blockDim.x) acc[6] += (double)loss_part[(size_t)v * part_stride + i];
  }
  const int w = l / 64;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const double s = wave_sum_d(acc[k]);
    if (l % 64 == 0) sh[k][w] = s;
  }
  __syncthreads();
  if (l >= 64) return;
  double g[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) g[k] = sh[k][0] + sh[k][1] + sh[k][2] + sh[k][3];
  const double loss = (sh[6][0] + sh[6][1] + sh[6][2] + sh[6][3]) / (double)HW;
  float* pose_history = ctrl->pose_history;
  const int max_hist = ctrl->max_hist;
  // warm-start fallback: at the first iteration, a start pose whose unmasked loss is
  // above the fallback's (or not finite) gives way to the fallback pose, without a step;
  // the histories record the rejected pose's loss and gradient and the fallback pose
  if (it == 0 && loss_in_part && ctrl->fb_armed[v]) {
    const double loss_un = (sh[7][0] + sh[7][1] + sh[7][2] + sh[7][3]) / (double)HW;
    if (!(loss_un <= ctrl->fb_loss[v])) {
      if (l == 0) {
        ctrl->fb_used[v] = 1;
        ctrl->loss[v] = loss;
        float* loss_history = ctrl->loss_history;
        if (loss_history && max_hist > 0) loss_history[v] = (float)loss;
        double* grad_history = ctrl->grad_history;
        if (grad_history && max_hist > 0)
#pragma unroll
          for (int k = 0; k < 6; ++k) grad_history[(size_t)v * 6 + k] = g[k];
        ctrl->iter_v[v] = 1;
      }
      if (l < 12) {
        const double P = ctrl->fb_pose[v][l];
        ctrl->master_pose[v][l] = P;
        pose_out[l] = (float)P;
        if (pose_history && max_hist > 0) pose_history[(size_t)v * 12 + l] = (float)P;
      }
      return;
    }
  }
  // guards: a problem that has stopped keeps its pose; a non-finite loss or gradient
  // stops it at the pose it has (the last finite one); with a patience, `patience`
  // iterations without a lower loss stop it at the pose of the lowest loss
  const int32_t status_old = ctrl->status[v];
  bool finite = isfinite(loss);
#pragma unroll
  for (int k = 0; k < 6; ++k) finite = finite && isfinite(g[k]);
  int32_t status = status_old;
  const bool improved = finite && loss < ctrl->best_loss[v];
  if (status == kTrackRan && !finite) status = kTrackNonFinite;
  if (status == kTrackRan && !improved && adam.patience > 0 && ctrl->rising[v] + 1 >= adam.patience)
    status = kTrackDiverged;
  if (status != kTrackRan) {
    // no step: the pose stays (or returns to the best one), the history repeats it
    const bool to_best = status == kTrackDiverged && status_old == kTrackRan;
    if (l == 0) {
      ctrl->status[v] = status;
      ctrl->loss[v] = loss;
      float* loss_history = ctrl->loss_history;
      if (loss_history && (int)it < max_hist) loss_history[(size_t)it * n_views + v] = (float)loss;
      double* grad_history = ctrl->grad_history;
      if (grad_history && (int)it < max_hist)
#pragma unroll
        for (int k = 0; k < 6; ++k) grad_history[((size_t)it * n_views + v) * 6 + k] = g[k];
      ctrl->iter_v[v] = it + 1;
    }
    if (l < 12) {
      const double P = to_best ? ctrl->best_pose[v][l] : T_old;
      if (to_best) {
        ctrl->master_pose[v][l] = P;
        pose_out[l] = (float)P;
      }
      if (pose_history && (int)it < max_hist) pose_history[((size_t)it * n_views + v) * 12 + l] = (float)P;
    }
    return;
  }
  if (l < 12 && improved) ctrl->best_pose[v][l] = T_old;
  if (l == 0) {
    if (improved) {
      ctrl->best_loss[v] = loss;
      ctrl->rising[v] = 0;
    } else {
      ctrl->rising[v] += 1;
    }
  }
  const double b1 = adam.beta1, b2 = adam.beta2;
  // bias corrections 1 - beta^t from running powers (t = it + 1)
  const double b1t = b1t_old * b1, b2t = b2t_old * b2;
  const double c1 = 1.0 - b1t, c2 = 1.0 - b2t;
  if (l == 0) {
#pragma unroll
    for (int k = 0; k < 6; ++k) ctrl->last_grad[v][k] = g[k];
    ctrl->loss[v] = loss;
    float* loss_history = ctrl->loss_history;
    if (loss_history && (int)it < max_hist) loss_history[(size_t)it * n_views + v] = (float)loss;
    double* grad_history = ctrl->grad_history;
    if (grad_history && (int)it < max_hist)
#pragma unroll
      for (int k = 0; k < 6; ++k) grad_history[((size_t)it * n_views + v) * 6 + k] = g[k];
    ctrl->adam_b1t[v] = b1t;
    ctrl->adam_b2t[v] = b2t;
    ctrl->iter_v[v] = it + 1;
  }
  double tau_l = 0.0;
  if (l < 6) {
    double gl = g[0];
#pragma unroll
    for (int k = 1; k < 6; ++k) gl = l == k ? g[k] : gl;
    const double m = b1 * m_old + (1.0 - b1) * gl;
    const double vv = b2 * v_old + (1.0 - b2) * gl * gl;
    ctrl->adam_m[v][l] = m;
    ctrl->adam_v[v][l] = vv;
    double lr = (double)adam.lr[0];
#pragma unroll
    for (int k = 1; k < 6; ++k) lr = l == k ? (double)adam.lr[k] : lr;
    tau_l = -lr * (m / c1) / (sqrt(vv / c2) + (double)adam.eps);
  }
  double tau[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) tau[k] = __shfl(tau_l, k, 64);
  double Re[9], te[3];
  se3_exp(tau, Re, te);
  // entry (r, c) of the new pose from column c of the old one
  const int r = l / 4, c = l % 4;
  double col[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) col[q] = __shfl(T_old, q * 4 + c, 64);
  if (l < 12) {
    double s = Re[r * 3 + 0] * col[0] + Re[r * 3 + 1] * col[1] + Re[r * 3 + 2] * col[2];
    if (c == 3) s += te[r];
    ctrl->master_pose[v][l] = s;
    pose_out[l] = (float)s;
    if (pose_history && (int)it < max_hist) pose_history[((size_t)it * n_views + v) * 12 + l] = (float)s;
  }
}

}  // namespace gs2d

#endif  // GS2D_POSE_STEP_H
