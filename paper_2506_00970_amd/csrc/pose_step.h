// The pose step of tracking, shared by its own kernel and the fused tracking walk.
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
// the step on one thread.
__device__ inline void pose_step_view(int v, int n_views, const ViewDesc* __restrict__ views,
                                      const float* __restrict__ pose_part, int loss_in_part,
                                      const float* __restrict__ loss_part, int part_stride, const AdamArgs& adam,
                                      Ctrl* __restrict__ ctrl) {
  __shared__ double sh[7][4];
  const ViewDesc& V = views[v];
  const int HW = V.cam.width * V.cam.height;
  const int rows = V.tiles_x * V.tiles_y;
  const float* pp = pose_part + (size_t)V.tile_base * 8;
  // the six pose sums and the loss in one pass and one block reduction (fixed order)
  double acc[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < rows; i += blockDim.x)
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[k] += (double)pp[(size_t)i * 8 + k];
  if (loss_in_part) {
    for (int i = threadIdx.x; i < rows; i += blockDim.x) acc[6] += (double)pp[(size_t)i * 8 + 6];
  } else {
    const int nl = (HW + kLossThreads - 1) / kLossThreads;
    for (int i = threadIdx.x; i < nl; i += blockDim.x) acc[6] += (double)loss_part[(size_t)v * part_stride + i];
  }
  const int w = threadIdx.x / 64;
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    const double s = wave_sum_d(acc[k]);
    if (threadIdx.x % 64 == 0) sh[k][w] = s;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double g[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) g[k] = sh[k][0] + sh[k][1] + sh[k][2] + sh[k][3];
  const double loss = (sh[6][0] + sh[6][1] + sh[6][2] + sh[6][3]) / (double)HW;
#pragma unroll
  for (int k = 0; k < 6; ++k) ctrl->last_grad[v][k] = g[k];
  const uint32_t it = ctrl->iter_v[v];
  float* pose_history = ctrl->pose_history;
  float* loss_history = ctrl->loss_history;
  const int max_hist = ctrl->max_hist;
  ctrl->loss[v] = loss;
  if (loss_history && (int)it < max_hist) loss_history[(size_t)it * n_views + v] = (float)loss;
  const double b1 = adam.beta1, b2 = adam.beta2;
  // bias corrections 1 - beta^t from running powers (t = it + 1)
  const double b1t = ctrl->adam_b1t[v] * b1, b2t = ctrl->adam_b2t[v] * b2;
  ctrl->adam_b1t[v] = b1t;
  ctrl->adam_b2t[v] = b2t;
  const double c1 = 1.0 - b1t, c2 = 1.0 - b2t;
  double tau[6];
  for (int k = 0; k < 6; ++k) {
    const double m = b1 * ctrl->adam_m[v][k] + (1.0 - b1) * g[k];
    const double vv = b2 * ctrl->adam_v[v][k] + (1.0 - b2) * g[k] * g[k];
    ctrl->adam_m[v][k] = m;
    ctrl->adam_v[v][k] = vv;
    tau[k] = -(double)adam.lr[k] * (m / c1) / (sqrt(vv / c2) + (double)adam.eps);
  }
  double Re[9], te[3];
  se3_exp(tau, Re, te);
  double* T = ctrl->master_pose[v];
  double Tn[12];
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 4; ++c) {
      double s = Re[r * 3 + 0] * T[0 * 4 + c] + Re[r * 3 + 1] * T[1 * 4 + c] + Re[r * 3 + 2] * T[2 * 4 + c];
      if (c == 3) s += te[r];
      Tn[r * 4 + c] = s;
    }
  }
  for (int k = 0; k < 12; ++k) {
    T[k] = Tn[k];
    V.pose[k] = (float)Tn[k];
    if (pose_history && (int)it < max_hist) pose_history[((size_t)it * n_views + v) * 12 + k] = (float)Tn[k];
  }
  ctrl->iter_v[v] = it + 1;
}

}  // namespace gs2d

#endif  // GS2D_POSE_STEP_H
