// Internal declarations shared by the HIP translation units of libgs2d.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/gs2d.h"

namespace gs2d {

// The library's constants of the method (see the rules in gs2d.h).
constexpr float kRhoCutoff = 9.0f;        // 3-sigma footprint, u^2 + v^2 <= 9
constexpr float kAlphaMax = 0.99f;        // opacity clamp
constexpr float kAlphaMin = 1.0f / 255.0f;  // pairs below this opacity are skipped
constexpr float kTMin = 1e-4f;            // stop before transmittance drops below this
constexpr float kFilterScale = 2.0f;      // low-pass term 2 |p - c|^2 (sigma^2 = 1/2 px^2)
constexpr float kOpacityMask = 0.95f;     // tracking-loss opacity mask threshold

// Per-surfel blend record: 6 float4 = 96 bytes, written by the preprocess kernel
// and staged through LDS by the blend kernels.
//   [0] footprint box px0, px1, py0, py1 (inclusive pixel bounds, for wave culling)
//   [1] cx, cy, Dt, k0      [2] k1, P0, P1, Q0      [3] Q1, m0, m1, m2
//   [4] opacity, r, g, b    [5] n.xyz, 0
// With M = K [s_u t_uc | s_v t_vc | mu_c] (rows M0, M1, M2 = m) and the projected
// centre c = (M02, M12) / m2, the record holds the centre-relative rows
// P = M0 - cx m, Q = M1 - cy m (whose third entries vanish), and
// Dt = P0 Q1 - P1 Q0, k0 = m0 Q1 - m1 Q0, k1 = P0 m1 - P1 m0, so that for a
// pixel at offset (dx, dy) from c the homogeneous intersection h_u x h_v is
// (m2 (Q1 dx - P1 dy), m2 (P0 dy - Q0 dx), Dt - k0 dx - k1 dy).
constexpr int kRecF4 = 6;

struct CamF {
  int width, height;
  float fx, fy, cx, cy;
};

struct Ctrl {            // device-resident counters
  uint32_t n_pairs;
  uint32_t n_visible;
  uint32_t overflow;
  uint32_t iter;         // tracking iteration (graph replays)
  double adam_m[6];
  double adam_v[6];
  double master_pose[12];
  double loss;
  float* pose_history;   // set per gs2d_track call, read by the pose step
  float* loss_history;
  int32_t max_hist;
  int32_t pad;
  unsigned long long work[4];  // profile counters: fwd evaluated, fwd covering, bwd evaluated, bwd covering
};

// Kernel families timed by the profiler.
enum Family { kPre, kDepthSort, kScan, kDup, kTileSort, kRanges, kBlendFwd, kLoss, kBlendBwd, kPreBwd, kPose,
              kReduce, kNumFamilies };

}  // namespace gs2d

struct gs2d_ctx {
  int device = 0;
  gs2d_options opt{};
  int last_hip_error = 0;

  // capacities
  int64_t n_cap = 0, p_cap = 0, hw_cap = 0, tile_cap = 0, part_cap = 0, gacc_cap = 0;
  bool pair_fixed = false;

  // per-surfel buffers [n_cap]
  float4* rec = nullptr;
  uint2* rect = nullptr;
  uint32_t* count = nullptr;
  uint32_t* dkey[2] = {nullptr, nullptr};
  uint32_t* dval[2] = {nullptr, nullptr};
  uint32_t* offs = nullptr;
  uint32_t* block_sums = nullptr;
  uint32_t* hist = nullptr;
  int64_t hist_cap = 0;
  float* gacc = nullptr;       // [n][16]

  // pairs [p_cap]
  uint32_t* pkey[2] = {nullptr, nullptr};
  uint32_t* pval[2] = {nullptr, nullptr};
  uint32_t* pkey_keep = nullptr;
  uint32_t* pval_keep = nullptr;

  // tiles, pixels, partials
  uint2* ranges = nullptr;
  float* t_final = nullptr;
  uint32_t* last = nullptr;
  float* lgrad = nullptr;      // [4][hw]: loss gradients used by gs2d_track
  float* limg = nullptr;       // [8][hw]: rendered images used by gs2d_track
  float* part = nullptr;       // [part_cap][8] per-workgroup pose partials
  float* lpart = nullptr;      // [hw_cap / 256 + 1] per-workgroup loss partials
  float* pose0 = nullptr;      // [12] start pose of gs2d_track (for a restart)
  float* saved_pose = nullptr; // [12] pose of the last render
  gs2d::Ctrl* ctrl = nullptr;
  gs2d::Ctrl* host_ctrl = nullptr;  // pinned mirror for readbacks
  hipStream_t graph_stream = nullptr;  // capture stream of gs2d_track (default priority)

  // cached tracking graph (invalidated whenever a workspace buffer moves)
  hipGraphExec_t track_exec = nullptr;
  hipGraph_t track_graph = nullptr;
  unsigned char track_key[256] = {0};
  bool track_valid = false;

  // profiling: HIP events around kernel families (eager calls only)
  struct EvPair { hipEvent_t a, b; int fam; };
  EvPair* ev = nullptr;
  int ev_used = 0, ev_cap = 0;
  double prof_ms[gs2d::kNumFamilies] = {0};
  long long prof_launches[gs2d::kNumFamilies] = {0};
  long long prof_renders = 0;

  // autotuner cache: (width, height, log2 n class) -> (tile_w, tile_h, batch, ms)
  struct TuneEntry { int w, h, ncls, tw, th, batch; float ms; };
  TuneEntry tune[32];
  int n_tune = 0;

  // state of the last render
  uint32_t generation = 0;
  int64_t last_n = 0;
  gs2d_camera last_cam{};
  const float* last_params = nullptr;
  int pair_buf = 0;            // which pkey/pval holds the sorted pairs
  int tiles_x = 0, tiles_y = 0, n_tiles = 0;
  bool have_forward = false;
  bool last_blank = false;
};

namespace gs2d {

// preprocess.hip
void launch_preprocess(const float* params, int n, const float* pose, CamF cam, float z_near, int filter,
                       int tile_w, int tile_h, int tiles_x, int tiles_y, float4* rec, uint2* rect,
                       uint32_t* count, uint32_t* dkey, uint32_t* dval, float* saved_pose,
                       hipStream_t s);
void launch_preprocess_bwd(const float* params, int n, const float* pose, const float* gacc,
                           float* d_params, int accumulate, float* part, hipStream_t s);

// sort.hip
constexpr int kScanItems = 2048;   // items per block of the scans and radix passes
void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
void launch_fill_f32(float* p, float v, int64_t n, hipStream_t s);
void launch_scan_counts(const uint32_t* count, const uint32_t* perm, int n, uint32_t* offs,
                        uint32_t* block_sums, Ctrl* ctrl, hipStream_t s);
// Stable LSD radix sort of (key, value) u32 pairs over bits [0, bits).  n is taken from
// *n_dev when n_dev is non-null (capacity-sized grid), else n_host.  Returns the index
// (0 or 1) of the buffer holding the result.
int radix_sort(uint32_t* keys[2], uint32_t* vals[2], int64_t cap, int64_t n_host,
               const uint32_t* n_dev, int bits, uint32_t* hist, hipStream_t s);
void launch_duplicate(const uint32_t* sorted_ids, const uint32_t* count, const uint32_t* offs,
                      const uint2* rect, int n, int tiles_x, int64_t p_cap, uint32_t* pkey,
                      uint32_t* pval, Ctrl* ctrl, hipStream_t s);
void launch_ranges(const uint32_t* skey, const Ctrl* ctrl, int64_t p_cap, uint2* ranges, int n_tiles,
                   hipStream_t s);
void launch_copy_u32(const uint32_t* src, uint32_t* dst, int64_t n, hipStream_t s);

// blend.hip
struct BlendArgs {
  const uint2* ranges;
  const uint32_t* pval;
  const float4* rec;
  CamF cam;
  float z_near;
  int filter;
  int tiles_x, n_tiles, batch;
};
// work (may be null): profile counters, see Ctrl::work
void launch_blend_fwd(const BlendArgs& a, int tile_w, int tile_h, float* rgb, float* depth,
                      float* normal, float* alpha, float* t_final, uint32_t* last,
                      unsigned long long* work, hipStream_t s);
void launch_blend_bwd(const BlendArgs& a, int tile_w, int tile_h, const float* t_final,
                      const uint32_t* last, const float* g_rgb, const float* g_depth,
                      const float* g_normal, const float* g_alpha, float* gacc, float* part,
                      unsigned long long* work, hipStream_t s);

// loss_pose.hip
void launch_tracking_loss(CamF cam, const float* rgb, const float* depth, const float* normal,
                          const float* alpha, const float* tgt_rgb, const float* tgt_depth,
                          float lambda_d, int use_masks, float* d_rgb, float* d_depth, float* part,
                          int* n_parts, hipStream_t s);
int loss_blocks(int hw);
void launch_reduce_loss(const float* part, int n_parts, float inv_hw, float* loss, Ctrl* ctrl,
                        hipStream_t s);
void launch_reduce_pose(const float* part, int n_parts, float* d_pose, int accumulate,
                        hipStream_t s);
struct AdamArgs {
  float lr[6];
  float beta1, beta2, eps, weight_decay;
};
void launch_pose_exp(const float* tau, const float* pose_in, float* pose_out, hipStream_t s);
void launch_pose_tau_grad(const float* tau, const float* d_pose, float* d_tau, hipStream_t s);
void launch_track_init(const float* pose, Ctrl* ctrl, float* pose_history, float* loss_history,
                       int max_hist, hipStream_t s);
void launch_pose_step(const float* pose_part, int n_pose_parts, const float* loss_part,
                      int n_loss_parts, float inv_hw, AdamArgs adam, float* pose, Ctrl* ctrl,
                      hipStream_t s);

}  // namespace gs2d
