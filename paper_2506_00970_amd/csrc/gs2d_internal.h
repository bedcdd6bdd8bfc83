// Internal declarations shared by the HIP translation units of libgs2d.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/gs2d.h"

namespace gs2d {

// The library's constants of the method (see the rules in gs2d.h).
constexpr float kRhoCutoff = 9.0f;        // 3-sigma footprint, u^2 + v^2 <= 9
constexpr float kAlphaMax = 0.99f;        // opacity clamp
constexpr float kAlphaMin = 1.0f / 255.0f;  // pairs below this opacity are skipped
constexpr float kTMin = 1e-4f;            // stop before transmittance drops below this
constexpr float kFilterScale = 2.0f;      // low-pass term 2 |p - c|^2 (sigma^2 = 1/2 px^2)
constexpr float kOpacityMask = 0.95f;     // tracking-loss opacity mask threshold

// Per-surfel blend record: 7 float4 = 112 bytes, written by the preprocess kernel
// and staged through LDS by the blend kernels.
//   [0] footprint box x0, x1, y0, y1 (inclusive integer pixel bounds, not clipped to
//       the image; wave culling, and the origin of the centre below)
//   [1] cx - x0, cy - y0, Dt, k0      [2] k1, P0, P1, Q0      [3] Q1, m0, m1, m2
//   [4] opacity, r, g, b    [5] n.xyz, Syy
//   [6] ex - x0, ey - y0, Sxx, Sxy: the 3-sigma ellipse (centre e, extent sqrt(d^T S d)
//       along a unit direction d), for the waves' separating-direction cull
// With M = K [s_u t_uc | s_v t_vc | mu_c] (rows M0, M1, M2 = m) and the projected
// centre c = (M02, M12) / m2, the record holds the centre-relative rows
// P = M0 - cx m, Q = M1 - cy m (whose third entries vanish), and
// Dt = P0 Q1 - P1 Q0, k0 = m0 Q1 - m1 Q0, k1 = P0 m1 - P1 m0, so that for a
// pixel at offset (dx, dy) from c the homogeneous intersection h_u x h_v is
// (m2 (Q1 dx - P1 dy), m2 (P0 dy - Q0 dx), Dt - k0 dx - k1 dy).
constexpr int kRecF4 = 7;
constexpr int kMaxViews = GS2D_MAX_VIEWS;

struct CamF {
  int width, height;
  float fx, fy, cx, cy;
};

// One view of a (possibly batched) launch: its surfels, pose, camera, images and
// gradients, and where its items, tiles and pixels sit in the shared work arrays.
// The single-view entry points are batches of one.
struct ViewDesc {
  const float* params;   // [15][n]
  float* pose;           // [12] (written only by the tracking step)
  float* rgb;            // images (forward outputs; tracking-loss inputs)
  float* depth;
  float* normal;
  float* alpha;
  float* g_rgb;          // image gradients (backward inputs; tracking-loss outputs)
  float* g_depth;
  float* g_normal;       // (the image loss writes it when it has a normal term)
  const float* g_alpha;
  const float* tgt_rgb;  // tracking targets
  const float* tgt_depth;
  const float* tgt_normal;  // image loss with a normal term
  float* d_pose;         // [6] pose gradient out (nullable)
  float* contrib;        // [n] per-surfel contribution out (nullable; forward blend)
  float* depth_norm;     // [H][W] D / O out (nullable; forward blend)
  float* depth_median;   // [H][W] median depth out (nullable; forward blend)
  CamF cam;
  int n;                 // surfels of this view
  int item_base;         // first (view, surfel) item
  int tile_base;         // first global tile
  int tiles_x, tiles_y;
  int pix_base;          // first pixel of the view in the per-pixel work arrays
};

struct Ctrl {            // device-resident counters and tracking state
  uint32_t n_pairs;
  uint32_t n_visible;
  uint32_t overflow;
  uint32_t iter;         // unused (kept for layout); see iter_v
  float* pose_history;   // set per tracking call, read by the pose step
  float* loss_history;
  double* grad_history;  // [max_hist][n_views][6] or null
  int32_t max_hist;
  int32_t n_views;
  unsigned long long work[4];  // profile counters: fwd evaluated, fwd covering, bwd evaluated, bwd covering
  uint32_t iter_v[kMaxViews];  // tracking iteration of each view (graph replays)
  double loss[kMaxViews];
  double adam_m[kMaxViews][6];
  double adam_v[kMaxViews][6];
  double last_grad[kMaxViews][6];  // each view's pose gradient of the last tracking step
  double adam_b1t[kMaxViews];   // beta1^t, beta2^t of each view's AdamW step
  double adam_b2t[kMaxViews];
  double master_pose[kMaxViews][12];
  // guards: nonzero when a render met a surfel or pose that is not finite (those items
  // are culled; cleared when a render uploads its views); per tracking problem, the
  // status (kTrackRan, kTrackDiverged, kTrackNonFinite), the iterations since the loss
  // last fell, and the lowest loss with the pose it was measured at
  uint32_t nonfinite;
  uint32_t check_bits;   // device checks that failed (builds with GS2D_DEVICE_CHECKS; sticky)
  int32_t status[kMaxViews];
  int32_t rising[kMaxViews];
  double best_loss[kMaxViews];
  double best_pose[kMaxViews][12];
  // warm-start fallback per tracking problem: armed, the pose and unmasked loss to fall
  // back to, and whether the first iteration did
  int32_t fb_armed[kMaxViews];
  int32_t fb_used[kMaxViews];
  double fb_loss[kMaxViews];
  double fb_pose[kMaxViews][12];
};

// Device checks of the debug build (GS2D_DEVICE_CHECKS): a failed check sets its bit
// in Ctrl::check_bits instead of trapping; release builds compile them away.
constexpr uint32_t kCheckRect = 1u;         // an item's tile rectangle lies inside its view's grid
constexpr uint32_t kCheckPairKey = 2u;      // a pair's tile key is below the tile count
constexpr uint32_t kCheckPairIndex = 4u;    // a pair's slot is below the pair capacity
constexpr uint32_t kCheckRangeTile = 8u;    // a sorted key names a tile below the tile count
constexpr uint32_t kCheckBlendRange = 16u;  // a blended tile exists and its range is ordered
#ifdef GS2D_DEVICE_CHECKS
#define GS2D_DCHECK(bits, cond, bit)                       \
  do {                                                     \
    if ((bits) != nullptr && !(cond)) atomicOr((bits), (bit)); \
  } while (0)
#else
#define GS2D_DCHECK(bits, cond, bit) \
  do {                               \
  } while (0)
#endif

constexpr int32_t kTrackRan = 0;        // every iteration stepped
constexpr int32_t kTrackDiverged = 1;   // stopped at the best pose after `patience` rising losses
constexpr int32_t kTrackNonFinite = 2;  // stopped at the last finite pose on a non-finite loss or step

// Kernel families timed by the profiler.
enum Family { kPre, kDepthSort, kScan, kDup, kTileSort, kRanges, kBlendFwd, kLoss, kBlendBwd, kPreBwd, kPose,
              kReduce, kBlendTrack, kNumFamilies };

// Host copy of a launch's view table.
struct ViewSet {
  ViewDesc v[kMaxViews];
  int n_views = 0;
  int64_t items = 0, tiles = 0, pixels = 0;
  int max_hw = 0;
};

// Binary search of the view owning item / tile `i` (n_views <= 32).
__device__ __forceinline__ int view_of_item(const ViewDesc* v, int nv, int i) {
  int lo = 0;
#pragma unroll
  for (int s = 16; s > 0; s >>= 1)
    if (lo + s < nv && v[lo + s].item_base <= i) lo += s;
  return lo;
}
__device__ __forceinline__ int view_of_tile(const ViewDesc* v, int nv, int g) {
  int lo = 0;
#pragma unroll
  for (int s = 16; s > 0; s >>= 1)
    if (lo + s < nv && v[lo + s].tile_base <= g) lo += s;
  return lo;
}

}  // namespace gs2d

struct gs2d_ctx {
  int device = 0;
  gs2d_options opt{};
  int last_hip_error = 0;

  // capacities
  int64_t n_cap = 0, p_cap = 0, hw_cap = 0, tile_cap = 0, part_cap = 0, gacc_cap = 0, img_cap = 0;
  bool pair_fixed = false;

  // per-item buffers [n_cap] (an item is one surfel of one view)
  float4* rec = nullptr;
  uint2* rect = nullptr;
  uint32_t* count = nullptr;
  uint32_t* dkey = nullptr;     // per-item depth keys
  uint32_t* parts = nullptr;   // per-block pair and visible counts of preprocessing
  uint32_t* hist = nullptr;    // the sort planes and row totals (gs2d::SortPlanes)
  int64_t hist_cap = 0;
  int hist_stride = 0;
  bool hist_fresh = false;     // allocated but not yet cleared on the stream
  float* gacc = nullptr;       // [items][16]

  // pairs [p_cap]
  uint32_t* pkey[2] = {nullptr, nullptr};
  uint32_t* pval[2] = {nullptr, nullptr};
  uint32_t* pdk[2] = {nullptr, nullptr};  // each pair's depth key, moved with pval by the tile sort
  uint32_t* pkey_keep = nullptr;
  uint32_t* pval_keep = nullptr;

  // tiles, pixels, partials, view tables
  uint2* ranges = nullptr;
  uint32_t* queue = nullptr;   // [kQueueOrder + tile_cap]: the blends' work queue
  bool queue_on = false;       // the last render built the queue (persistent blends)
  float* t_final = nullptr;
  uint32_t* last = nullptr;
  float* lgrad = nullptr;      // [4][pixels]: loss gradients of the tracking loop
  float* limg = nullptr;       // [8][pixels]: rendered images of the tracking loop
  float* part = nullptr;       // [part_cap][8] per-workgroup pose partials
  float* lpart = nullptr;      // [kMaxViews][loss blocks] per-workgroup loss partials
  int64_t lpart_cap = 0;
  float* pose0 = nullptr;      // [kMaxViews][12] start poses of a tracking call (for a restart)
  float* saved_pose = nullptr; // [kMaxViews][12] poses of the last render
  gs2d::ViewDesc* views = nullptr;  // device view table [kMaxViews]
  gs2d::Ctrl* ctrl = nullptr;
  gs2d::Ctrl* host_ctrl = nullptr;  // pinned mirror for readbacks
  // a pinned, device-mapped host word that the render's scan or duplication writes the
  // pair total to: the render waits for it without a copy (np_dev: its device address)
  volatile uint32_t* np_host = nullptr;
  uint32_t* np_dev = nullptr;
  hipStream_t graph_stream = nullptr;  // capture stream of the tracking loop (default priority)

  // cached tracking graph (invalidated whenever a workspace buffer moves)
  hipGraphExec_t track_exec = nullptr;
  hipGraph_t track_graph = nullptr;
  std::vector<unsigned char> track_key;
  bool track_valid = false;

  // profiling: HIP events around kernel families (eager calls only)
  struct EvPair { hipEvent_t a, b; int fam; };
  EvPair* ev = nullptr;
  int ev_used = 0, ev_cap = 0;
  double prof_ms[gs2d::kNumFamilies] = {0};
  long long prof_launches[gs2d::kNumFamilies] = {0};

  // autotuner cache: (width, height, log2 n class) -> (tile_w, tile_h, batch, ms)
  struct TuneEntry { int w, h, ncls, flags, tw, th, batch; float ms; };
  TuneEntry tune[32];
  int n_tune = 0;

  // state of the last render
  uint32_t generation = 0;
  gs2d::ViewSet last_views;    // views of the last render (host copy)
  int pair_buf = 0;            // which pkey/pval holds the sorted pairs
  bool have_forward = false;
};

namespace gs2d {

// preprocess.hip
// Copies the view table to the device; with ctrl (a render's upload) also clears the
// non-finite flag.
void launch_upload_views(const ViewSet& vs, ViewDesc* dst, hipStream_t s, Ctrl* ctrl = nullptr);
constexpr int kPartItems = 256;  // items per preprocessing block (per-block pair counts)
// Per item: record, tile rectangle, tile count and depth key (0xFFFFFFFF for items
// that touch no tile); per block of kPartItems items: the pair count and the count of
// items that touch a tile.  clear_overflow: clears ctrl->overflow (a tracking loop
// keeps it from the start of the call, so that an overflow in any iteration is seen).
void launch_preprocess(const ViewDesc* views, int n_views, int64_t items, float z_near, int filter, int tile_w,
                       int tile_h, float4* rec, uint2* rect, uint32_t* count, uint32_t* dkey, float* saved_pose,
                       uint32_t* part_pairs, uint32_t* part_vis, Ctrl* ctrl, hipStream_t s,
                       bool clear_overflow = true);
// Zero the 16-float accumulator rows of the items whose tile count is nonzero.
void launch_clear_rows(const uint32_t* count, float* gacc, int64_t items, hipStream_t s);
// count: the items' tile counts (rows of items with none are not read)
void launch_preprocess_bwd(const float* params, int n, const float* pose, const uint32_t* count, const float* gacc,
                           float* d_params, int accumulate, float* part, hipStream_t s);
// The same for n_views (1..32) views that share params, n and d_params, in one pass:
// view g's pose terms go to partial rows [g * rows, (g + 1) * rows), rows =
// 4 ceil(n / 256) (one per wave).  Returns -1 (and launches nothing) for an
// unsupported n_views.
constexpr int kGroupRowsPerBlock = 4;  // partial rows per 256-surfel block of the group backward
int launch_preprocess_bwd_group(const float* params, int n, int n_views, const float* const* poses,
                                const uint32_t* const* counts, const float* const* gaccs, float* d_params,
                                int accumulate, float* part, hipStream_t s);

// sort.hip
constexpr int kScanItems = 1024;   // keys per block of the radix passes
constexpr int kMaxDigitBits = 11;  // widest radix digit (2048 bins)
void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
void launch_fill_f32(float* p, float v, int64_t n, hipStream_t s);
// Digit histograms of the tile sort's passes: two digit-major planes of 2048 rows by
// `stride` columns (one per block of kScanItems pairs) and the row totals.  Between
// renders both planes are all zero.
struct SortPlanes {
  uint32_t* plane[2];
  int stride;
  uint32_t* dtot;
};
// Bits of pass p of a stable LSD sort over `bits` key bits in passes of at most 11.
int radix_pass_bits(int bits, int p);
// Whether `items` take the scan below (many preprocessing blocks); otherwise the
// duplication sums the per-block counts itself.
bool part_scan_needed(int64_t items);
// Exclusive scan of the per-block pair counts in place, and ctrl->n_pairs / n_visible
// (n_pairs also to *np_host, a host-visible word, if not NULL).
void launch_part_scan(uint32_t* part_pairs, const uint32_t* part_vis, int64_t items, Ctrl* ctrl, uint32_t* np_host,
                      hipStream_t s);
// The (tile, item) pairs of every item, in item order, placed by the per-block pair
// counts of preprocessing (an exclusive prefix when `scanned`; otherwise the kernel
// also stores ctrl->n_pairs, and *np_host if not NULL, and ctrl->n_visible); sets
// ctrl->overflow when the pairs exceed p_cap.  Fills plane 1 with the first tile
// pass's histogram.  Each pair's depth key (dkey of its item) goes to pdk beside pval.
void launch_duplicate(const SortPlanes& ws, const uint32_t* count, const uint32_t* part_pairs,
                      const uint32_t* part_vis, bool scanned, const uint2* rect, const ViewDesc* views, int n_views,
                      int64_t items, int64_t p_cap, int tile_bits, uint32_t* pkey, uint32_t* pval, Ctrl* ctrl,
                      uint2* ranges, int n_tiles, const uint32_t* dkey, uint32_t* pdk, uint32_t* np_host,
                      hipStream_t s);
// Stable sort of the min(n_pairs, p_cap) pairs by tile key over `bits` bits, moving
// vals and dks with the keys.  A single pass also writes the tile ranges (empty after
// an overflow).  Returns the buffer index.
int tile_sort(const SortPlanes& ws, uint32_t* keys[2], uint32_t* vals[2], uint32_t* dks[2], int64_t p_cap, int bits,
              Ctrl* ctrl, uint2* ranges, int n_tiles, hipStream_t s);
// Orders every tile's items (ids[ranges[t].x .. ranges[t].y), ascending on entry) by
// depth key, stably: each list then ascends in (depth key, item).  pdk: the pairs'
// depth keys beside ids; scratch: a buffer of the same size as ids for lists longer
// than one workgroup's LDS (those read the keys through dkey[id]).
void launch_tile_order(const uint2* ranges, int n_tiles, uint32_t* ids, uint32_t* scratch, const uint32_t* pdk,
                       const uint32_t* dkey, hipStream_t s);
void launch_ranges(const uint32_t* skey, Ctrl* ctrl, int64_t p_cap, uint2* ranges, int n_tiles,
                   hipStream_t s);
// The blends' work queue of a view set: tiles by descending list length (counting
// order over 64 buckets of 32 entries; within a bucket any order), both heads zero.
void launch_queue_order(const uint2* ranges, int n_tiles, uint32_t* queue, hipStream_t s);
void launch_copy_u32(const uint32_t* src, uint32_t* dst, int64_t n, hipStream_t s);

struct AdamArgs {  // the tracking pose step's AdamW settings and divergence guard
  float lr[6];
  float beta1, beta2, eps, weight_decay;
  int patience;     // stop after this many iterations without a lower loss (0: never)
};

// blend.hip
struct BlendArgs {
  const uint2* ranges;
  const uint32_t* pval;
  const float4* rec;
  const ViewDesc* views;
  int n_views;
  int n_tiles;           // global tiles over all views
  float z_near;
  int filter;
  int batch;
  // workgroup i blends tile (i * tile_stride) mod n_tiles (tile_stride coprime to
  // n_tiles): neighbouring tiles, which have lists of similar length, start at
  // different times and on different compute units
  int tile_stride = 1;
  // the tracking walk's tile rows (pose gradient in slots 0-5, loss in slot 6), and
  // the loss's depth weight and masks
  float* loss_part = nullptr;
  float lambda_d = 0.f;
  int use_masks = 0;
  // the learned warm start's input from the forward blend of one view with targets
  // (its sides multiples of 8; its images are not written): per 8 x 8 pixel block
  // (row-major, width / 8 per row), the BF16 block means of (image - target) for R,
  // G, B and depth in res_x[block][4], and |dR| + |dG| + |dB| + lambda_d |dD| summed
  // over the block in res_part[block]
  uint16_t* res_x = nullptr;
  float* res_part = nullptr;
  // tracking walk with 256-thread tiles: with order_ids, each workgroup first orders
  // its own tile's list (order_ids = the tile-sorted ids, order_scratch a buffer of the
  // same size, dkey the per-item depth keys), so no separate depth-order kernel runs
  uint32_t* order_ids = nullptr;
  uint32_t* order_scratch = nullptr;
  const uint32_t* dkey = nullptr;
  const uint32_t* order_keys = nullptr;  // the pairs' depth keys beside order_ids
  // persistent launch of the forward and backward blends (many more tiles than fit on
  // the GPU at once): queue[kQueueHeadFwd], queue[kQueueHeadBwd] are the next items,
  // queue[kQueueOrder + i] the tiles by descending list length; null: one workgroup
  // per tile
  uint32_t* queue = nullptr;
  uint32_t* check = nullptr;  // Ctrl::check_bits (device checks)
};

constexpr int kQueueHeadFwd = 0;
constexpr int kQueueHeadBwd = 1;
constexpr int kQueueOrder = 2;
// Batched renders with more tiles than this use the persistent blends.
constexpr int kQueueMinTiles = 4096;
// Tracking: forward blend, tracking loss and pose-only gradient in one walk; needs
// a.loss_part (tile rows: pose gradient in slots 0-5, loss in slot 6), lambda_d,
// use_masks, and views with targets.  work: the forward's profile counters.
void launch_blend_track(const BlendArgs& a, int tile_w, int tile_h, unsigned long long* work, hipStream_t s);
// work (may be null): profile counters, see Ctrl::work
void launch_blend_fwd(const BlendArgs& a, int tile_w, int tile_h, float* t_final, uint32_t* last,
                      unsigned long long* work, hipStream_t s);
// has_normal / has_alpha: some view has that gradient (views without it read zeros).
// gacc null selects the pose-only mode; part gets one row of 8 floats per global tile.
void launch_blend_bwd(const BlendArgs& a, int tile_w, int tile_h, const float* t_final, const uint32_t* last,
                      bool has_normal, bool has_alpha, float* gacc, float* part, unsigned long long* work,
                      hipStream_t s);

// loss_pose.hip
int loss_blocks(int hw);
// Weights and masks of the masked L1 image loss (the tracking loss is {1, lambda_d, 0,
// masks, masks}).
struct LossW {
  float w_rgb, w_d, w_n;
  int normal_mask, opacity_mask;
};
// Image loss of every view: images, targets and gradient outputs at the view table's
// pointers (colour, normal and gradient pointers may be null: term or output skipped);
// partial sums at part[v * part_stride + block].
void launch_image_loss(const ViewDesc* views, int n_views, int max_hw, LossW w, float* part, int part_stride,
                       hipStream_t s);
inline void launch_tracking_loss(const ViewDesc* views, int n_views, int max_hw, float lambda_d, int use_masks,
                                 float* part, int part_stride, hipStream_t s) {
  launch_image_loss(views, n_views, max_hw, LossW{1.0f, lambda_d, 0.0f, use_masks, use_masks}, part, part_stride,
                    s);
}
void launch_reduce_loss(const float* part, int n_parts, float inv_hw, float* loss, hipStream_t s);
// losses[v] = (sum of view v's partials, rows [v * part_stride, ...)) / HW_v, one wave per view.
void launch_reduce_loss_views(const ViewDesc* views, int n_views, const float* part, int part_stride, float* losses,
                              hipStream_t s);
// d_pose = sum of rows [row0, row0 + rows) of `part` (one launch).
void launch_reduce_pose(const float* part, int row0, int rows, float* d_pose, int accumulate, hipStream_t s);
// d_pose[g] (for g < n_views, skipped when NULL) = the sum of partial rows
// [g * rows, (g + 1) * rows), one workgroup per view.
void launch_reduce_pose_group(const float* part, int rows, int n_views, float* const* d_pose, int accumulate,
                              hipStream_t s);
// Per view: d_pose (from the view table) = sum of the rows of the view's tiles.
void launch_reduce_pose_views(const ViewDesc* views, int n_views, const float* part, int accumulate,
                              hipStream_t s);
void launch_pose_exp(const float* tau, const float* pose_in, float* pose_out, hipStream_t s);
// A render of one view (n > 0 surfels; its sides multiples of 8) whose forward blend
// writes, instead of the images, the learned warm start's input against the targets:
// x[block][4] and part[block] as BlendArgs::res_x and res_part describe.
int render_residual(gs2d_ctx* ctx, const float* params, int64_t n, const gs2d_camera* camera, const float* pose,
                    const float* tgt_rgb, const float* tgt_depth, float lambda_d, uint16_t* x, float* part,
                    hipStream_t s);
void launch_pose_tau_grad(const float* tau, const float* d_pose, float* d_tau, hipStream_t s);
// Resets the tracking state and the pair-overflow flag.  fallback (nullable): per view
// the device pose [12] and unmasked loss [1] of the warm start's fallback (either null:
// none for that view).
struct Fallbacks {
  const float* pose[kMaxViews];
  const float* loss[kMaxViews];
};
void launch_track_init(const ViewDesc* views, int n_views, Ctrl* ctrl, float* pose_history, float* loss_history,
                       double* grad_history, int max_hist, hipStream_t s, const Fallbacks* fallback = nullptr);
// One AdamW + Exp step per view: pose partials are the rows of each view's tiles,
// loss partials part[v * part_stride + block].
// loss_in_part: each view's loss is the sum of its tiles' pose_part[tile * 8 + 6]
// (fused into the forward blend), else of its row of loss_part.
void launch_pose_step(const ViewDesc* views, int n_views, const float* pose_part, bool loss_in_part,
                      const float* loss_part, int part_stride, AdamArgs adam, Ctrl* ctrl, hipStream_t s);

}  // namespace gs2d
