// C ABI of libgs2d.so: context and workspace management, render, backward,
// tracking loss, the graph-captured tracking loop and diagnostics.
#include <cmath>
#include <cstring>
#include <new>

#include "gs2d_internal.h"

using namespace gs2d;

namespace {

int fail_hip(gs2d_ctx* ctx, hipError_t e) {
  ctx->last_hip_error = (int)e;
  (void)hipGetLastError();  // clear the sticky launch error, if any
  return e == hipErrorOutOfMemory ? GS2D_ERR_OOM : GS2D_ERR_HIP;
}

#define GS2D_HIP(ctx, expr)                    \
  do {                                         \
    hipError_t e_ = (expr);                    \
    if (e_ != hipSuccess) return fail_hip((ctx), e_); \
  } while (0)

#define GS2D_TRY(expr)            \
  do {                            \
    int r_ = (expr);              \
    if (r_ != GS2D_OK) return r_; \
  } while (0)

void invalidate_graph(gs2d_ctx* ctx) {
  if (ctx->track_exec) (void)hipGraphExecDestroy(ctx->track_exec);
  if (ctx->track_graph) (void)hipGraphDestroy(ctx->track_graph);
  ctx->track_exec = nullptr;
  ctx->track_graph = nullptr;
  ctx->track_valid = false;
}

// Every workspace (re)allocation moves a buffer, so it also drops the cached
// tracking graph, whose kernels hold the old addresses.
template <class T>
int realloc_dev(gs2d_ctx* ctx, T** p, int64_t count) {
  invalidate_graph(ctx);
  if (*p) {
    (void)hipFree(*p);
    *p = nullptr;
  }
  if (count <= 0) return GS2D_OK;
  hipError_t e = hipMalloc((void**)p, (size_t)count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail_hip(ctx, e);
  }
  return GS2D_OK;
}

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

const char* kFamilyNames[kNumFamilies] = {"preprocess", "depth_order", "count_scan", "duplicate",
                                          "tile_sort",  "ranges",     "blend_fwd", "loss",
                                          "blend_bwd",  "preprocess_bwd", "pose_step", "reduce",
                                          "blend_track"};

// Records a HIP event pair around a kernel family on the launch stream when the
// context profiles and the stream is not being captured.
struct ProfScope {
  gs2d_ctx* ctx = nullptr;
  hipStream_t s = nullptr;
  int idx = -1;
  ProfScope(gs2d_ctx* c, int fam, hipStream_t st) {
    if (!c->opt.profile) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    if (c->ev_used == c->ev_cap) {
      const int cap = c->ev_cap ? 2 * c->ev_cap : 64;
      auto* nev = new (std::nothrow) gs2d_ctx::EvPair[cap];
      if (!nev) return;
      for (int i = 0; i < c->ev_cap; ++i) nev[i] = c->ev[i];
      for (int i = c->ev_cap; i < cap; ++i) {
        nev[i].a = nev[i].b = nullptr;
        if (hipEventCreate(&nev[i].a) != hipSuccess || hipEventCreate(&nev[i].b) != hipSuccess) {
          (void)hipGetLastError();
          delete[] nev;
          return;
        }
      }
      delete[] c->ev;
      c->ev = nev;
      c->ev_cap = cap;
    }
    idx = c->ev_used++;
    c->ev[idx].fam = fam;
    ctx = c;
    s = st;
    (void)hipEventRecord(c->ev[idx].a, st);
  }
  ~ProfScope() {
    if (ctx) (void)hipEventRecord(ctx->ev[idx].b, s);
  }
};

unsigned long long* work_ptr(gs2d_ctx* ctx, hipStream_t s) {
  if (ctx->opt.profile != 1) return nullptr;  // level 2 times the kernels without counting
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return nullptr;
  return ctx->ctrl->work;
}

int stream_capturing(hipStream_t s, bool* cap) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing(s, &st);
  if (e != hipSuccess) return (int)e;
  *cap = st == hipStreamCaptureStatusActive;
  return 0;
}

int ensure_hist(gs2d_ctx* ctx) {
  const int64_t items = ctx->n_cap > ctx->p_cap ? ctx->n_cap : ctx->p_cap;
  // two planes of 2048 digit rows by one column per block, plus the row totals
  const int64_t stride = (items + kScanItems - 1) / kScanItems > 0 ? (items + kScanItems - 1) / kScanItems : 1;
  if (stride <= ctx->hist_stride) return GS2D_OK;
  const int64_t need = 2 * stride * (1 << kMaxDigitBits) + (1 << kMaxDigitBits);
  GS2D_TRY(realloc_dev(ctx, &ctx->hist, need));
  ctx->hist_cap = need;
  ctx->hist_stride = (int)stride;
  ctx->hist_fresh = true;  // cleared on the stream before its first use
  return GS2D_OK;
}

SortPlanes sort_planes(gs2d_ctx* ctx) {
  const size_t plane = (size_t)ctx->hist_stride << kMaxDigitBits;
  return SortPlanes{{ctx->hist, ctx->hist + plane}, ctx->hist_stride, ctx->hist + 2 * plane};
}

// The sort planes must be all zero before a render; fresh allocations are cleared here.
void clear_fresh_hist(gs2d_ctx* ctx, hipStream_t s) {
  if (!ctx->hist_fresh) return;
  launch_fill_u32(ctx->hist, 0u, ctx->hist_cap, s);
  ctx->hist_fresh = false;
}

int ensure_surfels(gs2d_ctx* ctx, int64_t n) {
  if (n <= ctx->n_cap) return GS2D_OK;
  const int64_t cap = round_up(n, kScanItems);
  GS2D_TRY(realloc_dev(ctx, &ctx->rec, cap * kRecF4));
  GS2D_TRY(realloc_dev(ctx, &ctx->rect, cap));
  GS2D_TRY(realloc_dev(ctx, &ctx->count, cap));
  GS2D_TRY(realloc_dev(ctx, &ctx->dkey, cap));
  GS2D_TRY(realloc_dev(ctx, &ctx->parts, 2 * (cap / kPartItems + 1)));
  ctx->n_cap = cap;
  return ensure_hist(ctx);
}

int ensure_pairs(gs2d_ctx* ctx, int64_t p) {
  if (p <= ctx->p_cap) return GS2D_OK;
  const int64_t cap = round_up(p, kScanItems);
  for (int k = 0; k < 2; ++k) {
    GS2D_TRY(realloc_dev(ctx, &ctx->pkey[k], cap));
    GS2D_TRY(realloc_dev(ctx, &ctx->pval[k], cap));
    GS2D_TRY(realloc_dev(ctx, &ctx->pdk[k], cap));
  }
  if (ctx->opt.keep_unsorted) {
    GS2D_TRY(realloc_dev(ctx, &ctx->pkey_keep, cap));
    GS2D_TRY(realloc_dev(ctx, &ctx->pval_keep, cap));
  }
  ctx->p_cap = cap;
  return ensure_hist(ctx);
}

int ensure_pixels(gs2d_ctx* ctx, int64_t hw) {
  if (hw <= ctx->hw_cap) return GS2D_OK;
  GS2D_TRY(realloc_dev(ctx, &ctx->t_final, hw));
  GS2D_TRY(realloc_dev(ctx, &ctx->last, hw));
  ctx->hw_cap = hw;
  return GS2D_OK;
}

int ensure_tiles(gs2d_ctx* ctx, int64_t tiles) {
  if (tiles <= ctx->tile_cap) return GS2D_OK;
  GS2D_TRY(realloc_dev(ctx, &ctx->ranges, tiles));
  GS2D_TRY(realloc_dev(ctx, &ctx->queue, kQueueOrder + tiles));
  ctx->tile_cap = tiles;
  return GS2D_OK;
}

int ensure_parts(gs2d_ctx* ctx, int64_t rows) {
  if (rows <= ctx->part_cap) return GS2D_OK;
  GS2D_TRY(realloc_dev(ctx, &ctx->part, rows * 8));
  ctx->part_cap = rows;
  return GS2D_OK;
}

int ensure_gacc(gs2d_ctx* ctx, int64_t n) {
  if (n <= ctx->gacc_cap) return GS2D_OK;
  const int64_t cap = round_up(n, kScanItems);
  GS2D_TRY(realloc_dev(ctx, &ctx->gacc, cap * 16));
  ctx->gacc_cap = cap;
  return GS2D_OK;
}

int tile_bits(int n_tiles) {
  int b = 1;
  while ((1 << b) < n_tiles) ++b;
  return b;
}

bool valid_tile(int tw, int th) {
  return (tw == 8 && th == 8) || (tw == 16 && th == 8) || (tw == 16 && th == 16) || (tw == 32 && th == 16);
}

bool valid_batch(int b) { return b == 32 || b == 64 || b == 128 || b == 256; }

CamF camf(const gs2d_camera& c) { return CamF{c.width, c.height, c.fx, c.fy, c.cx, c.cy}; }

bool valid_camera(const gs2d_camera* c) {
  return c && c->width > 0 && c->height > 0 && c->width <= 16384 && c->height <= 16384 &&
         std::isfinite(c->fx) && std::isfinite(c->fy) && c->fx > 0.f && c->fy > 0.f &&
         std::isfinite(c->cx) && std::isfinite(c->cy);
}


int ensure_lpart(gs2d_ctx* ctx, int64_t n) {
  if (n <= ctx->lpart_cap) return GS2D_OK;
  GS2D_TRY(realloc_dev(ctx, &ctx->lpart, n));
  ctx->lpart_cap = n;
  return GS2D_OK;
}

// Lays out a view table: items, tiles and pixels of view v follow those of view v - 1.
int build_views(gs2d_ctx* ctx, const gs2d_view* in, int nv, ViewSet& vs) {
  if (!in || nv < 1 || nv > kMaxViews) return GS2D_ERR_INVALID_ARG;
  const int tw = ctx->opt.tile_w, th = ctx->opt.tile_h;
  vs = ViewSet();
  vs.n_views = nv;
  for (int k = 0; k < nv; ++k) {
    const gs2d_view& g = in[k];
    if (!valid_camera(&g.camera) || g.n < 0 || (g.n > 0 && !g.params) || !g.pose) return GS2D_ERR_INVALID_ARG;
    ViewDesc& d = vs.v[k];
    std::memset(&d, 0, sizeof(d));
    d.params = g.params;
    d.pose = const_cast<float*>(g.pose);
    d.rgb = g.rgb;
    d.depth = g.depth;
    d.normal = g.normal;
    d.alpha = g.alpha;
    d.contrib = g.contrib;
    d.depth_norm = g.depth_norm;
    d.depth_median = g.depth_median;
    d.cam = camf(g.camera);
    d.n = (int)g.n;
    d.tiles_x = (g.camera.width + tw - 1) / tw;
    d.tiles_y = (g.camera.height + th - 1) / th;
    d.item_base = (int)vs.items;
    d.tile_base = (int)vs.tiles;
    d.pix_base = (int)vs.pixels;
    const int hw = g.camera.width * g.camera.height;
    vs.max_hw = hw > vs.max_hw ? hw : vs.max_hw;
    vs.items += g.n;
    vs.tiles += (int64_t)d.tiles_x * d.tiles_y;
    vs.pixels += hw;
    if (vs.items > 0x7FFFFFFF || vs.pixels > 0x7FFFFFFF) return GS2D_ERR_UNSUPPORTED;
  }
  if (vs.tiles > (1 << 24)) return GS2D_ERR_UNSUPPORTED;
  return GS2D_OK;
}

// A stride near 97 that is coprime to n: the blend's workgroup -> tile map.
int tile_stride(int64_t n) {
  int s = 97;
  auto gcd = [](int64_t a, int64_t b) {
    while (b) {
      const int64_t t = a % b;
      a = b;
      b = t;
    }
    return a;
  };
  while (n > 1 && gcd(s, n) != 1) ++s;
  return s;
}

BlendArgs blend_args(gs2d_ctx* ctx) {
  BlendArgs a{ctx->ranges, ctx->pval[ctx->pair_buf], ctx->rec, ctx->views, ctx->last_views.n_views,
              (int)ctx->last_views.tiles, ctx->opt.z_near, ctx->opt.filter, ctx->opt.batch};
  a.tile_stride = tile_stride(ctx->last_views.tiles);
  a.queue = ctx->queue_on ? ctx->queue : nullptr;
  a.check = &ctx->ctrl->check_bits;
  return a;
}

// Forward pass of a view set.  With allow_sync the pair count is read back after the
// scan and the pair buffers grow to fit; without it (graph capture, tracking loop) an
// overflow only raises the device flag.
// upload = false: the device view table already holds vs (the tracking loop uploads
// it once, outside the captured iteration).  ro: the forward blend of a one-view set
// with targets forms the learned warm start's input instead of the images.
constexpr uint32_t kNpPending = 0xFFFFFFFFu;  // the pair-total word before the device writes it

struct ResidualOut {
  uint16_t* x;
  float* part;
  float lambda_d;
};
// tracking: a render of the tracking loop (the pair-overflow flag is kept from the
// call's start, so that an overflow in any iteration restarts the call).
int render_views(gs2d_ctx* ctx, const ViewSet& vs, hipStream_t s, bool allow_sync, bool upload = true,
                 const ResidualOut* ro = nullptr, bool blend = true, bool order = true, bool tracking = false) {
  const int64_t items = vs.items;
  const int nv = vs.n_views;
  bool capturing = false;
  if (stream_capturing(s, &capturing) != 0) return GS2D_ERR_INVALID_ARG;
  const bool grow_ok = !capturing;
  // partial rows: one per tile, or per wave of 256-surfel blocks of every view (the
  // parameter backward of views that share their surfels writes them side by side)
  int64_t rows = 0;
  for (int k = 0; k < nv; ++k) rows += (int64_t)kGroupRowsPerBlock * ((vs.v[k].n + 255) / 256);
  if (rows < vs.tiles) rows = vs.tiles;
  if ((items > ctx->n_cap || vs.pixels > ctx->hw_cap || vs.tiles > ctx->tile_cap || rows > ctx->part_cap ||
       ctx->p_cap == 0) &&
      !grow_ok)
    return GS2D_ERR_CAPACITY;
  GS2D_TRY(ensure_surfels(ctx, items > 0 ? items : 1));
  GS2D_TRY(ensure_pixels(ctx, vs.pixels));
  GS2D_TRY(ensure_tiles(ctx, vs.tiles));
  GS2D_TRY(ensure_parts(ctx, rows));
  if (ctx->p_cap == 0)
    GS2D_TRY(ensure_pairs(ctx, ctx->opt.pair_capacity > 0 ? ctx->opt.pair_capacity : 4 * (items > 0 ? items : 1)));
  if (upload) launch_upload_views(vs, ctx->views, s, ctx->ctrl);
  const int tw = ctx->opt.tile_w, th = ctx->opt.tile_h;
  int pbuf = 0;
  if (items == 0) {
    for (int k = 0; k < nv; ++k) {
      const ViewDesc& d = vs.v[k];
      const int64_t hw = (int64_t)d.cam.width * d.cam.height;
      if (d.rgb) launch_fill_f32(d.rgb, 0.f, 3 * hw, s);
      if (d.depth) launch_fill_f32(d.depth, 0.f, hw, s);
      if (d.normal) launch_fill_f32(d.normal, 0.f, 3 * hw, s);
      if (d.alpha) launch_fill_f32(d.alpha, 0.f, hw, s);
    }
    launch_fill_f32(ctx->t_final, 1.f, vs.pixels, s);
    launch_fill_u32(ctx->last, 0u, vs.pixels, s);
    launch_fill_u32(reinterpret_cast<uint32_t*>(ctx->ranges), 0u, 2 * vs.tiles, s);
    launch_fill_u32(reinterpret_cast<uint32_t*>(ctx->ctrl), 0u, 3, s);
    ctx->queue_on = false;
  } else {
    clear_fresh_hist(ctx, s);
    SortPlanes ws = sort_planes(ctx);
    uint32_t* part_pairs = ctx->parts;
    uint32_t* part_vis = ctx->parts + ctx->n_cap / kPartItems + 1;
    {
      ProfScope ps(ctx, kPre, s);
      launch_preprocess(ctx->views, nv, items, ctx->opt.z_near, ctx->opt.filter, tw, th, ctx->rec, ctx->rect,
                        ctx->count, ctx->dkey, ctx->saved_pose, part_pairs, part_vis, ctx->ctrl, s, !tracking);
    }
    // the pair total is read back (and the pair buffers grown) unless capturing
    const bool read_np = allow_sync && !capturing && !ctx->pair_fixed;
    uint32_t* const np_out = read_np ? ctx->np_dev : nullptr;
    // no render in flight writes the word (each one that does is waited for below)
    if (read_np) *ctx->np_host = kNpPending;
    const bool scanned = part_scan_needed(items);
    if (scanned) {
      ProfScope ps(ctx, kScan, s);
      launch_part_scan(part_pairs, part_vis, items, ctx->ctrl, np_out, s);
    }
    // pairs in item order; a tile sort of one pass (up to 2048 tiles) writes the tile
    // ranges itself
    const int tbits = tile_bits((int)vs.tiles);
    const bool fused_ranges = tbits <= kMaxDigitBits;
    auto duplicate = [&](uint32_t* np_dst) {
      ProfScope ps(ctx, kDup, s);
      launch_duplicate(ws, ctx->count, part_pairs, part_vis, scanned, ctx->rect, ctx->views, nv, items, ctx->p_cap,
                       tbits, ctx->pkey[0], ctx->pval[0], ctx->ctrl, ctx->ranges, (int)vs.tiles, ctx->dkey,
                       ctx->pdk[0], np_dst, s);
    };
    duplicate(np_out);
    if (read_np) {
      // the total is written early (by the scan, or by the duplication's first
      // workgroup): wait for the word itself rather than the whole stream, so that the
      // launches below are queued before the duplication ends
      uint32_t np32 = *ctx->np_host;
      while (np32 == kNpPending) {
        const hipError_t q = hipStreamQuery(s);
        np32 = *ctx->np_host;
        if (q == hipErrorNotReady || np32 != kNpPending) continue;
        GS2D_HIP(ctx, q);
        // the stream is idle and the word unwritten: read the device's copy
        GS2D_HIP(ctx, hipMemcpy(&np32, &ctx->ctrl->n_pairs, sizeof(uint32_t), hipMemcpyDeviceToHost));
        break;
      }
      const int64_t np = np32;
      ctx->host_ctrl->n_pairs = np32;  // for callers that size buffers from this render
      if (np > ctx->p_cap) {
        GS2D_HIP(ctx, hipStreamSynchronize(s));
        // grow and duplicate again (the first pass counted part of its pairs into plane 1)
        GS2D_TRY(ensure_pairs(ctx, np + np / 4));
        if (ctx->hist_fresh) {
          clear_fresh_hist(ctx, s);
        } else {
          launch_fill_u32(ctx->hist + ((size_t)ctx->hist_stride << kMaxDigitBits), 0u,
                          (int64_t)ctx->hist_stride << kMaxDigitBits, s);
        }
        ws = sort_planes(ctx);
        launch_fill_u32(&ctx->ctrl->overflow, 0u, 1, s);  // set by the first pass
        duplicate(nullptr);
      }
    }
    if (ctx->opt.keep_unsorted && ctx->pkey_keep) {
      launch_copy_u32(ctx->pkey[0], ctx->pkey_keep, ctx->p_cap, s);
      launch_copy_u32(ctx->pval[0], ctx->pval_keep, ctx->p_cap, s);
    }
    {
      ProfScope ps(ctx, kTileSort, s);
      pbuf = tile_sort(ws, ctx->pkey, ctx->pval, ctx->pdk, ctx->p_cap, tbits, ctx->ctrl, ctx->ranges, (int)vs.tiles,
                       s);
    }
    if (!fused_ranges) {
      ProfScope ps(ctx, kRanges, s);
      launch_ranges(ctx->pkey[pbuf], ctx->ctrl, ctx->p_cap, ctx->ranges, (int)vs.tiles, s);
    }
    if (order) {
      // each tile's items, ascending on entry, stably into depth order
      ProfScope ps(ctx, kDepthSort, s);
      launch_tile_order(ctx->ranges, (int)vs.tiles, ctx->pval[pbuf], ctx->pval[pbuf ^ 1], ctx->pdk[pbuf], ctx->dkey,
                        s);
    }
    // many more tiles than fit on the GPU at once: the blends pull tiles from a queue,
    // longest lists first
    ctx->queue_on = blend && vs.tiles > kQueueMinTiles;
    if (ctx->queue_on) launch_queue_order(ctx->ranges, (int)vs.tiles, ctx->queue, s);
    BlendArgs ba{ctx->ranges, ctx->pval[pbuf], ctx->rec, ctx->views, nv, (int)vs.tiles, ctx->opt.z_near,
                 ctx->opt.filter, ctx->opt.batch};
    ba.tile_stride = tile_stride(vs.tiles);
    ba.queue = ctx->queue_on ? ctx->queue : nullptr;
    ba.check = &ctx->ctrl->check_bits;
    if (ro) {
      ba.res_x = ro->x;
      ba.res_part = ro->part;
      ba.lambda_d = ro->lambda_d;
    }
    if (blend) {
      for (int k = 0; k < nv; ++k)
        if (vs.v[k].contrib) launch_fill_f32(vs.v[k].contrib, 0.f, vs.v[k].n, s);
      ProfScope ps(ctx, kBlendFwd, s);
      launch_blend_fwd(ba, tw, th, ctx->t_final, ctx->last, work_ptr(ctx, s), s);
    }
  }
  GS2D_HIP(ctx, hipGetLastError());
  ctx->generation += 1;
  ctx->last_views = vs;
  ctx->pair_buf = pbuf;
  ctx->have_forward = true;
  return GS2D_OK;
}

// Reverse mode of the last render for per-view gradients.
int backward_views(gs2d_ctx* ctx, const gs2d_view_grad* grads, int nv, int acc, hipStream_t s) {
  ViewSet vs = ctx->last_views;
  if (nv != vs.n_views) return GS2D_ERR_INVALID_ARG;
  bool full = false, hn = false, ho = false;
  for (int k = 0; k < nv; ++k) {
    ViewDesc& d = vs.v[k];
    d.g_rgb = const_cast<float*>(grads[k].d_rgb);
    d.g_depth = const_cast<float*>(grads[k].d_depth);
    d.g_normal = const_cast<float*>(grads[k].d_normal);
    d.g_alpha = grads[k].d_alpha;
    d.d_pose = grads[k].d_pose;
    full = full || grads[k].d_params != nullptr;
    hn = hn || grads[k].d_normal != nullptr;
    ho = ho || grads[k].d_alpha != nullptr;
  }
  if (vs.items == 0) {
    if (!acc)
      for (int k = 0; k < nv; ++k)
        if (grads[k].d_pose) launch_fill_f32(grads[k].d_pose, 0.f, 6, s);
    GS2D_HIP(ctx, hipGetLastError());
    return GS2D_OK;
  }
  bool capturing = false;
  if (stream_capturing(s, &capturing) != 0) return GS2D_ERR_INVALID_ARG;
  if (full) {
    if (vs.items > ctx->gacc_cap && capturing) return GS2D_ERR_CAPACITY;
    GS2D_TRY(ensure_gacc(ctx, vs.items));
  }
  launch_upload_views(vs, ctx->views, s);
  const BlendArgs ba = blend_args(ctx);
  if (ba.queue) launch_fill_u32(ba.queue + kQueueHeadBwd, 0u, 1, s);
  if (!full) {
    {
      ProfScope ps(ctx, kBlendBwd, s);
      launch_blend_bwd(ba, ctx->opt.tile_w, ctx->opt.tile_h, ctx->t_final, ctx->last, hn, ho, nullptr, ctx->part,
                       work_ptr(ctx, s), s);
    }
    ProfScope ps(ctx, kReduce, s);
    launch_reduce_pose_views(ctx->views, nv, ctx->part, acc, s);
  } else {
    launch_clear_rows(ctx->count, ctx->gacc, vs.items, s);
    {
      ProfScope ps(ctx, kBlendBwd, s);
      launch_blend_bwd(ba, ctx->opt.tile_w, ctx->opt.tile_h, ctx->t_final, ctx->last, hn, ho, ctx->gacc,
                       ctx->part, work_ptr(ctx, s), s);
    }
    // views that share the surfel set and d_params (the mapping window): one pass
    bool group = nv <= GS2D_MAX_VIEWS && vs.v[0].n > 0 && grads[0].d_params != nullptr;
    for (int k = 1; k < nv && group; ++k)
      group = vs.v[k].params == vs.v[0].params && vs.v[k].n == vs.v[0].n && grads[k].d_params == grads[0].d_params;
    if (group && nv > 1) {
      const ViewDesc& d0 = vs.v[0];
      const int rows = kGroupRowsPerBlock * ((d0.n + 255) / 256);
      const float* poses[GS2D_MAX_VIEWS];
      const uint32_t* counts[GS2D_MAX_VIEWS];
      const float* gaccs[GS2D_MAX_VIEWS];
      for (int k = 0; k < nv; ++k) {
        poses[k] = ctx->saved_pose + 12 * k;
        counts[k] = ctx->count + vs.v[k].item_base;
        gaccs[k] = ctx->gacc + (size_t)16 * vs.v[k].item_base;
      }
      {
        ProfScope ps(ctx, kPreBwd, s);
        if (launch_preprocess_bwd_group(d0.params, d0.n, nv, poses, counts, gaccs, grads[0].d_params, acc, ctx->part,
                                        s) != 0)
          return GS2D_ERR_INVALID_ARG;
      }
      float* d_poses[GS2D_MAX_VIEWS];
      for (int k = 0; k < nv; ++k) d_poses[k] = grads[k].d_pose;
      {
        ProfScope ps(ctx, kReduce, s);
        launch_reduce_pose_group(ctx->part, rows, nv, d_poses, acc, s);
      }
      GS2D_HIP(ctx, hipGetLastError());
      return GS2D_OK;
    }
    for (int k = 0; k < nv; ++k) {
      const ViewDesc& d = vs.v[k];
      if (d.n == 0) {
        if (!acc && grads[k].d_pose) launch_fill_f32(grads[k].d_pose, 0.f, 6, s);
        continue;
      }
      // views that share a d_params buffer add into it after the first
      int acc_k = acc;
      for (int j = 0; j < k && grads[k].d_params; ++j)
        if (grads[j].d_params == grads[k].d_params && vs.v[j].n > 0) acc_k = 1;
      {
        ProfScope ps(ctx, kPreBwd, s);
        launch_preprocess_bwd(d.params, d.n, ctx->saved_pose + 12 * k, ctx->count + d.item_base,
                              ctx->gacc + (size_t)16 * d.item_base,
                              grads[k].d_params, acc_k, ctx->part, s);
      }
      if (grads[k].d_pose) {
        ProfScope ps(ctx, kReduce, s);
        launch_reduce_pose(ctx->part, 0, (d.n + 255) / 256, grads[k].d_pose, acc, s);
      }
    }
  }
  GS2D_HIP(ctx, hipGetLastError());
  return GS2D_OK;
}

int set_device(gs2d_ctx* ctx) {
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != ctx->device) GS2D_HIP(ctx, hipSetDevice(ctx->device));
  return GS2D_OK;
}

// Everything a captured tracking iteration bakes into its kernel arguments.
struct TrackKeyHead {
  int32_t n_problems;
  float lambda_d;
  int32_t use_masks;
  float lr[6];
  float beta1, beta2, eps, weight_decay;
  int32_t patience, pad0;
  int64_t p_cap;
  int32_t tile_w, tile_h, batch, pad;
};

std::vector<unsigned char> make_key(gs2d_ctx* ctx, const gs2d_track_problem* p, int np, const gs2d_track_args* a) {
  TrackKeyHead h;
  std::memset(&h, 0, sizeof(h));
  h.n_problems = np;
  h.lambda_d = a->lambda_d;
  h.use_masks = a->use_masks;
  for (int i = 0; i < 6; ++i) h.lr[i] = a->lr[i];
  h.beta1 = a->beta1;
  h.beta2 = a->beta2;
  h.eps = a->eps;
  h.weight_decay = a->weight_decay;
  h.patience = a->diverge_patience;
  h.p_cap = ctx->p_cap;
  h.tile_w = ctx->opt.tile_w;
  h.tile_h = ctx->opt.tile_h;
  h.batch = ctx->opt.batch;
  std::vector<unsigned char> key(sizeof(h) + (size_t)np * sizeof(gs2d_track_problem));
  std::memcpy(key.data(), &h, sizeof(h));
  for (int k = 0; k < np; ++k) {
    gs2d_track_problem q;
    std::memset(&q, 0, sizeof(q));
    q.params = p[k].params;
    q.n = p[k].n;
    q.camera = p[k].camera;
    q.pose = p[k].pose;
    q.tgt_rgb = p[k].tgt_rgb;
    q.tgt_depth = p[k].tgt_depth;
    std::memcpy(key.data() + sizeof(h) + (size_t)k * sizeof(q), &q, sizeof(q));
  }
  return key;
}

// The view set of a tracking batch: images and gradients in the context's buffers.
int track_views(gs2d_ctx* ctx, const gs2d_track_problem* probs, int np, ViewSet& vs) {
  gs2d_view in[kMaxViews];
  for (int k = 0; k < np; ++k) {
    std::memset(&in[k], 0, sizeof(in[k]));
    in[k].params = probs[k].params;
    in[k].n = probs[k].n;
    in[k].camera = probs[k].camera;
    in[k].pose = probs[k].pose;
  }
  GS2D_TRY(build_views(ctx, in, np, vs));
  for (int k = 0; k < np; ++k) {
    ViewDesc& d = vs.v[k];
    const int64_t hw = (int64_t)d.cam.width * d.cam.height;
    float* img = ctx->limg + (size_t)8 * d.pix_base;
    float* grad = ctx->lgrad + (size_t)4 * d.pix_base;
    d.rgb = img;
    d.depth = img + 3 * hw;
    d.normal = img + 4 * hw;
    d.alpha = img + 7 * hw;
    d.g_rgb = grad;
    d.g_depth = grad + 3 * hw;
    d.tgt_rgb = probs[k].tgt_rgb;
    d.tgt_depth = probs[k].tgt_depth;
  }
  return GS2D_OK;
}

// One tracking iteration of every problem: batched render, tracking losses, batched
// pose-only backward, one AdamW + Exp step per problem.  No allocation and no
// synchronisation (capturable).
int track_iteration(gs2d_ctx* ctx, const ViewSet& vs, const gs2d_track_args* a, hipStream_t s) {
  AdamArgs adam;
  for (int k = 0; k < 6; ++k) adam.lr[k] = a->lr[k];
  adam.beta1 = a->beta1;
  adam.beta2 = a->beta2;
  adam.eps = a->eps;
  adam.weight_decay = a->weight_decay;
  adam.patience = a->diverge_patience;
  // sorts, then one walk per tile for the forward blend, the tracking loss and the
  // pose gradient; with no surfel there is no walk and the loss kernel forms the loss
  // with 256-pixel tiles each workgroup of the walk orders its own tile's list
  const bool walk_orders = ctx->opt.tile_w * ctx->opt.tile_h == 256;
  GS2D_TRY(render_views(ctx, vs, s, false, false, nullptr, false, !walk_orders, true));
  const int stride = loss_blocks(vs.max_hw);
  if (vs.items > 0) {
    BlendArgs ba = blend_args(ctx);
    ba.loss_part = ctx->part;
    ba.lambda_d = a->lambda_d;
    ba.use_masks = a->use_masks;
    if (walk_orders) {
      ba.order_ids = ctx->pval[ctx->pair_buf];
      ba.order_scratch = ctx->pval[ctx->pair_buf ^ 1];
      ba.dkey = ctx->dkey;
      ba.order_keys = ctx->pdk[ctx->pair_buf];
    }
    ProfScope ps(ctx, kBlendTrack, s);
    launch_blend_track(ba, ctx->opt.tile_w, ctx->opt.tile_h, work_ptr(ctx, s), s);
  } else {
    ProfScope ps(ctx, kLoss, s);
    launch_fill_f32(ctx->part, 0.f, 8 * vs.tiles, s);
    launch_tracking_loss(ctx->views, vs.n_views, vs.max_hw, a->lambda_d, a->use_masks, ctx->lpart, stride, s);
  }
  {
    ProfScope ps(ctx, kPose, s);
    launch_pose_step(ctx->views, vs.n_views, ctx->part, vs.items > 0, ctx->lpart, stride, adam, ctx->ctrl, s);
  }
  GS2D_HIP(ctx, hipGetLastError());
  return GS2D_OK;
}

int track_impl(gs2d_ctx* ctx, const gs2d_track_problem* probs, int np, const gs2d_track_args* a,
               hipStream_t caller_stream) {
  if (!ctx || !probs || !a || np < 1 || np > kMaxViews || a->n_iters < 0) return GS2D_ERR_INVALID_ARG;
  Fallbacks fb{};
  for (int k = 0; k < np; ++k) {
    if (!valid_camera(&probs[k].camera) || probs[k].n < 0 || (probs[k].n > 0 && !probs[k].params) ||
        !probs[k].pose || !probs[k].tgt_rgb || !probs[k].tgt_depth ||
        (probs[k].fallback_pose == nullptr) != (probs[k].fallback_loss == nullptr))
      return GS2D_ERR_INVALID_ARG;
    fb.pose[k] = probs[k].fallback_pose;
    fb.loss[k] = probs[k].fallback_loss;
  }
  for (int k = 0; k < 6; ++k)
    if (!std::isfinite(a->lr[k]) || a->lr[k] < 0.f) return GS2D_ERR_INVALID_ARG;
  if (!(a->beta1 >= 0.f && a->beta1 < 1.f && a->beta2 >= 0.f && a->beta2 < 1.f && a->eps > 0.f) ||
      !std::isfinite(a->lambda_d) || a->diverge_patience < 0)
    return GS2D_ERR_INVALID_ARG;
  GS2D_TRY(set_device(ctx));
  bool capturing = false;
  if (stream_capturing(caller_stream, &capturing) != 0 || capturing) return GS2D_ERR_INVALID_ARG;
  // The loop runs on the caller's stream, or, to be captured into a graph, on a
  // stream of the context (the legacy null stream cannot be captured).
  hipStream_t s = caller_stream;
  if (a->use_graph) {
    if (!ctx->graph_stream) GS2D_HIP(ctx, hipStreamCreateWithFlags(&ctx->graph_stream, hipStreamNonBlocking));
    GS2D_HIP(ctx, hipStreamSynchronize(caller_stream));
    s = ctx->graph_stream;
  }
  // pixel layout first (buffers for the loop's images and gradients)
  int64_t pixels = 0, max_hw = 0;
  for (int k = 0; k < np; ++k) {
    const int64_t hw = (int64_t)probs[k].camera.width * probs[k].camera.height;
    pixels += hw;
    max_hw = hw > max_hw ? hw : max_hw;
  }
  GS2D_TRY(ensure_pixels(ctx, pixels));
  if (ctx->img_cap < ctx->hw_cap || !ctx->limg || !ctx->lgrad) {
    GS2D_TRY(realloc_dev(ctx, &ctx->limg, 8 * ctx->hw_cap));
    GS2D_TRY(realloc_dev(ctx, &ctx->lgrad, 4 * ctx->hw_cap));
    ctx->img_cap = ctx->hw_cap;
  }
  GS2D_TRY(ensure_lpart(ctx, (int64_t)np * loss_blocks((int)max_hw)));
  ViewSet vs;
  GS2D_TRY(track_views(ctx, probs, np, vs));
  for (int k = 0; k < np; ++k)
    GS2D_HIP(ctx, hipMemcpyAsync(ctx->pose0 + 12 * k, probs[k].pose, 12 * sizeof(float), hipMemcpyDeviceToDevice,
                                 s));
  const bool was_fixed = ctx->pair_fixed;
  int result = GS2D_ERR_CAPACITY;
  for (int attempt = 0; attempt < 3; ++attempt) {
    if (attempt > 0)
      for (int k = 0; k < np; ++k)
        GS2D_HIP(ctx, hipMemcpyAsync(probs[k].pose, ctx->pose0 + 12 * k, 12 * sizeof(float),
                                     hipMemcpyDeviceToDevice, s));
    std::vector<unsigned char> key = make_key(ctx, probs, np, a);
    const bool reuse = a->use_graph && attempt == 0 && ctx->track_valid && ctx->track_key == key;
    if (!reuse) {
      // size the pair buffers on the start poses, with headroom for the moving poses
      ctx->pair_fixed = false;
      int r = render_views(ctx, vs, s, true);
      if (r == GS2D_OK) {
        const int64_t npairs = ctx->host_ctrl->n_pairs;
        r = ensure_pairs(ctx, (npairs + npairs / 2 + 1024) << attempt);
      }
      if (r == GS2D_OK) r = ensure_lpart(ctx, (int64_t)np * loss_blocks((int)max_hw));
      if (r != GS2D_OK) {
        ctx->pair_fixed = was_fixed;
        return r;
      }
    }
    ctx->pair_fixed = true;
    launch_upload_views(vs, ctx->views, s, ctx->ctrl);
    launch_track_init(ctx->views, np, ctx->ctrl, a->pose_history, a->loss_history, a->grad_history, a->n_iters,
                      s, &fb);
    int r = GS2D_OK;
    if (a->use_graph && a->n_iters > 0) {
      if (!reuse) {
        invalidate_graph(ctx);
        GS2D_HIP(ctx, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        const int ri = track_iteration(ctx, vs, a, s);
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(s, &graph);
        if (ri != GS2D_OK || ec != hipSuccess) {
          if (graph) (void)hipGraphDestroy(graph);
          ctx->pair_fixed = was_fixed;
          return ri != GS2D_OK ? ri : fail_hip(ctx, ec);
        }
        hipGraphExec_t exec = nullptr;
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
          (void)hipGraphDestroy(graph);
          ctx->pair_fixed = was_fixed;
          return fail_hip(ctx, ei);
        }
        ctx->track_graph = graph;
        ctx->track_exec = exec;
        ctx->track_key = make_key(ctx, probs, np, a);
        ctx->track_valid = true;
      }
      for (int it = 0; it < a->n_iters; ++it) {
        const hipError_t el = hipGraphLaunch(ctx->track_exec, s);
        if (el != hipSuccess) {
          ctx->pair_fixed = was_fixed;
          return fail_hip(ctx, el);
        }
      }
    } else {
      for (int it = 0; it < a->n_iters && r == GS2D_OK; ++it) r = track_iteration(ctx, vs, a, s);
    }
    if (r != GS2D_OK) {
      ctx->pair_fixed = was_fixed;
      return r;
    }
    GS2D_HIP(ctx, hipMemcpyAsync(ctx->host_ctrl, ctx->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
    GS2D_HIP(ctx, hipStreamSynchronize(s));
    if (!ctx->host_ctrl->overflow) {
      result = GS2D_OK;
      bool bad = ctx->host_ctrl->nonfinite != 0u;
      for (int k = 0; k < np; ++k) bad = bad || ctx->host_ctrl->status[k] == kTrackNonFinite;
      if (a->status) {
        int32_t st[kMaxViews];
        for (int k = 0; k < np; ++k)
          st[k] = ctx->host_ctrl->status[k] | (ctx->host_ctrl->fb_used[k] ? GS2D_TRACK_FELL_BACK : 0);
        GS2D_HIP(ctx, hipMemcpyAsync(a->status, st, (size_t)np * sizeof(int32_t), hipMemcpyHostToDevice, s));
        GS2D_HIP(ctx, hipStreamSynchronize(s));
      }
      if (bad) result = GS2D_ERR_NONFINITE;
      if (ctx->host_ctrl->check_bits) result = GS2D_ERR_DEVICE_CHECK;
      break;
    }
    invalidate_graph(ctx);
  }
  ctx->pair_fixed = was_fixed;
  ctx->have_forward = false;  // the loop's internal render state is not a public forward
  return result;
}

}  // namespace

namespace gs2d {

int render_residual(gs2d_ctx* ctx, const float* params, int64_t n, const gs2d_camera* camera, const float* pose,
                    const float* tgt_rgb, const float* tgt_depth, float lambda_d, uint16_t* x, float* part,
                    hipStream_t s) {
  if (!ctx || !valid_camera(camera) || n <= 0 || !params || !pose || !tgt_rgb || !tgt_depth || !x || !part)
    return GS2D_ERR_INVALID_ARG;
  if (camera->width % 8 || camera->height % 8) return GS2D_ERR_UNSUPPORTED;
  gs2d_view v{params, n, *camera, pose, nullptr, nullptr, nullptr, nullptr};
  ViewSet vs;
  GS2D_TRY(build_views(ctx, &v, 1, vs));
  vs.v[0].tgt_rgb = tgt_rgb;
  vs.v[0].tgt_depth = tgt_depth;
  GS2D_TRY(set_device(ctx));
  const ResidualOut ro{x, part, lambda_d};
  return render_views(ctx, vs, s, true, true, &ro);
}

}  // namespace gs2d

extern "C" {

GS2D_API int gs2d_default_options(gs2d_options* opt) {
  if (!opt) return GS2D_ERR_INVALID_ARG;
  std::memset(opt, 0, sizeof(*opt));
  opt->tile_w = 16;
  opt->tile_h = 16;
  opt->batch = 128;
  opt->filter = 1;
  opt->z_near = 0.2f;
  opt->pair_capacity = 0;
  opt->keep_unsorted = 0;
  opt->profile = 0;
  return GS2D_OK;
}

GS2D_API int gs2d_create(gs2d_ctx** out, int device, const gs2d_options* opt) {
  if (!out) return GS2D_ERR_INVALID_ARG;
  *out = nullptr;
  gs2d_options o;
  gs2d_default_options(&o);
  if (opt) o = *opt;
  if (!valid_tile(o.tile_w, o.tile_h) || !valid_batch(o.batch) || !(o.z_near > 0.f) ||
      !std::isfinite(o.z_near) || o.pair_capacity < 0 || (o.filter != 0 && o.filter != 1) ||
      o.profile < 0 || o.profile > 2)
    return GS2D_ERR_INVALID_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return GS2D_ERR_INVALID_ARG;
  }
  gs2d_ctx* ctx = new (std::nothrow) gs2d_ctx();
  if (!ctx) return GS2D_ERR_OOM;
  ctx->device = device;
  ctx->opt = o;
  int r = set_device(ctx);
  if (r == GS2D_OK) r = realloc_dev(ctx, &ctx->ctrl, 1);
  if (r == GS2D_OK) r = realloc_dev(ctx, &ctx->saved_pose, 12 * kMaxViews);
  if (r == GS2D_OK) r = realloc_dev(ctx, &ctx->pose0, 12 * kMaxViews);
  if (r == GS2D_OK) r = realloc_dev(ctx, &ctx->views, kMaxViews);
  if (r == GS2D_OK) {
    hipError_t e = hipHostMalloc((void**)&ctx->host_ctrl, sizeof(Ctrl), hipHostMallocDefault);
    if (e != hipSuccess) r = fail_hip(ctx, e);
  }
  if (r == GS2D_OK) {
    uint32_t* p = nullptr;
    hipError_t e = hipHostMalloc((void**)&p, 64, hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) {
      ctx->np_host = p;
      e = hipHostGetDevicePointer((void**)&ctx->np_dev, p, 0);
    }
    if (e != hipSuccess) r = fail_hip(ctx, e);
  }
  if (r == GS2D_OK && o.pair_capacity > 0) {
    r = ensure_pairs(ctx, o.pair_capacity);
    ctx->pair_fixed = true;
  }
  if (r == GS2D_OK) {
    hipError_t e = hipMemset(ctx->ctrl, 0, sizeof(Ctrl));
    if (e != hipSuccess) r = fail_hip(ctx, e);
  }
  if (r != GS2D_OK) {
    gs2d_destroy(ctx);
    return r;
  }
  *out = ctx;
  return GS2D_OK;
}

GS2D_API int gs2d_destroy(gs2d_ctx* ctx) {
  if (!ctx) return GS2D_OK;
  (void)set_device(ctx);
  invalidate_graph(ctx);
  void* bufs[] = {ctx->rec,       ctx->rect,       ctx->count,     ctx->dkey,      ctx->parts,     ctx->hist,
                  ctx->gacc,      ctx->pkey[0],    ctx->pkey[1],   ctx->pval[0],   ctx->pval[1],   ctx->pkey_keep,
                  ctx->pval_keep, ctx->ranges,     ctx->t_final,   ctx->last,      ctx->lgrad,     ctx->limg,
                  ctx->part,      ctx->lpart,      ctx->pose0,     ctx->saved_pose, ctx->views,    ctx->ctrl,
                  ctx->queue,     ctx->pdk[0],     ctx->pdk[1]};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  if (ctx->host_ctrl) (void)hipHostFree(ctx->host_ctrl);
  if (ctx->np_host) (void)hipHostFree(const_cast<uint32_t*>(ctx->np_host));
  if (ctx->graph_stream) (void)hipStreamDestroy(ctx->graph_stream);
  for (int i = 0; i < ctx->ev_cap; ++i) {
    (void)hipEventDestroy(ctx->ev[i].a);
    (void)hipEventDestroy(ctx->ev[i].b);
  }
  delete[] ctx->ev;
  delete ctx;
  return GS2D_OK;
}

GS2D_API int gs2d_render(gs2d_ctx* ctx, const float* params, int64_t n, const gs2d_camera* camera,
                         const float* pose, float* rgb, float* depth, float* normal, float* alpha,
                         uint32_t* generation, hipStream_t stream) {
  if (!ctx || !valid_camera(camera) || n < 0 || (n > 0 && !params) || !pose) return GS2D_ERR_INVALID_ARG;
  gs2d_view v{params, n, *camera, pose, rgb, depth, normal, alpha};
  return gs2d_render_batch(ctx, &v, 1, generation, stream);
}

GS2D_API int gs2d_render_batch(gs2d_ctx* ctx, const gs2d_view* views, int32_t n_views, uint32_t* generation,
                               hipStream_t stream) {
  if (!ctx) return GS2D_ERR_INVALID_ARG;
  ViewSet vs;
  GS2D_TRY(build_views(ctx, views, n_views, vs));
  GS2D_TRY(set_device(ctx));
  GS2D_TRY(render_views(ctx, vs, stream, true));
  if (generation) *generation = ctx->generation;
  return GS2D_OK;
}

GS2D_API int gs2d_render_backward(gs2d_ctx* ctx, const float* d_rgb, const float* d_depth,
                                  const float* d_normal, const float* d_alpha, float* d_params,
                                  float* d_pose, uint32_t generation, int32_t flags, hipStream_t stream) {
  if (!ctx) return GS2D_ERR_INVALID_ARG;
  gs2d_view_grad g{d_rgb, d_depth, d_normal, d_alpha, d_params, d_pose};
  return gs2d_render_backward_batch(ctx, &g, 1, generation, flags, stream);
}

GS2D_API int gs2d_render_backward_batch(gs2d_ctx* ctx, const gs2d_view_grad* grads, int32_t n_views,
                                        uint32_t generation, int32_t flags, hipStream_t stream) {
  if (!ctx || !grads || n_views < 1 || n_views > kMaxViews) return GS2D_ERR_INVALID_ARG;
  if ((flags & ~GS2D_ACCUMULATE) != 0) return GS2D_ERR_INVALID_ARG;
  if (!ctx->have_forward || generation != ctx->generation) return GS2D_ERR_STATE;
  if (n_views != ctx->last_views.n_views) return GS2D_ERR_INVALID_ARG;
  GS2D_TRY(set_device(ctx));
  return backward_views(ctx, grads, n_views, (flags & GS2D_ACCUMULATE) ? 1 : 0, stream);
}

GS2D_API int gs2d_tracking_loss(gs2d_ctx* ctx, const gs2d_camera* camera, const float* rgb, const float* depth,
                                const float* normal, const float* alpha, const float* tgt_rgb,
                                const float* tgt_depth, float lambda_d, int32_t use_masks, float* loss,
                                float* d_rgb, float* d_depth, hipStream_t stream) {
  if (!ctx || !valid_camera(camera) || !rgb || !depth || !tgt_rgb || !tgt_depth || !loss || !d_rgb || !d_depth)
    return GS2D_ERR_INVALID_ARG;
  if (use_masks && (!normal || !alpha)) return GS2D_ERR_INVALID_ARG;
  if (!std::isfinite(lambda_d)) return GS2D_ERR_INVALID_ARG;
  GS2D_TRY(set_device(ctx));
  const int hw = camera->width * camera->height;
  bool capturing = false;
  if (stream_capturing(stream, &capturing) != 0) return GS2D_ERR_INVALID_ARG;
  if (loss_blocks(hw) > ctx->lpart_cap && capturing) return GS2D_ERR_CAPACITY;
  GS2D_TRY(ensure_lpart(ctx, loss_blocks(hw)));
  ViewSet vs;
  vs.n_views = 1;
  ViewDesc& d = vs.v[0];
  std::memset(&d, 0, sizeof(d));
  d.cam = camf(*camera);
  d.rgb = const_cast<float*>(rgb);
  d.depth = const_cast<float*>(depth);
  d.normal = const_cast<float*>(normal);
  d.alpha = const_cast<float*>(alpha);
  d.tgt_rgb = tgt_rgb;
  d.tgt_depth = tgt_depth;
  d.g_rgb = d_rgb;
  d.g_depth = d_depth;
  launch_upload_views(vs, ctx->views, stream);
  {
    ProfScope ps(ctx, kLoss, stream);
    launch_tracking_loss(ctx->views, 1, hw, lambda_d, use_masks, ctx->lpart, loss_blocks(hw), stream);
  }
  {
    ProfScope ps(ctx, kReduce, stream);
    launch_reduce_loss(ctx->lpart, loss_blocks(hw), 1.0f / (float)hw, loss, stream);
  }
  GS2D_HIP(ctx, hipGetLastError());
  return GS2D_OK;
}

GS2D_API int gs2d_image_loss(gs2d_ctx* ctx, const gs2d_camera* camera, const float* rgb, const float* depth,
                             const float* normal, const float* alpha, const float* tgt_rgb, const float* tgt_depth,
                             const float* tgt_normal, const gs2d_loss_weights* w, float* loss, float* d_rgb,
                             float* d_depth, float* d_normal, hipStream_t stream) {
  if (!ctx || !valid_camera(camera) || !w || !loss || !depth || !tgt_depth) return GS2D_ERR_INVALID_ARG;
  if (!std::isfinite(w->w_rgb) || !std::isfinite(w->w_depth) || !std::isfinite(w->w_normal))
    return GS2D_ERR_INVALID_ARG;
  if ((w->w_rgb != 0.f || d_rgb) && (!rgb || !tgt_rgb)) return GS2D_ERR_INVALID_ARG;
  if ((w->w_normal != 0.f || d_normal) && (!normal || !tgt_normal)) return GS2D_ERR_INVALID_ARG;
  if ((w->normal_mask && !normal) || (w->opacity_mask && !alpha)) return GS2D_ERR_INVALID_ARG;
  GS2D_TRY(set_device(ctx));
  const int hw = camera->width * camera->height;
  bool capturing = false;
  if (stream_capturing(stream, &capturing) != 0) return GS2D_ERR_INVALID_ARG;
  if (loss_blocks(hw) > ctx->lpart_cap && capturing) return GS2D_ERR_CAPACITY;
  GS2D_TRY(ensure_lpart(ctx, loss_blocks(hw)));
  ViewSet vs;
  vs.n_views = 1;
  ViewDesc& d = vs.v[0];
  std::memset(&d, 0, sizeof(d));
  d.cam = camf(*camera);
  const bool colour = w->w_rgb != 0.f || d_rgb, normals = w->w_normal != 0.f || d_normal;
  d.rgb = colour ? const_cast<float*>(rgb) : nullptr;
  d.tgt_rgb = colour ? tgt_rgb : nullptr;
  d.depth = const_cast<float*>(depth);
  d.tgt_depth = tgt_depth;
  d.normal = const_cast<float*>(normal);
  d.tgt_normal = normals ? tgt_normal : nullptr;
  d.alpha = const_cast<float*>(alpha);
  d.g_rgb = d_rgb;
  d.g_depth = d_depth;
  d.g_normal = d_normal;
  launch_upload_views(vs, ctx->views, stream);
  {
    ProfScope ps(ctx, kLoss, stream);
    launch_image_loss(ctx->views, 1, hw, LossW{w->w_rgb, w->w_depth, w->w_normal, w->normal_mask, w->opacity_mask},
                      ctx->lpart, loss_blocks(hw), stream);
  }
  {
    ProfScope ps(ctx, kReduce, stream);
    launch_reduce_loss(ctx->lpart, loss_blocks(hw), 1.0f / (float)hw, loss, stream);
  }
  GS2D_HIP(ctx, hipGetLastError());
  return GS2D_OK;
}

GS2D_API int gs2d_image_loss_batch(gs2d_ctx* ctx, const gs2d_loss_view* views, int32_t n_views,
                                   const gs2d_loss_weights* w, float* losses, hipStream_t stream) {
  if (!ctx || !views || !w || !losses || n_views < 1 || n_views > GS2D_MAX_VIEWS) return GS2D_ERR_INVALID_ARG;
  if (!std::isfinite(w->w_rgb) || !std::isfinite(w->w_depth) || !std::isfinite(w->w_normal))
    return GS2D_ERR_INVALID_ARG;
  int max_hw = 0;
  for (int k = 0; k < n_views; ++k) {
    const gs2d_loss_view& v = views[k];
    if (!valid_camera(&v.camera) || !v.depth || !v.tgt_depth) return GS2D_ERR_INVALID_ARG;
    if ((w->w_rgb != 0.f || v.d_rgb) && (!v.rgb || !v.tgt_rgb)) return GS2D_ERR_INVALID_ARG;
    if ((w->w_normal != 0.f || v.d_normal) && (!v.normal || !v.tgt_normal)) return GS2D_ERR_INVALID_ARG;
    if ((w->normal_mask && !v.normal) || (w->opacity_mask && !v.alpha)) return GS2D_ERR_INVALID_ARG;
    const int hw = v.camera.width * v.camera.height;
    if (hw > max_hw) max_hw = hw;
  }
  GS2D_TRY(set_device(ctx));
  const int stride = loss_blocks(max_hw);
  bool capturing = false;
  if (stream_capturing(stream, &capturing) != 0) return GS2D_ERR_INVALID_ARG;
  if ((int64_t)n_views * stride > ctx->lpart_cap && capturing) return GS2D_ERR_CAPACITY;
  GS2D_TRY(ensure_lpart(ctx, (int64_t)n_views * stride));
  ViewSet vs;
  vs.n_views = n_views;
  for (int k = 0; k < n_views; ++k) {
    const gs2d_loss_view& v = views[k];
    ViewDesc& d = vs.v[k];
    std::memset(&d, 0, sizeof(d));
    d.cam = camf(v.camera);
    const bool colour = w->w_rgb != 0.f || v.d_rgb, normals = w->w_normal != 0.f || v.d_normal;
    d.rgb = colour ? const_cast<float*>(v.rgb) : nullptr;
    d.tgt_rgb = colour ? v.tgt_rgb : nullptr;
    d.depth = const_cast<float*>(v.depth);
    d.tgt_depth = v.tgt_depth;
    d.normal = const_cast<float*>(v.normal);
    d.tgt_normal = normals ? v.tgt_normal : nullptr;
    d.alpha = const_cast<float*>(v.alpha);
    d.g_rgb = v.d_rgb;
    d.g_depth = v.d_depth;
    d.g_normal = v.d_normal;
  }
  launch_upload_views(vs, ctx->views, stream);
  {
    ProfScope ps(ctx, kLoss, stream);
    launch_image_loss(ctx->views, n_views, max_hw,
                      LossW{w->w_rgb, w->w_depth, w->w_normal, w->normal_mask, w->opacity_mask}, ctx->lpart, stride,
                      stream);
  }
  {
    ProfScope ps(ctx, kReduce, stream);
    launch_reduce_loss_views(ctx->views, n_views, ctx->lpart, stride, losses, stream);
  }
  GS2D_HIP(ctx, hipGetLastError());
  return GS2D_OK;
}

GS2D_API int gs2d_tracking_error(gs2d_ctx* ctx, const gs2d_camera* camera, const float* depth, const float* normal,
                                 const float* alpha, const float* tgt_depth, float* error, hipStream_t stream) {
  if (!ctx || !valid_camera(camera) || !depth || !normal || !alpha || !tgt_depth || !error)
    return GS2D_ERR_INVALID_ARG;
  GS2D_TRY(set_device(ctx));
  const int hw = camera->width * camera->height;
  bool capturing = false;
  if (stream_capturing(stream, &capturing) != 0) return GS2D_ERR_INVALID_ARG;
  if (loss_blocks(hw) > ctx->lpart_cap && capturing) return GS2D_ERR_CAPACITY;
  GS2D_TRY(ensure_lpart(ctx, loss_blocks(hw)));
  ViewSet vs;
  vs.n_views = 1;
  ViewDesc& d = vs.v[0];
  std::memset(&d, 0, sizeof(d));
  d.cam = camf(*camera);
  d.depth = const_cast<float*>(depth);
  d.normal = const_cast<float*>(normal);
  d.alpha = const_cast<float*>(alpha);
  d.tgt_depth = tgt_depth;
  launch_upload_views(vs, ctx->views, stream);
  {
    ProfScope ps(ctx, kLoss, stream);
    launch_tracking_loss(ctx->views, 1, hw, 1.0f, 1, ctx->lpart, loss_blocks(hw), stream);
  }
  {
    ProfScope ps(ctx, kReduce, stream);
    launch_reduce_loss(ctx->lpart, loss_blocks(hw), 1.0f / (float)hw, error, stream);
  }
  GS2D_HIP(ctx, hipGetLastError());
  return GS2D_OK;
}

GS2D_API int gs2d_track(gs2d_ctx* ctx, const gs2d_track_args* a, hipStream_t caller_stream) {
  if (!ctx || !a) return GS2D_ERR_INVALID_ARG;
  gs2d_track_problem p{a->params,  a->n,         a->camera,        a->pose,
                       a->tgt_rgb, a->tgt_depth, a->fallback_pose, a->fallback_loss};
  return track_impl(ctx, &p, 1, a, caller_stream);
}

GS2D_API int gs2d_track_batch(gs2d_ctx* ctx, const gs2d_track_problem* problems, int32_t n_problems,
                              const gs2d_track_args* common, hipStream_t stream) {
  return track_impl(ctx, problems, n_problems, common, stream);
}

GS2D_API int gs2d_get_counts(gs2d_ctx* ctx, gs2d_counts* out, hipStream_t stream) {
  if (!ctx || !out) return GS2D_ERR_INVALID_ARG;
  GS2D_TRY(set_device(ctx));
  GS2D_HIP(ctx, hipMemcpyAsync(ctx->host_ctrl, ctx->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, stream));
  GS2D_HIP(ctx, hipStreamSynchronize(stream));
  const bool blank = ctx->last_views.items == 0;
  out->n_surfels = ctx->last_views.items;
  out->n_visible = blank ? 0 : ctx->host_ctrl->n_visible;
  out->n_pairs = blank ? 0 : ctx->host_ctrl->n_pairs;
  out->pair_capacity = ctx->p_cap;
  out->overflow = ctx->host_ctrl->overflow ? 1 : 0;
  out->n_tiles = (int32_t)ctx->last_views.tiles;
  out->nonfinite = ctx->host_ctrl->nonfinite ? 1 : 0;
  out->device_checks = (int32_t)ctx->host_ctrl->check_bits;
  return GS2D_OK;
}

GS2D_API int gs2d_debug_copy(gs2d_ctx* ctx, int32_t which, void* host_dst, size_t* bytes, hipStream_t stream) {
  if (!ctx || !bytes || (!host_dst && *bytes > 0)) return GS2D_ERR_INVALID_ARG;
  if (which == 10) {  // the tracking loop's last pose gradients (no forward state needed)
    const size_t need = sizeof(ctx->ctrl->last_grad);
    if (*bytes < need) {
      *bytes = need;
      return GS2D_ERR_INVALID_ARG;
    }
    GS2D_TRY(set_device(ctx));
    GS2D_HIP(ctx, hipStreamSynchronize(stream));
    GS2D_HIP(ctx, hipMemcpy(host_dst, ctx->ctrl->last_grad, need, hipMemcpyDeviceToHost));
    *bytes = need;
    return GS2D_OK;
  }
  if (!ctx->have_forward) return GS2D_ERR_STATE;
  gs2d_counts c;
  GS2D_TRY(gs2d_get_counts(ctx, &c, stream));
  const int64_t items = ctx->last_views.items, pixels = ctx->last_views.pixels;
  const void* src = nullptr;
  size_t need = 0;
  const int64_t np = c.n_pairs < ctx->p_cap ? c.n_pairs : ctx->p_cap;
  switch (which) {
    case 0: src = ctx->pkey[ctx->pair_buf]; need = (size_t)np * 4; break;
    case 1: src = ctx->pval[ctx->pair_buf]; need = (size_t)np * 4; break;
    case 2: src = ctx->ranges; need = (size_t)ctx->last_views.tiles * 8; break;
    case 3: src = ctx->dkey; need = (size_t)items * 4; break;
    case 4: src = ctx->rect; need = (size_t)items * 8; break;
    case 5: src = ctx->t_final; need = (size_t)pixels * 4; break;
    case 6: src = ctx->last; need = (size_t)pixels * 4; break;
    case 7: src = ctx->pkey_keep; need = (size_t)np * 4; break;
    case 8: src = ctx->pval_keep; need = (size_t)np * 4; break;
    default: return GS2D_ERR_INVALID_ARG;
  }
  if (!src) return GS2D_ERR_UNSUPPORTED;
  if (*bytes < need) {
    *bytes = need;
    return GS2D_ERR_INVALID_ARG;
  }
  if (need > 0) GS2D_HIP(ctx, hipMemcpy(host_dst, src, need, hipMemcpyDeviceToHost));
  *bytes = need;
  return GS2D_OK;
}

GS2D_API int gs2d_pose_exp(gs2d_ctx* ctx, const float* tau, const float* pose_in, float* pose_out,
                           hipStream_t stream) {
  if (!ctx || !tau || !pose_in || !pose_out) return GS2D_ERR_INVALID_ARG;
  GS2D_TRY(set_device(ctx));
  launch_pose_exp(tau, pose_in, pose_out, stream);
  GS2D_HIP(ctx, hipGetLastError());
  return GS2D_OK;
}

GS2D_API int gs2d_pose_tau_grad(gs2d_ctx* ctx, const float* tau, const float* d_pose, float* d_tau,
                                hipStream_t stream) {
  if (!ctx || !tau || !d_pose || !d_tau) return GS2D_ERR_INVALID_ARG;
  GS2D_TRY(set_device(ctx));
  launch_pose_tau_grad(tau, d_pose, d_tau, stream);
  GS2D_HIP(ctx, hipGetLastError());
  return GS2D_OK;
}

GS2D_API int gs2d_autotune(gs2d_ctx* ctx, const float* params, int64_t n, const gs2d_camera* camera,
                           const float* pose, int32_t reps, int32_t flags, gs2d_tuning* out, hipStream_t stream) {
  if (!ctx || !out || !valid_camera(camera) || n <= 0 || !params || !pose || reps < 1 || reps > 1000 ||
      (flags & ~GS2D_TUNE_FULL_BACKWARD) != 0 || n > INT32_MAX)
    return GS2D_ERR_INVALID_ARG;
  const bool full = (flags & GS2D_TUNE_FULL_BACKWARD) != 0;
  GS2D_TRY(set_device(ctx));
  bool capturing = false;
  if (stream_capturing(stream, &capturing) != 0 || capturing) return GS2D_ERR_INVALID_ARG;
  std::memset(out, 0, sizeof(*out));
  int ncls = 0;
  while ((1ll << ncls) < n) ++ncls;
  for (int i = 0; i < ctx->n_tune; ++i) {
    const auto& e = ctx->tune[i];
    if (e.w == camera->width && e.h == camera->height && e.ncls == ncls && e.flags == flags) {
      if (ctx->opt.tile_w != e.tw || ctx->opt.tile_h != e.th || ctx->opt.batch != e.batch) invalidate_graph(ctx);
      ctx->opt.tile_w = e.tw;
      ctx->opt.tile_h = e.th;
      ctx->opt.batch = e.batch;
      *out = gs2d_tuning{e.tw, e.th, e.batch, e.ms, 16, 1};
      return GS2D_OK;
    }
  }
  const int64_t HW = (int64_t)camera->width * camera->height;
  // images (also the tracking targets and image gradients of the timed passes), the
  // timed backward's pose gradient, and a copy of the pose for the timed pose steps
  float* img = nullptr;
  GS2D_HIP(ctx, hipMalloc((void**)&img, (size_t)(8 * HW + 24) * sizeof(float)));
  float* pose_copy = img + 8 * HW + 8;
  float* dpar = nullptr;  // the timed full backward's parameter gradient
  if (full) {
    const hipError_t e = hipMalloc((void**)&dpar, (size_t)15 * n * sizeof(float));
    if (e != hipSuccess) {
      (void)hipFree(img);
      return fail_hip(ctx, e);
    }
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const int tiles[4][2] = {{8, 8}, {16, 8}, {16, 16}, {32, 16}};
  const int batches[4] = {32, 64, 128, 256};
  const gs2d_options saved = ctx->opt;
  const bool saved_fixed = ctx->pair_fixed;
  ctx->opt.profile = 0;
  float best = 1e30f;
  int bt = saved.tile_w, bh = saved.tile_h, bb = saved.batch;
  int r = GS2D_OK;
  // pose-only mode: the timed work is the tracking iteration gs2d_track runs (sorts,
  // the fused walk and the pose step), on a copy of the pose with zero learning rates
  gs2d_track_args ta;
  std::memset(&ta, 0, sizeof(ta));
  ta.lambda_d = 1.0f;
  ta.use_masks = 1;
  ta.beta1 = 0.9f;
  ta.beta2 = 0.999f;
  ta.eps = 1e-8f;
  GS2D_HIP(ctx, hipMemcpyAsync(pose_copy, pose, 12 * sizeof(float), hipMemcpyDeviceToDevice, stream));
  gs2d_view v{params, n, *camera, full ? pose : pose_copy, img, img + 3 * HW, img + 4 * HW, img + 7 * HW};
  for (int ti = 0; ti < 4 && r == GS2D_OK; ++ti)
    for (int bi = 0; bi < 4 && r == GS2D_OK; ++bi) {
      ctx->opt.tile_w = tiles[ti][0];
      ctx->opt.tile_h = tiles[ti][1];
      ctx->opt.batch = batches[bi];
      ViewSet vs;
      r = build_views(ctx, &v, 1, vs);
      if (r != GS2D_OK) break;
      // the image buffer doubles as the image gradient of the timed backward, and as
      // the tracking target of the timed walk
      vs.v[0].g_rgb = img;
      vs.v[0].g_depth = img + 3 * HW;
      vs.v[0].d_pose = img + 8 * HW;
      vs.v[0].tgt_rgb = img;
      vs.v[0].tgt_depth = img + 3 * HW;
      ctx->pair_fixed = false;
      // one synchronising warm-up sizes the pair buffers for this tile shape (and,
      // for the full backward, its accumulator rows)
      r = render_views(ctx, vs, stream, true);
      if (r != GS2D_OK) break;
      gs2d_view_grad g{img, img + 3 * HW, nullptr, nullptr, dpar, img + 8 * HW};
      if (full) {
        r = backward_views(ctx, &g, 1, 0, stream);
      } else {
        // the tracking loop's headroom for moving poses, and its state
        const int64_t npairs = ctx->host_ctrl->n_pairs;
        r = ensure_pairs(ctx, npairs + npairs / 2 + 1024);
        if (r == GS2D_OK) {
          launch_upload_views(vs, ctx->views, stream);
          launch_track_init(ctx->views, 1, ctx->ctrl, nullptr, nullptr, nullptr, 0, stream);
          r = track_iteration(ctx, vs, &ta, stream);
        }
      }
      if (r != GS2D_OK) break;
      ctx->pair_fixed = true;
      (void)hipEventRecord(e0, stream);
      for (int k = 0; k < reps && r == GS2D_OK; ++k) {
        if (full) {
          r = render_views(ctx, vs, stream, false);
          if (r == GS2D_OK) r = backward_views(ctx, &g, 1, 0, stream);
        } else {
          r = track_iteration(ctx, vs, &ta, stream);
        }
      }
      (void)hipEventRecord(e1, stream);
      if (r != GS2D_OK) break;
      if (hipEventSynchronize(e1) != hipSuccess) {
        r = fail_hip(ctx, hipGetLastError());
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      ms /= (float)reps;
      (void)hipMemcpy(ctx->host_ctrl, ctx->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost);
      if (!ctx->host_ctrl->overflow && ms < best) {
        best = ms;
        bt = tiles[ti][0];
        bh = tiles[ti][1];
        bb = batches[bi];
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(stream);
  (void)hipFree(img);
  if (dpar) (void)hipFree(dpar);
  ctx->pair_fixed = saved_fixed;
  ctx->opt.profile = saved.profile;
  ctx->opt.tile_w = bt;
  ctx->opt.tile_h = bh;
  ctx->opt.batch = bb;
  ctx->have_forward = false;
  invalidate_graph(ctx);
  if (r != GS2D_OK) {
    ctx->opt = saved;
    return r;
  }
  if (ctx->n_tune < 32) ctx->tune[ctx->n_tune++] = {camera->width, camera->height, ncls, flags, bt, bh, bb, best};
  *out = gs2d_tuning{bt, bh, bb, best, 16, 0};
  return GS2D_OK;
}

GS2D_API const char* gs2d_profile_family(int i) {
  return (i >= 0 && i < kNumFamilies) ? kFamilyNames[i] : nullptr;
}

GS2D_API int gs2d_get_profile(gs2d_ctx* ctx, gs2d_profile* out, int32_t reset, hipStream_t stream) {
  if (!ctx || !out) return GS2D_ERR_INVALID_ARG;
  if (!ctx->opt.profile) return GS2D_ERR_UNSUPPORTED;
  GS2D_TRY(set_device(ctx));
  GS2D_HIP(ctx, hipStreamSynchronize(stream));
  if (ctx->graph_stream) GS2D_HIP(ctx, hipStreamSynchronize(ctx->graph_stream));
  for (int i = 0; i < ctx->ev_used; ++i) {
    float ms = 0.f;
    GS2D_HIP(ctx, hipEventSynchronize(ctx->ev[i].b));
    GS2D_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev[i].a, ctx->ev[i].b));
    ctx->prof_ms[ctx->ev[i].fam] += ms;
    ctx->prof_launches[ctx->ev[i].fam] += 1;
  }
  ctx->ev_used = 0;
  GS2D_HIP(ctx, hipMemcpy(ctx->host_ctrl, ctx->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost));
  std::memset(out, 0, sizeof(*out));
  for (int f = 0; f < kNumFamilies; ++f) {
    out->ms[f] = ctx->prof_ms[f];
    out->launches[f] = ctx->prof_launches[f];
  }
  out->fwd_evaluated = (int64_t)ctx->host_ctrl->work[0];
  out->fwd_covering = (int64_t)ctx->host_ctrl->work[1];
  out->bwd_evaluated = (int64_t)ctx->host_ctrl->work[2];
  out->bwd_covering = (int64_t)ctx->host_ctrl->work[3];
  if (reset) {
    for (int f = 0; f < kNumFamilies; ++f) {
      ctx->prof_ms[f] = 0.0;
      ctx->prof_launches[f] = 0;
    }
    launch_fill_u32(reinterpret_cast<uint32_t*>(ctx->ctrl->work), 0u, 8, stream);
    GS2D_HIP(ctx, hipStreamSynchronize(stream));
  }
  return GS2D_OK;
}

GS2D_API int gs2d_last_hip_error(gs2d_ctx* ctx) { return ctx ? ctx->last_hip_error : 0; }

GS2D_API int gs2d_build_info(void) {
#ifdef GS2D_DEVICE_CHECKS
  return GS2D_BUILD_DEVICE_CHECKS;
#else
  return 0;
#endif
}

GS2D_API const char* gs2d_error_string(int code) {
  switch (code) {
    case GS2D_OK: return "ok";
    case GS2D_ERR_INVALID_ARG: return "invalid argument";
    case GS2D_ERR_OOM: return "out of device memory";
    case GS2D_ERR_HIP: return "HIP runtime error (see gs2d_last_hip_error)";
    case GS2D_ERR_CAPACITY: return "tile-pair capacity exceeded; outputs of the last render are invalid";
    case GS2D_ERR_STATE: return "backward without a matching forward (generation mismatch)";
    case GS2D_ERR_UNSUPPORTED: return "unsupported configuration";
    case GS2D_ERR_NONFINITE: return "a surfel, pose, loss or gradient was not finite";
    case GS2D_ERR_DEVICE_CHECK: return "a device check failed (see gs2d_counts.device_checks)";
    default: return "unknown error code";
  }
}

}  // extern "C"
