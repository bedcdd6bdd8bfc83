// Per-tile front-to-back blending (forward) and its reverse mode (backward).
//
// Forward (Sec. "2D Gaussian Splatting", eq:alpha_blending): one workgroup per
// screen tile, one lane per pixel, each wave owning an 8x8 block of the tile.
// The tile's depth-ordered surfel list is staged through LDS in batches of
// records; every wave tests each record's footprint box against its own
// 8x8 block (a scalar, wave-uniform branch) before any lane evaluates it.  Per
// (pixel, surfel) pair the ray-splat intersection is solved in the surfel's uv
// frame from the centre-relative homography rows (see gs2d_internal.h), the
// Gaussian G = exp(-(u^2+v^2)/2) (or the low-pass filter term) gives
// alpha = min(0.99, o G), and colour, depth, normal and opacity are composited
// until the transmittance would fall below 1e-4.
//
// Backward (Sec. "Camera Pose Optimization"): the same lists walked back to front
// from each pixel's last composited entry.  The transmittance in front of each
// surfel is recovered by division, T_i = T_{i+1} / (1 - alpha_i), starting from
// the stored final transmittance, and the colour/depth/normal/opacity behind it
// by B_{i-1} = alpha_i v_i + (1 - alpha_i) B_i, so dL/dalpha_i =
// T_i sum_ch g_ch (v_i,ch - B_i,ch) needs no per-surfel blend state.  For every
// pair the gradient to the camera-frame surfel frame H_c (columns a = s_u t_uc,
// b = s_v t_vc, mu_c) is rank one, V (u, v, 1)^T, where V = K^T V' collects the
// image-space gradient of the pair (the paper's W^T dL/dT); the filter branch
// has (u, v) = (0, 0).  Hence the pose gradient of eq:derivatives is, pair by
// pair, rho += V and phi += X x V (+ n x g_n) with X = mu_c + u a + v b the
// intersection point.  Pose-only mode accumulates those six numbers in
// registers and reduces them once per workgroup (no per-surfel atomics); the
// full mode reduces the 16 per-surfel terms over each wave and adds them
// atomically.
#include <mutex>
#include <vector>

#include "tile_order.h"

namespace gs2d {
namespace {

struct Hit {
  float alpha, G, d, u, v, rq, dx, dy;
  bool b3d, clamped;
};

// One (pixel, surfel) evaluation; the forward and backward kernels call this same
// function so that every decision is reproduced bit for bit.  Returns 0 outside
// the footprint (rho > 9 or depth < z_near), 1 inside it but below the opacity
// threshold, 2 when the pair is composited.
__device__ __forceinline__ int evaluate(float px, float py, float ox, float oy, const float4 g1, const float4 g2,
                                        const float4 g3, float o, float z_near, int filter, Hit& h) {
  // (ox, oy): the integer box corner; g1.xy: the projected centre relative to it
  const float cxr = g1.x, cyr = g1.y, Dt = g1.z, k0 = g1.w;
  const float k1 = g2.x, P0 = g2.y, P1 = g2.z, Q0 = g2.w;
  const float Q1 = g3.x, m0 = g3.y, m1 = g3.z, m2 = g3.w;
  h.dx = (px - ox) - cxr;  // px - ox is exact (integers below 2^24)
  h.dy = (py - oy) - cyr;
  const float q2 = fmaf(-h.dy, k1, fmaf(-h.dx, k0, Dt));
  const float e0 = fmaf(Q1, h.dx, -(P1 * h.dy));
  const float e1 = fmaf(P0, h.dy, -(Q0 * h.dx));
  h.rq = __builtin_amdgcn_rcpf(q2);
  const float sc = m2 * h.rq;
  h.u = e0 * sc;
  h.v = e1 * sc;
  const float rho3 = fmaf(h.u, h.u, h.v * h.v);
  const float rho2 = filter ? kFilterScale * fmaf(h.dx, h.dx, h.dy * h.dy) : __builtin_inff();
  h.b3d = rho3 <= rho2;  // NaN (q2 = 0) selects the filter branch
  const float rho = h.b3d ? rho3 : rho2;
  h.d = h.b3d ? fmaf(m0, h.u, fmaf(m1, h.v, m2)) : m2;
  if (!(rho <= kRhoCutoff) || !(h.d >= z_near)) return 0;
  h.G = __builtin_amdgcn_exp2f(rho * -0.72134752044448170368f);  // exp(-rho / 2)
  const float og = o * h.G;
  h.clamped = og > kAlphaMax;
  h.alpha = h.clamped ? kAlphaMax : og;
  return h.alpha >= kAlphaMin ? 2 : 1;
}

__device__ __forceinline__ void add_work(unsigned long long* work, int lane, int a, int b) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    a += __shfl_xor(a, m, 64);
    b += __shfl_xor(b, m, 64);
  }
  if (lane == 0) {
    atomicAdd(work, (unsigned long long)a);
    atomicAdd(work + 1, (unsigned long long)b);
  }
}

__device__ __forceinline__ float uniformf(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

// Issue priority of a wave by the length of the list it walks: all tiles' workgroups
// are resident at once, and a long list is the critical path of the launch, so its
// waves take the SIMD before the short ones (which fill the remaining slots).
__device__ __forceinline__ void prioritise(int len) {
  __builtin_amdgcn_s_setprio(0);  // a persistent workgroup's next tile starts from 0
  if (len >= 192)
    __builtin_amdgcn_s_setprio(3);
  else if (len >= 128)
    __builtin_amdgcn_s_setprio(2);
  else if (len >= 64)
    __builtin_amdgcn_s_setprio(1);
}

// The tile of a workgroup of a direct (one workgroup per tile) launch: workgroups are
// dealt round-robin to the 8 XCDs, so each XCD gets every 8th tile of the stride:
// an even share of the dense and sparse image regions.
__device__ __forceinline__ int grid_tile(const BlendArgs& a) {
  return (int)(((uint64_t)blockIdx.x * (uint64_t)a.tile_stride) % (uint64_t)a.n_tiles);
}

// The next item of a persistent launch's queue for the whole workgroup (every thread
// calls it; the previous item's LDS is free once everyone has passed the first barrier).
__device__ __forceinline__ int next_queue_item(uint32_t* head) {
  __shared__ int s_item;
  __syncthreads();
  if (threadIdx.x == 0) s_item = (int)atomicAdd(head, 1u);
  __syncthreads();
  return s_item;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v = max(v, __shfl_xor(v, m, 64));
  return v;
}

// Per staged entry, what the waves' cull reads: the footprint box, the 3-sigma
// ellipse (centre relative to the box corner, support matrix Sxx, Sxy) and
// (Syy, low-pass disc centre relative to the box corner, free word; the backward
// keeps the entry's surfel id there).
constexpr int kLdsRec = 6;  // record float4 kept per staged entry ([6] feeds the cull only)

struct CullLds {
  float4* box;
  float4* ell;
  float4* ell2;
};
__device__ __forceinline__ void stage_cull(const CullLds& c, int j, int f, const float4& v) {
  if (f == 0) c.box[j] = v;
  if (f == 6) c.ell[j] = v;
  if (f == 5) c.ell2[j].x = v.w;
  if (f == 1) {
    c.ell2[j].y = v.x;
    c.ell2[j].z = v.y;
  }
}

// Entries [c0, c0 + 64) of a staged batch of nb: the mask of those whose list
// position is below `limit` and whose footprint may touch the wave's 8x8 block
// [bx0, bx0 + 7] x [by0, by0 + 7] (lane k tests entry c0 + k; the mask is
// wave-uniform).  The footprint (rho <= 9) is the union of the projected 3-sigma
// ellipse and, with the low-pass filter, the disc of radius 3/sqrt(2) about the
// projected centre.  An entry is dropped when its box misses the block, or when
// both the ellipse and the disc are separated from it: the ellipse along the
// direction from its centre to the block's centre, the disc by its distance.  Half
// a pixel of slack keeps the test conservative against the per-pixel FP32
// evaluation, so dropping changes no image.
__device__ __forceinline__ uint64_t overlap_mask(const CullLds& c, int c0, int nb, int lane, float bx0, float by0,
                                                 int filter, int pos0, int limit) {
  const int j = c0 + lane;
  bool hit = false;
  if (j < nb && pos0 + j < limit) {
    const float4 bb = c.box[j];
    hit = !(bb.y < bx0 || bb.x > bx0 + 7.0f || bb.w < by0 || bb.z > by0 + 7.0f);
    if (hit) {
      const float4 e = c.ell[j], e2 = c.ell2[j];
      // block corner relative to the box corner (integers: exact)
      const float rx = bx0 - bb.x, ry = by0 - bb.z;
      float nx = rx + 3.5f - e.x, ny = ry + 3.5f - e.y;
      const float n2 = nx * nx + ny * ny;
      bool sep_e = false;
      if (n2 > 0.0f) {
        const float inv = __builtin_amdgcn_rsqf(n2);
        nx *= inv;
        ny *= inv;
        const float ext = __builtin_amdgcn_sqrtf(fmaxf(nx * nx * e.z + 2.0f * nx * ny * e.w + ny * ny * e2.x, 0.0f));
        const float box_lo = nx * (rx + 3.5f) + ny * (ry + 3.5f) - 3.5f * (fabsf(nx) + fabsf(ny));
        sep_e = box_lo > nx * e.x + ny * e.y + ext + 0.5f;
      }
      bool sep_d = true;
      if (filter) {
        const float qx = fminf(fmaxf(e2.y, rx), rx + 7.0f), qy = fminf(fmaxf(e2.z, ry), ry + 7.0f);
        const float dx = e2.y - qx, dy = e2.z - qy;
        const float r = 2.12132034f + 0.5f;  // sqrt(9 / 2) + slack
        sep_d = dx * dx + dy * dy > r * r;
      }
      hit = !(sep_e && sep_d);
    }
  }
  return __ballot(hit);
}

// A staged record: box corner (x0, y0), rows g1..g3, (o, rgb), normal.
struct Rec {
  float ox, oy;
  float4 g1, g2, g3, c4, nv;
};
__device__ __forceinline__ Rec load_rec(const float4* srec, int j) {
  Rec r;
  const float4 bb = srec[j * kLdsRec];
  r.ox = bb.x;
  r.oy = bb.z;
  r.g1 = srec[j * kLdsRec + 1];
  r.g2 = srec[j * kLdsRec + 2];
  r.g3 = srec[j * kLdsRec + 3];
  r.c4 = srec[j * kLdsRec + 4];
  r.nv = srec[j * kLdsRec + 5];
  return r;
}

struct FwdPix {
  float T, cr, cg, cb, cd, n0, n1, n2, co;
  float dmed;  // median depth: of the last composited entry with incoming T > 1/2
  int lastj;
  bool done;
};

// Front-to-back compositing of one evaluated entry (list position pos); returns the
// entry's blending weight at this pixel (0 when it is not composited).
__device__ __forceinline__ float composite(FwdPix& s, int code, const Hit& h, const Rec& r, int pos) {
  if (s.done || code != 2) return 0.f;
  const float Tn = s.T * (1.0f - h.alpha);
  if (Tn < kTMin) {
    s.done = true;
    return 0.f;
  }
  const float w = h.alpha * s.T;
  s.cr = fmaf(w, r.c4.y, s.cr);
  s.cg = fmaf(w, r.c4.z, s.cg);
  s.cb = fmaf(w, r.c4.w, s.cb);
  s.cd = fmaf(w, h.d, s.cd);
  s.n0 = fmaf(w, r.nv.x, s.n0);
  s.n1 = fmaf(w, r.nv.y, s.n1);
  s.n2 = fmaf(w, r.nv.z, s.n2);
  s.co += w;
  if (s.T > 0.5f) s.dmed = h.d;
  s.T = Tn;
  s.lastj = pos + 1;
  return w;
}

// Sum over the wave, left in lane 63 (other lanes hold partial sums): an inclusive scan
// inside each 16-lane row by DPP row shifts, then the row totals carried forward by the
// row broadcasts of lanes 15 and 31.  Every lane of the wave must be active.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float x) {
  return x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xf, false));
}
__device__ __forceinline__ float wave_total_lane63(float x) {
  x = dpp_add<0x111, 0xf>(x);  // row_shr:1
  x = dpp_add<0x112, 0xf>(x);  // row_shr:2
  x = dpp_add<0x114, 0xf>(x);  // row_shr:4
  x = dpp_add<0x118, 0xf>(x);  // row_shr:8
  x = dpp_add<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
  x = dpp_add<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
  return x;
}

// eq:contribution: the wave's weights of one entry, added to the surfel's sum (one
// atomic per wave and entry, none where the wave has no weight for it).  Every lane of
// the wave calls it.
__device__ __forceinline__ void add_contribution(float* contrib, uint32_t surfel, float w, int lane) {
  if (__ballot(w != 0.f) == 0ull) return;
  const float ws = wave_total_lane63(w);
  // a global (not flat) atomic: flat ones also hold the LDS counter the walk waits on
  using gfloat = __attribute__((address_space(1))) float;
  if (lane == 63)
    __hip_atomic_fetch_add((gfloat*)(contrib + surfel), ws, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int TW, int TH, bool PROF>
__device__ __forceinline__ void blend_fwd_tile(const BlendArgs& a, const int tile, float* __restrict__ t_final,
                                               uint32_t* __restrict__ last_out,
                                               unsigned long long* __restrict__ work) {
  constexpr int NT = TW * TH, WX = TW / 8;
  extern __shared__ float4 srec[];
  const CullLds cull{srec + (size_t)a.batch * kLdsRec, srec + (size_t)a.batch * (kLdsRec + 1),
                     srec + (size_t)a.batch * (kLdsRec + 2)};
  uint32_t* const sids = reinterpret_cast<uint32_t*>(srec + (size_t)a.batch * (kLdsRec + 3));
  const ViewDesc& V = a.views[view_of_tile(a.views, a.n_views, tile)];
  const int lt = tile - V.tile_base;
  const int tx = lt % V.tiles_x, ty = lt / V.tiles_x;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int wx0 = tx * TW + (wave % WX) * 8, wy0 = ty * TH + (wave / WX) * 8;
  const int px = wx0 + (lane & 7), py = wy0 + (lane >> 3);
  const bool inside = px < V.cam.width && py < V.cam.height;
  const float fpx = (float)px, fpy = (float)py;
  const float bx0 = (float)wx0, by0 = (float)wy0;
  const uint2 rg = a.ranges[tile];
  GS2D_DCHECK(a.check, tile < a.n_tiles && rg.x <= rg.y, kCheckBlendRange);
  const int start = (int)rg.x, end = (int)rg.y;
  prioritise(end - start);
  FwdPix s{1.0f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0, !inside};
  // read once: the contribution atomics could alias the view table for the compiler
  float* const contrib = V.contrib;
  const uint32_t item_base = (uint32_t)V.item_base;
  int n_eval = 0, n_cov = 0;
  for (int b0 = start; b0 < end; b0 += a.batch) {
    if (__syncthreads_count(!s.done) == 0) break;
    const int nb = min(a.batch, end - b0);
    for (int k = t; k < nb * kRecF4; k += NT) {
      const int j = k / kRecF4, f = k - j * kRecF4;
      const uint32_t id = a.pval[b0 + j];
      const float4 v = a.rec[(size_t)id * kRecF4 + f];
      if (f < kLdsRec) srec[j * kLdsRec + f] = v;
      if (f == 0) sids[j] = id;
      stage_cull(cull, j, f, v);
    }
    __syncthreads();
    const int pos0 = b0 - start;
    for (int c0 = 0; c0 < nb; c0 += 64) {
      if (__ballot(!s.done) == 0ull) break;
      uint64_t m = overlap_mask(cull, c0, nb, lane, bx0, by0, a.filter, 0, nb);
      // two overlapping entries per step: their evaluations are independent, the
      // compositing stays in list order
      while (m != 0ull) {
        const int j1 = c0 + __builtin_ctzll(m);
        m &= m - 1ull;
        const bool two = m != 0ull;
        const int j2 = two ? c0 + __builtin_ctzll(m) : j1;
        if (two) m &= m - 1ull;
        float w1 = 0.f, w2 = 0.f;
        if (!s.done) {
          const Rec r1 = load_rec(srec, j1), r2 = load_rec(srec, j2);
          Hit h1, h2;
          const int k1 = evaluate(fpx, fpy, r1.ox, r1.oy, r1.g1, r1.g2, r1.g3, r1.c4.x, a.z_near, a.filter, h1);
          const int k2 = evaluate(fpx, fpy, r2.ox, r2.oy, r2.g1, r2.g2, r2.g3, r2.c4.x, a.z_near, a.filter, h2);
          if (PROF) {
            n_eval += 1;
            n_cov += k1 > 0;
          }
          w1 = composite(s, k1, h1, r1, pos0 + j1);
          if (two && !s.done) {
            if (PROF) {
              n_eval += 1;
              n_cov += k2 > 0;
            }
            w2 = composite(s, k2, h2, r2, pos0 + j2);
          }
        }
        if (contrib) {  // the view, and so this branch, is uniform over the workgroup
          add_contribution(contrib, sids[j1] - item_base, w1, lane);
          if (two) add_contribution(contrib, sids[j2] - item_base, w2, lane);
        }
        if (__ballot(!s.done) == 0ull) break;
      }
    }
  }
  if (PROF) add_work(work, lane, n_eval, n_cov);
  const int HW = V.cam.width * V.cam.height;
  const int p = py * V.cam.width + px;
  if (inside) {
    if (V.rgb) {
      V.rgb[p] = s.cr;
      V.rgb[HW + p] = s.cg;
      V.rgb[2 * HW + p] = s.cb;
    }
    if (V.depth) V.depth[p] = s.cd;
    if (V.normal) {
      V.normal[p] = s.n0;
      V.normal[HW + p] = s.n1;
      V.normal[2 * HW + p] = s.n2;
    }
    if (V.alpha) V.alpha[p] = s.co;
    if (V.depth_norm) V.depth_norm[p] = s.co > 0.f ? s.cd / s.co : 0.f;
    if (V.depth_median) V.depth_median[p] = s.dmed;
    t_final[V.pix_base + p] = s.T;
    last_out[V.pix_base + p] = (uint32_t)s.lastj;
  }
  if (a.res_x && wx0 < V.cam.width && wy0 < V.cam.height) {
    // the learned warm start's input and the unmasked tracking loss's terms of this
    // wave's 8 x 8 pixel block (the frame's sides are multiples of 8: every lane is
    // inside), each a sum over the wave's lanes in butterfly order
    float d[4];
    d[0] = s.cr - V.tgt_rgb[p];
    d[1] = s.cg - V.tgt_rgb[HW + p];
    d[2] = s.cb - V.tgt_rgb[2 * HW + p];
    d[3] = s.cd - V.tgt_depth[p];
    float l = fabsf(d[0]) + fabsf(d[1]) + fabsf(d[2]) + a.lambda_d * fabsf(d[3]);
    l = wave_sum(l);
#pragma unroll
    for (int c = 0; c < 4; ++c) d[c] = wave_sum(d[c]) * (1.0f / 64.0f);
    if (lane == 0) {
      const int blk = (wy0 >> 3) * (V.cam.width >> 3) + (wx0 >> 3);
      uint2 q;
      q.x = (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)d[0]) |
            ((uint32_t)__builtin_bit_cast(uint16_t, (__bf16)d[1]) << 16);
      q.y = (uint32_t)__builtin_bit_cast(uint16_t, (__bf16)d[2]) |
            ((uint32_t)__builtin_bit_cast(uint16_t, (__bf16)d[3]) << 16);
      *reinterpret_cast<uint2*>(a.res_x + (size_t)blk * 4) = q;
      a.res_part[blk] = l;
    }
  }
}

template <int TW, int TH, bool PROF>
__global__ __launch_bounds__(TW* TH) void blend_fwd_kernel(BlendArgs a, float* __restrict__ t_final,
                                                           uint32_t* __restrict__ last_out,
                                                           unsigned long long* __restrict__ work) {
  if (a.queue) {
    // persistent: tiles in the queue's order (longest lists first) until it is empty
    for (;;) {
      const int item = next_queue_item(a.queue + kQueueHeadFwd);
      if (item >= a.n_tiles) break;
      blend_fwd_tile<TW, TH, PROF>(a, (int)a.queue[kQueueOrder + item], t_final, last_out, work);
    }
  } else {
    blend_fwd_tile<TW, TH, PROF>(a, grid_tile(a), t_final, last_out, work);
  }
}

// Per-pixel state of the backward walk.
struct BwdPix {
  float T;                                   // transmittance in front of the next entry
  float gr, gg, gb, gd, gn0, gn1, gn2, go;   // image-space gradients of the pixel
  float Br, Bg, Bb, Bd, Bn0, Bn1, Bn2, Bo;   // blended values behind the next entry
  float pr0, pr1, pr2, pp0, pp1, pp2;        // pose gradient (pose-only mode)
};

// Reverse mode of one composited entry: updates the walk state and either the
// pose sums (pose-only) or the entry's 16 per-surfel terms acc.
template <bool POSE_ONLY, bool HAS_N, bool HAS_O>
__device__ __forceinline__ void reverse_entry(BwdPix& s, const Hit& h, const Rec& r, const CamF& cam, float xh,
                                              float yh, float ifx, float ify, float* acc) {
  const float4 c4 = r.c4, nv = r.nv;
  const float al = h.alpha;
  const float Tj = s.T * __builtin_amdgcn_rcpf(1.0f - al);
  const float w = al * Tj;
  float dLda = s.gr * (c4.y - s.Br) + s.gg * (c4.z - s.Bg) + s.gb * (c4.w - s.Bb) + s.gd * (h.d - s.Bd);
  if (HAS_N) dLda += s.gn0 * (nv.x - s.Bn0) + s.gn1 * (nv.y - s.Bn1) + s.gn2 * (nv.z - s.Bn2);
  if (HAS_O) dLda += s.go * (1.0f - s.Bo);
  dLda *= Tj;
  s.Br = fmaf(al, c4.y - s.Br, s.Br);
  s.Bg = fmaf(al, c4.z - s.Bg, s.Bg);
  s.Bb = fmaf(al, c4.w - s.Bb, s.Bb);
  s.Bd = fmaf(al, h.d - s.Bd, s.Bd);
  if (HAS_N) {
    s.Bn0 = fmaf(al, nv.x - s.Bn0, s.Bn0);
    s.Bn1 = fmaf(al, nv.y - s.Bn1, s.Bn1);
    s.Bn2 = fmaf(al, nv.z - s.Bn2, s.Bn2);
  }
  if (HAS_O) s.Bo = fmaf(al, 1.0f - s.Bo, s.Bo);
  s.T = Tj;
  const float g_d = w * s.gd;
  float g_o = 0.f, dLdG = 0.f;
  if (!h.clamped) {
    g_o = h.G * dLda;
    dLdG = c4.x * dLda;
  }
  const float dLdrho = -0.5f * h.G * dLdG;
  const float m0 = r.g3.y, m1 = r.g3.z, m2 = r.g3.w;
  float Vx, Vy, Vz, ue, ve, Xx, Xy, Xz;
  if (h.b3d) {
    // u = q0/q2, v = q1/q2; depth d = m . (u, v, 1)
    const float gu = fmaf(2.0f * h.u, dLdrho, m0 * g_d);
    const float gv = fmaf(2.0f * h.v, dLdrho, m1 * g_d);
    const float gq0 = gu * h.rq, gq1 = gv * h.rq;
    // h_u = P - dx m, h_v = Q - dy m (third entries -dx m2, -dy m2)
    const float hu0 = fmaf(-h.dx, m0, r.g2.y), hu1 = fmaf(-h.dx, m1, r.g2.z);
    const float hv0 = fmaf(-h.dy, m0, r.g2.w), hv1 = fmaf(-h.dy, m1, r.g3.x);
    const float V0 = hv0 * gq1 - hv1 * gq0;  // (h_v x g_q)_z
    const float V1 = gq0 * hu1 - gq1 * hu0;  // (g_q x h_u)_z
    Vx = cam.fx * V0;
    Vy = cam.fy * V1;
    Vz = g_d - xh * Vx - yh * Vy;
    ue = h.u;
    ve = h.v;
    Xx = h.d * xh;
    Xy = h.d * yh;
    Xz = h.d;
  } else {
    // rho = 2 |p - c|^2 with c = (M02, M12) / m2; depth = m2
    const float gcx = -2.0f * kFilterScale * h.dx * dLdrho;
    const float gcy = -2.0f * kFilterScale * h.dy * dLdrho;
    const float im2 = __builtin_amdgcn_rcpf(m2);
    Vx = cam.fx * gcx * im2;
    Vy = cam.fy * gcy * im2;
    const float xc = ((r.ox + r.g1.x) - cam.cx) * ifx, yc = ((r.oy + r.g1.y) - cam.cy) * ify;
    Vz = g_d - xc * Vx - yc * Vy;
    ue = 0.f;
    ve = 0.f;
    Xx = m2 * xc;
    Xy = m2 * yc;
    Xz = m2;
  }
  if (POSE_ONLY) {
    s.pr0 += Vx;
    s.pr1 += Vy;
    s.pr2 += Vz;
    s.pp0 += Xy * Vz - Xz * Vy;
    s.pp1 += Xz * Vx - Xx * Vz;
    s.pp2 += Xx * Vy - Xy * Vx;
    if (HAS_N) {
      const float w0 = w * s.gn0, w1 = w * s.gn1, w2 = w * s.gn2;
      s.pp0 += nv.y * w2 - nv.z * w1;
      s.pp1 += nv.z * w0 - nv.x * w2;
      s.pp2 += nv.x * w1 - nv.y * w0;
    }
  } else {
    acc[0] = Vx;
    acc[1] = Vy;
    acc[2] = Vz;
    acc[3] = ue * Vx;
    acc[4] = ue * Vy;
    acc[5] = ue * Vz;
    acc[6] = ve * Vx;
    acc[7] = ve * Vy;
    acc[8] = ve * Vz;
    acc[9] = w * s.gn0;
    acc[10] = w * s.gn1;
    acc[11] = w * s.gn2;
    acc[12] = w * s.gr;
    acc[13] = w * s.gg;
    acc[14] = w * s.gb;
    acc[15] = g_o;
  }
}

// The value of x at the lane that DPP control CTRL selects (all rows and banks on).
template <int CTRL>
__device__ __forceinline__ float dpp_get(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, false));
}

// Full mode: the wave's sums of one entry's 16 terms, added to the surfel's row.  A
// transposing butterfly halves the values per lane at each exchange, so that lane bits
// 5, 4, 3, 2 pick the term, then sums the four lanes of each quad.  Every exchange is a
// VALU lane move: v_permlane32_swap (lanes L, L^32), v_permlane16_swap (rows 0-1 and
// 2-3), DPP row_ror:8 (L^8 within a row), DPP row_half_mirror (a lane of the other
// half of its 8-lane group) and quad_perm.  Lanes 4k hold term k and add it into the
// entry's 16-float slot of the workgroup's LDS accumulator (one 16-lane ds_add, 16
// banks), which the block adds to the surfel's row in HBM once per batch.  Every lane
// of the wave must be active.
__device__ __forceinline__ void flush_entry(const float* acc, bool contrib, float* sacc, int j, int lane) {
  if (__ballot(contrib) == 0ull) return;
  float v16[16], v8[8], v4[4], v2[2];
#pragma unroll
  for (int k = 0; k < 16; ++k) v16[k] = contrib ? acc[k] : 0.f;
  // lanes 0-31 keep terms 0-7 and add lane L+32's; lanes 32-63 keep 8-15 and add L-32's
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v16[i]), __float_as_uint(v16[8 + i]), false,
                                                    false);
    v8[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  // rows 0 and 2 keep the lower four, rows 1 and 3 the upper four
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v8[i]), __float_as_uint(v8[4 + i]), false,
                                                    false);
    v4[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  const bool h8 = (lane & 8) != 0, h4 = (lane & 4) != 0;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const float mine = h8 ? v4[2 + i] : v4[i], give = h8 ? v4[i] : v4[2 + i];
    v2[i] = mine + dpp_get<0x128>(give);  // row_ror:8
  }
  float v = (h4 ? v2[1] : v2[0]) + dpp_get<0x141>(h4 ? v2[0] : v2[1]);  // row_half_mirror
  v += dpp_get<0x4E>(v);  // quad_perm [2, 3, 0, 1]
  v += dpp_get<0xB1>(v);  // quad_perm [1, 0, 3, 2]
  const int k = ((lane >> 5) & 1) * 8 + ((lane >> 4) & 1) * 4 + ((lane >> 3) & 1) * 2 + ((lane >> 2) & 1);
  using lfloat = __attribute__((address_space(3))) float;
  if ((lane & 3) == 0)
    __hip_atomic_fetch_add((lfloat*)(sacc + j * 16 + k), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <int TW, int TH, bool POSE_ONLY, bool HAS_N, bool HAS_O, bool PROF>
__device__ __forceinline__ void blend_bwd_tile(const BlendArgs& a, const int tile, const float* __restrict__ t_final,
                                               const uint32_t* __restrict__ last_in, float* __restrict__ gacc,
                                               float* __restrict__ part, unsigned long long* __restrict__ work) {
  constexpr int NT = TW * TH, WX = TW / 8, NW = NT / 64;
  extern __shared__ float4 srec[];
  const CullLds cull{srec + (size_t)a.batch * kLdsRec, srec + (size_t)a.batch * (kLdsRec + 1),
                     srec + (size_t)a.batch * (kLdsRec + 2)};
  // full mode: per staged entry the block's sums of its 16 terms (zero between
  // batches); the entry's surfel id rides in the unused last word of its cull data,
  // which keeps a 256-entry batch within a third of the CU's LDS
  float* sacc = reinterpret_cast<float*>(srec + (size_t)a.batch * (kLdsRec + 3));
  __shared__ int s_wmax[NW];
  __shared__ float s_red[NW][6];
  const ViewDesc& V = a.views[view_of_tile(a.views, a.n_views, tile)];
  const CamF cam = V.cam;
  const int lt = tile - V.tile_base;
  const int tx = lt % V.tiles_x, ty = lt / V.tiles_x;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  if (!POSE_ONLY)
    for (int k = t; k < a.batch * 16; k += NT) sacc[k] = 0.f;
  const int wx0 = tx * TW + (wave % WX) * 8, wy0 = ty * TH + (wave / WX) * 8;
  const int px = wx0 + (lane & 7), py = wy0 + (lane >> 3);
  const bool inside = px < cam.width && py < cam.height;
  const float fpx = (float)px, fpy = (float)py;
  const float bx0 = (float)wx0, by0 = (float)wy0;
  const int HW = cam.width * cam.height;
  const int p = py * cam.width + px;
  int my_last = 0;
  BwdPix s{};
  s.T = 1.0f;
  if (inside) {
    my_last = (int)last_in[V.pix_base + p];
    s.T = t_final[V.pix_base + p];
    if (V.g_rgb) {
      s.gr = V.g_rgb[p];
      s.gg = V.g_rgb[HW + p];
      s.gb = V.g_rgb[2 * HW + p];
    }
    if (V.g_depth) s.gd = V.g_depth[p];
    if (HAS_N && V.g_normal) {
      s.gn0 = V.g_normal[p];
      s.gn1 = V.g_normal[HW + p];
      s.gn2 = V.g_normal[2 * HW + p];
    }
    if (HAS_O && V.g_alpha) s.go = V.g_alpha[p];
  }
  const float xh = (fpx - cam.cx) / cam.fx, yh = (fpy - cam.cy) / cam.fy;
  const float ifx = 1.0f / cam.fx, ify = 1.0f / cam.fy;
  int n_eval = 0, n_cov = 0;
  const uint2 rg = a.ranges[tile];
  GS2D_DCHECK(a.check, tile < a.n_tiles && rg.x <= rg.y, kCheckBlendRange);
  const int start = (int)rg.x;

  const int wlast = wave_max(my_last);
  if (lane == 0) s_wmax[wave] = wlast;
  __syncthreads();
  int blast = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) blast = max(blast, s_wmax[w]);
  prioritise(blast);

  for (int bend = blast; bend > 0; bend -= a.batch) {
    const int bstart = max(0, bend - a.batch);
    const int nb = bend - bstart;
    __syncthreads();
    for (int k = t; k < nb * kRecF4; k += NT) {
      const int j = k / kRecF4, f = k - j * kRecF4;
      const uint32_t id = a.pval[start + bstart + j];
      const float4 v = a.rec[(size_t)id * kRecF4 + f];
      if (f < kLdsRec) srec[j * kLdsRec + f] = v;
      stage_cull(cull, j, f, v);
      if (f == 0) cull.ell2[j].w = __uint_as_float(id);
    }
    __syncthreads();
    // chunks of 64 from the back; within a chunk the overlapping entries below the
    // wave's last position, highest first (two per step in the pose-only mode)
    for (int c1 = nb; c1 > 0; c1 -= 64) {
      const int c0 = max(0, c1 - 64);
      uint64_t m = overlap_mask(cull, c0, c1, lane, bx0, by0, a.filter, bstart, wlast);
      while (m != 0ull) {
        const int b1 = 63 - __builtin_clzll(m);
        m &= ~(1ull << b1);
        // the full mode takes one entry per step: its 16 terms per entry then fit
        // 70-80 VGPRs (about 110-120 with two), which doubles the waves per SIMD
        const bool two = POSE_ONLY && m != 0ull;
        const int b2 = two ? 63 - __builtin_clzll(m) : b1;
        if (two) m &= ~(1ull << b2);
        const int j1 = c0 + b1, j2 = c0 + b2;
        const Rec r1 = load_rec(srec, j1), r2 = load_rec(srec, j2);
        const bool live1 = bstart + j1 < my_last, live2 = two && bstart + j2 < my_last;
        Hit h1, h2;
        const int k1 = evaluate(fpx, fpy, r1.ox, r1.oy, r1.g1, r1.g2, r1.g3, r1.c4.x, a.z_near, a.filter, h1);
        const int k2 = evaluate(fpx, fpy, r2.ox, r2.oy, r2.g1, r2.g2, r2.g3, r2.c4.x, a.z_near, a.filter, h2);
        if (PROF) {
          n_eval += (int)live1 + (int)live2;
          n_cov += (int)(live1 && k1 > 0) + (int)(live2 && k2 > 0);
        }
        float acc1[16], acc2[16];
        const bool c1on = live1 && k1 == 2, c2on = live2 && k2 == 2;
        if (c1on) reverse_entry<POSE_ONLY, HAS_N, HAS_O>(s, h1, r1, cam, xh, yh, ifx, ify, acc1);
        if (!POSE_ONLY) flush_entry(acc1, c1on, sacc, j1, lane);
        if (c2on) reverse_entry<POSE_ONLY, HAS_N, HAS_O>(s, h2, r2, cam, xh, yh, ifx, ify, acc2);
        if (!POSE_ONLY && two) flush_entry(acc2, c2on, sacc, j2, lane);
      }
    }
    if (!POSE_ONLY) {
      // the batch's sums into the surfel rows: one atomic per nonzero term, 16
      // consecutive floats (one 64 B row) per entry; the slots are left zero
      __syncthreads();
      using gfloat = __attribute__((address_space(1))) float;
      for (int k = t; k < nb * 16; k += NT) {
        const float v = sacc[k];
        if (v != 0.f) {
          const uint32_t id = __float_as_uint(cull.ell2[k >> 4].w);
          __hip_atomic_fetch_add((gfloat*)(gacc + (size_t)id * 16 + (k & 15)), v, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
          sacc[k] = 0.f;
        }
      }
    }
  }
  if (PROF) add_work(work + 2, lane, n_eval, n_cov);
  if (POSE_ONLY) {
    float v[6] = {s.pr0, s.pr1, s.pr2, s.pp0, s.pp1, s.pp2};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const float sum = wave_sum(v[k]);
      if (lane == 0) s_red[wave][k] = sum;
    }
    __syncthreads();
    if (t < 6) {  // slots 6 and 7 of the row belong to the forward's tracking loss
      float sum = 0.f;
#pragma unroll
      for (int w = 0; w < NW; ++w) sum += s_red[w][t];
      part[(size_t)tile * 8 + t] = sum;
    }
  }
}

template <int TW, int TH, bool POSE_ONLY, bool HAS_N, bool HAS_O, bool PROF>
__global__ __launch_bounds__(TW* TH) void blend_bwd_kernel(BlendArgs a, const float* __restrict__ t_final,
                                                           const uint32_t* __restrict__ last_in,
                                                           float* __restrict__ gacc, float* __restrict__ part,
                                                           unsigned long long* __restrict__ work) {
  if (a.queue) {
    for (;;) {
      const int item = next_queue_item(a.queue + kQueueHeadBwd);
      if (item >= a.n_tiles) break;
      blend_bwd_tile<TW, TH, POSE_ONLY, HAS_N, HAS_O, PROF>(a, (int)a.queue[kQueueOrder + item], t_final, last_in,
                                                            gacc, part, work);
    }
  } else {
    blend_bwd_tile<TW, TH, POSE_ONLY, HAS_N, HAS_O, PROF>(a, grid_tile(a), t_final, last_in, gacc, part, work);
  }
}

// float4 slots before the ordered list in the tracking walk's LDS: the staged records
// and their cull data, or the ordering's scratch, whichever is larger (both are used
// one after the other)
__host__ __device__ constexpr int track_stage_f4(int batch) {
  return batch * (kLdsRec + 3) > (kOrderScratchWords + 3) / 4 ? batch * (kLdsRec + 3) : (kOrderScratchWords + 3) / 4;
}

// Tracking: the forward blend, the tracking loss and the pose-only gradient in one
// walk of each tile's list.  For pixel loss gradients g_ch (known only once the
// pixel is composited) the pose gradient of eq:derivatives is
//   sum_ch g_ch A_ch + g_D G_D,  A_ch = sum_i v_i,ch (T_i J_i - w_i Q_<i),
//   Q_<i = sum_{j<i} J_j / (1 - alpha_j),  G_D = sum_i w_i K_i,
// where v_i are the colours and the depth of composited entry i, w_i = alpha_i T_i,
// J_i = dalpha_i/dtau (zero when the opacity clamp is active) and K_i = dd_i/dtau,
// both rank-one pair terms [V; X x V] as in the backward kernel.  This is the
// back-to-front recurrence dL/dalpha_i = T_i sum_ch g_ch (v_i,ch - B_i,ch) with the
// colour behind i, T_{i+1} B_i = sum_{j>i} w_j v_j, regrouped by j: every term is
// accumulated front to back, and no total is subtracted from a prefix.  A_D and G_D
// share one accumulator (both take g_D).  Entries are walked one per step: the
// walk's registers then allow five waves per SIMD, which hides more latency than
// two independent evaluations per step at four.
template <int TW, int TH, bool PROF>
__global__ __launch_bounds__(TW* TH) __attribute__((amdgpu_waves_per_eu(5))) void blend_track_kernel(BlendArgs a, unsigned long long* __restrict__ work) {
  constexpr int NT = TW * TH, WX = TW / 8, NW = NT / 64;
  extern __shared__ float4 srec[];
  const CullLds cull{srec + (size_t)a.batch * kLdsRec, srec + (size_t)a.batch * (kLdsRec + 1),
                     srec + (size_t)a.batch * (kLdsRec + 2)};
  __shared__ float s_red[NW][8];
  const int tile = (int)(((uint64_t)blockIdx.x * (uint64_t)a.tile_stride) % (uint64_t)a.n_tiles);
  const ViewDesc& V = a.views[view_of_tile(a.views, a.n_views, tile)];
  const CamF cam = V.cam;
  const int lt = tile - V.tile_base;
  const int tx = lt % V.tiles_x, ty = lt / V.tiles_x;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int wx0 = tx * TW + (wave % WX) * 8, wy0 = ty * TH + (wave / WX) * 8;
  const int px = wx0 + (lane & 7), py = wy0 + (lane >> 3);
  const bool inside = px < cam.width && py < cam.height;
  const float fpx = (float)px, fpy = (float)py;
  const float bx0 = (float)wx0, by0 = (float)wy0;
  const float xh = (fpx - cam.cx) / cam.fx, yh = (fpy - cam.cy) / cam.fy;
  const float ifx = 1.0f / cam.fx, ify = 1.0f / cam.fy;
  const uint2 rg = a.ranges[tile];
  GS2D_DCHECK(a.check, tile < a.n_tiles && rg.x <= rg.y, kCheckBlendRange);
  const int start = (int)rg.x, end = (int)rg.y;
  prioritise(end - start);
  // the tile's depth order, in LDS when the list fits (see tile_order.h); the staged
  // records are then gathered through the ordered ids in LDS
  uint32_t* const sid = reinterpret_cast<uint32_t*>(srec + track_stage_f4(a.batch));
  bool lds_list = false;
  if constexpr (NT == kBlockThreads) {
    if (a.order_ids)
      lds_list = order_list(a.order_ids, a.order_scratch, a.dkey, start, end - start,
                            order_lds(reinterpret_cast<uint32_t*>(srec), sid), false, a.order_keys);
  }
  FwdPix s{1.0f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0, !inside};
  float Q[6], Ar[6], Ag[6], Ab[6], AD[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) Q[k] = Ar[k] = Ag[k] = Ab[k] = AD[k] = 0.f;
  int n_eval = 0, n_cov = 0;
  // one composited entry: the forward blend and the gradient terms
  auto step = [&](int code, const Hit& h, const Rec& r) {
    if (s.done || code != 2) return;
    const float al = h.alpha;
    const float Tn = s.T * (1.0f - al);
    if (Tn < kTMin) {
      s.done = true;
      return;
    }
    const float T = s.T, w = al * T;
    const float m0 = r.g3.y, m1 = r.g3.z, m2 = r.g3.w;
    // V = dLdrho V_rho + g_d V_d for the pair (see the backward kernel); J and K are
    // [V; X x V] with X = d (xr, yr, 1) the intersection point: X x V = d (r x V)
    // with r = (xr, yr, 1) the ray through the pixel (or, in the filter branch, through
    // the projected centre).
    float Vr0, Vr1, Vd0, Vd1, Vd2, d;
    if (h.b3d) {
      const float hu0 = fmaf(-h.dx, m0, r.g2.y), hu1 = fmaf(-h.dx, m1, r.g2.z);
      const float hv0 = fmaf(-h.dy, m0, r.g2.w), hv1 = fmaf(-h.dy, m1, r.g3.x);
      // d(rho)/d(q-row entries) 2 (u, v) rq; d(depth) (m0, m1) rq, in which the pixel
      // offsets cancel: h_v0 m1 - h_v1 m0 = Q0 m1 - Q1 m0, m0 h_u1 - m1 h_u0 = m0 P1 - m1 P0
      const float r2 = 2.0f * h.rq;
      Vr0 = (cam.fx * r2) * fmaf(hv0, h.v, -(hv1 * h.u));
      Vr1 = (cam.fy * r2) * fmaf(hu1, h.u, -(hu0 * h.v));
      Vd0 = (cam.fx * h.rq) * fmaf(r.g2.w, m1, -(r.g3.x * m0));
      Vd1 = (cam.fy * h.rq) * fmaf(m0, r.g2.z, -(m1 * r.g2.y));
      d = h.d;
    } else {
      // filter branch: rho = 2 |p - c|^2 about the projected centre c, depth m2; its
      // intersection point is the centre's ray at depth m2
      const float im2 = __builtin_amdgcn_rcpf(m2);
      Vr0 = cam.fx * (-2.0f * kFilterScale * h.dx) * im2;
      Vr1 = cam.fy * (-2.0f * kFilterScale * h.dy) * im2;
      Vd0 = 0.f;
      Vd1 = 0.f;
      d = m2;
    }
    float xr = xh, yr = yh;
    if (!h.b3d) {
      xr = ((r.ox + r.g1.x) - cam.cx) * ifx;
      yr = ((r.oy + r.g1.y) - cam.cy) * ify;
    }
    const float axy = xr * yr, bx = fmaf(xr, xr, 1.0f), by = fmaf(yr, yr, 1.0f);
    const float Vr2 = fmaf(-xr, Vr0, -(yr * Vr1));
    Vd2 = fmaf(-xr, Vd0, fmaf(-yr, Vd1, 1.0f));
    // J = dalpha/dtau = dLdrho-direction times drho/dalpha = -G o / 2 (unclamped)
    const float jc = h.clamped ? 0.f : -0.5f * h.G * r.c4.x;
    const float jd = jc * d;
    float J[6], K[6];
    J[0] = jc * Vr0;
    J[1] = jc * Vr1;
    J[2] = jc * Vr2;
    // r x Vr with Vr2 = -xr Vr0 - yr Vr1: (-xr yr Vr0 - (1 + yr^2) Vr1, (1 + xr^2) Vr0 + xr yr Vr1, xr Vr1 - yr Vr0)
    J[3] = jd * fmaf(-axy, Vr0, -(by * Vr1));
    J[4] = jd * fmaf(bx, Vr0, axy * Vr1);
    J[5] = jd * fmaf(xr, Vr1, -(yr * Vr0));
    K[0] = Vd0;
    K[1] = Vd1;
    K[2] = Vd2;
    K[3] = d * fmaf(yr, Vd2, -Vd1);
    K[4] = d * fmaf(-xr, Vd2, Vd0);
    K[5] = d * fmaf(xr, Vd1, -(yr * Vd0));
    const float ia = __builtin_amdgcn_rcpf(1.0f - al);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const float U = fmaf(T, J[k], -w * Q[k]);
      Ar[k] = fmaf(r.c4.y, U, Ar[k]);
      Ag[k] = fmaf(r.c4.z, U, Ag[k]);
      Ab[k] = fmaf(r.c4.w, U, Ab[k]);
      AD[k] = fmaf(h.d, U, fmaf(w, K[k], AD[k]));
      Q[k] = fmaf(J[k], ia, Q[k]);
    }
    s.cr = fmaf(w, r.c4.y, s.cr);
    s.cg = fmaf(w, r.c4.z, s.cg);
    s.cb = fmaf(w, r.c4.w, s.cb);
    s.cd = fmaf(w, h.d, s.cd);
    // the normal mask needs only N . r: blended as the scalar n . r of each entry
    s.n0 = fmaf(w, fmaf(r.nv.x, xh, fmaf(r.nv.y, yh, r.nv.z)), s.n0);
    s.co += w;
    s.T = Tn;
  };
  for (int b0 = start; b0 < end; b0 += a.batch) {
    if (__syncthreads_count(!s.done) == 0) break;
    const int nb = min(a.batch, end - b0);
    for (int k = t; k < nb * kRecF4; k += NT) {
      const int j = k / kRecF4, f = k - j * kRecF4;
      const uint32_t id = lds_list ? sid[b0 - start + j] : a.pval[b0 + j];
      const float4 v = a.rec[(size_t)id * kRecF4 + f];
      if (f < kLdsRec) srec[j * kLdsRec + f] = v;
      stage_cull(cull, j, f, v);
    }
    __syncthreads();
    for (int c0 = 0; c0 < nb; c0 += 64) {
      if (__ballot(!s.done) == 0ull) break;
      uint64_t m = overlap_mask(cull, c0, nb, lane, bx0, by0, a.filter, 0, nb);
      while (m != 0ull) {
        const int j1 = c0 + __builtin_ctzll(m);
        m &= m - 1ull;
        if (!s.done) {
          const Rec r1 = load_rec(srec, j1);
          Hit h1;
          const int k1 = evaluate(fpx, fpy, r1.ox, r1.oy, r1.g1, r1.g2, r1.g3, r1.c4.x, a.z_near, a.filter, h1);
          if (PROF) {
            n_eval += 1;
            n_cov += k1 > 0;
          }
          step(k1, h1, r1);
        }
        if (__ballot(!s.done) == 0ull) break;
      }
    }
  }
  if (PROF) add_work(work, lane, n_eval, n_cov);
  // the pixel's tracking loss (eq:tracking_loss with the masks of eq:normal_mask
  // and eq:opacity_mask) and its gradient to the rendered colour and depth
  const int HW = cam.width * cam.height;
  const int p = py * cam.width + px;
  // (and the same sum without the masks, which the warm start's fallback compares)
  float l = 0.f, lu = 0.f, pg[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (inside) {
    bool mk = true;
    if (a.use_masks) {
      const float ndr = s.n0;
      mk = (ndr > 0.0f) && (s.co > kOpacityMask);
    }
    const float d0 = s.cr - V.tgt_rgb[p];
    const float d1 = s.cg - V.tgt_rgb[HW + p];
    const float d2 = s.cb - V.tgt_rgb[2 * HW + p];
    const float dd = s.cd - V.tgt_depth[p];
    lu = fabsf(d0) + fabsf(d1) + fabsf(d2) + a.lambda_d * fabsf(dd);
    if (mk) {
      const float inv = 1.0f / (float)HW;
      auto sgn = [](float v) { return v > 0.f ? 1.f : (v < 0.f ? -1.f : 0.f); };
      l = lu;
      const float gr = sgn(d0) * inv, gg = sgn(d1) * inv, gb = sgn(d2) * inv, gd = a.lambda_d * sgn(dd) * inv;
#pragma unroll
      for (int k = 0; k < 6; ++k) pg[k] = gr * Ar[k] + gg * Ag[k] + gb * Ab[k] + gd * AD[k];
    }
  }
  // tile sums: pose gradient in slots 0-5, loss in slot 6, unmasked loss in slot 7
  float v8[8] = {pg[0], pg[1], pg[2], pg[3], pg[4], pg[5], l, lu};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float sum = wave_sum(v8[k]);
    if (lane == 0) s_red[wave][k] = sum;
  }
  __syncthreads();
  if (t < 8) {
    float sum = 0.f;
#pragma unroll
    for (int w = 0; w < NW; ++w) sum += s_red[w][t];
    a.loss_part[(size_t)tile * 8 + t] = sum;
  }
}

// Workgroups of `kernel` that fit on the current device at once (occupancy per CU
// times the CUs), cached per kernel and LDS size: the grid of a persistent launch.
template <typename K>
int resident_workgroups(K kernel, int threads, size_t lds) {
  struct Entry {
    const void* k;
    size_t lds;
    int dev, n;
  };
  static std::mutex mu;
  static std::vector<Entry> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  std::lock_guard<std::mutex> lock(mu);
  for (const Entry& e : cache)
    if (e.k == reinterpret_cast<const void*>(kernel) && e.lds == lds && e.dev == dev) return e.n;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  const int n = per_cu * cus;
  cache.push_back(Entry{reinterpret_cast<const void*>(kernel), lds, dev, n});
  return n;
}

// Grid of a blend launch: one workgroup per tile, or with a queue the workgroups that
// fit at once (each then pulls tiles until the queue is empty; never more than the
// tiles).  A failed occupancy query falls back to one workgroup per tile.
template <typename K>
int blend_grid(const BlendArgs& a, K kernel, int threads, size_t lds) {
  if (!a.queue) return a.n_tiles;
  const int n = resident_workgroups(kernel, threads, lds);
  return n > 0 && n < a.n_tiles ? n : a.n_tiles;
}

template <int TW, int TH>
void fwd_shape(const BlendArgs& a, float* t_final, uint32_t* last, unsigned long long* work, hipStream_t s) {
  // staged records and their cull data, then the staged surfel ids
  const size_t lds = (size_t)a.batch * ((kLdsRec + 3) * sizeof(float4) + sizeof(uint32_t));
  if (work) {
    auto k = blend_fwd_kernel<TW, TH, true>;
    k<<<blend_grid(a, k, TW * TH, lds), TW * TH, lds, s>>>(a, t_final, last, work);
  } else {
    auto k = blend_fwd_kernel<TW, TH, false>;
    k<<<blend_grid(a, k, TW * TH, lds), TW * TH, lds, s>>>(a, t_final, last, work);
  }
}

template <int TW, int TH, bool PO, bool HN, bool HO>
void bwd_variant(const BlendArgs& a, const float* t_final, const uint32_t* last, float* gacc, float* part,
                 unsigned long long* work, hipStream_t s) {
  // staged records and their cull data, and in full mode the per-entry term sums
  const size_t lds = (size_t)a.batch * ((kLdsRec + 3) * sizeof(float4) + (PO ? 0 : 16 * sizeof(float)));
  if (work) {
    auto k = blend_bwd_kernel<TW, TH, PO, HN, HO, true>;
    k<<<blend_grid(a, k, TW * TH, lds), TW * TH, lds, s>>>(a, t_final, last, gacc, part, work);
  } else {
    auto k = blend_bwd_kernel<TW, TH, PO, HN, HO, false>;
    k<<<blend_grid(a, k, TW * TH, lds), TW * TH, lds, s>>>(a, t_final, last, gacc, part, work);
  }
}

template <int TW, int TH>
void bwd_shape(const BlendArgs& a, const float* t_final, const uint32_t* last, bool hn, bool ho, float* gacc,
               float* part, unsigned long long* work, hipStream_t s) {
  const bool po = gacc == nullptr;
#define GS2D_BWD(PO, HN, HO) bwd_variant<TW, TH, PO, HN, HO>(a, t_final, last, gacc, part, work, s)
  if (po) {
    if (hn && ho) GS2D_BWD(true, true, true);
    else if (hn) GS2D_BWD(true, true, false);
    else if (ho) GS2D_BWD(true, false, true);
    else GS2D_BWD(true, false, false);
  } else {
    if (hn && ho) GS2D_BWD(false, true, true);
    else if (hn) GS2D_BWD(false, true, false);
    else if (ho) GS2D_BWD(false, false, true);
    else GS2D_BWD(false, false, false);
  }
#undef GS2D_BWD
}

}  // namespace

void launch_blend_fwd(const BlendArgs& a, int tile_w, int tile_h, float* t_final, uint32_t* last,
                      unsigned long long* work, hipStream_t s) {
  if (tile_w == 8 && tile_h == 8) fwd_shape<8, 8>(a, t_final, last, work, s);
  else if (tile_w == 16 && tile_h == 8) fwd_shape<16, 8>(a, t_final, last, work, s);
  else if (tile_w == 32 && tile_h == 16) fwd_shape<32, 16>(a, t_final, last, work, s);
  else fwd_shape<16, 16>(a, t_final, last, work, s);
}

template <int TW, int TH>
void track_shape(const BlendArgs& a, unsigned long long* work, hipStream_t s) {
  // staging (or, before it, the ordering's scratch), then the ordered list
  const size_t lds = (size_t)track_stage_f4(a.batch) * sizeof(float4) + kOrderMax * sizeof(uint32_t);
  if (work)
    blend_track_kernel<TW, TH, true><<<a.n_tiles, TW * TH, lds, s>>>(a, work);
  else
    blend_track_kernel<TW, TH, false><<<a.n_tiles, TW * TH, lds, s>>>(a, work);
}

void launch_blend_track(const BlendArgs& a, int tile_w, int tile_h, unsigned long long* work, hipStream_t s) {
  if (tile_w == 8 && tile_h == 8) track_shape<8, 8>(a, work, s);
  else if (tile_w == 16 && tile_h == 8) track_shape<16, 8>(a, work, s);
  else if (tile_w == 32 && tile_h == 16) track_shape<32, 16>(a, work, s);
  else track_shape<16, 16>(a, work, s);
}

void launch_blend_bwd(const BlendArgs& a, int tile_w, int tile_h, const float* t_final, const uint32_t* last,
                      bool has_normal, bool has_alpha, float* gacc, float* part, unsigned long long* work,
                      hipStream_t s) {
  if (tile_w == 8 && tile_h == 8) bwd_shape<8, 8>(a, t_final, last, has_normal, has_alpha, gacc, part, work, s);
  else if (tile_w == 16 && tile_h == 8)
    bwd_shape<16, 8>(a, t_final, last, has_normal, has_alpha, gacc, part, work, s);
  else if (tile_w == 32 && tile_h == 16)
    bwd_shape<32, 16>(a, t_final, last, has_normal, has_alpha, gacc, part, work, s);
  else
    bwd_shape<16, 16>(a, t_final, last, has_normal, has_alpha, gacc, part, work, s);
}

}  // namespace gs2d
