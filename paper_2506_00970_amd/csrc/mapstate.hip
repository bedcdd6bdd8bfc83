// Map bookkeeping kernels (include/gs2d_map.h): covisibility and the keyframe test
// (Sec. "Tracking and Keyframe Selection"), pruning and stable compaction, the map
// state update (Sec. "Mapping", eq:map) and map correction (Sec. "Map Correction").
//
// All are HBM-bound streams over the splats: one thread per splat for the state update
// and the correction, four for the covisibility counts, the prune mask and the Adam
// step over the parameters, and for the compaction 1024 splats per workgroup in four
// wave-contiguous rounds.  Decisions on distances and scores are taken in
// double, as in their definitions.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/gs2d_map.h"

namespace gs2d {
namespace map {
namespace {

constexpr int kThreads = 256;
constexpr int kPer = 4;                      // splats per thread in the compaction
constexpr int kBlockItems = kThreads * kPer;  // 1024 splats per compaction workgroup

inline int blocks_for(int64_t n, int per) {
  const int64_t b = (n + per - 1) / per;
  return b > 0 ? (int)b : 1;
}

__device__ inline uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += (uint32_t)__shfl_xor((int)v, m, 64);
  return v;
}

// Exclusive scan over the 256 threads of a block; *total = the block's sum.
__device__ inline uint32_t block_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[wave] = x;
  __syncthreads();
  uint32_t below = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) {
    below += w < wave ? sh[w] : 0u;
    all += sh[w];
  }
  __syncthreads();
  if (total) *total = all;
  return below + x - v;
}

constexpr int kCovisMaxBlocks = 1024;

inline int covis_blocks(int64_t n) {
  const int64_t b = (n / 4 + kThreads - 1) / kThreads;
  return b < 1 ? 1 : (b > kCovisMaxBlocks ? kCovisMaxBlocks : (int)b);
}

// |G_A & G_B| and |G_A | G_B|, stage 1: each workgroup counts a grid-strided share
// (four splats per thread and step, 16-byte loads when both arrays allow them) and
// writes its two counts to work[2 b], work[2 b + 1].
template <bool VEC>
__global__ __launch_bounds__(kThreads) void covis_partial_kernel(const float* __restrict__ a,
                                                                 const float* __restrict__ b, int64_t n, float thr,
                                                                 uint32_t* __restrict__ work) {
  __shared__ uint32_t sh[2][kThreads / 64];
  uint32_t ci = 0, cu = 0;
  const int64_t n4 = n / 4, stride = (int64_t)gridDim.x * kThreads;
  for (int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x; g < n4; g += stride) {
    float va[4], vb[4];
    if (VEC) {
      const float4 x = reinterpret_cast<const float4*>(a)[g], y = reinterpret_cast<const float4*>(b)[g];
      va[0] = x.x, va[1] = x.y, va[2] = x.z, va[3] = x.w;
      vb[0] = y.x, vb[1] = y.y, vb[2] = y.z, vb[3] = y.w;
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) va[q] = a[4 * g + q], vb[q] = b[4 * g + q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bool pa = va[q] > thr, pb = vb[q] > thr;
      ci += (pa && pb) ? 1u : 0u;
      cu += (pa || pb) ? 1u : 0u;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x < (int)(n - 4 * n4)) {  // the last n mod 4 splats
    const int64_t k = 4 * n4 + threadIdx.x;
    const bool pa = a[k] > thr, pb = b[k] > thr;
    ci += (pa && pb) ? 1u : 0u;
    cu += (pa || pb) ? 1u : 0u;
  }
  ci = wave_sum_u32(ci);
  cu = wave_sum_u32(cu);
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = ci;
    sh[1][threadIdx.x >> 6] = cu;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    uint32_t t = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) t += sh[threadIdx.x][w];
    work[2 * blockIdx.x + threadIdx.x] = t;
  }
}

// Stage 2 (one workgroup): counts = the sums of the nb partial pairs.
__global__ __launch_bounds__(kThreads) void covis_final_kernel(const uint32_t* __restrict__ work, int nb,
                                                               uint32_t* __restrict__ counts) {
  __shared__ uint32_t sh[2][kThreads / 64];
  uint32_t ci = 0, cu = 0;
  for (int e = threadIdx.x; e < nb; e += kThreads) {
    ci += work[2 * e];
    cu += work[2 * e + 1];
  }
  ci = wave_sum_u32(ci);
  cu = wave_sum_u32(cu);
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = ci;
    sh[1][threadIdx.x >> 6] = cu;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    uint32_t t = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) t += sh[threadIdx.x][w];
    counts[threadIdx.x] = t;
  }
}

__global__ void keyframe_kernel(const uint32_t* __restrict__ counts, const float* __restrict__ pc,
                                const float* __restrict__ pk, double c_k, double d_k, int32_t* __restrict__ out) {
  if (threadIdx.x != 0) return;
  const double score = counts[1] ? (double)counts[0] / (double)counts[1] : 0.0;
  const double dx = (double)pc[3] - (double)pk[3], dy = (double)pc[7] - (double)pk[7],
               dz = (double)pc[11] - (double)pk[11];
  const double dist = sqrt(dx * dx + dy * dy + dz * dz);
  *out = (score < c_k || dist > d_k) ? 1 : 0;
}

// Four splats per thread: 16-byte contribution and frame loads and one 4-byte mask
// store when the three arrays allow them.
template <bool VEC>
__global__ __launch_bounds__(kThreads) void prune_kernel(const float* __restrict__ contrib,
                                                         const int32_t* __restrict__ closest, int32_t frame,
                                                         float thr, int64_t n, uint8_t* __restrict__ remove) {
  const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x, k0 = 4 * g;
  if (k0 >= n) return;
  if (VEC && k0 + 4 <= n) {
    const float4 c = reinterpret_cast<const float4*>(contrib)[g];
    const int4 f = reinterpret_cast<const int4*>(closest)[g];
    const uint32_t m = (f.x == frame && c.x < thr ? 1u : 0u) | (f.y == frame && c.y < thr ? 1u << 8 : 0u) |
                       (f.z == frame && c.z < thr ? 1u << 16 : 0u) | (f.w == frame && c.w < thr ? 1u << 24 : 0u);
    reinterpret_cast<uint32_t*>(remove)[g] = m;
    return;
  }
  for (int64_t k = k0; k < n && k < k0 + 4; ++k) remove[k] = (closest[k] == frame && contrib[k] < thr) ? 1 : 0;
}

// Compaction, pass 1: the kept count of each block of 1024 splats (item q * 256 + t of
// the block in round q, so every load is contiguous over the wave).
__device__ inline bool kept(const uint8_t* __restrict__ remove, int64_t k, int64_t n) {
  return k < n && !(remove && remove[k]);
}

__global__ __launch_bounds__(kThreads) void compact_count_kernel(const uint8_t* __restrict__ remove, int64_t n,
                                                                 uint32_t* __restrict__ block_counts) {
  __shared__ uint32_t sh[kThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kBlockItems + threadIdx.x;
  uint32_t c = 0;
#pragma unroll
  for (int q = 0; q < kPer; ++q) c += (uint32_t)__popcll(__ballot(kept(remove, base + q * kThreads, n)));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) t += sh[w];
    block_counts[blockIdx.x] = t;
  }
}

// Pass 2 (one workgroup): exclusive scan of the block counts in place; the total.
__global__ __launch_bounds__(kThreads) void compact_scan_kernel(uint32_t* __restrict__ block_counts, int nb,
                                                                uint32_t* __restrict__ n_out) {
  __shared__ uint32_t sh[kThreads / 64];
  uint32_t carry = 0;
  for (int c0 = 0; c0 < nb; c0 += kThreads * kPer) {
    uint32_t v[kPer], s = 0;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = c0 + (int)threadIdx.x * kPer + q;
      v[q] = e < nb ? block_counts[e] : 0u;
      s += v[q];
    }
    uint32_t total;
    uint32_t run = carry + block_scan(s, sh, &total);
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = c0 + (int)threadIdx.x * kPer + q;
      if (e < nb) block_counts[e] = run;
      run += v[q];
    }
    carry += total;
  }
  if (threadIdx.x == 0) *n_out = carry;
}

// Pass 3: each kept splat's columns to its slot: the block's base, the kept splats of
// earlier rounds, of earlier waves in this round, and of lower lanes in this wave.
__global__ __launch_bounds__(kThreads) void compact_scatter_kernel(const uint32_t* __restrict__ in,
                                                                   int64_t in_stride, int n_planes, int64_t n,
                                                                   const uint8_t* __restrict__ remove,
                                                                   uint32_t* __restrict__ out, int64_t out_stride,
                                                                   const uint32_t* __restrict__ block_base) {
  constexpr int kWaves = kThreads / 64;
  __shared__ uint32_t sh[kPer * kWaves];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  const int64_t base = (int64_t)blockIdx.x * kBlockItems + threadIdx.x;
  bool keep[kPer];
  uint32_t rank[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    keep[q] = kept(remove, base + q * kThreads, n);
    const uint64_t m = __ballot(keep[q]);
    rank[q] = (uint32_t)__popcll(m & below);
    if (lane == 0) sh[q * kWaves + wave] = (uint32_t)__popcll(m);
  }
  __syncthreads();
  uint32_t run = block_base[blockIdx.x];
  uint32_t slot[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      before += w < wave ? sh[q * kWaves + w] : 0u;
      all += sh[q * kWaves + w];
    }
    slot[q] = run + before + rank[q];
    run += all;
  }
  // planes five at a time: 20 independent loads in flight per thread
  constexpr int kPlanes = 5;
  int p = 0;
  for (; p + kPlanes <= n_planes; p += kPlanes) {
    uint32_t v[kPlanes][kPer];
#pragma unroll
    for (int i = 0; i < kPlanes; ++i)
#pragma unroll
      for (int q = 0; q < kPer; ++q)
        v[i][q] = keep[q] ? in[(size_t)(p + i) * in_stride + base + q * kThreads] : 0u;
#pragma unroll
    for (int i = 0; i < kPlanes; ++i)
#pragma unroll
      for (int q = 0; q < kPer; ++q)
        if (keep[q]) out[(size_t)(p + i) * out_stride + slot[q]] = v[i][q];
  }
  for (; p < n_planes; ++p) {
#pragma unroll
    for (int q = 0; q < kPer; ++q)
      if (keep[q]) out[(size_t)p * out_stride + slot[q]] = in[(size_t)p * in_stride + base + q * kThreads];
  }
}

__global__ __launch_bounds__(kThreads) void state_kernel(const float* __restrict__ params, int64_t n,
                                                         const float* __restrict__ contrib,
                                                         const float* __restrict__ pose, int32_t frame,
                                                         int32_t inactive_after, int32_t loop_frame,
                                                         int32_t* __restrict__ t_closest,
                                                         float* __restrict__ d_closest, int32_t* __restrict__ t_last,
                                                         int32_t* __restrict__ active) {
  const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (k >= n) return;
  // camera centre of the world-to-camera pose: -R^T t
  double cc[3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
    cc[c] = -((double)pose[0 * 4 + c] * pose[3] + (double)pose[1 * 4 + c] * pose[7] + (double)pose[2 * 4 + c] * pose[11]);
  const bool vis = contrib[k] > 0.5f;
  bool act = active[k] != 0;
  int32_t tc = t_closest[k], tl = t_last[k];
  if (loop_frame >= 0 && !act && vis && tc > loop_frame) {
    act = true;
    tl = frame;
  }
  if (act && vis) {
    tl = frame;
    const double dx = (double)params[k] - cc[0], dy = (double)params[n + k] - cc[1],
                 dz = (double)params[2 * n + k] - cc[2];
    const double dist = sqrt(dx * dx + dy * dy + dz * dz);
    if (dist < (double)d_closest[k]) {
      d_closest[k] = (float)dist;
      tc = frame;
    }
  }
  if (act && (int64_t)frame - (int64_t)tl > (int64_t)inactive_after) act = false;
  t_closest[k] = tc;
  t_last[k] = tl;
  active[k] = act ? 1 : 0;
}

__global__ __launch_bounds__(kThreads) void correct_kernel(float* __restrict__ params, int64_t n,
                                                           const int32_t* __restrict__ closest,
                                                           const float* __restrict__ delta, int32_t n_frames) {
  const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (k >= n) return;
  const int32_t f = closest[k];
  if (f < 0 || f >= n_frames) return;
  const float* D = delta + (size_t)f * 12;
  double R[9], t[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    R[r * 3 + 0] = D[r * 4 + 0];
    R[r * 3 + 1] = D[r * 4 + 1];
    R[r * 3 + 2] = D[r * 4 + 2];
    t[r] = D[r * 4 + 3];
  }
  // rows 0-2: mu (rotated and moved); rows 3-5, 6-8: t_u, t_v (rotated)
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    double v[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = params[(size_t)(3 * g + c) * n + k];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      double s = R[r * 3 + 0] * v[0] + R[r * 3 + 1] * v[1] + R[r * 3 + 2] * v[2];
      if (g == 0) s += t[r];
      params[(size_t)(3 * g + r) * n + k] = (float)s;
    }
  }
}

// Adam over the surfel parameters [15][n]: row blockIdx.y, four surfels per thread
// (16-byte accesses when n and the four arrays allow them).
struct AdamP {
  float lr[6];
  float b1, b2, eps, wd;
  float ic1, ic2;  // 1 / (1 - b1^t), 1 / (1 - b2^t)
  float s_min, o_min, o_max;
};

__device__ __forceinline__ float adam_one(float p, float g, float& m, float& v, float lr, const AdamP& a, int row) {
  m = fmaf(a.b1, m, (1.0f - a.b1) * g);
  v = fmaf(a.b2, v, (1.0f - a.b2) * g * g);
  const float step = (m * a.ic1) / (sqrtf(v * a.ic2) + a.eps);
  p -= lr * fmaf(a.wd, p, step);
  if (row == 9 || row == 10) p = fmaxf(p, a.s_min);
  if (row == 11) p = fminf(fmaxf(p, a.o_min), a.o_max);
  return p;
}

template <bool VEC>
__global__ __launch_bounds__(kThreads) void params_adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                                               float* __restrict__ m, float* __restrict__ v,
                                                               int64_t n, AdamP a) {
  const int row = blockIdx.y;
  const int grp = row < 3 ? 0 : row < 6 ? 1 : row < 9 ? 2 : row < 11 ? 3 : row == 11 ? 4 : 5;
  const float lr = a.lr[grp];
  const int64_t k0 = 4 * ((int64_t)blockIdx.x * kThreads + threadIdx.x);
  if (k0 >= n) return;
  const size_t base = (size_t)row * (size_t)n;
  if (VEC && k0 + 4 <= n) {
    float4 pp = *reinterpret_cast<float4*>(p + base + k0), gg = *reinterpret_cast<const float4*>(g + base + k0);
    float4 mm = *reinterpret_cast<float4*>(m + base + k0), vv = *reinterpret_cast<float4*>(v + base + k0);
    pp.x = adam_one(pp.x, gg.x, mm.x, vv.x, lr, a, row);
    pp.y = adam_one(pp.y, gg.y, mm.y, vv.y, lr, a, row);
    pp.z = adam_one(pp.z, gg.z, mm.z, vv.z, lr, a, row);
    pp.w = adam_one(pp.w, gg.w, mm.w, vv.w, lr, a, row);
    *reinterpret_cast<float4*>(p + base + k0) = pp;
    *reinterpret_cast<float4*>(m + base + k0) = mm;
    *reinterpret_cast<float4*>(v + base + k0) = vv;
    return;
  }
  for (int64_t k = k0; k < n && k < k0 + 4; ++k) {
    float mk = m[base + k], vk = v[base + k];
    p[base + k] = adam_one(p[base + k], g[base + k], mk, vk, lr, a, row);
    m[base + k] = mk;
    v[base + k] = vk;
  }
}

}  // namespace
}  // namespace map
}  // namespace gs2d

using namespace gs2d::map;

#define MAP_LAUNCHED() (hipGetLastError() == hipSuccess ? GS2D_OK : GS2D_ERR_HIP)

GS2D_API int64_t gs2d_covisibility_workspace(int64_t n) { return n < 0 ? 0 : 2 * (int64_t)covis_blocks(n); }

GS2D_API int gs2d_covisibility(const float* contrib_a, const float* contrib_b, int64_t n, float threshold,
                               uint32_t* counts, uint32_t* work, hipStream_t stream) {
  if (n < 0 || !counts || !work || (n > 0 && (!contrib_a || !contrib_b))) return GS2D_ERR_INVALID_ARG;
  const int nb = covis_blocks(n);
  const bool vec = ((reinterpret_cast<uintptr_t>(contrib_a) | reinterpret_cast<uintptr_t>(contrib_b)) & 15) == 0;
  if (vec)
    covis_partial_kernel<true><<<nb, kThreads, 0, stream>>>(contrib_a, contrib_b, n, threshold, work);
  else
    covis_partial_kernel<false><<<nb, kThreads, 0, stream>>>(contrib_a, contrib_b, n, threshold, work);
  covis_final_kernel<<<1, kThreads, 0, stream>>>(work, nb, counts);
  return MAP_LAUNCHED();
}

GS2D_API int gs2d_keyframe_test(const uint32_t* counts, const float* pose_cur, const float* pose_kf, double c_k,
                                double d_k, int32_t* is_keyframe, hipStream_t stream) {
  if (!counts || !pose_cur || !pose_kf || !is_keyframe) return GS2D_ERR_INVALID_ARG;
  keyframe_kernel<<<1, 64, 0, stream>>>(counts, pose_cur, pose_kf, c_k, d_k, is_keyframe);
  return MAP_LAUNCHED();
}

GS2D_API int gs2d_prune_mask(const float* contrib, const int32_t* closest_frame, int32_t frame, float threshold,
                             int64_t n, uint8_t* remove, hipStream_t stream) {
  if (n < 0 || (n > 0 && (!contrib || !closest_frame || !remove))) return GS2D_ERR_INVALID_ARG;
  if (n == 0) return GS2D_OK;
  const int nb = blocks_for((n + 3) / 4, kThreads);
  const bool vec = ((reinterpret_cast<uintptr_t>(contrib) | reinterpret_cast<uintptr_t>(closest_frame)) & 15) == 0 &&
                   (reinterpret_cast<uintptr_t>(remove) & 3) == 0;
  if (vec)
    prune_kernel<true><<<nb, kThreads, 0, stream>>>(contrib, closest_frame, frame, threshold, n, remove);
  else
    prune_kernel<false><<<nb, kThreads, 0, stream>>>(contrib, closest_frame, frame, threshold, n, remove);
  return MAP_LAUNCHED();
}

GS2D_API int64_t gs2d_compact_workspace(int64_t n) { return n < 0 ? 0 : (int64_t)blocks_for(n, kBlockItems); }

GS2D_API int gs2d_compact(const void* in, int64_t in_stride, int32_t n_planes, int64_t n, const uint8_t* remove,
                          void* out, int64_t out_stride, uint32_t* n_out, uint32_t* work, hipStream_t stream) {
  if (n < 0 || n_planes < 1 || !n_out || !work || in_stride < n || out_stride < 0 ||
      (n > 0 && (!in || !out)) || n > 0xFFFFFFFFll)
    return GS2D_ERR_INVALID_ARG;
  const int nb = blocks_for(n, kBlockItems);
  compact_count_kernel<<<nb, kThreads, 0, stream>>>(remove, n, work);
  compact_scan_kernel<<<1, kThreads, 0, stream>>>(work, nb, n_out);
  if (n > 0)
    compact_scatter_kernel<<<nb, kThreads, 0, stream>>>(static_cast<const uint32_t*>(in), in_stride, n_planes, n,
                                                        remove, static_cast<uint32_t*>(out), out_stride, work);
  return MAP_LAUNCHED();
}

GS2D_API int gs2d_map_state_update(const float* params, int64_t n, const float* contrib, const float* pose_kf,
                                   int32_t frame, int32_t inactive_after, int32_t loop_frame, int32_t* t_closest,
                                   float* d_closest, int32_t* t_last, int32_t* active, hipStream_t stream) {
  if (n < 0 || !pose_kf ||
      (n > 0 && (!params || !contrib || !t_closest || !d_closest || !t_last || !active)))
    return GS2D_ERR_INVALID_ARG;
  if (n == 0) return GS2D_OK;
  state_kernel<<<blocks_for(n, kThreads), kThreads, 0, stream>>>(params, n, contrib, pose_kf, frame, inactive_after,
                                                                 loop_frame, t_closest, d_closest, t_last, active);
  return MAP_LAUNCHED();
}

GS2D_API int gs2d_map_correct(float* params, int64_t n, const int32_t* closest_frame, const float* delta,
                              int32_t n_frames, hipStream_t stream) {
  if (n < 0 || n_frames < 0 || (n > 0 && (!params || !closest_frame)) || (n_frames > 0 && !delta))
    return GS2D_ERR_INVALID_ARG;
  if (n == 0 || n_frames == 0) return GS2D_OK;
  correct_kernel<<<blocks_for(n, kThreads), kThreads, 0, stream>>>(params, n, closest_frame, delta, n_frames);
  return MAP_LAUNCHED();
}

GS2D_API int gs2d_params_adam(float* params, const float* grad, float* m, float* v, int64_t n,
                              const gs2d_adam_args* args, hipStream_t stream) {
  if (n < 0 || !args || args->step < 1 || (n > 0 && (!params || !grad || !m || !v))) return GS2D_ERR_INVALID_ARG;
  if (!(args->beta1 >= 0.f && args->beta1 < 1.f) || !(args->beta2 >= 0.f && args->beta2 < 1.f) || !(args->eps >= 0.f))
    return GS2D_ERR_INVALID_ARG;
  if (n == 0) return GS2D_OK;
  AdamP a;
  for (int k = 0; k < 6; ++k) a.lr[k] = args->lr[k];
  a.b1 = args->beta1;
  a.b2 = args->beta2;
  a.eps = args->eps;
  a.wd = args->weight_decay;
  a.ic1 = (float)(1.0 / (1.0 - std::pow((double)args->beta1, (double)args->step)));
  a.ic2 = (float)(1.0 / (1.0 - std::pow((double)args->beta2, (double)args->step)));
  a.s_min = args->s_min;
  a.o_min = args->o_min;
  a.o_max = args->o_max;
  const dim3 grid((unsigned)blocks_for((n + 3) / 4, kThreads), 15);
  const bool vec = (n % 4) == 0 && ((reinterpret_cast<uintptr_t>(params) | reinterpret_cast<uintptr_t>(grad) |
                                      reinterpret_cast<uintptr_t>(m) | reinterpret_cast<uintptr_t>(v)) & 15) == 0;
  if (vec)
    params_adam_kernel<true><<<grid, kThreads, 0, stream>>>(params, grad, m, v, n, a);
  else
    params_adam_kernel<false><<<grid, kThreads, 0, stream>>>(params, grad, m, v, n, a);
  return MAP_LAUNCHED();
}
