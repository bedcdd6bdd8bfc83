// Scans, the stable LSD radix sort, pair duplication and tile ranges.
//
// The paper composites surfels "sorted by depth" per pixel (Sec. "2D Gaussian
// Splatting", eq:alpha_blending).  The tile rasterizer realises that order with
// two stable sorts: (view, surfel) items by float32 camera depth (ties keep the
// item order, i.e. the surfel index within a view), then the (tile, item) pairs,
// emitted in that depth order and keyed by a global tile index (each view's tiles
// follow the previous view's), stably by tile.  Each tile's list is therefore
// ascending (depth, index), the order of the per-pixel definition.
//
// Radix pass (digits of up to 11 bits: 256 or 2048 bins) = three kernels over blocks
// of kScanItems keys:
//   hist    per-block digit histogram (LDS atomics, one sub-histogram per wave),
//           stored digit-major: row d holds digit d's count in every block
//   offsets one workgroup per digit: exclusive scan of that digit's row (its
//           offset within the digit) and the row total
//   scatter per block: the digit bases (an LDS scan of the row totals) plus the
//           row prefix give each digit's first output slot; then 8 rounds of 256
//           keys: a wave-level multi-split (ballots over the digit bits give each
//           lane the mask of lanes holding the same digit), the same digit's keys
//           in the lower waves of the round (per-wave counts in LDS, stamped with
//           the round so that they need no clearing), and the running per-digit
//           offset across rounds keep the pass stable.
// 32-bit depth keys take 3 passes (11, 11, 10 bits); tile keys of up to 2048 tiles
// take one, whose digit bases and totals are the tile ranges.
// The depth sort's first pass also compacts: items whose key is kDropKey (surfels
// that touch no tile) are left out of the histogram and the scatter, so the pass
// writes only the visible items, in stable order, and counts them on the device;
// the remaining passes and everything after them run over that count.
// Kernels whose item count lives on the device read it and exit early, so a
// capacity-sized launch can be captured in a graph.
#include "gs2d_internal.h"

namespace gs2d {
namespace {

constexpr int kThreads = 256;
constexpr int kRounds = kScanItems / kThreads;  // 8
constexpr int kWaves = kThreads / 64;
constexpr uint32_t kDropKey = 0xFFFFFFFFu;

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void fill_f32_kernel(float* p, float v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void copy_u32_kernel(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
  // Hillis-Steele over 256 threads in LDS; sh has 256 entries.
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kThreads; off <<= 1) {
    uint32_t x = t >= off ? sh[t - off] : 0u;
    __syncthreads();
    sh[t] += x;
    __syncthreads();
  }
  const uint32_t incl = sh[t];
  if (total) *total = sh[kThreads - 1];
  __syncthreads();
  return incl - v;
}

__device__ inline uint32_t load_count(const uint32_t* count, const uint32_t* perm, int i, int n) {
  if (i >= n) return 0u;
  return perm ? count[perm[i]] : count[i];
}

// Item count of a pass: the device count clamped to the buffer capacity
// (`limit`), or `limit` itself when there is no device count.
__device__ inline int64_t item_count(const uint32_t* n_dev, int64_t limit) {
  if (!n_dev) return limit;
  const int64_t n = (int64_t)(*n_dev);
  return n < limit ? n : limit;
}

__global__ __launch_bounds__(kThreads) void scan_reduce_kernel(const uint32_t* __restrict__ count,
                                                               const uint32_t* __restrict__ perm,
                                                               const uint32_t* __restrict__ n_dev, int limit,
                                                               uint32_t* __restrict__ block_sums) {
  const int n = (int)item_count(n_dev, limit);
  if ((int64_t)blockIdx.x * kScanItems >= n) return;
  __shared__ uint32_t sh[kThreads];
  const int base = blockIdx.x * kScanItems + threadIdx.x * kRounds;
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kRounds; ++k) s += load_count(count, perm, base + k, n);
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) block_sums[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kThreads) void scan_blocks_kernel(uint32_t* __restrict__ block_sums,
                                                               const uint32_t* __restrict__ n_dev, int limit,
                                                               Ctrl* __restrict__ ctrl) {
  // one block: exclusive scan of the active blocks' sums, in chunks of 256
  const int n = (int)item_count(n_dev, limit);
  const int nb = (n + kScanItems - 1) / kScanItems;
  __shared__ uint32_t sh[kThreads];
  uint32_t carry = 0;
  for (int c0 = 0; c0 < nb; c0 += kThreads) {
    const int i = c0 + threadIdx.x;
    const uint32_t v = i < nb ? block_sums[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(v, sh, &tot);
    if (i < nb) block_sums[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    ctrl->n_pairs = carry;
    ctrl->overflow = 0;
  }
}

__global__ __launch_bounds__(kThreads) void scan_final_kernel(const uint32_t* __restrict__ count,
                                                              const uint32_t* __restrict__ perm,
                                                              const uint32_t* __restrict__ n_dev, int limit,
                                                              const uint32_t* __restrict__ block_sums,
                                                              uint32_t* __restrict__ offs) {
  const int n = (int)item_count(n_dev, limit);
  if ((int64_t)blockIdx.x * kScanItems >= n) return;
  __shared__ uint32_t sh[kThreads];
  const int base = blockIdx.x * kScanItems + threadIdx.x * kRounds;
  uint32_t v[kRounds];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kRounds; ++k) {
    v[k] = load_count(count, perm, base + k, n);
    s += v[k];
  }
  uint32_t run = block_sums[blockIdx.x] + block_exclusive_scan(s, sh, nullptr);
#pragma unroll
  for (int k = 0; k < kRounds; ++k) {
    if (base + k < n) offs[base + k] = run;
    run += v[k];
  }
}

// Radix passes take up to 11 bits: R = 256 or 2048 bins (kDigits8, kDigits11).
constexpr int kDigits8 = 256, kDigits11 = 2048;

// Per-block digit histogram, digit-major (row d = digit d's count in every block).
// drop: leave kDropKey keys out and add the kept count to *n_kept (zero beforehand).
template <int R>
__global__ __launch_bounds__(kThreads) void radix_hist_kernel(const uint32_t* __restrict__ keys,
                                                              const uint32_t* __restrict__ n_dev,
                                                              int64_t n_host, int shift, int bits, int drop,
                                                              uint32_t* __restrict__ hist,
                                                              uint32_t* __restrict__ n_kept) {
  constexpr int PER = R / kThreads;  // digits per thread
  const int64_t n = item_count(n_dev, n_host);
  const int64_t base = (int64_t)blockIdx.x * kScanItems;
  if (base >= n) return;
  __shared__ uint32_t h[kWaves][R];
  const int wave = threadIdx.x / 64;
  const uint32_t dmask = (1u << bits) - 1u;
  for (int k = threadIdx.x; k < kWaves * R; k += kThreads) (&h[0][0])[k] = 0u;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int64_t i = base + r * kThreads + threadIdx.x;
    if (i < n) {
      const uint32_t k = keys[i];
      if (!(drop && k == kDropKey)) atomicAdd(&h[wave][(k >> shift) & dmask], 1u);
    }
  }
  __syncthreads();
  uint32_t kept = 0;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int d = q * kThreads + threadIdx.x;
    uint32_t s = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) s += h[w][d];
    hist[(size_t)d * gridDim.x + blockIdx.x] = s;
    kept += s;
  }
  if (drop) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) kept += __shfl_xor(kept, m, 64);
    if ((threadIdx.x & 63) == 0 && kept) atomicAdd(n_kept, kept);
  }
}

// One workgroup per digit d (grid = R): exclusive scan, in place, of row d of the
// digit-major histogram over the active blocks (each thread four consecutive
// entries per chunk of 1024), and the row total into dtot[d].  The grid's block
// count is the row stride.
__global__ __launch_bounds__(kThreads) void radix_offsets_kernel(uint32_t* __restrict__ hist, int nb_grid,
                                                                 const uint32_t* __restrict__ n_dev,
                                                                 int64_t n_host, uint32_t* __restrict__ dtot) {
  const int64_t n = item_count(n_dev, n_host);
  const int nb = (int)((n + kScanItems - 1) / kScanItems);
  uint32_t* __restrict__ row = hist + (size_t)blockIdx.x * nb_grid;
  __shared__ uint32_t sh[kThreads];
  const int t = threadIdx.x;
  uint32_t carry = 0;
  for (int c0 = 0; c0 < nb; c0 += 4 * kThreads) {
    uint32_t v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = c0 + 4 * t + k;
      v[k] = e < nb ? row[e] : 0u;
    }
    uint32_t tot;
    uint32_t run = carry + block_exclusive_scan(v[0] + v[1] + v[2] + v[3], sh, &tot);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = c0 + 4 * t + k;
      if (e < nb) row[e] = run;
      run += v[k];
    }
    carry += tot;
  }
  if (t == 0) dtot[blockIdx.x] = carry;
}

// Scatter of one pass.  With `ranges` (a pass over every tile bit of the pair keys),
// block 0 also writes each tile's [start, end) -- the digit bases and totals -- for
// tiles < n_tiles (empty ranges after a pair overflow).
template <int R>
__global__ __launch_bounds__(kThreads) void radix_scatter_kernel(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint32_t* __restrict__ kout,
    uint32_t* __restrict__ vout, const uint32_t* __restrict__ n_dev, int64_t n_host, int shift,
    int bits, int drop, const uint32_t* __restrict__ hist, const uint32_t* __restrict__ dtot,
    uint2* __restrict__ ranges, int n_tiles, const uint32_t* __restrict__ overflow) {
  constexpr int PER = R / kThreads;
  const int64_t n = item_count(n_dev, n_host);
  const int64_t base = (int64_t)blockIdx.x * kScanItems;
  if (base >= n) return;
  __shared__ uint32_t doff[R];
  __shared__ uint32_t wcnt[kWaves][R];  // (round stamp << 16) | count of the wave's keys of a digit
  __shared__ uint32_t sh[kThreads];
  const int t = threadIdx.x, wave = t / 64, lane = t % 64;
  for (int k = t; k < kWaves * R; k += kThreads) (&wcnt[0][0])[k] = 0u;
  // first slot of digit d: the keys of all smaller digits, then this digit's keys in
  // the blocks before this one (thread t holds digits PER t .. PER t + PER - 1)
  uint32_t tot[PER], pre = 0;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    tot[q] = dtot[PER * t + q];
    pre += tot[q];
  }
  uint32_t run = block_exclusive_scan(pre, sh, nullptr);
  const bool write_ranges = ranges && blockIdx.x == 0;
  const bool empty = write_ranges && *overflow != 0u;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int d = PER * t + q;
    doff[d] = run + hist[(size_t)d * gridDim.x + blockIdx.x];
    if (write_ranges && d < n_tiles) ranges[d] = empty ? make_uint2(0u, 0u) : make_uint2(run, run + tot[q]);
    run += tot[q];
  }
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  // all of the block's keys up front: the rounds' loads overlap instead of each
  // round waiting for its own
  uint32_t kr[kRounds], vr[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int64_t i = base + r * kThreads + t;
    kr[r] = i < n ? kin[i] : 0u;
    vr[r] = i < n ? vin[i] : 0u;
  }
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const uint32_t stamp = (uint32_t)(r + 1) << 16;
    const int64_t i = base + r * kThreads + t;
    const uint32_t key = kr[r], val = vr[r];
    bool valid = i < n;
    const uint32_t digit = valid ? (key >> shift) & ((1u << bits) - 1u) : 0u;
    valid = valid && !(drop && key == kDropKey);
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < bits; ++b) {
      const bool set = (digit >> b) & 1u;
      const uint64_t bal = __ballot(valid && set);
      peers &= set ? bal : ~bal;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    const uint32_t cnt = (uint32_t)__popcll(peers);
    const bool leader = valid && rank == 0;
    if (leader) wcnt[wave][digit] = stamp | cnt;
    __syncthreads();
    // the group's first slot: the digit's running offset plus the same digit's keys
    // in the lower waves of this round
    uint32_t pb = 0;
    if (leader) {
      pb = doff[digit];
      for (int w = 0; w < wave; ++w) {
        const uint32_t e = wcnt[w][digit];
        if ((e & 0xFFFF0000u) == stamp) pb += e & 0xFFFFu;
      }
    }
    __syncthreads();
    if (leader) atomicAdd(&doff[digit], cnt);
    const int src = peers ? (int)__ffsll((long long)peers) - 1 : lane;
    const uint32_t gb = (uint32_t)__shfl((int)pb, src, 64);
    if (valid) {
      const uint32_t pos = gb + rank;
      kout[pos] = key;
      vout[pos] = val;
    }
  }
}

__global__ __launch_bounds__(kThreads) void duplicate_kernel(
    const uint32_t* __restrict__ sorted_ids, const uint32_t* __restrict__ count,
    const uint32_t* __restrict__ offs, const uint2* __restrict__ rect, const ViewDesc* __restrict__ views,
    int n_views, const uint32_t* __restrict__ n_dev, int limit, int64_t p_cap, uint32_t* __restrict__ pkey,
    uint32_t* __restrict__ pval, Ctrl* __restrict__ ctrl, uint2* __restrict__ ranges, int n_tiles) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  // clear the tile ranges for the ranges kernel (which runs after the tile sort)
  for (int k = j; k < n_tiles; k += gridDim.x * blockDim.x) ranges[k] = make_uint2(0u, 0u);
  const int n = (int)item_count(n_dev, limit);
  const uint32_t id = j < n ? sorted_ids[j] : 0u;
  const uint32_t c = j < n ? count[id] : 0u;
  if (c == 0) return;
  uint32_t off = offs[j];
  if ((int64_t)off + c > p_cap) {
    ctrl->overflow = 1u;
    return;
  }
  // key = the view's first global tile + the tile's index within the view
  const ViewDesc& V = views[view_of_item(views, n_views, (int)id)];
  const uint32_t base = (uint32_t)V.tile_base, tiles_x = (uint32_t)V.tiles_x;
  const uint2 rc = rect[id];
  const uint32_t tx0 = rc.x & 0xFFFFu, tx1 = rc.x >> 16, ty0 = rc.y & 0xFFFFu, ty1 = rc.y >> 16;
  for (uint32_t ty = ty0; ty <= ty1; ++ty)
    for (uint32_t tx = tx0; tx <= tx1; ++tx) {
      pkey[off] = base + ty * tiles_x + tx;
      pval[off] = id;
      ++off;
    }
}

__global__ __launch_bounds__(kThreads) void ranges_kernel(const uint32_t* __restrict__ skey,
                                                          const Ctrl* __restrict__ ctrl, int64_t p_cap,
                                                          uint2* __restrict__ ranges) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t np = ctrl->n_pairs;
  if (ctrl->overflow) np = 0;
  if (np > p_cap) np = p_cap;
  if (i >= np) return;
  const uint32_t t = skey[i];
  if (i == 0 || skey[i - 1] != t) ranges[t].x = (uint32_t)i;
  if (i == np - 1 || skey[i + 1] != t) ranges[t].y = (uint32_t)(i + 1);
}

inline int blocks_for(int64_t n, int per) { return (int)((n + per - 1) / per) > 0 ? (int)((n + per - 1) / per) : 1; }

}  // namespace

void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  fill_u32_kernel<<<blocks_for(n, 256), 256, 0, s>>>(p, v, n);
}
void launch_fill_f32(float* p, float v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  fill_f32_kernel<<<blocks_for(n, 256), 256, 0, s>>>(p, v, n);
}
void launch_copy_u32(const uint32_t* src, uint32_t* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  copy_u32_kernel<<<blocks_for(n, 256), 256, 0, s>>>(src, dst, n);
}

void launch_scan_counts(const uint32_t* count, const uint32_t* perm, const uint32_t* n_dev, int limit,
                        uint32_t* offs, uint32_t* block_sums, Ctrl* ctrl, hipStream_t s) {
  const int nb = blocks_for(limit, kScanItems);
  scan_reduce_kernel<<<nb, kThreads, 0, s>>>(count, perm, n_dev, limit, block_sums);
  scan_blocks_kernel<<<1, kThreads, 0, s>>>(block_sums, n_dev, limit, ctrl);
  scan_final_kernel<<<nb, kThreads, 0, s>>>(count, perm, n_dev, limit, block_sums, offs);
}

int radix_sort(uint32_t* keys[2], uint32_t* vals[2], int64_t cap, int64_t n_host, const uint32_t* n_dev,
               int bits, uint32_t* hist, uint32_t* n_kept, uint2* ranges, int n_tiles, const uint32_t* overflow,
               hipStream_t s) {
  const int nb = blocks_for(cap, kScanItems);
  const int64_t limit = n_dev ? cap : n_host;
  uint32_t* dtot = hist + (size_t)kDigits11 * nb;
  const int passes = (bits + 10) / 11;
  int cur = 0, shift = 0;
  for (int p = 0; p < passes; ++p) {
    const int pb = (bits - shift + (passes - p) - 1) / (passes - p);  // split the bits evenly
    const int drop = (n_kept && p == 0) ? 1 : 0;
    // after a dropping first pass the kept count is the item count
    const uint32_t* nd = (n_kept && p > 0) ? n_kept : n_dev;
    const int64_t lim = (n_kept && p > 0) ? cap : limit;
    uint2* rg = (ranges && passes == 1) ? ranges : nullptr;
    if (pb <= 8) {
      radix_hist_kernel<kDigits8><<<nb, kThreads, 0, s>>>(keys[cur], nd, lim, shift, pb, drop, hist, n_kept);
      radix_offsets_kernel<<<kDigits8, kThreads, 0, s>>>(hist, nb, nd, lim, dtot);
      radix_scatter_kernel<kDigits8><<<nb, kThreads, 0, s>>>(keys[cur], vals[cur], keys[cur ^ 1], vals[cur ^ 1],
                                                             nd, lim, shift, pb, drop, hist, dtot, rg, n_tiles,
                                                             overflow);
    } else {
      radix_hist_kernel<kDigits11><<<nb, kThreads, 0, s>>>(keys[cur], nd, lim, shift, pb, drop, hist, n_kept);
      radix_offsets_kernel<<<kDigits11, kThreads, 0, s>>>(hist, nb, nd, lim, dtot);
      radix_scatter_kernel<kDigits11><<<nb, kThreads, 0, s>>>(keys[cur], vals[cur], keys[cur ^ 1], vals[cur ^ 1],
                                                              nd, lim, shift, pb, drop, hist, dtot, rg, n_tiles,
                                                              overflow);
    }
    cur ^= 1;
    shift += pb;
  }
  return cur;
}

void launch_duplicate(const uint32_t* sorted_ids, const uint32_t* count, const uint32_t* offs,
                      const uint2* rect, const ViewDesc* views, int n_views, const uint32_t* n_dev, int limit,
                      int64_t p_cap, uint32_t* pkey, uint32_t* pval, Ctrl* ctrl, uint2* ranges, int n_tiles,
                      hipStream_t s) {
  duplicate_kernel<<<blocks_for(limit, 256), 256, 0, s>>>(sorted_ids, count, offs, rect, views, n_views, n_dev,
                                                          limit, p_cap, pkey, pval, ctrl, ranges, n_tiles);
}

void launch_ranges(const uint32_t* skey, const Ctrl* ctrl, int64_t p_cap, uint2* ranges, int n_tiles,
                   hipStream_t s) {
  (void)n_tiles;  // cleared by the duplicate kernel
  ranges_kernel<<<blocks_for(p_cap, 256), 256, 0, s>>>(skey, ctrl, p_cap, ranges);
}

}  // namespace gs2d
