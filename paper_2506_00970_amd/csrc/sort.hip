// Pair duplication, the tile sort, the per-tile depth order and the tile ranges.
//
// The paper composites surfels "sorted by depth" per pixel (Sec. "2D Gaussian
// Splatting", eq:alpha_blending).  Here every tile's list ends up ascending in
// (float32 camera depth, item), the order of the per-pixel definition, in three steps:
//   1. duplication  each item (view, surfel) that touches a tile emits one (tile,
//                   item) pair per tile of its rectangle, in item order: its first
//                   slot is the pair count of all earlier items (per-block counts
//                   from preprocessing, plus a block scan);
//   2. tile sort    a stable LSD radix sort of the pairs by the global tile index (each
//                   view's tiles follow the previous view's), so that each tile's
//                   items stay in ascending item order;
//   3. depth order  one workgroup per tile stably sorts the tile's items by depth key;
//                   with the items ascending on entry, ties keep item order (see
//                   tile_order.h; the tracking walk orders its own tile instead).
//
// Radix pass of the tile sort (digits of up to 11 bits: 256 or 2048 bins) over blocks
// of kScanItems keys, with a digit-major histogram plane: cell (d, b) = the keys of
// digit d in block b.  The duplication fills the first pass's plane (and a two-pass
// sort's first scatter fills the second's), with atomics at each key's block.  The
// pass itself is two kernels:
//   offsets one workgroup per digit: exclusive scan of row d over the active blocks,
//           in place, and the row total
//   scatter per block: the digit bases (an LDS scan of the row totals) plus the
//           block's column give each digit's first output slot, and the block then
//           clears its column, so that a plane is all zero again once its pass is
//           done; then 4 rounds of 256 keys: a wave-level multi-split (ballots over
//           the digit bits give each lane the mask of lanes holding the same digit),
//           the same digit's keys in the lower waves of the round (per-wave counts in
//           LDS, stamped with the round so that they need no clearing), and the
//           running per-digit offset across rounds keep the pass stable.
// Up to 2048 tiles take one pass, whose digit bases and totals are the tile ranges.
// Kernels whose item count lives on the device read it and exit early, so a
// capacity-sized launch can be captured in a graph.
#include "tile_order.h"

namespace gs2d {
namespace {

constexpr int kThreads = kBlockThreads;
constexpr int kRounds = kScanItems / kThreads;  // 4
constexpr int kWaves = kBlockWaves;
constexpr int kBlockShift = 10;  // log2(kScanItems)
static_assert(kScanItems == 1 << kBlockShift, "block shift");
static_assert(kPartItems == kThreads, "duplication blocks are preprocessing blocks");
constexpr int kDirectParts = 4096;  // up to this many item blocks, each block sums the counts before it

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

// Item count of a pass: the device count clamped to the buffer capacity
// (`limit`), or `limit` itself when there is no device count.
__device__ inline int64_t item_count(const uint32_t* n_dev, int64_t limit) {
  if (!n_dev) return limit;
  const int64_t n = (int64_t)(*n_dev);
  return n < limit ? n : limit;
}

// One workgroup per digit d (grid = the pass's bins): exclusive scan, in place, of
// row d of the plane over the active blocks (each thread four consecutive entries
// per chunk of 1024), and the row total into dtot[d].
__global__ __launch_bounds__(kThreads) void radix_offsets_kernel(uint32_t* __restrict__ hist, int stride,
                                                                 const uint32_t* __restrict__ n_dev,
                                                                 int64_t n_host, uint32_t* __restrict__ dtot) {
  const int64_t n = item_count(n_dev, n_host);
  const int nb = (int)((n + kScanItems - 1) / kScanItems);
  uint32_t* __restrict__ row = hist + (size_t)blockIdx.x * stride;
  __shared__ uint32_t sh[kWaves];
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

// The same for the 2048-bin passes, whose rows are short (the tile sorts of up to 2048
// tiles: one entry per 1024 pairs): one wave per digit, four digits per workgroup,
// each lane four consecutive entries per chunk of 256, a wave-level scan with a carry.
__global__ __launch_bounds__(kThreads) void radix_offsets_wave_kernel(uint32_t* __restrict__ hist, int stride,
                                                                      const uint32_t* __restrict__ n_dev,
                                                                      int64_t n_host, uint32_t* __restrict__ dtot) {
  const int64_t n = item_count(n_dev, n_host);
  const int nb = (int)((n + kScanItems - 1) / kScanItems);
  const int lane = threadIdx.x & 63;
  const int d = blockIdx.x * kWaves + (threadIdx.x >> 6);
  uint32_t* __restrict__ row = hist + (size_t)d * stride;
  uint32_t carry = 0;
  for (int c0 = 0; c0 < nb; c0 += 4 * 64) {
    uint32_t v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = c0 + 4 * lane + k;
      v[k] = e < nb ? row[e] : 0u;
    }
    const uint32_t mine = v[0] + v[1] + v[2] + v[3];
    uint32_t x = mine;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = (uint32_t)__shfl_up((int)x, o, 64);
      if (lane >= o) x += y;
    }
    uint32_t run = carry + x - mine;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = c0 + 4 * lane + k;
      if (e < nb) row[e] = run;
      run += v[k];
    }
    carry += (uint32_t)__shfl((int)x, 63, 64);
  }
  if (lane == 0) dtot[d] = carry;
}

// One radix pass's scatter (see the top of the file).
struct PassArgs {
  const uint32_t* kin;
  const uint32_t* vin;
  uint32_t* kout;
  uint32_t* vout;
  const uint32_t* n_dev;  // item count on the device (clamped to n_host), or null: n_host
  int64_t n_host;
  int shift, bits;        // digit = (key >> shift) mod 2^bits
  uint32_t* hist;         // this pass's plane: offsets in, cleared out
  int stride;             // row stride of the planes
  const uint32_t* dtot;   // row totals
  uint32_t* hnext;        // the next pass's plane, or null
  int nshift, nbits;      // the next pass's digit
  uint2* ranges;          // a pass over every tile bit: block 0 writes each tile's [start, end)
  int n_tiles;            //   for tiles < n_tiles (empty ranges when *overflow != 0)
  const uint32_t* overflow;
  uint32_t* check;        // Ctrl::check_bits (device checks)
  const uint32_t* din;    // a second value moved with the keys (the pairs' depth keys), or null
  uint32_t* dout;
};

template <int R>
__global__ __launch_bounds__(kThreads) void radix_scatter_kernel(PassArgs a) {
  constexpr int PER = R / kThreads;
  const int64_t n = item_count(a.n_dev, a.n_host);
  const int64_t base = (int64_t)blockIdx.x * kScanItems;
  if (base >= n) return;
  __shared__ uint32_t doff[R];
  __shared__ uint32_t wcnt[kWaves][R];  // (round stamp << 16) | count of the wave's keys of a digit
  __shared__ uint32_t sh[kWaves];
  const int t = threadIdx.x;
  for (int k = t; k < kWaves * R; k += kThreads) (&wcnt[0][0])[k] = 0u;
  // first slot of digit d: the keys of all smaller digits, then this digit's keys in
  // the blocks before this one (thread t holds digits PER t .. PER t + PER - 1)
  uint32_t tot[PER], pre = 0;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    tot[q] = a.dtot[PER * t + q];
    pre += tot[q];
  }
  uint32_t run = block_exclusive_scan(pre, sh, nullptr);
  const bool write_ranges = a.ranges && blockIdx.x == 0;
  const bool empty = write_ranges && *a.overflow != 0u;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int d = PER * t + q;
    uint32_t* cell = a.hist + (size_t)d * a.stride + blockIdx.x;
    const uint32_t c = *cell;
    if (c) *cell = 0u;  // only this block reads this column
    doff[d] = run + c;
    if (write_ranges && d < a.n_tiles) a.ranges[d] = empty ? make_uint2(0u, 0u) : make_uint2(run, run + tot[q]);
    GS2D_DCHECK(a.check, !write_ranges || empty || d < a.n_tiles || tot[q] == 0u, kCheckRangeTile);
    run += tot[q];
  }
  __syncthreads();
  const uint32_t nmask = (1u << a.nbits) - 1u;
  // all of the block's keys up front: the rounds' loads overlap instead of each
  // round waiting for its own
  uint32_t kr[kRounds], vr[kRounds], dr[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int64_t i = base + r * kThreads + t;
    kr[r] = i < n ? a.kin[i] : 0u;
    vr[r] = i < n ? a.vin[i] : 0u;
    dr[r] = i < n && a.din ? a.din[i] : 0u;
  }
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const bool valid = base + r * kThreads + t < n;
    const uint32_t key = kr[r];
    const uint32_t digit = valid ? (key >> a.shift) & ((1u << a.bits) - 1u) : 0u;
    const uint32_t pos = rank_round<R>(digit, valid, a.bits, (uint32_t)(r + 1) << 16, &wcnt[0][0], doff);
    if (valid) {
      a.kout[pos] = key;
      a.vout[pos] = vr[r];
      if (a.dout) a.dout[pos] = dr[r];
      if (a.hnext)
        atomicAdd(&a.hnext[(size_t)((key >> a.nshift) & nmask) * a.stride + (pos >> kBlockShift)], 1u);
    }
  }
}

// With more item blocks than kDirectParts: exclusive scan, in place, of the per-block
// pair counts (one workgroup, chunks of kScanItems), and the totals.
__global__ __launch_bounds__(kThreads) void scan_parts_kernel(uint32_t* __restrict__ part_pairs,
                                                              const uint32_t* __restrict__ part_vis, int n_parts,
                                                              Ctrl* __restrict__ ctrl, uint32_t* __restrict__ np_host) {
  __shared__ uint32_t sh[kWaves];
  const int t = threadIdx.x;
  uint32_t carry = 0, vis = 0;
  for (int c0 = 0; c0 < n_parts; c0 += kScanItems) {
    uint32_t v[kRounds], s = 0;
#pragma unroll
    for (int k = 0; k < kRounds; ++k) {
      const int e = c0 + kRounds * t + k;
      v[k] = e < n_parts ? part_pairs[e] : 0u;
      vis += e < n_parts ? part_vis[e] : 0u;
      s += v[k];
    }
    uint32_t tot;
    uint32_t run = carry + block_exclusive_scan(s, sh, &tot);
#pragma unroll
    for (int k = 0; k < kRounds; ++k) {
      const int e = c0 + kRounds * t + k;
      if (e < n_parts) part_pairs[e] = run;
      run += v[k];
    }
    carry += tot;
  }
  uint32_t vt;
  (void)block_exclusive_scan(vis, sh, &vt);
  if (t == 0) {
    ctrl->n_pairs = carry;
    ctrl->n_visible = vt;
    if (np_host) __hip_atomic_store(np_host, carry, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// The pairs of every item, in item order (one thread per item, the blocks of
// preprocessing).  Item j's first slot is the pair count of the items before it: the
// earlier blocks' counts (summed here, or scanned beforehand for many blocks) plus a
// block scan.  Each pair also counts into the first tile pass's plane at its output
// block.
struct DupArgs {
  const uint32_t* count;       // tile count per item
  const uint32_t* part_pairs;  // per-block pair counts (exclusive prefix when scanned)
  const uint32_t* part_vis;    // per-block visible-item counts
  int n_parts;
  int scanned;
  const uint2* rect;
  const ViewDesc* views;
  int n_views;
  int64_t items;
  int64_t p_cap;
  uint32_t* pkey;
  uint32_t* pval;
  Ctrl* ctrl;
  const uint32_t* dkey;
  uint32_t* pdk;
  uint2* ranges;  // cleared here for the ranges kernel (multi-pass tile sorts)
  int n_tiles;
  uint32_t* hist;  // the first tile pass's plane
  int stride;
  int bits;        // the first tile pass's digit: key mod 2^bits
  uint32_t* np_host;  // nullable: the pair total also to this host-visible word
};

__global__ __launch_bounds__(kThreads) void duplicate_kernel(DupArgs a) {
  const int t = threadIdx.x;
  const int g = blockIdx.x;
  const int64_t j = (int64_t)g * kThreads + t;
  // the loads that do not wait on the scan go first, all three at once
  uint32_t c = 0u, dk = 0u;
  uint2 rc = make_uint2(1u, 0u);
  if (j < a.items) {
    c = a.count[j];
    rc = a.rect[j];
    dk = a.dkey[j];
  }
  if (c == 0u) rc = make_uint2(1u, 0u);
  for (int64_t k = j; k < a.n_tiles; k += (int64_t)gridDim.x * kThreads) a.ranges[k] = make_uint2(0u, 0u);
  __shared__ uint32_t sh[kWaves];
  __shared__ unsigned long long sh64[kWaves];
  uint32_t before, off;
  if (a.scanned) {
    before = a.part_pairs[g];
    off = before + block_exclusive_scan(c, sh, nullptr);
  } else {
    // one scan of (earlier blocks' counts, this item's count) packed in 64 bits: the
    // high half's total is the pair count before the block, the low half's exclusive
    // prefix the item's place within it
    // (the counts of blocks 0 .. g - 1, 8 per thread at a time, all loads issued before
    // the first addition: reads past block g - 1 return 0)
    uint32_t s = 0;
    const __amdgpu_buffer_rsrc_t prs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t*>(a.part_pairs), (short)0, 4 * g, 0x00020000);
    for (int k0 = t; k0 < g; k0 += 8 * kThreads) {
      uint32_t v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        v[u] = __builtin_amdgcn_raw_buffer_load_b32(prs, 4u * (uint32_t)(k0 + u * kThreads), 0, 0);
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    const int lane = t & 63, wave = t >> 6;
    const unsigned long long v = ((unsigned long long)s << 32) | c;
    unsigned long long x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const unsigned long long y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) sh64[wave] = x;
    __syncthreads();
    unsigned long long below = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const unsigned long long sw = sh64[w];
      below += w < wave ? sw : 0ull;
      all += sw;
    }
    before = (uint32_t)(all >> 32);
    off = before + (uint32_t)((below + x - v) & 0xFFFFFFFFull);
    if (g == 0) {
      uint32_t sp = 0, sv = 0;
      for (int k = t; k < a.n_parts; k += kThreads) {
        sp += a.part_pairs[k];
        sv += a.part_vis[k];
      }
      uint32_t tp, tv;
      (void)block_exclusive_scan(sp, sh, &tp);
      (void)block_exclusive_scan(sv, sh, &tv);
      if (t == 0) {
        a.ctrl->n_pairs = tp;
        a.ctrl->n_visible = tv;
        if (a.np_host) __hip_atomic_store(a.np_host, tp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      }
    }
  }
  if (c == 0) return;
  if ((int64_t)off + c > a.p_cap) {
    a.ctrl->overflow = 1u;
    return;
  }
  // key = the view's first global tile + the tile's index within the view
  const int item = (int)j;
  const ViewDesc& V = a.views[a.n_views == 1 ? 0 : view_of_item(a.views, a.n_views, item)];
  const uint32_t tbase = (uint32_t)V.tile_base, tiles_x = (uint32_t)V.tiles_x;
  const uint32_t tx0 = rc.x & 0xFFFFu, tx1 = rc.x >> 16, ty0 = rc.y & 0xFFFFu, ty1 = rc.y >> 16;
  const uint32_t dmask = (1u << a.bits) - 1u;
  for (uint32_t ty = ty0; ty <= ty1; ++ty)
    for (uint32_t tx = tx0; tx <= tx1; ++tx) {
      const uint32_t key = tbase + ty * tiles_x + tx;
      GS2D_DCHECK(&a.ctrl->check_bits, key < (uint32_t)a.n_tiles, kCheckPairKey);
      GS2D_DCHECK(&a.ctrl->check_bits, (int64_t)off < a.p_cap, kCheckPairIndex);
      a.pkey[off] = key;
      a.pval[off] = (uint32_t)item;
      a.pdk[off] = dk;
      atomicAdd(&a.hist[(size_t)(key & dmask) * a.stride + (off >> kBlockShift)], 1u);
      ++off;
    }
}

__global__ __launch_bounds__(kThreads) void ranges_kernel(const uint32_t* __restrict__ skey, Ctrl* __restrict__ ctrl,
                                                          int64_t p_cap, uint2* __restrict__ ranges, int n_tiles) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t np = ctrl->n_pairs;
  if (ctrl->overflow) np = 0;
  if (np > p_cap) np = p_cap;
  if (i >= np) return;
  const uint32_t t = skey[i];
  GS2D_DCHECK(&ctrl->check_bits, t < (uint32_t)n_tiles, kCheckRangeTile);
  (void)n_tiles;
  if (i == 0 || skey[i - 1] != t) ranges[t].x = (uint32_t)i;
  if (i == np - 1 || skey[i + 1] != t) ranges[t].y = (uint32_t)(i + 1);
}

// Depth order of one tile's list: one workgroup per tile (see tile_order.h).
__global__ __launch_bounds__(kBlockThreads) void tile_order_kernel(const uint2* __restrict__ ranges,
                                                                   uint32_t* __restrict__ ids,
                                                                   uint32_t* __restrict__ scratch,
                                                                   const uint32_t* __restrict__ pdk,
                                                                   const uint32_t* __restrict__ dkey) {
  const uint2 rg = ranges[blockIdx.x];
  const int64_t start = rg.x, L = (int64_t)rg.y - (int64_t)rg.x;
  if (L <= 1) return;
  __shared__ __align__(16) uint32_t lds[kOrderScratchWords];
  __shared__ uint32_t sid[kOrderMax];
  (void)order_list(ids, scratch, dkey, start, L, order_lds(lds, sid), true, pdk);
}

inline int blocks_for(int64_t n, int per) { return (int)((n + per - 1) / per) > 0 ? (int)((n + per - 1) / per) : 1; }

void launch_pass(const PassArgs& a, int grid, hipStream_t s) {
  if (a.bits <= 8) {
    radix_offsets_kernel<<<256, kThreads, 0, s>>>(a.hist, a.stride, a.n_dev, a.n_host, const_cast<uint32_t*>(a.dtot));
    radix_scatter_kernel<256><<<grid, kThreads, 0, s>>>(a);
  } else {
    radix_offsets_wave_kernel<<<2048 / kWaves, kThreads, 0, s>>>(a.hist, a.stride, a.n_dev, a.n_host,
                                                                 const_cast<uint32_t*>(a.dtot));
    radix_scatter_kernel<2048><<<grid, kThreads, 0, s>>>(a);
  }
}

// The blends' work queue: tiles by descending list length.  One workgroup: a
// histogram of the lengths over 64 buckets of 32 entries, bucket offsets from the
// longest bucket down, then each tile's slot by an atomic on its bucket's offset.
constexpr int kQueueThreads = 1024;
constexpr int kQueueBuckets = 64;
__device__ inline int queue_bucket(uint2 r) {
  const uint32_t len = r.y - r.x;
  return len >= (uint32_t)(32 * (kQueueBuckets - 1)) ? kQueueBuckets - 1 : (int)((len + 31u) >> 5);
}
__global__ __launch_bounds__(kQueueThreads) void queue_order_kernel(const uint2* __restrict__ ranges, int n_tiles,
                                                                    uint32_t* __restrict__ queue) {
  __shared__ uint32_t hist[kQueueBuckets], off[kQueueBuckets];
  const int t = threadIdx.x;
  if (t < kQueueBuckets) hist[t] = 0u;
  if (t == 0) {
    queue[kQueueHeadFwd] = 0u;
    queue[kQueueHeadBwd] = 0u;
  }
  __syncthreads();
  for (int i = t; i < n_tiles; i += kQueueThreads) atomicAdd(&hist[queue_bucket(ranges[i])], 1u);
  __syncthreads();
  if (t == 0) {
    uint32_t run = 0u;
    for (int b = kQueueBuckets - 1; b >= 0; --b) {
      off[b] = run;
      run += hist[b];
    }
  }
  __syncthreads();
  for (int i = t; i < n_tiles; i += kQueueThreads) {
    const uint32_t pos = atomicAdd(&off[queue_bucket(ranges[i])], 1u);
    queue[kQueueOrder + pos] = (uint32_t)i;
  }
}

}  // namespace

int radix_pass_bits(int bits, int p) {
  const int passes = (bits + kMaxDigitBits - 1) / kMaxDigitBits;
  int shift = 0, pb = 0;
  for (int k = 0; k <= p; ++k) {
    pb = (bits - shift + (passes - k) - 1) / (passes - k);  // split the bits evenly
    shift += pb;
  }
  return pb;
}

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

bool part_scan_needed(int64_t items) { return blocks_for(items, kPartItems) > kDirectParts; }

void launch_part_scan(uint32_t* part_pairs, const uint32_t* part_vis, int64_t items, Ctrl* ctrl, uint32_t* np_host,
                      hipStream_t s) {
  scan_parts_kernel<<<1, kThreads, 0, s>>>(part_pairs, part_vis, blocks_for(items, kPartItems), ctrl, np_host);
}

void launch_duplicate(const SortPlanes& ws, const uint32_t* count, const uint32_t* part_pairs,
                      const uint32_t* part_vis, bool scanned, const uint2* rect, const ViewDesc* views, int n_views,
                      int64_t items, int64_t p_cap, int tile_bits, uint32_t* pkey, uint32_t* pval, Ctrl* ctrl,
                      uint2* ranges, int n_tiles, const uint32_t* dkey, uint32_t* pdk, uint32_t* np_host,
                      hipStream_t s) {
  const int n_parts = blocks_for(items, kPartItems);
  DupArgs a{count,  part_pairs, part_vis, n_parts, scanned ? 1 : 0, rect,   views,   n_views,
            items,  p_cap,      pkey,     pval,    ctrl,            dkey,   pdk,     ranges,
            n_tiles, ws.plane[1], ws.stride, radix_pass_bits(tile_bits, 0), np_host};
  duplicate_kernel<<<n_parts, kThreads, 0, s>>>(a);
}

int tile_sort(const SortPlanes& ws, uint32_t* keys[2], uint32_t* vals[2], uint32_t* dks[2], int64_t p_cap, int bits,
              Ctrl* ctrl, uint2* ranges, int n_tiles, hipStream_t s) {
  const int grid = blocks_for(p_cap, kScanItems);
  const int passes = (bits + kMaxDigitBits - 1) / kMaxDigitBits;
  int cur = 0, shift = 0;
  for (int p = 0; p < passes; ++p) {
    const int pb = radix_pass_bits(bits, p);
    PassArgs a{};
    a.kin = keys[cur];
    a.vin = vals[cur];
    a.kout = keys[cur ^ 1];
    a.vout = vals[cur ^ 1];
    a.din = dks[cur];
    a.dout = dks[cur ^ 1];
    a.n_dev = &ctrl->n_pairs;
    a.n_host = p_cap;
    a.shift = shift;
    a.bits = pb;
    a.hist = ws.plane[(p + 1) & 1];  // the duplication fills plane 1
    a.stride = ws.stride;
    a.dtot = ws.dtot;
    if (p + 1 < passes) {
      a.hnext = ws.plane[p & 1];
      a.nshift = shift + pb;
      a.nbits = radix_pass_bits(bits, p + 1);
    }
    if (passes == 1) {
      a.ranges = ranges;
      a.n_tiles = n_tiles;
      a.overflow = &ctrl->overflow;
      a.check = &ctrl->check_bits;
    }
    launch_pass(a, grid, s);
    cur ^= 1;
    shift += pb;
  }
  return cur;
}

void launch_ranges(const uint32_t* skey, Ctrl* ctrl, int64_t p_cap, uint2* ranges, int n_tiles, hipStream_t s) {
  // the ranges were cleared by the duplicate kernel
  ranges_kernel<<<blocks_for(p_cap, 256), 256, 0, s>>>(skey, ctrl, p_cap, ranges, n_tiles);
}

void launch_queue_order(const uint2* ranges, int n_tiles, uint32_t* queue, hipStream_t s) {
  queue_order_kernel<<<1, kQueueThreads, 0, s>>>(ranges, n_tiles, queue);
}

void launch_tile_order(const uint2* ranges, int n_tiles, uint32_t* ids, uint32_t* scratch, const uint32_t* pdk,
                       const uint32_t* dkey, hipStream_t s) {
  if (n_tiles <= 0) return;
  tile_order_kernel<<<n_tiles, kThreads, 0, s>>>(ranges, ids, scratch, pdk, dkey);
}

}  // namespace gs2d
