// Block-level building blocks of the sorts, and the depth order of one tile's list.
//
// The per-pixel lists of the paper's blending (Sec. "2D Gaussian Splatting",
// eq:alpha_blending) ascend in (float32 camera depth, item).  A tile's list arrives
// in ascending item order (the pairs are emitted in item order and sorted stably by
// tile), so a stable sort by depth key alone gives that order.  One 256-thread
// workgroup orders one list:
//   up to 512 entries  each entry's slot is counted directly against the others: the
//                      entries whose (depth key, item) is smaller, as one 64-bit key;
//   up to kOrderMax    a stable LSD radix sort in LDS and registers, four passes of
//                      8 bits, each a counting pass (histogram, digit offsets, ranked
//                      rounds of 256); a digit that every entry shares is skipped;
//   longer lists       the same passes through global memory, alternating between the
//                      list and a scratch buffer (four passes end in the list).
#ifndef GS2D_TILE_ORDER_H
#define GS2D_TILE_ORDER_H

#include "gs2d_internal.h"

namespace gs2d {

constexpr int kBlockThreads = 256;  // workgroup size of the sort kernels and of the ordering
constexpr int kBlockWaves = kBlockThreads / 64;
constexpr int kOrderBits = 8;
constexpr int kOrderBins = 1 << kOrderBits;
constexpr int kOrderMax = 2048;  // lists up to this length are ordered in LDS
constexpr int kOrderCounted = 2 * kBlockThreads;  // lists up to this length are ranked by counting
constexpr int kOrderRounds = kOrderMax / kBlockThreads;
// LDS words of the ordering's scratch, besides the ordered list itself: keys, per-wave
// digit counts, digit offsets, histogram and the block scan's wave totals
constexpr int kOrderScratchWords = kOrderMax + kBlockWaves * kOrderBins + 2 * kOrderBins + kBlockWaves;

// Exclusive scan over the 256 threads of a block: a scan within each wave, then the
// totals of the lower waves (sh: kBlockWaves words of LDS).  *total = the block's sum.
// Every thread of the block must call it.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
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
  for (int w = 0; w < kBlockWaves; ++w) {
    const uint32_t sw = sh[w];
    below += w < wave ? sw : 0u;
    all += sw;
  }
  __syncthreads();
  if (total) *total = all;
  return below + x - v;
}

// Slot of each key of one round of up to 256 keys in a stable counting pass (every
// thread of the block calls it).  digit: the key's digit (< R); valid: the lane holds
// a key; doff[d]: the next free slot of digit d (advanced here); wcnt[w * R + d]:
// per-wave digit counts, stamped with the round (stamp = round << 16, never 0) so that
// stale entries need no clearing.
template <int R>
__device__ inline uint32_t rank_round(uint32_t digit, bool valid, int bits, uint32_t stamp, uint32_t* wcnt,
                                      uint32_t* doff) {
  const int t = threadIdx.x, wave = t / 64, lane = t % 64;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint64_t peers = __ballot(valid);
  for (int b = 0; b < bits; ++b) {
    const bool set = (digit >> b) & 1u;
    const uint64_t bal = __ballot(valid && set);
    peers &= set ? bal : ~bal;
  }
  const uint32_t rank = (uint32_t)__popcll(peers & lt);
  const uint32_t cnt = (uint32_t)__popcll(peers);
  const bool leader = valid && rank == 0;
  if (leader) wcnt[wave * R + digit] = stamp | cnt;
  __syncthreads();
  // the group's first slot: the digit's running offset plus the same digit's keys
  // in the lower waves of this round
  uint32_t pb = 0;
  if (leader) {
    pb = doff[digit];
    for (int w = 0; w < wave; ++w) {
      const uint32_t e = wcnt[w * R + digit];
      if ((e & 0xFFFF0000u) == stamp) pb += e & 0xFFFFu;
    }
  }
  __syncthreads();
  if (leader) atomicAdd(&doff[digit], cnt);
  const int src = peers ? (int)__ffsll((long long)peers) - 1 : lane;
  return (uint32_t)__shfl((int)pb, src, 64) + rank;
}

// LDS of one ordering: `scratch` holds kOrderScratchWords words (16-byte aligned),
// `sid` kOrderMax words (the ordered list, when it fits).
struct OrderLds {
  uint32_t* skey;
  uint32_t* sid;
  uint32_t* wcnt;
  uint32_t* doff;
  uint32_t* hcnt;
  uint32_t* sh;
};
__device__ inline OrderLds order_lds(uint32_t* scratch, uint32_t* sid) {
  OrderLds m;
  m.skey = scratch;
  m.wcnt = scratch + kOrderMax;
  m.doff = m.wcnt + kBlockWaves * kOrderBins;
  m.hcnt = m.doff + kOrderBins;
  m.sh = m.hcnt + kOrderBins;
  m.sid = sid;
  return m;
}

// Orders ids[start .. start + L) (ascending on entry) by (dkey[id], id), that is
// stably by dkey[id]; every thread of the 256-thread block calls it.  pkeys (nullable):
// the same keys stored beside the ids, pkeys[start + e] = dkey[ids[start + e]], read
// instead of gathering through the ids (not by the global-memory path, which permutes
// the ids).  Lists of up to kOrderMax entries end in m.sid[0 .. L) (and, with
// write_back, in ids as well) and the call returns true; longer lists are ordered in ids
// (scratch: a buffer of the same size) and the call returns false.  Ends with a block
// barrier: the scratch may be reused at once.
__device__ inline bool order_list(uint32_t* __restrict__ ids, uint32_t* __restrict__ scratch,
                                  const uint32_t* __restrict__ dkey, int64_t start, int64_t L, const OrderLds& m,
                                  bool write_back, const uint32_t* __restrict__ pkeys = nullptr) {
  constexpr int RB = kOrderBins;
  const int t = threadIdx.x;
  if (L <= kOrderCounted) {
    // up to two entries per thread, ranked by counting the entries whose (key, id),
    // one 64-bit key, is smaller (ids within a list are distinct; slots past the end
    // read as 2^64 - 1, above every entry)
    static_assert(kOrderCounted * 2 <= kOrderMax, "the 64-bit keys fit the key scratch");
    uint64_t* k64 = reinterpret_cast<uint64_t*>(m.skey);
    const bool v0 = t < L, v1 = t + kBlockThreads < L;
    const uint32_t id0 = v0 ? ids[start + t] : 0u;
    const uint32_t id1 = v1 ? ids[start + t + kBlockThreads] : 0u;
    const uint32_t dk0 = v0 ? (pkeys ? pkeys[start + t] : dkey[id0]) : 0u;
    const uint32_t dk1 = v1 ? (pkeys ? pkeys[start + t + kBlockThreads] : dkey[id1]) : 0u;
    const uint64_t key0 = v0 ? ((uint64_t)dk0 << 32) | id0 : ~0ull;
    const uint64_t key1 = v1 ? ((uint64_t)dk1 << 32) | id1 : ~0ull;
    k64[t] = key0;
    k64[t + kBlockThreads] = key1;
    __syncthreads();
    // 16 keys per trip (every slot below 512 holds a key or 2^64 - 1), the eight LDS
    // reads of a trip issued before its compares: the loop is bound by LDS latency
    constexpr int kTrip = 16;
    const int n16 = (int)((L + kTrip - 1) & ~(int64_t)(kTrip - 1));
    uint32_t r0 = 0, r1 = 0;
    if (L <= kBlockThreads) {
      for (int j = 0; j < n16; j += kTrip) {
        ulonglong2 q[kTrip / 2];
#pragma unroll
        for (int u = 0; u < kTrip / 2; ++u) q[u] = *reinterpret_cast<const ulonglong2*>(&k64[j + 2 * u]);
#pragma unroll
        for (int u = 0; u < kTrip / 2; ++u) r0 += (q[u].x < key0) + (q[u].y < key0);
      }
    } else {
      for (int j = 0; j < n16; j += kTrip) {
        ulonglong2 q[kTrip / 2];
#pragma unroll
        for (int u = 0; u < kTrip / 2; ++u) q[u] = *reinterpret_cast<const ulonglong2*>(&k64[j + 2 * u]);
#pragma unroll
        for (int u = 0; u < kTrip / 2; ++u) {
          r0 += (q[u].x < key0) + (q[u].y < key0);
          r1 += (q[u].x < key1) + (q[u].y < key1);
        }
      }
    }
    if (v0) {
      m.sid[r0] = id0;
      if (write_back) ids[start + r0] = id0;
    }
    if (v1) {
      m.sid[r1] = id1;
      if (write_back) ids[start + r1] = id1;
    }
    __syncthreads();
    return true;
  }
  for (int k = t; k < kBlockWaves * RB; k += kBlockThreads) m.wcnt[k] = 0u;
  uint32_t stamp = 0;  // round counter across the whole sort: stamps never repeat
  if (L <= kOrderMax) {
    const int nr = (int)((L + kBlockThreads - 1) / kBlockThreads);
    uint32_t key[kOrderRounds], id[kOrderRounds];
#pragma unroll
    for (int r = 0; r < kOrderRounds; ++r) {
      const int e = r * kBlockThreads + t;
      id[r] = e < L ? ids[start + e] : 0u;
      key[r] = e < L ? (pkeys ? pkeys[start + e] : dkey[id[r]]) : 0u;
    }
    for (int p = 0; p < 32 / kOrderBits; ++p) {
      const int shift = p * kOrderBits;
      m.hcnt[t] = 0u;
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kOrderRounds; ++r)
        if (r * kBlockThreads + t < L) atomicAdd(&m.hcnt[(key[r] >> shift) & (RB - 1)], 1u);
      __syncthreads();
      const uint32_t h = m.hcnt[t];
      // a digit that every entry shares leaves the order as it is
      const bool uniform = __syncthreads_or(h == (uint32_t)L) != 0;
      if (uniform) continue;
      m.doff[t] = block_exclusive_scan(h, m.sh, nullptr);
      __syncthreads();
      uint32_t pos[kOrderRounds];
#pragma unroll
      for (int r = 0; r < kOrderRounds; ++r) {
        if (r < nr) {
          const bool valid = r * kBlockThreads + t < L;
          const uint32_t digit = valid ? (key[r] >> shift) & (RB - 1) : 0u;
          stamp += 1u << 16;
          pos[r] = rank_round<RB>(digit, valid, kOrderBits, stamp, m.wcnt, m.doff);
        }
      }
#pragma unroll
      for (int r = 0; r < kOrderRounds; ++r) {
        if (r * kBlockThreads + t < L) {
          m.skey[pos[r]] = key[r];
          m.sid[pos[r]] = id[r];
        }
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kOrderRounds; ++r) {
        const int e = r * kBlockThreads + t;
        if (e < L) {
          key[r] = m.skey[e];
          id[r] = m.sid[e];
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < kOrderRounds; ++r) {
      const int e = r * kBlockThreads + t;
      if (e < L) {
        m.sid[e] = id[r];
        if (write_back) ids[start + e] = id[r];
      }
    }
    __syncthreads();
    return true;
  }
  // long lists: the same passes through global memory, chunk by chunk
  for (int p = 0; p < 32 / kOrderBits; ++p) {
    const int shift = p * kOrderBits;
    const uint32_t* __restrict__ src = (p & 1) ? scratch : ids;
    uint32_t* __restrict__ dst = (p & 1) ? ids : scratch;
    m.hcnt[t] = 0u;
    __syncthreads();
    for (int64_t e = t; e < L; e += kBlockThreads) atomicAdd(&m.hcnt[(dkey[src[start + e]] >> shift) & (RB - 1)], 1u);
    __syncthreads();
    m.doff[t] = block_exclusive_scan(m.hcnt[t], m.sh, nullptr);
    __syncthreads();
    for (int64_t e0 = 0; e0 < L; e0 += kBlockThreads) {
      if ((stamp >> 16) == 0xFFFFu) {  // stamps used up: clear the counts and start again
        __syncthreads();
        for (int k = t; k < kBlockWaves * RB; k += kBlockThreads) m.wcnt[k] = 0u;
        __syncthreads();
        stamp = 0;
      }
      const int64_t e = e0 + t;
      const bool valid = e < L;
      const uint32_t v = valid ? src[start + e] : 0u;
      const uint32_t digit = valid ? (dkey[v] >> shift) & (RB - 1) : 0u;
      stamp += 1u << 16;
      const uint32_t pos = rank_round<RB>(digit, valid, kOrderBits, stamp, m.wcnt, m.doff);
      if (valid) dst[start + pos] = v;
    }
    __syncthreads();
  }
  return false;
}

}  // namespace gs2d

#endif  // GS2D_TILE_ORDER_H
