// Binning: the scan + emission of tile instances and the tile ranges (the
// radix sort itself is in radix.hip; the gather of records into sorted order
// happens batch by batch inside the composite).
//
// Front-to-back order inside each tile (Sec. 3: splats sorted by depth) is
// obtained in two sorts instead of one wide one:
//   1. the projected slots are sorted by their float32 depth bits (stable,
//      so equal depths keep ascending Gaussian index);
//   2. instances are emitted in that order and sorted stably by global tile.
// The result is ordered by (tile, depth bits, Gaussian index), the same as a
// single sort on the 64-bit key (tile << 32 | depth bits) with ties by index,
// while moving 32-bit keys over fewer bits.
//
#include "nxs_internal.h"

#include <algorithm>

namespace nxs {

namespace {


// Block-wide exclusive scan of one value per thread (256 threads).
template <int NW = 4>   // waves in the work-group
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t* s_tmp,
                                                         uint32_t* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t incl = wave_inclusive_scan_u32(x);
  if (lane == 63) s_tmp[wid] = incl;
  __syncthreads();
  uint32_t wave_off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    uint32_t v = s_tmp[w];
    if (w < wid) wave_off += v;
    tot += v;
  }
  __syncthreads();
  *total = tot;
  return wave_off + incl - x;
}

// ---------------------------------------------------------------- scan + emit

constexpr int kScanBlock = 256;
constexpr int kScanItems = 2;
constexpr int kScanChunk = kScanBlock * kScanItems;

// Block-local exclusive scan of the slots' tile counts: nt_sorted in
// depth-sorted order, or (nt_sorted null) the counts in the projection's
// rectangles, in slot order.
__global__ __launch_bounds__(kScanBlock) void scan_local_kernel(
    const uint32_t* __restrict__ nt_sorted, const uint2* __restrict__ trect, int64_t n,
    uint32_t* __restrict__ local, uint32_t* __restrict__ block_sums) {
  __shared__ uint32_t s_tmp[kScanBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + threadIdx.x * kScanItems;
  uint32_t v[kScanItems], sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + k;
    v[k] = i < n ? (nt_sorted ? nt_sorted[i] : rect_tile_count(trect[i])) : 0u;
    sum += v[k];
  }
  uint32_t tot;
  uint32_t ex = block_exclusive_scan(sum, s_tmp, &tot);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + k;
    if (i < n) local[i] = ex;
    ex += v[k];
  }
  if (threadIdx.x == 0) {
    block_sums[blockIdx.x] = tot;                 // scanned later if needed
    block_sums[gridDim.x + blockIdx.x] = tot;     // kept as is
  }
}

// Single work-group exclusive scan of the block sums (in place): 1,024
// threads of 16 consecutive sums each, so that 16,384 sums take one round of
// loads, one scan and one round of stores (93,750 block sums of a 48M-slot
// batch: 6 rounds; with 256 threads of 4 sums, 92 rounds took 91 us).
constexpr int kSumThreads = 1024;
constexpr int kSumItems = 16;
__global__ __launch_bounds__(kSumThreads) void scan_blocks_kernel(uint32_t* __restrict__ sums,
                                                                  int nblocks) {
  __shared__ uint32_t s_tmp[kSumThreads / 64];
  uint32_t running = 0;
  for (int b = 0; b < nblocks; b += kSumThreads * kSumItems) {
    uint32_t v[kSumItems], sum = 0;
#pragma unroll
    for (int k = 0; k < kSumItems; ++k) {
      const int idx = b + threadIdx.x * kSumItems + k;
      v[k] = idx < nblocks ? sums[idx] : 0u;
      sum += v[k];
    }
    uint32_t tot;
    uint32_t ex = block_exclusive_scan<kSumThreads / 64>(sum, s_tmp, &tot) + running;
#pragma unroll
    for (int k = 0; k < kSumItems; ++k) {
      const int idx = b + threadIdx.x * kSumItems + k;
      if (idx < nblocks) sums[idx] = ex;
      ex += v[k];
    }
    running += tot;
  }
}

// One work-group per 512 sorted slots writes all of their instances as one
// contiguous run, consecutive threads at consecutive addresses however
// unevenly the Gaussians' tile counts are spread: the run is taken in windows
// of kEmitWindow positions, each slot first marks the positions of its
// instances in the window with its index (an owner map in LDS), then each
// position is written from its owner's record.
// Blocks up to this count find their output offset by summing the totals of
// the blocks before them (no separate scan launch); beyond it the totals are
// scanned by scan_blocks_kernel first.
constexpr int kInlineBlocks = 2048;
constexpr uint32_t kEmitWindow = 4096;   // positions per owner map (8 KB)
constexpr uint32_t kEmitShort = 32;      // longer runs are marked by a whole wave

// sorted_slots null: the slots in their own order, rectangles from trect.
__global__ __launch_bounds__(kScanBlock) void emit_kernel(
    const uint32_t* __restrict__ sorted_slots, const uint2* __restrict__ rect_sorted,
    const uint2* __restrict__ trect, int64_t n,
    int32_t n_gauss, int n_views, const ViewDev* __restrict__ views,
    const uint32_t* __restrict__ local, const uint32_t* __restrict__ block_sums, int nblocks,
    uint32_t capacity, uint32_t* __restrict__ inst_tile, uint32_t* __restrict__ inst_val) {
  __shared__ uint32_t s_off[kScanChunk + 1];
  __shared__ uint32_t s_slot[kScanChunk];
  __shared__ uint32_t s_tile0[kScanChunk];   // global tile of the rectangle's first tile
  __shared__ uint32_t s_geom[kScanChunk];    // width | tiles_x << 16
  __shared__ uint32_t s_tmp[kScanBlock / 64];
  __shared__ uint16_t s_owner[kEmitWindow];   // block-local slot of each position
  const int64_t b0 = (int64_t)blockIdx.x * kScanChunk;
  const int cnt = (int)min((int64_t)kScanChunk, n - b0);
  // This block's output offset: with the inline sum (many loads and a block
  // scan) before the slots' loads, else after them (measured both ways: the
  // 1080p frame's 1,954 blocks 20.9 against 21.8 us with the sum first; the
  // eight 720p views' 7,813 pre-scanned blocks 149 against 154 us with the
  // loads first).
  const bool inline_sum = nblocks <= kInlineBlocks;
  uint32_t out0 = 0, out1 = 0;
  auto block_offset = [&]() {
    if (inline_sum) {
      // the sum of the totals of the blocks before this one (all of a
      // thread's loads issued before the first is added)
      constexpr int kInlinePerT = kInlineBlocks / kScanBlock;
      static_assert(kInlineBlocks % kScanBlock == 0, "whole rounds of block totals");
      uint32_t v[kInlinePerT];
#pragma unroll
      for (int q = 0; q < kInlinePerT; ++q) {
        const int b = q * kScanBlock + threadIdx.x;
        v[q] = b < (int)blockIdx.x ? block_sums[b] : 0u;
      }
      uint32_t part = 0;
#pragma unroll
      for (int q = 0; q < kInlinePerT; ++q) part += v[q];
      uint32_t all;
      (void)block_exclusive_scan(part, s_tmp, &all);
      out0 = all;
      out1 = out0 + block_sums[blockIdx.x];
    } else {
      out0 = block_sums[blockIdx.x];   // scanned in place
      out1 = out0 + block_sums[nblocks + blockIdx.x];
    }
  };
  if (inline_sum) block_offset();
  // the slots' loads (all independent), then the LDS tables
  constexpr int kPerT = kScanChunk / kScanBlock;
  uint32_t slot_r[kPerT], off_r[kPerT];
  uint2 rect_r[kPerT];
#pragma unroll
  for (int q = 0; q < kPerT; ++q) {
    const int k = q * kScanBlock + threadIdx.x;
    slot_r[q] = k < cnt ? (sorted_slots ? sorted_slots[b0 + k] : (uint32_t)(b0 + k)) : 0u;
    off_r[q] = k < cnt ? local[b0 + k] : 0u;
  }
#pragma unroll
  for (int q = 0; q < kPerT; ++q) {
    const int k = q * kScanBlock + threadIdx.x;
    if (k >= cnt) {
      rect_r[q] = make_uint2(0xFFFFFFFFu, 0xFFFFFFFFu);
    } else if (sorted_slots) {
      rect_r[q] = rect_sorted[b0 + k];
    } else {
      rect_r[q] = trect[b0 + k];
    }
  }
  if (!inline_sum) block_offset();
#pragma unroll
  for (int q = 0; q < kPerT; ++q) {
    const int k = q * kScanBlock + threadIdx.x;
    if (k >= cnt) continue;
    s_slot[k] = slot_r[q];
    s_off[k] = off_r[q];
    const uint2 r = rect_r[q];
    if (r.x != 0xFFFFFFFFu) {
      const uint32_t vi = n_views == 1 ? 0u : slot_r[q] / (uint32_t)n_gauss;
      const uint32_t tile_off = (uint32_t)views[vi].tile_off;
      const uint32_t tiles_x = (uint32_t)views[vi].tiles_x;
      const uint32_t tx0 = r.x & 0xFFFF, tx1 = r.x >> 16, ty0 = r.y & 0xFFFF;
      s_tile0[k] = tile_off + ty0 * tiles_x + tx0;
      s_geom[k] = (tx1 - tx0 + 1) | (tiles_x << 16);
    } else {
      s_tile0[k] = 0;
      s_geom[k] = 1;
    }
  }
  __syncthreads();
  const uint32_t tot = out1 - out0;
  // slot k owns positions [s_off[k], s_off[k + 1]) (the last one: up to tot)
  const int lane = threadIdx.x & 63;
  uint32_t end_r[kPerT];
#pragma unroll
  for (int q = 0; q < kPerT; ++q) {
    const int k = q * kScanBlock + threadIdx.x;
    end_r[q] = k + 1 < cnt ? s_off[k + 1] : (k < cnt ? tot : off_r[q]);
  }
  for (uint32_t w0 = 0; w0 < tot; w0 += kEmitWindow) {
    const uint32_t w1 = min(tot, w0 + kEmitWindow);
    // a short run is marked by its slot's thread, a long one by the whole
    // wave (the slot's lane broadcasts its bounds)
#pragma unroll
    for (int q = 0; q < kPerT; ++q) {
      const int k = q * kScanBlock + threadIdx.x;
      const uint32_t a = off_r[q], e = end_r[q];
      const bool longrun = e - a > kEmitShort;
      if (!longrun)
        for (uint32_t j = max(a, w0); j < min(e, w1); ++j) s_owner[j - w0] = (uint16_t)k;
      uint64_t runs = __ballot(longrun);
      while (runs) {
        const int b = __builtin_ctzll(runs);
        runs &= runs - 1;
        // (b is the same on every lane: the bounds come by readlane)
        const uint32_t ba = (uint32_t)__builtin_amdgcn_readlane((int)a, b);
        const uint32_t be = (uint32_t)__builtin_amdgcn_readlane((int)e, b);
        const uint16_t bk = (uint16_t)(k - lane + b);
        for (uint32_t j = max(ba, w0) + lane; j < min(be, w1); j += 64) s_owner[j - w0] = bk;
      }
    }
    __syncthreads();
    for (uint32_t q = w0 + threadIdx.x; q < w1; q += kScanBlock) {
      const int k = s_owner[q - w0];
      const uint32_t geom = s_geom[k];
      const uint32_t w = geom & 0xFFFF, tiles_x = geom >> 16;
      const uint32_t l = q - s_off[k];
      // row = l / w in float (exact for l < 2^24 after the +-1 fix-up)
      uint32_t row = (uint32_t)((float)l * __frcp_rn((float)w));
      if (row * w > l) --row;
      if ((row + 1) * w <= l) ++row;
      if (out0 + q < capacity) {
        inst_tile[out0 + q] = s_tile0[k] + row * tiles_x + (l - row * w);
        inst_val[out0 + q] = s_slot[k];
      }
    }
    __syncthreads();   // the next window's marks overwrite this one's
  }
}

// ----------------------------------------------------------------- ranges

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, int64_t n, uint32_t value) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

// Entry j starts its tile's range if the entry before it has another tile,
// and ends it if the entry after it has another tile.  A thread takes
// kRangeItems consecutive entries (16-byte loads) and their two neighbours;
// eight per thread keep the 1080p frame's 2.69M entries within one round of
// resident work-groups.
constexpr int kRangeItems = 8;
static_assert(kRangeItems % 4 == 0, "whole 16-byte loads");

__global__ __launch_bounds__(256) void ranges_kernel(const uint32_t* __restrict__ inst_tile,
                                                     int64_t m, uint2* __restrict__ ranges,
                                                     const Counters* __restrict__ dn) {
  if (dn) m = min(m, live_count(dn));
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * kRangeItems;
  for (int64_t j0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kRangeItems; j0 < m;
       j0 += stride) {
    uint32_t t[kRangeItems];
    if (j0 + kRangeItems <= m) {
#pragma unroll
      for (int h = 0; h < kRangeItems / 4; ++h) {
        const uint4 q = *reinterpret_cast<const uint4*>(inst_tile + j0 + 4 * h);   // (j0 % 4 == 0)
        t[4 * h + 0] = q.x;
        t[4 * h + 1] = q.y;
        t[4 * h + 2] = q.z;
        t[4 * h + 3] = q.w;
      }
    } else {
#pragma unroll
      for (int k = 0; k < kRangeItems; ++k) t[k] = j0 + k < m ? inst_tile[j0 + k] : 0u;
    }
    // (no tile is ~0: the neighbour outside the list never matches)
    const uint32_t prev = j0 > 0 ? inst_tile[j0 - 1] : ~0u;
    const uint32_t next = j0 + kRangeItems < m ? inst_tile[j0 + kRangeItems] : ~0u;
#pragma unroll
    for (int k = 0; k < kRangeItems; ++k) {
      const int64_t j = j0 + k;
      if (j >= m) break;
      const uint32_t before = k == 0 ? prev : t[k - 1];
      const uint32_t after = j == m - 1 ? ~0u : (k == kRangeItems - 1 ? next : t[k + 1]);
      if (before != t[k]) ranges[t[k]].x = (uint32_t)j;
      if (after != t[k]) ranges[t[k]].y = (uint32_t)(j + 1);
    }
  }
}

}  // namespace

size_t scan_blocks_size(int64_t n) {
  return 2 * (size_t)((n + kScanChunk - 1) / kScanChunk) + 1;
}

void launch_emit_scan(const uint32_t* nt_sorted, const uint2* trect, int64_t n_slots,
                      uint32_t* scan_local, uint32_t* block_sums, hipStream_t s) {
  if (n_slots <= 0) return;
  const int nblocks = (int)((n_slots + kScanChunk - 1) / kScanChunk);
  hipLaunchKernelGGL(scan_local_kernel, dim3(nblocks), dim3(kScanBlock), 0, s, nt_sorted, trect,
                     n_slots, scan_local, block_sums);
  if (nblocks > kInlineBlocks)
    hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(kSumThreads), 0, s, block_sums,
                       nblocks);
}

void launch_emit_write(const uint32_t* sorted_slots, const uint2* rect_sorted,
                       const uint2* trect, int64_t n_slots, int32_t n_gauss,
                       const ViewDev* views, const uint32_t* scan_local,
                       const uint32_t* block_sums, uint32_t capacity, uint32_t* inst_tile,
                       uint32_t* inst_val, hipStream_t s) {
  if (n_slots <= 0) return;
  const int nblocks = (int)((n_slots + kScanChunk - 1) / kScanChunk);
  const int n_views = (int)(n_slots / n_gauss);
  hipLaunchKernelGGL(emit_kernel, dim3(nblocks), dim3(kScanBlock), 0, s, sorted_slots,
                     rect_sorted, trect, n_slots, n_gauss, n_views, views, scan_local,
                     block_sums, nblocks, capacity, inst_tile, inst_val);
}

void launch_fill_u32(uint32_t* p, int64_t n, uint32_t value, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     p, n, value);
}

void launch_ranges(const uint32_t* inst_tile, int64_t m, uint2* ranges, hipStream_t s,
                   const Counters* dn, int64_t m_plan) {
  if (m <= 0) return;
  const int64_t g = dn && m_plan > 0 ? std::min(m_plan, m) : m;
  const int64_t per_group = 256 * kRangeItems;
  hipLaunchKernelGGL(ranges_kernel, dim3((unsigned)((g + per_group - 1) / per_group)), dim3(256),
                     0, s, inst_tile, m, ranges, dn);
}

}  // namespace nxs
