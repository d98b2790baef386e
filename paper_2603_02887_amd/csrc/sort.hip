// Binning: the scan + emission of tile instances, tile ranges and the gather
// of the composite records into sorted order (the radix sort itself is in
// radix.hip).
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
#include <hip/hip_fp16.h>

#include "nxs_internal.h"

namespace nxs {

namespace {

constexpr uint32_t kXcds = 8;   // accelerator complex dies of an MI355X

// Block-wide exclusive scan of one value per thread (256 threads).
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t* s_tmp,
                                                         uint32_t* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t incl = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) s_tmp[wid] = incl;
  __syncthreads();
  uint32_t wave_off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
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
constexpr int kScanItems = 4;
constexpr int kScanChunk = kScanBlock * kScanItems;

// Block-local exclusive scan of ntiles in sorted-slot order.
__global__ __launch_bounds__(kScanBlock) void scan_local_kernel(
    const uint32_t* __restrict__ nt_sorted, int64_t n, uint32_t* __restrict__ local,
    uint32_t* __restrict__ block_sums) {
  __shared__ uint32_t s_tmp[kScanBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + threadIdx.x * kScanItems;
  uint32_t v[kScanItems], sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + k;
    v[k] = i < n ? nt_sorted[i] : 0u;
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

// Single work-group exclusive scan of the block sums (in place).
__global__ __launch_bounds__(kScanBlock) void scan_blocks_kernel(uint32_t* __restrict__ sums,
                                                                 int nblocks) {
  __shared__ uint32_t s_tmp[kScanBlock / 64];
  uint32_t running = 0;
  for (int b = 0; b < nblocks; b += kScanBlock * 4) {
    uint32_t v[4], sum = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int idx = b + threadIdx.x * 4 + k;
      v[k] = idx < nblocks ? sums[idx] : 0u;
      sum += v[k];
    }
    uint32_t tot;
    uint32_t ex = block_exclusive_scan(sum, s_tmp, &tot) + running;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int idx = b + threadIdx.x * 4 + k;
      if (idx < nblocks) sums[idx] = ex;
      ex += v[k];
    }
    running += tot;
  }
}

// One work-group per 1024 sorted slots writes all of their instances as one
// contiguous run: each output position finds its slot by binary search over
// the block's offsets in LDS, so consecutive threads write consecutive
// addresses however unevenly the Gaussians' tile counts are spread.
// Blocks up to this count find their output offset by summing the totals of
// the blocks before them (no separate scan launch); beyond it the totals are
// scanned by scan_blocks_kernel first.
constexpr int kInlineBlocks = 2048;

__global__ __launch_bounds__(kScanBlock) void emit_kernel(
    const uint32_t* __restrict__ sorted_slots, const uint2* __restrict__ rect_sorted, int64_t n,
    int32_t n_gauss, int n_views, const ViewDev* __restrict__ views,
    const uint32_t* __restrict__ local, const uint32_t* __restrict__ block_sums, int nblocks,
    uint32_t capacity, uint32_t* __restrict__ inst_tile, uint32_t* __restrict__ inst_val) {
  __shared__ uint32_t s_off[kScanChunk + 1];
  __shared__ uint32_t s_slot[kScanChunk];
  __shared__ uint32_t s_tile0[kScanChunk];   // global tile of the rectangle's first tile
  __shared__ uint32_t s_geom[kScanChunk];    // width | tiles_x << 16
  __shared__ uint32_t s_tmp[kScanBlock / 64];
  const int64_t b0 = (int64_t)blockIdx.x * kScanChunk;
  const int cnt = (int)min((int64_t)kScanChunk, n - b0);
  uint32_t out0;
  if (nblocks <= kInlineBlocks) {
    // the sum of the totals of the blocks before this one
    uint32_t part = 0;
    for (int b = threadIdx.x; b < (int)blockIdx.x; b += kScanBlock) part += block_sums[b];
    uint32_t all;
    (void)block_exclusive_scan(part, s_tmp, &all);
    out0 = all;
  } else {
    out0 = block_sums[blockIdx.x];   // scanned in place
  }
  const uint32_t out1 = out0 + (nblocks <= kInlineBlocks ? block_sums[blockIdx.x]
                                                         : block_sums[nblocks + blockIdx.x]);
  // loads first (all independent), then the LDS tables
  constexpr int kPerT = kScanChunk / kScanBlock;
  uint32_t slot_r[kPerT], off_r[kPerT];
  uint2 rect_r[kPerT];
#pragma unroll
  for (int q = 0; q < kPerT; ++q) {
    const int k = q * kScanBlock + threadIdx.x;
    slot_r[q] = k < cnt ? sorted_slots[b0 + k] : 0u;
    off_r[q] = k < cnt ? local[b0 + k] : 0u;
  }
#pragma unroll
  for (int q = 0; q < kPerT; ++q) {
    const int k = q * kScanBlock + threadIdx.x;
    rect_r[q] = k < cnt ? rect_sorted[b0 + k] : make_uint2(0xFFFFFFFFu, 0xFFFFFFFFu);
  }
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
  for (uint32_t q = threadIdx.x; q < tot; q += kScanBlock) {
    int lo = 0, hi = cnt - 1;   // last slot whose offset is <= q (it has q inside)
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_off[mid] <= q) lo = mid; else hi = mid - 1;
    }
    const uint32_t geom = s_geom[lo];
    const uint32_t w = geom & 0xFFFF, tiles_x = geom >> 16;
    const uint32_t l = q - s_off[lo];
    // row = l / w in float (exact for l < 2^24 after the +-1 fix-up)
    uint32_t row = (uint32_t)((float)l * __frcp_rn((float)w));
    if (row * w > l) --row;
    if ((row + 1) * w <= l) ++row;
    if (out0 + q < capacity) {
      inst_tile[out0 + q] = s_tile0[lo] + row * tiles_x + (l - row * w);
      inst_val[out0 + q] = s_slot[lo];
    }
  }
}

// ----------------------------------------------------- ranges + gather


__global__ void fill_u32_kernel(uint32_t* __restrict__ p, int64_t n, uint32_t value) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

__device__ __forceinline__ int view_of_tile(const ViewDev* views, int n_views, uint32_t tile) {
  int lo = 0, hi = n_views - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((uint32_t)views[mid].tile_off <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(256) void ranges_gather_kernel(
    const uint32_t* __restrict__ inst_tile, const uint32_t* __restrict__ inst_val,
    int64_t m, ProjDev proj, const ViewDev* __restrict__ views, int n_views, int tile_w,
    int tile_h, float log2_alpha_min, uint2* __restrict__ ranges,
    float4* __restrict__ crec, uint32_t per_xcd) {
  // Work-groups go to the 8 XCDs round-robin; give each XCD one contiguous
  // eighth of the sorted list (a band of tile rows), so that the records of
  // Gaussians shared by neighbouring tiles are re-read from that XCD's L2.
  const uint32_t lb = (blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
  const int64_t j = (int64_t)lb * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const uint32_t tile = inst_tile[j];
  if (j == 0 || inst_tile[j - 1] != tile) ranges[tile].x = (uint32_t)j;
  if (j == m - 1 || inst_tile[j + 1] != tile) ranges[tile].y = (uint32_t)(j + 1);
  const uint32_t slot = inst_val[j];
  const int vi = view_of_tile(views, n_views, tile);
  const ViewDev& v = views[vi];
  const int lt = (int)(tile - (uint32_t)v.tile_off);
  const int tx = lt % v.tiles_x, ty = lt / v.tiles_x;
  const float4 r0 = proj.rec[3 * (int64_t)slot + 0];
  const float4 r1 = proj.rec[3 * (int64_t)slot + 1];
  const float4 r2 = proj.rec[3 * (int64_t)slot + 2];
  // centre relative to the tile corner: (hi - corner) is exact, then + lo
  const float du = (r0.x - (float)(tx * tile_w)) + r0.y;
  const float dv = (r0.z - (float)(ty * tile_h)) + r0.w;
  // half-extents of the alpha >= alpha_min box, packed as two fp16 (rounded up)
  const uint32_t hx = __float_as_uint(r2.w);
  const float rx = __half2float(__ushort_as_half((unsigned short)(hx & 0xFFFFu)));
  const float ry = __half2float(__ushort_as_half((unsigned short)(hx >> 16)));
  // which 8x8 pixel blocks of the tile (bit by * (tile_w / 8) + bx) the
  // footprint reaches, judged at pixel centres; the composite's waves skip the
  // others.  A block passes the box test, then the exact one: the largest
  // exponent e = lo + A' dx^2 + B' dx dy + C' dy^2 over the rectangle spanned
  // by its pixel centres must reach log2(alpha_min) (with a margin of 2e-3 in
  // log2 units, so float32 rounding here can only keep a block, never drop one
  // that some pixel needs).
  const float qa = -r1.x, qb = -r1.y, qc = -r1.z;    // Q = -(e - lo) >= 0
  const float qlim = r1.w - log2_alpha_min + 2e-3f;  // e >= log2(alpha_min) <=> Q <= qlim
  const float ia = 0.5f / qa, ic = 0.5f / qc;
  uint32_t mask = 0;
  const int nbx = tile_w >> 3, nby = tile_h >> 3;
  for (int by = 0; by < nby; ++by) {
    const float y0 = (float)(8 * by) + 0.5f, y1 = (float)(8 * by) + 7.5f;
    if (dv - ry > y1 || dv + ry < y0) continue;
    const float ylo = y0 - dv, yhi = y1 - dv;          // dy range over the block
    for (int bx = 0; bx < nbx; ++bx) {
      const float x0 = (float)(8 * bx) + 0.5f, x1 = (float)(8 * bx) + 7.5f;
      if (du - rx > x1 || du + rx < x0) continue;
      const float xlo = x0 - du, xhi = x1 - du;        // dx range over the block
      float qmin = 0.0f;
      if (!(xlo <= 0.0f && xhi >= 0.0f && ylo <= 0.0f && yhi >= 0.0f)) {
        // the centre is outside: the minimum lies on an edge of the rectangle
        qmin = __builtin_inff();
        const float xs[2] = {xlo, xhi}, ys[2] = {ylo, yhi};
#pragma unroll
        for (int e2 = 0; e2 < 2; ++e2) {
          const float X = xs[e2];
          const float y = fminf(fmaxf(-qb * X * ic, ylo), yhi);
          qmin = fminf(qmin, X * (qa * X + qb * y) + qc * y * y);
          const float Y = ys[e2];
          const float x = fminf(fmaxf(-qb * Y * ia, xlo), xhi);
          qmin = fminf(qmin, Y * (qc * Y + qb * x) + qa * x * x);
        }
      }
      if (qmin <= qlim) mask |= 1u << (by * nbx + bx);
    }
  }
  crec[3 * j + 0] = make_float4(du, dv, r1.x, r1.y);
  crec[3 * j + 1] = make_float4(r1.z, r1.w, r2.x, r2.y);
  crec[3 * j + 2] = make_float4(r2.z, __uint_as_float(mask), __uint_as_float(slot), 0.0f);
}

}  // namespace

size_t scan_blocks_size(int64_t n) {
  return 2 * (size_t)((n + kScanChunk - 1) / kScanChunk) + 1;
}

void launch_emit_scan(const uint32_t* nt_sorted, int64_t n_slots, uint32_t* scan_local,
                      uint32_t* block_sums, hipStream_t s) {
  if (n_slots <= 0) return;
  const int nblocks = (int)((n_slots + kScanChunk - 1) / kScanChunk);
  hipLaunchKernelGGL(scan_local_kernel, dim3(nblocks), dim3(kScanBlock), 0, s, nt_sorted,
                     n_slots, scan_local, block_sums);
  if (nblocks > kInlineBlocks)
    hipLaunchKernelGGL(scan_blocks_kernel, dim3(1), dim3(kScanBlock), 0, s, block_sums,
                       nblocks);
}

void launch_emit_write(const uint32_t* sorted_slots, const uint2* rect_sorted, int64_t n_slots,
                       int32_t n_gauss, const ViewDev* views, const uint32_t* scan_local,
                       const uint32_t* block_sums, uint32_t capacity, uint32_t* inst_tile,
                       uint32_t* inst_val, hipStream_t s) {
  if (n_slots <= 0) return;
  const int nblocks = (int)((n_slots + kScanChunk - 1) / kScanChunk);
  const int n_views = (int)(n_slots / n_gauss);
  hipLaunchKernelGGL(emit_kernel, dim3(nblocks), dim3(kScanBlock), 0, s, sorted_slots,
                     rect_sorted, n_slots, n_gauss, n_views, views, scan_local, block_sums,
                     nblocks, capacity, inst_tile, inst_val);
}

void launch_fill_u32(uint32_t* p, int64_t n, uint32_t value, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     p, n, value);
}

void launch_ranges_gather(const uint32_t* inst_tile, const uint32_t* inst_val, int64_t m,
                          const ProjDev& proj, const ViewDev* views, int n_views,
                          int tile_w, int tile_h, float log2_alpha_min, uint2* ranges,
                          float4* crec, hipStream_t s) {
  if (m <= 0) return;
  const uint32_t nb = (uint32_t)((m + 255) / 256);
  const uint32_t per = (nb + kXcds - 1) / kXcds;
  hipLaunchKernelGGL(ranges_gather_kernel, dim3(per * kXcds), dim3(256), 0, s, inst_tile,
                     inst_val, m, proj, views, n_views, tile_w, tile_h, log2_alpha_min,
                     ranges, crec, per);
}

}  // namespace nxs
