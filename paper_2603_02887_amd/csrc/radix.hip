// Stable LSD radix sort of (u32 key, u32 value) pairs, reduce-then-scan.
//
// Digits of up to 9 bits (as few passes as that allows, widths balanced) over
// chunks of 1,024 keys below 3.5M keys (many work-groups, short per-group
// latency, which is what bounds these passes at 1-3 million keys) and of
// 4,096 keys above (longer digit runs per chunk, and a grid that four
// work-groups per CU cover in fewer rounds).  Each pass is three kernels:
//   count    per chunk and digit                counts[d * nchunks + c]
//            (one LDS atomic add per key)
//   scan     per digit over chunks (one work-group per digit) -> exclusive
//            offsets in place, digit totals
//   scatter  per chunk: stable local ranks via wave ballots, a reorder by
//            digit in LDS, then the digit runs written out.
// Work-groups are dealt to the 8 XCDs round-robin; chunk c goes to the
// work-group that puts a contiguous range of chunks on each XCD.  A digit's
// runs from consecutive chunks are adjacent in the output, so the partial
// cache lines at their seams are merged in one XCD's L2 instead of reaching
// HBM as several partial writes.  No kernel waits on another work-group.
#include "nxs_internal.h"

#include <algorithm>

namespace nxs {

namespace {

constexpr int kRThreads = 256;
constexpr int kRWaves = kRThreads / 64;
// Keys per thread: 4 (chunks of 1,024) keeps the per-group latency short,
// which is what bounds a pass at up to about 3.5 million keys; 16 (chunks of
// 4,096) gives each digit runs four times longer in a chunk's output (fewer
// partial cache lines at run ends) and needs a quarter of the work-groups
// (4M keys: 2.5 rounds of the small chunks' grid, one of the large).
constexpr int kRItemsSmall = 4;
constexpr int kRItemsLarge = 16;
// Planned keys from which the large chunks are used; a deferred render plans
// its tile sort for the expected count plus a quarter (the 1080p frame's
// 2.69M instances: 3.37M planned, faster in small chunks).
constexpr int64_t kRLargeFrom = int64_t(7) << 19;   // 3.5M keys
constexpr int kRChunkMin = kRThreads * kRItemsSmall;
constexpr int kRBins = 1 << kMaxDigitBits;     // digits of up to 9 bits
constexpr int kRBinsPerThread = kRBins / kRThreads;
static_assert(kRBinsPerThread == 2, "the scans below take two digits per thread");
constexpr uint32_t kRXcds = 8;

// The chunks of work-group b out of a grid of 8 * per_g when nlive chunks
// hold keys: XCD x = b % 8 (work-groups are dealt to the XCDs round-robin)
// owns the contiguous chunks [x * per_c, (x + 1) * per_c), per_c =
// ceil(nlive / 8), and its work-groups take them in turn from x * per_c +
// b / 8 in steps of per_g.  A grid planned for the chunk count gives every
// work-group one chunk; a smaller grid loops.
struct ChunkWalk {
  uint32_t first, end, step;
};
__device__ __forceinline__ ChunkWalk chunk_walk(uint32_t b, uint32_t per_g, uint32_t nlive) {
  const uint32_t per_c = (nlive + kRXcds - 1) / kRXcds;
  const uint32_t x = b % kRXcds;
  ChunkWalk w;
  w.first = x * per_c + b / kRXcds;
  w.end = min((x + 1) * per_c, nlive);
  w.step = per_g;
  return w;
}

// lanes of the wave whose digit equals this lane's (valid lanes only)
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, int width, bool valid) {
  uint64_t peers = __ballot(valid);
  for (int b = 0; b < width; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

// A pass's digit is (key >> shift) & (2^width - 1); with `plan` the pair comes
// from device memory (plan[pass] = shift | width << 8 | kPassActive), so a
// sort can be enqueued before the host knows how many bits vary.  Returns
// false for an inactive pass (every kernel of it does nothing).
__device__ __forceinline__ bool pass_digit(const uint32_t* plan, int pass, int& shift,
                                           int& width) {
  if (plan) {
    const uint32_t w = plan[pass];
    shift = (int)(w & 0xFFu);
    width = (int)((w >> 8) & 0xFFu);
    return (w & kPassActive) != 0;
  }
  return true;
}

// Only the first pass of a plan is optional: when it is inactive, the
// second pass reads the sort's input (keys_first, vals_first) instead of the
// first pass's output, and the result still lands where four passes put it.
__device__ __forceinline__ void select_input(const uint32_t* plan, int pass,
                                             const uint32_t* keys_first,
                                             const uint32_t* vals_first, const uint32_t*& keys,
                                             const uint32_t*& vals) {
  if (plan && pass == 1 && !(plan[0] & kPassActive)) {
    keys = keys_first;
    vals = vals_first;
  }
}

// The number of keys: n, or with dn the count read on the device (n is then
// its upper bound).
__device__ __forceinline__ int64_t key_count(int64_t n, const Counters* dn) {
  return dn ? min(live_count(dn), n) : n;
}

template <int ITEMS>
__device__ __forceinline__ uint32_t live_chunks(int64_t n) {
  return (uint32_t)((n + kRThreads * ITEMS - 1) / (kRThreads * ITEMS));
}

template <int ITEMS>
__global__ __launch_bounds__(kRThreads) void rx_count(const uint32_t* keys,
                                                      const uint32_t* keys_first, int64_t n,
                                                      int shift, int width,
                                                      const uint32_t* __restrict__ plan,
                                                      int pass, uint32_t nchunks, uint32_t per,
                                                      uint32_t* __restrict__ counts,
                                                      const Counters* __restrict__ dn) {
  __shared__ uint32_t h[kRBins];
  if (!pass_digit(plan, pass, shift, width)) return;   // the whole grid
  n = key_count(n, dn);
  const ChunkWalk walk = chunk_walk(blockIdx.x, per, min(nchunks, live_chunks<ITEMS>(n)));
  {
    const uint32_t* unused = nullptr;
    select_input(plan, pass, keys_first, nullptr, keys, unused);
  }
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const uint32_t mask = (1u << width) - 1u;
  for (uint32_t c = walk.first; c < walk.end; c += walk.step) {   // (uniform per group)
    for (int d = t; d < kRBins; d += kRThreads) h[d] = 0;
    __syncthreads();
    const int64_t base = (int64_t)c * (kRThreads * ITEMS);
    const int chunk_n = (int)min((int64_t)(kRThreads * ITEMS), n - base);
    uint32_t k[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      const int li = wid * (64 * ITEMS) + r * 64 + lane;
      k[r] = li < chunk_n ? keys[base + li] : 0u;
    }
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      const int li = wid * (64 * ITEMS) + r * 64 + lane;
      const bool valid = li < chunk_n;
      const uint32_t d = (k[r] >> shift) & mask;
      if (valid) atomicAdd(&h[d], 1u);
    }
    __syncthreads();
    for (int d = t; d <= (int)mask; d += kRThreads) counts[(int64_t)d * nchunks + c] = h[d];
    __syncthreads();   // h is cleared for the next chunk
  }
}

__device__ __forceinline__ uint32_t rx_block_scan(uint32_t x, uint32_t* s_tmp, uint32_t* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint32_t incl = wave_inclusive_scan_u32(x);
  if (lane == 63) s_tmp[wid] = incl;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kRWaves; ++w) {
    const uint32_t v = s_tmp[w];
    if (w < wid) off += v;
    tot += v;
  }
  __syncthreads();
  *total = tot;
  return off + incl - x;
}

// One work-group per digit: exclusive scan of counts[d][0..live chunks) in
// place (rows of nchunks entries).
template <int ITEMS>
__global__ __launch_bounds__(kRThreads) void rx_scan(uint32_t* __restrict__ counts,
                                                     uint32_t nchunks,
                                                     uint32_t* __restrict__ totals, int width,
                                                     const uint32_t* __restrict__ plan,
                                                     int pass, int64_t n,
                                                     const Counters* __restrict__ dn) {
  __shared__ uint32_t s_tmp[kRWaves];
  int shift = 0;
  if (!pass_digit(plan, pass, shift, width)) return;   // the whole grid
  if (blockIdx.x >= (1u << width)) return;    // the whole work-group
  uint32_t* row = counts + (int64_t)blockIdx.x * nchunks;
  nchunks = min(nchunks, live_chunks<ITEMS>(key_count(n, dn)));
  uint32_t running = 0;
  for (uint32_t b = 0; b < nchunks; b += kRThreads * 4) {
    uint32_t v[4], sum = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t i = b + threadIdx.x * 4 + q;
      v[q] = i < nchunks ? row[i] : 0u;
      sum += v[q];
    }
    uint32_t tot;
    uint32_t ex = rx_block_scan(sum, s_tmp, &tot) + running;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t i = b + threadIdx.x * 4 + q;
      if (i < nchunks) row[i] = ex;
      ex += v[q];
    }
    running += tot;
  }
  if (threadIdx.x == 0) totals[blockIdx.x] = running;
}

// vals_in == nullptr: the values are the input positions.  The last pass
// also writes each value's tile rectangle (from `trect`) and tile count when
// trect is given.
template <int ITEMS>
__global__ __launch_bounds__(kRThreads) void rx_scatter(
    const uint32_t* keys_in, const uint32_t* vals_in, const uint32_t* keys_first,
    const uint32_t* vals_first, uint32_t* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out, int64_t n, int shift, int width,
    const uint32_t* __restrict__ plan, int pass, uint32_t nchunks, uint32_t per,
    const uint32_t* __restrict__ counts, const uint32_t* __restrict__ totals,
    const uint2* __restrict__ trect, uint32_t* __restrict__ nt_out,
    uint2* __restrict__ rect_out, const Counters* __restrict__ dn) {
  // Per-wave digit counts (at most 64 * ITEMS), then each wave's first
  // position per digit in the chunk (below 256 * ITEMS), are kept in 16 bits:
  // at 4,096 keys the tables then leave room for four work-groups per CU.
  static_assert(kRThreads * ITEMS <= 0xFFFF, "local positions must fit 16 bits");
  __shared__ uint32_t s_key[(kRThreads * ITEMS)];
  __shared__ uint32_t s_val[(kRThreads * ITEMS)];
  __shared__ uint16_t s_wave[kRWaves][kRBins];
  __shared__ uint32_t s_delta[kRBins];   // global minus local start of each digit's run
  __shared__ uint32_t s_tmp[kRWaves];

  if (!pass_digit(plan, pass, shift, width)) return;   // the whole grid
  n = key_count(n, dn);
  const ChunkWalk walk = chunk_walk(blockIdx.x, per, min(nchunks, live_chunks<ITEMS>(n)));
  select_input(plan, pass, keys_first, vals_first, keys_in, vals_in);
  const int t = threadIdx.x;
  const int lane = t & 63, wid = t >> 6;
  const uint32_t mask = (1u << width) - 1u;
  const int nd = 1 << width;
  static_assert(sizeof(s_wave) == 16 * kRThreads, "one 16-byte store per thread clears s_wave");
  for (uint32_t c = walk.first; c < walk.end; c += walk.step) {   // (uniform per group)
    reinterpret_cast<uint4*>(&s_wave[0][0])[t] = make_uint4(0u, 0u, 0u, 0u);
    const int64_t base = (int64_t)c * (kRThreads * ITEMS);
    const int chunk_n = (int)min((int64_t)(kRThreads * ITEMS), n - base);

    uint32_t k_reg[ITEMS], v_reg[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      const int li = wid * (64 * ITEMS) + r * 64 + lane;
      k_reg[r] = 0u;
      v_reg[r] = 0u;
      if (li < chunk_n) {
        k_reg[r] = keys_in[base + li];
        v_reg[r] = vals_in ? vals_in[base + li] : (uint32_t)(base + li);
      }
    }
    // global start of this chunk's run of each digit: keys of smaller digits
    // plus keys of that digit in earlier chunks (thread t: digits 2t, 2t + 1;
    // the scan's barriers also order the cleared counters before the ranks)
    const int d0 = 2 * t, d1 = 2 * t + 1;
    uint32_t gbase0, gbase1;
    {
      const uint32_t tot0 = d0 < nd ? totals[d0] : 0u, tot1 = d1 < nd ? totals[d1] : 0u;
      const uint32_t off0 = d0 < nd ? counts[(int64_t)d0 * nchunks + c] : 0u;
      const uint32_t off1 = d1 < nd ? counts[(int64_t)d1 * nchunks + c] : 0u;
      uint32_t all;
      const uint32_t ex = rx_block_scan(tot0 + tot1, s_tmp, &all);
      gbase0 = ex + off0;
      gbase1 = ex + tot0 + off1;
    }
    // per-wave ranks: keys of the same digit earlier in this wave's part
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t rank[ITEMS], dig[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      const int li = wid * (64 * ITEMS) + r * 64 + lane;
      const bool valid = li < chunk_n;
      const uint32_t d = valid ? (k_reg[r] >> shift) & mask : 0u;
      const uint64_t peers = digit_peers(d, width, valid);
      dig[r] = d;
      rank[r] = 0;
      if (valid) {
        const uint32_t before = s_wave[wid][d];   // the same for every peer
        const uint32_t pos = (uint32_t)__popcll(peers & lt_mask);
        rank[r] = before + pos;
        if (pos == 0) s_wave[wid][d] = (uint16_t)(before + (uint32_t)__popcll(peers));
      }
    }
    __syncthreads();
    // local start of each digit's run in the chunk; each wave's count of a
    // digit then becomes the wave's first position for that digit (the run's
    // start plus the digit's keys in the waves before it)
    {
      uint32_t cnt0 = 0, cnt1 = 0, before0[kRWaves], before1[kRWaves];
#pragma unroll
      for (int w = 0; w < kRWaves; ++w) {
        before0[w] = cnt0;
        before1[w] = cnt1;
        cnt0 += s_wave[w][d0];
        cnt1 += s_wave[w][d1];
      }
      uint32_t all;
      const uint32_t ex = rx_block_scan(cnt0 + cnt1, s_tmp, &all);
#pragma unroll
      for (int w = 0; w < kRWaves; ++w) {
        s_wave[w][d0] = (uint16_t)(ex + before0[w]);
        s_wave[w][d1] = (uint16_t)(ex + cnt0 + before1[w]);
      }
      s_delta[d0] = gbase0 - ex;
      s_delta[d1] = gbase1 - (ex + cnt0);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      const int li = wid * (64 * ITEMS) + r * 64 + lane;
      if (li < chunk_n) {
        const uint32_t off = s_wave[wid][dig[r]] + rank[r];
        s_key[off] = k_reg[r];
        s_val[off] = v_reg[r];
      }
    }
    __syncthreads();
    // (unrolled by four: each group's LDS reads are issued together, and the
    // 4,096-key chunks keep the registers of four work-groups per CU)
#pragma unroll 4
    for (int r = 0; r < ITEMS; ++r) {
      const int i = r * kRThreads + t;
      if (i < chunk_n) {
        const uint32_t k = s_key[i];
        const uint32_t g = s_delta[(k >> shift) & mask] + (uint32_t)i;
        const uint32_t v = s_val[i];
        keys_out[g] = k;
        vals_out[g] = v;
        if (trect) {   // the slot's tile rectangle, now in sorted order
          const uint2 rc = trect[v];
          nt_out[g] = rect_tile_count(rc);
          rect_out[g] = rc;
        }
      }
    }
    __syncthreads();   // the LDS tables are rebuilt for the next chunk
  }
}

// ------------------------------------------------- per-tile depth sort

// One work-group sorts one tile's list (slots in slot order after the stable
// tile sort) stably by the slots' depth bits: LSD passes of balanced digits
// of up to kMaxDigitBits over the bits that vary among visible depths, each
// pass ranked like a scatter chunk (wave ballots, per-wave digit counters,
// a scan over the digits, two per thread).  Up to kSegMax entries live in
// LDS for all passes; a longer list is sorted through global memory in
// chunks of kSegMax, ping-ponging with `temp`.

// Per-wave digit counters -> each wave's first position per digit: s_wave[w][d]
// becomes base + (entries of digit d in waves < w) + (entries of digits < d),
// base[d] = run[d] (0 for a single chunk); run[d] then advances by the
// digit's count.  Threads t own digits 2t and 2t + 1.
__device__ __forceinline__ void seg_digit_offsets(uint32_t (*s_wave)[kRBins], uint32_t* s_run,
                                                  uint32_t* s_tmp, int nd, bool chained) {
  const int t = threadIdx.x;
  const int d0 = 2 * t, d1 = 2 * t + 1;
  uint32_t c0 = 0, c1 = 0;
  for (int w = 0; w < kRWaves; ++w) {
    c0 += d0 < nd ? s_wave[w][d0] : 0u;
    c1 += d1 < nd ? s_wave[w][d1] : 0u;
  }
  uint32_t all;
  const uint32_t ex = rx_block_scan(c0 + c1, s_tmp, &all);   // (synchronises)
  uint32_t r0 = chained ? s_run[d0] : ex, r1 = chained ? s_run[d1] : ex + c0;
  for (int w = 0; w < kRWaves; ++w) {
    if (d0 < nd) {
      const uint32_t x = s_wave[w][d0];
      s_wave[w][d0] = r0;
      r0 += x;
    }
    if (d1 < nd) {
      const uint32_t x = s_wave[w][d1];
      s_wave[w][d1] = r1;
      r1 += x;
    }
  }
  if (chained) {
    s_run[d0] = r0;
    s_run[d1] = r1;
  }
}

// Stable ranks of one chunk's digits within their wave; items of wave w,
// round r, lane l are chunk entries w * 64 * ITEMS + r * 64 + l.
template <int ITEMS>
__device__ __forceinline__ void seg_rank(const uint32_t (&k)[ITEMS], int m, int shift, int width,
                                         uint32_t (*s_wave)[kRBins], uint32_t (&dig)[ITEMS],
                                         uint32_t (&rank)[ITEMS]) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  const uint32_t mask = (1u << width) - 1u;
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const int li = wid * (64 * ITEMS) + r * 64 + lane;
    const bool valid = li < m;
    const uint32_t d = valid ? (k[r] >> shift) & mask : 0u;
    const uint64_t peers = digit_peers(d, width, valid);
    dig[r] = d;
    rank[r] = 0;
    if (valid) {
      const uint32_t before = s_wave[wid][d];   // the same for every peer
      const uint32_t pos = (uint32_t)__popcll(peers & lt);
      rank[r] = before + pos;
      if (pos == 0) s_wave[wid][d] = before + (uint32_t)__popcll(peers);
    }
  }
}

struct SegLds {
  uint32_t key[kSegMax];
  uint32_t val[kSegMax];
  uint32_t wave[kRWaves][kRBins];
  uint32_t run[kRBins];
  uint32_t tmp[kRWaves];
};

// All passes in LDS (m <= 256 * ITEMS <= kSegMax).
template <int ITEMS>
__device__ void seg_sort_lds(uint32_t* list, int m, const uint32_t* __restrict__ depth_key,
                             const int* shifts, const int* widths, int passes, SegLds& L) {
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  uint32_t k[ITEMS], v[ITEMS];
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const int li = wid * (64 * ITEMS) + r * 64 + lane;
    v[r] = li < m ? list[li] : 0u;
  }
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const int li = wid * (64 * ITEMS) + r * 64 + lane;
    k[r] = li < m ? depth_key[v[r]] : 0u;
  }
  for (int p = 0; p < passes; ++p) {
    for (int i = t; i < kRWaves * kRBins; i += kRThreads) (&L.wave[0][0])[i] = 0u;
    __syncthreads();
    uint32_t dig[ITEMS], rank[ITEMS];
    seg_rank<ITEMS>(k, m, shifts[p], widths[p], L.wave, dig, rank);
    __syncthreads();
    seg_digit_offsets(L.wave, L.run, L.tmp, 1 << widths[p], false);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      const int li = wid * (64 * ITEMS) + r * 64 + lane;
      if (li < m) {
        const uint32_t dst = L.wave[wid][dig[r]] + rank[r];
        L.key[dst] = k[r];
        L.val[dst] = v[r];
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      const int li = wid * (64 * ITEMS) + r * 64 + lane;
      if (li < m) {
        k[r] = L.key[li];
        v[r] = L.val[li];
      }
    }
  }
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const int li = wid * (64 * ITEMS) + r * 64 + lane;
    if (li < m) list[li] = v[r];
  }
}

// A list longer than kSegMax: every pass counts the whole list, then ranks
// and writes it chunk by chunk in order, between `list` and `temp`.
__device__ void seg_sort_global(uint32_t* list, uint32_t* temp, int m,
                                const uint32_t* __restrict__ depth_key, const int* shifts,
                                const int* widths, int passes, SegLds& L) {
  constexpr int ITEMS = kSegMax / kRThreads;
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  uint32_t* src = list;
  uint32_t* dst = temp;
  for (int p = 0; p < passes; ++p) {
    const int shift = shifts[p], width = widths[p], nd = 1 << width;
    const uint32_t mask = (1u << width) - 1u;
    for (int i = t; i < kRBins; i += kRThreads) L.run[i] = 0u;
    __syncthreads();
    for (int i = t; i < m; i += kRThreads)
      atomicAdd(&L.run[(depth_key[src[i]] >> shift) & mask], 1u);
    __syncthreads();
    {
      // exclusive scan of the digit totals: the first position of each digit
      const int d0 = 2 * t, d1 = 2 * t + 1;
      const uint32_t c0 = d0 < nd ? L.run[d0] : 0u, c1 = d1 < nd ? L.run[d1] : 0u;
      uint32_t all;
      const uint32_t ex = rx_block_scan(c0 + c1, L.tmp, &all);
      if (d0 < nd) L.run[d0] = ex;
      if (d1 < nd) L.run[d1] = ex + c0;
    }
    __syncthreads();
    for (int c = 0; c < m; c += kSegMax) {
      const int cm = min(kSegMax, m - c);
      uint32_t k[ITEMS], v[ITEMS];
#pragma unroll
      for (int r = 0; r < ITEMS; ++r) {
        const int li = wid * (64 * ITEMS) + r * 64 + lane;
        v[r] = li < cm ? src[c + li] : 0u;
      }
#pragma unroll
      for (int r = 0; r < ITEMS; ++r) {
        const int li = wid * (64 * ITEMS) + r * 64 + lane;
        k[r] = li < cm ? depth_key[v[r]] : 0u;
      }
      for (int i = t; i < kRWaves * kRBins; i += kRThreads) (&L.wave[0][0])[i] = 0u;
      __syncthreads();
      uint32_t dig[ITEMS], rank[ITEMS];
      seg_rank<ITEMS>(k, cm, shift, width, L.wave, dig, rank);
      __syncthreads();
      seg_digit_offsets(L.wave, L.run, L.tmp, nd, true);
      __syncthreads();
#pragma unroll
      for (int r = 0; r < ITEMS; ++r) {
        const int li = wid * (64 * ITEMS) + r * 64 + lane;
        if (li < cm) dst[L.wave[wid][dig[r]] + rank[r]] = v[r];
      }
      __syncthreads();   // the counters are cleared for the next chunk
    }
    uint32_t* x = src;
    src = dst;
    dst = x;
    __threadfence_block();   // this pass's writes before the next pass reads them
    __syncthreads();
  }
  if (src != list) {
    for (int i = t; i < m; i += kRThreads) list[i] = src[i];
  }
}

// Lists of up to kSegWaveMax entries are sorted by one wave with no
// work-group barrier: its items stay in registers (ITEMS per lane, entry
// r * 64 + lane), each pass ranks them with ballots against per-digit
// counters in LDS, a wave-wide scan turns the counters into each digit's
// first position, and the items go to their positions through LDS.  The
// wave's LDS accesses complete in order, so a fence that keeps the compiler
// from moving them is all the ordering a pass needs.
constexpr int kSegWaveMax = 1024;

__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct SegWaveLds {
  uint32_t key[kSegWaveMax];
  uint32_t val[kSegWaveMax];
  uint32_t cnt[kRBins];
};

template <int ITEMS>
__device__ void seg_sort_wave(uint32_t* list, int m, const uint32_t* __restrict__ depth_key,
                              const int* shifts, const int* widths, int passes,
                              SegWaveLds& L) {
  const int lane = threadIdx.x & 63;
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  uint32_t k[ITEMS], v[ITEMS];
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) v[r] = r * 64 + lane < m ? list[r * 64 + lane] : 0u;
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) k[r] = r * 64 + lane < m ? depth_key[v[r]] : 0u;
  for (int p = 0; p < passes; ++p) {
    const int shift = shifts[p], width = widths[p], nd = 1 << width;
    const uint32_t mask = (1u << width) - 1u;
    for (int d = lane; d < nd; d += 64) L.cnt[d] = 0u;
    wave_lds_fence();
    uint32_t dig[ITEMS], rank[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      const bool valid = r * 64 + lane < m;
      const uint32_t d = valid ? (k[r] >> shift) & mask : 0u;
      const uint64_t peers = digit_peers(d, width, valid);
      dig[r] = d;
      rank[r] = 0;
      uint32_t before = 0;
      if (valid) before = L.cnt[d];   // the same for every peer
      wave_lds_fence();
      const uint32_t pos = (uint32_t)__popcll(peers & lt);
      if (valid) {
        rank[r] = before + pos;
        if (pos == 0) L.cnt[d] = before + (uint32_t)__popcll(peers);
      }
      wave_lds_fence();
    }
    // each digit's first position: lane l scans digits [l * per, (l + 1) * per)
    {
      const int per = nd / 64 > 0 ? nd / 64 : 1;
      const int d0 = lane * per;
      uint32_t local = 0;
      for (int i = 0; i < per; ++i)
        if (d0 + i < nd) local += L.cnt[d0 + i];
      uint32_t run = wave_inclusive_scan_u32(local) - local;
      wave_lds_fence();
      for (int i = 0; i < per; ++i)
        if (d0 + i < nd) {
          const uint32_t c = L.cnt[d0 + i];
          L.cnt[d0 + i] = run;
          run += c;
        }
    }
    wave_lds_fence();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r)
      if (r * 64 + lane < m) {
        const uint32_t dst = L.cnt[dig[r]] + rank[r];
        L.key[dst] = k[r];
        L.val[dst] = v[r];
      }
    wave_lds_fence();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r)
      if (r * 64 + lane < m) {
        k[r] = L.key[r * 64 + lane];
        v[r] = L.val[r * 64 + lane];
      }
    wave_lds_fence();
  }
#pragma unroll
  for (int r = 0; r < ITEMS; ++r)
    if (r * 64 + lane < m) list[r * 64 + lane] = v[r];
}

// The digits of the per-tile sort: balanced digits of up to kMaxDigitBits
// over the bits that vary among the render's visible depths.  Returns the
// number of passes (0: equal depths).
__device__ __forceinline__ int seg_plan(const Counters* __restrict__ cnt, int* shifts,
                                        int* widths) {
  const uint32_t diff = cnt->dmin <= cnt->dmax ? (cnt->dmin ^ cnt->dmax) : 0u;
  const int nbits = diff ? 32 - __clz((int)diff) : 0;
  if (nbits == 0) return 0;
  const int passes = (nbits + kMaxDigitBits - 1) / kMaxDigitBits;
  int sh = 0;
  for (int p = 0; p < passes; ++p) {
    widths[p] = (nbits - sh + (passes - p) - 1) / (passes - p);
    shifts[p] = sh;
    sh += widths[p];
  }
  return passes;
}

// One wave per tile of at most kSegWaveMax entries (longer lists: skipped,
// for tile_depth_sort_kernel).
__global__ __launch_bounds__(64) void tile_depth_sort_wave_kernel(
    const uint2* __restrict__ ranges, uint32_t n_tiles, const uint32_t* __restrict__ depth_key,
    const Counters* __restrict__ cnt, uint32_t* __restrict__ list) {
  __shared__ SegWaveLds L;
  const uint32_t tile = blockIdx.x;
  if (tile >= n_tiles || cnt->fail) return;
  const uint2 rg = ranges[tile];
  const int m = (int)(rg.y - rg.x);
  if (m <= 1 || m > kSegWaveMax) return;
  int shifts[4], widths[4];
  const int passes = seg_plan(cnt, shifts, widths);
  if (passes == 0) return;   // equal depths: slot order is the order
  uint32_t* seg = list + rg.x;
  if (m <= 64)
    seg_sort_wave<1>(seg, m, depth_key, shifts, widths, passes, L);
  else if (m <= 128)
    seg_sort_wave<2>(seg, m, depth_key, shifts, widths, passes, L);
  else if (m <= 256)
    seg_sort_wave<4>(seg, m, depth_key, shifts, widths, passes, L);
  else if (m <= 512)
    seg_sort_wave<8>(seg, m, depth_key, shifts, widths, passes, L);
  else
    seg_sort_wave<16>(seg, m, depth_key, shifts, widths, passes, L);
}

__global__ __launch_bounds__(kRThreads) void tile_depth_sort_kernel(
    const uint2* __restrict__ ranges, uint32_t n_tiles, const uint32_t* __restrict__ depth_key,
    const Counters* __restrict__ cnt, uint32_t* __restrict__ list, uint32_t* __restrict__ temp) {
  __shared__ SegLds L;
  const uint32_t tile = blockIdx.x;
  if (tile >= n_tiles || cnt->fail) return;
  const uint2 rg = ranges[tile];
  const int m = (int)(rg.y - rg.x);
  if (m <= kSegWaveMax) return;   // (tile_depth_sort_wave_kernel's)
  int shifts[4], widths[4];
  const int passes = seg_plan(cnt, shifts, widths);
  if (passes == 0) return;   // equal depths: slot order is the order
  uint32_t* seg = list + rg.x;
  if (m <= 2048)
    seg_sort_lds<8>(seg, m, depth_key, shifts, widths, passes, L);
  else if (m <= kSegMax)
    seg_sort_lds<16>(seg, m, depth_key, shifts, widths, passes, L);
  else
    seg_sort_global(seg, temp + rg.x, m, depth_key, shifts, widths, passes, L);
}

}  // namespace

size_t radix_counts_words(int64_t n) {
  const int64_t nchunks = std::max<int64_t>((n + kRChunkMin - 1) / kRChunkMin, 1);
  return (size_t)nchunks * kRBins + kRBins;
}

namespace {

// Passes first..passes-1; pass p writes (k0, v0) if p is even, else (k1, v1),
// and the first launched pass reads the sort's input.  Returns which pair
// holds the result.
int run_passes(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* k0, uint32_t* v0,
               uint32_t* k1, uint32_t* v1, int64_t n, int first, int passes,
               const int* shifts, const int* widths, const uint32_t* plan, uint32_t* counts,
               const uint2* trect, uint32_t* nt_out, uint2* rect_out, hipStream_t s,
               const Counters* dn, int64_t n_plan) {
  // n bounds the keys (the counts layout); the grid is planned for n_plan
  // keys (with dn, the count expected on the device) and loops beyond it
  const bool large = n_plan >= kRLargeFrom;
  const int chunk = kRThreads * (large ? kRItemsLarge : kRItemsSmall);
  const uint32_t nchunks = (uint32_t)((n + chunk - 1) / chunk);
  const uint32_t plan_chunks =
      (uint32_t)std::max<int64_t>((std::min(n_plan, n) + chunk - 1) / chunk, 1);
  const uint32_t per = (plan_chunks + kRXcds - 1) / kRXcds;
  const unsigned grid = per * kRXcds;
  uint32_t* totals = counts + (size_t)nchunks * kRBins;
  const uint32_t* kin = keys_in;
  const uint32_t* vin = vals_in;
  for (int p = first; p < passes; ++p) {
    const int shift = shifts ? shifts[p] : 0, width = widths ? widths[p] : 8;
    uint32_t* kout = (p & 1) ? k1 : k0;
    uint32_t* vout = (p & 1) ? v1 : v0;
    const dim3 scan_grid(plan ? kRBins : (1u << width));
    const bool last = p == passes - 1;
    if (large) {
      hipLaunchKernelGGL(rx_count<kRItemsLarge>, dim3(grid), dim3(kRThreads), 0, s, kin,
                         keys_in, n, shift, width, plan, p, nchunks, per, counts, dn);
      hipLaunchKernelGGL(rx_scan<kRItemsLarge>, scan_grid, dim3(kRThreads), 0, s, counts,
                         nchunks, totals, width, plan, p, n, dn);
      hipLaunchKernelGGL(rx_scatter<kRItemsLarge>, dim3(grid), dim3(kRThreads), 0, s, kin, vin,
                         keys_in, vals_in, kout, vout, n, shift, width, plan, p, nchunks, per,
                         counts, totals, last ? trect : nullptr, nt_out, rect_out, dn);
    } else {
      hipLaunchKernelGGL(rx_count<kRItemsSmall>, dim3(grid), dim3(kRThreads), 0, s, kin,
                         keys_in, n, shift, width, plan, p, nchunks, per, counts, dn);
      hipLaunchKernelGGL(rx_scan<kRItemsSmall>, scan_grid, dim3(kRThreads), 0, s, counts,
                         nchunks, totals, width, plan, p, n, dn);
      hipLaunchKernelGGL(rx_scatter<kRItemsSmall>, dim3(grid), dim3(kRThreads), 0, s, kin, vin,
                         keys_in, vals_in, kout, vout, n, shift, width, plan, p, nchunks, per,
                         counts, totals, last ? trect : nullptr, nt_out, rect_out, dn);
    }
    kin = kout;
    vin = vout;
  }
  return (passes - 1) & 1;
}

}  // namespace

int radix_sort(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* k0, uint32_t* v0,
               uint32_t* k1, uint32_t* v1, int64_t n, int nbits, uint32_t* counts,
               hipStream_t s, const Counters* dn, int64_t n_plan) {
  if (n <= 0) return 0;
  nbits = std::max(nbits, 1);
  const int passes = (nbits + kMaxDigitBits - 1) / kMaxDigitBits;
  int shifts[4], widths[4], shift = 0;
  for (int p = 0; p < passes; ++p) {
    widths[p] = (nbits - shift + (passes - p) - 1) / (passes - p);
    shifts[p] = shift;
    shift += widths[p];
  }
  return run_passes(keys_in, vals_in, k0, v0, k1, v1, n, 0, passes, shifts, widths, nullptr,
                    counts, nullptr, nullptr, nullptr, s, dn,
                    dn && n_plan > 0 ? std::min(n_plan, n) : n);
}

int radix_sort_planned(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* k0,
                       uint32_t* v0, uint32_t* k1, uint32_t* v1, int64_t n,
                       const uint32_t* plan, int first_pass, uint32_t* counts,
                       const uint2* trect, uint32_t* nt_out, uint2* rect_out, hipStream_t s) {
  if (n <= 0) return 1;
  return run_passes(keys_in, vals_in, k0, v0, k1, v1, n, first_pass, kPlanPasses, nullptr,
                    nullptr, plan, counts, trect, nt_out, rect_out, s, nullptr, n);
}

void launch_tile_depth_sort(const uint2* ranges, int64_t n_tiles, const uint32_t* depth_key,
                            const Counters* counters, uint32_t* list, uint32_t* temp,
                            hipStream_t s) {
  if (n_tiles <= 0) return;
  hipLaunchKernelGGL(tile_depth_sort_wave_kernel, dim3((unsigned)n_tiles), dim3(64), 0, s,
                     ranges, (uint32_t)n_tiles, depth_key, counters, list);
  hipLaunchKernelGGL(tile_depth_sort_kernel, dim3((unsigned)n_tiles), dim3(kRThreads), 0, s,
                     ranges, (uint32_t)n_tiles, depth_key, counters, list, temp);
}

}  // namespace nxs
