// Per-tile front-to-back composite with a pluggable transmittance operator.
//
// One wave per 8x8 pixel block of a screen tile, one lane per pixel; waves
// run on their own (no barriers).  The tile's sorted list holds projected
// slots: a wave walks it in batches of 64, each lane fetching one slot's
// record and testing whether its footprint reaches the rows and columns of
// the wave's block that still hold a running pixel; the records that do are
// written in order to the wave's LDS (the gather to
// sorted order, done only for the part of the list the wave reaches before
// its pixels stop).  Each staged splat is then read by the whole wave with
// broadcast LDS reads.  Per pixel (Sec. 4, eq. generalized_gaussian and
// eq. nexp_p):
//   alpha = aleph exp(-q/2), evaluated as exp2 of a precomputed quadratic;
//   splats with alpha < alpha_min are skipped;
//   p = alpha * T                (exponential, T <- T (1 - alpha))
//     = alpha                    (linear)
//     = alpha (1 + c tau)        (quadratic; tau <- tau + alpha)
//   if the running sum of p would reach 1, p takes the remainder, T becomes
//   exactly 0 and the pixel stops (saturation); the exponential also stops
//   after the first splat that leaves T < t_eps;
//   L += E p, overdraw += 1 for every composited splat.
// A wave leaves the tile when a ballot finds all its pixels stopped.
//
// Four schedules of the same per-block work, with bitwise-identical results:
//   tile WGs     one work-group per tile, one wave per 8x8 block of it;
//   block waves  one single-wave work-group per 8x8 block, so the dispatcher
//                refills a wave slot as soon as any block finishes;
//   queue        all views' tiles in one queue ordered by decreasing
//                tile-list length (the longest start early instead of
//                forming the tail), consumed in order by the hardware
//                dispatcher, one single-wave work-group per 8x8 block, the
//                blocks of a tile on one XCD;
//   persistent   a fixed grid of single-wave work-groups taking whole tiles
//                (their 8x8 blocks one after another) from atomic counters
//                over the same order; one counter per XCD, each serving
//                every eighth tile, so a ticket is contended only within one
//                XCD.  Measured slower than the dispatcher on this GPU (a
//                contended device-scope atomic per ticket); kept for callers
//                that want a fixed grid.
// The first two give each XCD a contiguous band of tiles.
#include "nxs_internal.h"
#include "nxs_ops.h"
#include "nxs_stage.h"

#include <algorithm>

namespace nxs {

namespace {

// One wave composites the 8x8 block `wid` of global tile `tile`, gathering
// NB batches of 64 list entries per round (wlds holds NB * kStageF4).
template <int MODEL, int TW, int TH, bool STATE, int NB>
__device__ __forceinline__ void composite_block(
    const ViewDev* __restrict__ views, int n_views, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ inst_val, const float4* __restrict__ rec,
    const CompositeParams& prm, float4* __restrict__ pstate, float4* wlds, uint32_t tile,
    int wid, int lane) {
  static_assert(TW % 8 == 0 && TH % 8 == 0, "waves cover 8x8 blocks");
  int vi = 0;
  {
    int lo = 0, hi = n_views - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if ((uint32_t)views[mid].tile_off <= tile) lo = mid; else hi = mid - 1;
    }
    vi = lo;
  }
  const ViewDev& v = views[vi];
  const int lt = (int)(tile - (uint32_t)v.tile_off);
  const int tx = lt % v.tiles_x, ty = lt / v.tiles_x;
  const int bx = (wid % (TW / 8)) * 8, by = (wid / (TW / 8)) * 8;   // wave's 8x8 block
  const int lx = bx + (lane & 7), ly = by + (lane >> 3);
  const int px = tx * TW + lx, py = ty * TH + ly;
  const bool inside = px < v.width && py < v.height;
  const float fx = (float)lx + 0.5f, fy = (float)ly + 0.5f;
  const StageBlock sb = stage_block<TW>(tx, ty, TH, wid, prm.log2_alpha_min);

  const uint2 rg = ranges[tile];
  const float amin = prm.log2_alpha_min;
  const float t_eps = prm.t_eps;
  const float param = prm.param;
  Op<MODEL> op;

  if (!inside) op.stop();
  float L0 = 0.0f, L1 = 0.0f, L2 = 0.0f;
  int od = 0;
  // backward state (linear and quadratic): E_k, tau_k, U
  constexpr bool kSat = STATE && MODEL >= 1 && MODEL <= 4;
  float ek0 = prm.bg[0], ek1 = prm.bg[1], ek2 = prm.bg[2], tau_s = 0.0f;
  float u0 = 0.0f, u1 = 0.0f, u2 = 0.0f;

  // Rounds of NB batches of 64 list entries are staged in LDS (only the
  // splats that reach the block, in list order); each staged splat is then
  // visited by the whole wave.  The per-pixel update is branch-free: a lane
  // whose alpha is below alpha_min, or which has stopped, composites a = 0,
  // which leaves every operator's state unchanged, so the loop carries no
  // per-lane control flow.  Each round is staged against the rows and
  // columns that still hold a running pixel (act: the wave's running lanes).
  // Slot indices are read two rounds ahead and records one round ahead.
  constexpr uint32_t kRound = 64u * NB;
  bool running = !op.stopped(t_eps);
  uint64_t act = __builtin_amdgcn_ballot_w64(running);
  // (an empty tile fetches nothing: its range is [0, 0) or [x, x))
  StageSlot slots[NB];
  StageFetch fetched[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    slots[k] = StageSlot{0u, false};
    fetched[k] = StageFetch{};
  }
  if (rg.x < rg.y) {
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      slots[k] = stage_slot(inst_val, (uint64_t)rg.x + 64u * k, rg.y, lane);
      fetched[k] = stage_records(slots[k], rec);
      slots[k] = stage_slot(inst_val, (uint64_t)rg.x + kRound + 64u * k, rg.y, lane);
    }
  }
  auto composite_one = [&](const float4* r) {
    const float4 q0 = r[0], q1 = r[1];
    const float c[9] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w, r[2].x};
    const float dx = fx - c[0], dy = fy - c[1];
    const float e = fmaf(dx, fmaf(c[2], dx, c[3] * dy), fmaf(c[4] * dy, dy, c[5]));
    const bool valid = (e >= amin) && running;
    const float a = valid ? __builtin_amdgcn_exp2f(e) : 0.0f;
    const float s_before = op.S;
    const float p = op.step(a, param, t_eps);
    if (kSat) {
      // the saturating splat's emission, and the sums over the splats before it
      const bool sat_now = op.S >= 1.0f && s_before < 1.0f;
      ek0 = sat_now ? c[6] : ek0;
      ek1 = sat_now ? c[7] : ek1;
      ek2 = sat_now ? c[8] : ek2;
      const float a_pre = op.S >= 1.0f ? 0.0f : a;
      u0 = fmaf(c[6], a_pre, u0);
      u1 = fmaf(c[7], a_pre, u1);
      u2 = fmaf(c[8], a_pre, u2);
      tau_s += a_pre;
    }
    L0 = fmaf(c[6], p, L0);
    L1 = fmaf(c[7], p, L1);
    L2 = fmaf(c[8], p, L2);
    od += valid ? 1 : 0;
    running = !op.stopped(t_eps);
    act = __builtin_amdgcn_ballot_w64(running);
  };
  for (uint32_t base = rg.x; base < rg.y && act != 0; base += kRound) {
    const StageBlock sbr = stage_shrink(sb, act);
    uint32_t n = 0;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      n += stage_batch(fetched[k], sbr, wlds + 3 * n);
      fetched[k] = stage_records(slots[k], rec);                                 // next round
      slots[k] = stage_slot(inst_val, (uint64_t)base + 2 * kRound + 64u * k, rg.y, lane);
    }
    // two staged splats per trip: an odd count (below 64 NB, so the stage has
    // room) is padded with a splat whose exponent is -inf at every pixel
    // (alpha 0, no emission); a pair's second splat after every pixel stopped
    // composites a = 0 as well
    n = __builtin_amdgcn_readfirstlane(n);
    if (n & 1u) {
      if (lane < 3)
        wlds[3 * n + lane] = lane == 1 ? make_float4(0.0f, -__builtin_inff(), 0.0f, 0.0f)
                                       : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      wave_lds_order();
    }
    for (uint32_t i = 0; i < n && act != 0; i += 2) {
      composite_one(wlds + 3 * i);
      composite_one(wlds + 3 * i + 3);
    }
  }
  if (inside) {
    const float Tf = op.transmittance(param);
    const int64_t pix = (int64_t)py * v.width + px;
    v.rgb[3 * pix + 0] = L0 + prm.bg[0] * Tf;
    v.rgb[3 * pix + 1] = L1 + prm.bg[1] * Tf;
    v.rgb[3 * pix + 2] = L2 + prm.bg[2] * Tf;
    v.trans[pix] = Tf;
    if (v.od) v.od[pix] = od;
    if (STATE) {
      float4* st = pstate + 3 * (v.pix_off + pix);
      st[0] = make_float4(L0 + prm.bg[0] * Tf, L1 + prm.bg[1] * Tf, L2 + prm.bg[2] * Tf, Tf);
      st[1] = make_float4(ek0, ek1, ek2, tau_s);
      st[2] = make_float4(u0, u1, u2, 0.0f);
    }
  }
}

constexpr int kBlocksPerTile(int tw, int th) { return (tw / 8) * (th / 8); }

template <int MODEL, int TW, int TH, bool STATE, int NB>
__global__ __launch_bounds__(TW* TH) void composite_tiles_kernel(
    const ViewDev* __restrict__ views, int n_views, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ inst_val, const float4* __restrict__ rec, CompositeParams prm,
    float4* __restrict__ pstate, uint32_t n_tiles, uint32_t per_xcd) {
  __shared__ float4 stage[kBlocksPerTile(TW, TH) * NB * kStageF4];
  const uint32_t tile = xcd_banded(blockIdx.x, per_xcd);
  if (tile >= n_tiles) return;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  composite_block<MODEL, TW, TH, STATE, NB>(views, n_views, ranges, inst_val, rec, prm,
                                            pstate, stage + wid * NB * kStageF4, tile, wid,
                                            threadIdx.x & 63);
}

template <int MODEL, int TW, int TH, bool STATE, int NB>
__global__ __launch_bounds__(64) void composite_blocks_kernel(
    const ViewDev* __restrict__ views, int n_views, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ inst_val, const float4* __restrict__ rec, CompositeParams prm,
    float4* __restrict__ pstate, uint32_t n_items, uint32_t per_xcd) {
  __shared__ float4 stage[NB * kStageF4];
  constexpr int B = kBlocksPerTile(TW, TH);
  const uint32_t item = xcd_banded(blockIdx.x, per_xcd);
  if (item >= n_items) return;
  composite_block<MODEL, TW, TH, STATE, NB>(views, n_views, ranges, inst_val, rec, prm,
                                            pstate, stage, item / B, (int)(item % B),
                                            threadIdx.x);
}

// The ordered queue dealt to the 8 XCDs (which receive work-groups
// round-robin) at tile granularity: work-group w, the i-th on XCD x = w mod 8,
// takes block (i mod B) of the tile of rank 8 (i / B) + x in the order, so the
// longest tiles start first on every XCD and each tile's blocks share one L2.
template <int MODEL, int TW, int TH, bool STATE, int NB>
__global__ __launch_bounds__(64) void composite_ordered_kernel(
    const ViewDev* __restrict__ views, int n_views, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ inst_val, const float4* __restrict__ rec, CompositeParams prm,
    float4* __restrict__ pstate, const uint32_t* __restrict__ order, uint32_t n_tiles) {
  __shared__ float4 stage[NB * kStageF4];
  constexpr int B = kBlocksPerTile(TW, TH);
  const uint32_t x = blockIdx.x % kQueues, i = blockIdx.x / kQueues;
  const uint32_t r = (i / B) * kQueues + x;
  if (r >= n_tiles) return;
  composite_block<MODEL, TW, TH, STATE, NB>(views, n_views, ranges, inst_val, rec, prm,
                                            pstate, stage, order[r], (int)(i % B),
                                            threadIdx.x);
}

// Queue q (the work-group's XCD under round-robin dispatch) hands out the
// tiles order[q], order[q + 8], ...; the wave composites each tile's blocks in
// turn.  Every queue has work-groups (the grid is a multiple of 8), and every
// wave leaves once its queue is drained.
template <int MODEL, int TW, int TH, bool STATE, int NB>
__global__ __launch_bounds__(64) void composite_queue_kernel(
    const ViewDev* __restrict__ views, int n_views, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ inst_val, const float4* __restrict__ rec, CompositeParams prm,
    float4* __restrict__ pstate, const uint32_t* __restrict__ order, uint32_t n_tiles,
    uint32_t* __restrict__ queue) {
  __shared__ float4 stage[NB * kStageF4];
  constexpr int B = kBlocksPerTile(TW, TH);
  const int lane = threadIdx.x;
  const uint32_t q = blockIdx.x % kQueues;
  for (;;) {
    uint32_t k = 0;
    if (lane == 0) k = atomicAdd(queue + q, 1u);
    k = __builtin_amdgcn_readfirstlane(k);   // lane 0's ticket, wave-uniform
    const uint64_t i = (uint64_t)k * kQueues + q;
    if (i >= n_tiles) break;
    const uint32_t tile = order[i];
    for (int b = 0; b < B; ++b)
      composite_block<MODEL, TW, TH, STATE, NB>(views, n_views, ranges, inst_val, rec, prm,
                                                pstate, stage, tile, b, lane);
  }
}

// Tiles in order of decreasing list length, bucketed by floor(log2(length)),
// in two grid-wide passes: each tile takes a rank within its bucket from a
// global counter (lanes of a wave with equal buckets are matched by ballots
// and take one atomic together), then every work-group scans the bucket
// counts, longest bucket first, and scatters its tiles.  The counters start
// at zero (cleared with the tile ranges).  Order within a bucket is whatever
// the atomics give; it only changes which wave runs a tile, not any result.
constexpr int kOrderThreads = 256;
constexpr int kBuckets = 33;
constexpr int kBucketBits = 6;

__device__ __forceinline__ uint32_t length_bucket(const uint2 r) {
  const uint32_t len = r.y - r.x;
  return len ? 32u - (uint32_t)__clz(len) : 0u;   // 0 for empty, else 1 + floor(log2)
}

// lanes of the wave (valid ones only) whose bucket equals this lane's
__device__ __forceinline__ uint64_t bucket_peers(uint32_t b, bool valid) {
  uint64_t peers = __builtin_amdgcn_ballot_w64(valid);
#pragma unroll
  for (int k = 0; k < kBucketBits; ++k) {
    const bool bit = (b >> k) & 1u;
    const uint64_t m = __builtin_amdgcn_ballot_w64(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

__global__ __launch_bounds__(kOrderThreads) void order_rank_kernel(
    const uint2* __restrict__ ranges, uint32_t n_tiles, uint32_t* __restrict__ buckets,
    uint32_t* __restrict__ rank) {
  const uint32_t i = blockIdx.x * kOrderThreads + threadIdx.x;
  const int lane = (int)(threadIdx.x & 63);
  const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const bool valid = i < n_tiles;
  const uint32_t b = valid ? length_bucket(ranges[i]) : 0u;
  const uint64_t peers = bucket_peers(b, valid);
  const bool leader = valid && (peers & lt_mask) == 0;
  uint32_t base = 0;
  if (leader) base = atomicAdd(buckets + b, (uint32_t)__popcll(peers));
  // every lane takes its leader's base (the lowest lane among its peers)
  const int src = valid ? __builtin_ctzll(peers) : lane;
  base = (uint32_t)__shfl((int)base, src, 64);
  if (valid) rank[i] = base + (uint32_t)__popcll(peers & lt_mask);
}

__global__ __launch_bounds__(kOrderThreads) void order_scatter_kernel(
    const uint2* __restrict__ ranges, uint32_t n_tiles, const uint32_t* __restrict__ buckets,
    const uint32_t* __restrict__ rank, uint32_t* __restrict__ order) {
  __shared__ uint32_t start[kBuckets];
  const uint32_t t = threadIdx.x;
  if (t == 0) {
    uint32_t run = 0;
    for (int k = kBuckets - 1; k >= 0; --k) {   // longest lists first
      start[k] = run;
      run += buckets[k];
    }
  }
  __syncthreads();
  const uint32_t i = blockIdx.x * kOrderThreads + t;
  if (i < n_tiles) order[start[length_bucket(ranges[i])] + rank[i]] = i;
}

}  // namespace

void launch_composite_order(const CompositeLaunch& L, hipStream_t s) {
  if (L.n_tiles <= 0 ||
      (L.schedule != NXS_SCHED_QUEUE && L.schedule != NXS_SCHED_PERSISTENT))
    return;
  const unsigned grid = (unsigned)((L.n_tiles + kOrderThreads - 1) / kOrderThreads);
  uint32_t* rank = L.order + L.n_tiles;
  hipLaunchKernelGGL(order_rank_kernel, dim3(grid), dim3(kOrderThreads), 0, s, L.ranges,
                     (uint32_t)L.n_tiles, L.sched_counters + kQueues, rank);
  hipLaunchKernelGGL(order_scatter_kernel, dim3(grid), dim3(kOrderThreads), 0, s, L.ranges,
                     (uint32_t)L.n_tiles, L.sched_counters + kQueues, rank, L.order);
}

namespace {

template <int MODEL, int TW, int TH, bool STATE, int NB>
void launch_s(const CompositeLaunch& L, const CompositeParams& p, float4* pstate,
              hipStream_t s) {
  constexpr int B = kBlocksPerTile(TW, TH);
  if (L.schedule == NXS_SCHED_TILES) {
    const uint32_t per = (uint32_t)((L.n_tiles + 7) / 8);
    hipLaunchKernelGGL((composite_tiles_kernel<MODEL, TW, TH, STATE, NB>), dim3(per * 8),
                       dim3(TW * TH), 0, s, L.views, L.n_views, L.ranges, L.inst_val, L.rec, p,
                       pstate, (uint32_t)L.n_tiles, per);
  } else if (L.schedule == NXS_SCHED_BLOCKS) {
    const int64_t items = L.n_tiles * B;
    const uint32_t per = (uint32_t)((items + 7) / 8);
    hipLaunchKernelGGL((composite_blocks_kernel<MODEL, TW, TH, STATE, NB>), dim3(per * 8),
                       dim3(64), 0, s, L.views, L.n_views, L.ranges, L.inst_val, L.rec, p,
                       pstate, (uint32_t)items, per);
  } else if (L.schedule == NXS_SCHED_QUEUE) {
    const int64_t grid = (L.n_tiles + kQueues - 1) / kQueues * kQueues * B;
    hipLaunchKernelGGL((composite_ordered_kernel<MODEL, TW, TH, STATE, NB>), dim3((unsigned)grid),
                       dim3(64), 0, s, L.views, L.n_views, L.ranges, L.inst_val, L.rec, p,
                       pstate, L.order, (uint32_t)L.n_tiles);
  } else {
    int64_t grid = std::min<int64_t>(L.n_tiles, (int64_t)L.n_cu * kQueueWavesPerCU);
    grid = std::max<int64_t>((grid + kQueues - 1) / kQueues, 1) * kQueues;
    hipLaunchKernelGGL((composite_queue_kernel<MODEL, TW, TH, STATE, NB>), dim3((unsigned)grid),
                       dim3(64), 0, s, L.views, L.n_views, L.ranges, L.inst_val, L.rec, p,
                       pstate, L.order, (uint32_t)L.n_tiles, L.sched_counters);
  }
}

template <int MODEL, int TW, int TH, bool STATE>
void launch_b(const CompositeLaunch& L, const CompositeParams& p, float4* pstate,
              hipStream_t s) {
  if (p.lds_batch >= 256)
    launch_s<MODEL, TW, TH, STATE, 4>(L, p, pstate, s);
  else if (p.lds_batch >= 128)
    launch_s<MODEL, TW, TH, STATE, 2>(L, p, pstate, s);
  else
    launch_s<MODEL, TW, TH, STATE, 1>(L, p, pstate, s);
}

template <int MODEL, int TW, int TH>
void launch_t(const CompositeLaunch& L, const CompositeParams& p, float4* pstate,
              hipStream_t s) {
  // (state is kept only for the models that have a backward)
  if (MODEL <= 4 && pstate)
    launch_b<MODEL, TW, TH, MODEL <= 4>(L, p, pstate, s);
  else
    launch_b<MODEL, TW, TH, false>(L, p, pstate, s);
}

template <int MODEL>
void launch_m(const CompositeLaunch& L, const CompositeParams& p, float4* pstate,
              hipStream_t s) {
  if (L.tile_w == 8 && L.tile_h == 8)
    launch_t<MODEL, 8, 8>(L, p, pstate, s);
  else if (L.tile_w == 32 && L.tile_h == 8)
    launch_t<MODEL, 32, 8>(L, p, pstate, s);
  else
    launch_t<MODEL, 16, 16>(L, p, pstate, s);
}

}  // namespace

void launch_composite(int model, const CompositeLaunch& L, const CompositeParams& p,
                      float4* pstate, hipStream_t s) {
  if (L.n_tiles <= 0) return;
  switch (model) {
#define NXS_M(M) \
  case M: launch_m<M>(L, p, pstate, s); break;
    NXS_M(0) NXS_M(1) NXS_M(2) NXS_M(3) NXS_M(4) NXS_M(5) NXS_M(6) NXS_M(7)
#undef NXS_M
    default: break;
  }
}

}  // namespace nxs
