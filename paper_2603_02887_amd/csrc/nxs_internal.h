// Internal declarations shared by the HIP translation units of libnxs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nxs.h"

namespace nxs {

// Per-view parameters, one entry per view in a device table.
struct ViewDev {
  float R[9];
  float t[3];
  float fx, fy, cx, cy, znear;
  float campos[3];          // camera centre in world space, -R^T t
  int32_t width, height;
  int32_t tiles_x, tiles_y;
  int32_t tile_off;         // first global tile of this view
  int32_t pad_;
  int64_t pix_off;          // first pixel of this view in per-pixel state buffers
  float* rgb;               // [H, W, 3]
  float* trans;             // [H, W]
  int32_t* od;              // [H, W] or null
  const float* g_rgb;       // backward: dLoss/drgb [H, W, 3]
  const float* g_trans;     // backward: dLoss/dtrans [H, W] or null
};

struct GaussDev {
  const float* means;
  const float* scales;
  const float* quats;
  const float* opac;
  const float* sh;
  int32_t n;
  int32_t sh_degree;
};

// Per projected slot (slot = view * n + gaussian) arrays written by the projection.
struct ProjDev {
  uint32_t* depth_key;      // float32 depth bits; 0xFFFFFFFF when culled
  // tile rectangle (tx0 | tx1 << 16, ty0 | ty1 << 16), all ones when culled;
  // the covered tiles are rect_tile_count(trect[slot])
  uint2* trect;
  // 3 float4 per slot:
  //   (u_hi, u_lo, v_hi, v_lo)  image-plane centre as float hi + lo parts
  //   (A', B', C', log2 aleph)  log2(alpha) = log2 aleph + A' dx^2 + B' dx dy + C' dy^2
  //   (r, g, b, 0)              emission
  float4* rec;
};

// Device counters filled by the projection: total instances, depth-bit range.
struct Counters {
  unsigned long long total;
  uint32_t dmin, dmax;
  // the depth sort's digits (shift | width << 8 | kPassActive per pass),
  // from dmin ^ dmax
  uint32_t plan[4];
  // a deferred render that cannot complete (kFail* bits; 0 otherwise): the
  // kernels after the emission then do nothing
  uint32_t fail;
  uint32_t pad_;
};
constexpr uint32_t kFailCapacity = 1u;   // more instances than the capacity
constexpr uint32_t kFailPlan = 2u;       // the depth sort skipped a pass it needs

// The outcome of the deferred renders on a context since the host last read
// it (device memory, cleared by the host).
struct DeferredStatus {
  unsigned long long need;   // largest instance count a failed render needed
  unsigned long long last;   // instance count of the latest deferred render
  uint32_t fail;             // OR of their kFail* bits
  uint32_t count;            // failed renders
  uint32_t last_fail;        // kFail* bits of the latest deferred render
  uint32_t pad_;
};

// What the projection's final fold checks for a deferred render, and where
// it also writes its results in pinned host memory (so that no copy command
// follows it).
struct DeferCheck {
  unsigned long long capacity;   // instance capacity (~0: not deferred)
  int first_pass;                // first depth-sort pass launched (0 or 1)
  DeferredStatus* status;        // device status, updated by every deferred render
  DeferredStatus* status_host;   // pinned copy of it after the update, or null
  Counters* counters_host;       // pinned copy of the counters, or null
};

// Inclusive sum over the lanes of a wave (every lane active): within each
// 16-lane row by four DPP row shifts (a lane whose source lies before its
// row adds 0), then the three lower rows' totals, read by readlane.  Integer
// sums: the same result as any other order.
__device__ __forceinline__ uint32_t wave_inclusive_scan_u32(uint32_t x) {
  int v = (int)x;
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, false);   // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, false);   // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false);   // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, false);   // row_shr:8
  const int r0 = __builtin_amdgcn_readlane(v, 15);
  const int r1 = __builtin_amdgcn_readlane(v, 31);
  const int r2 = __builtin_amdgcn_readlane(v, 47);
  const int row = (int)(threadIdx.x & 63) >> 4;
  v += (row >= 1 ? r0 : 0) + (row >= 2 ? r1 : 0) + (row >= 3 ? r2 : 0);
  return (uint32_t)v;
}

// The tiles a slot's rectangle covers (0 for a culled slot).
__device__ __forceinline__ uint32_t rect_tile_count(uint2 r) {
  if (r.x == 0xFFFFFFFFu) return 0u;
  return ((r.x >> 16) - (r.x & 0xFFFFu) + 1u) * ((r.y >> 16) - (r.y & 0xFFFFu) + 1u);
}

// The instance count a kernel after the emission works on: 0 for a failed
// deferred render.
__device__ __forceinline__ int64_t live_count(const Counters* c) {
  return c->fail ? 0 : (int64_t)c->total;
}

// Up to this many views travel to the projection as a kernel argument (the
// projection then writes the device view table the later kernels read), so
// that a render needs no host-to-device copy.
constexpr int kArgViews = 8;
struct ViewArgs {
  ViewDev v[kArgViews];
};

// ---- launchers (all enqueue on `s`) ------------------------------------------
// `partials` needs project_partials_size(n) entries.  Also sets `counters`
// (total instances, depth-bit range, depth-sort plan, fail bits from `check`)
// and zeroes clear[0, n_clear).  host_views: null, or the n_views <=
// kArgViews views (host memory, read during the call), which the projection
// writes to `views`; otherwise `views` must already hold them.  Returns
// false if host_views was given but cannot be used (no Gaussians): the
// caller then copies the table itself.
size_t project_partials_size(int n);
bool launch_project(const GaussDev& g, ViewDev* views, const ViewDev* host_views, int n_views,
                    float kappa2, float alpha_min, int tile_w, int tile_h,
                    const ProjDev& out, uint4* partials, Counters* counters,
                    const DeferCheck& check, uint32_t* clear, int64_t n_clear,
                    hipStream_t s);

constexpr int kPlanPasses = 4;
constexpr int kMaxDigitBits = 9;
constexpr uint32_t kPassActive = 1u << 16;

// Stable LSD radix sort of (u32 key, u32 value) pairs (reduce-then-scan,
// digits of up to kMaxDigitBits): sorts (keys_in, vals_in) by the low nbits
// of the keys (at least one pass), ping-ponging through (k0, v0) and (k1, v1);
// returns which pair holds the result (0 or 1).  vals_in == nullptr: values
// are the input positions.  `counts` needs radix_counts_words(n) u32.
// With `dn`, the number of pairs is read on the device (live_count(dn)) and
// n is only its upper bound, which sizes the counts layout; the grids are
// planned for n_plan pairs (0: n) and their work-groups loop over the chunks
// of a larger count.
size_t radix_counts_words(int64_t n);
int radix_sort(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* k0, uint32_t* v0,
               uint32_t* k1, uint32_t* v1, int64_t n, int nbits, uint32_t* counts,
               hipStream_t s, const Counters* dn = nullptr, int64_t n_plan = 0);
// The same sort with its digits read from device memory: plan[p] = shift |
// width << 8 | kPassActive for kPlanPasses passes (an active pass of width 0
// copies).  Passes 1..3 are always active, pass 0 only when three digits of
// kMaxDigitBits do not cover the varying bits.  Enough for keys of up to 32
// varying bits.  first_pass = 0 launches all four passes (an inactive pass 0
// does nothing and pass 1 then reads the input); first_pass = 1 launches
// passes 1..3 only, which is right only if the plan leaves pass 0 inactive
// (the caller checks plan[0] once it has read the counters, and sorts again
// with first_pass = 0 otherwise).  The result is in (k1, v1); returns 1.
// The last pass also writes, in sorted order, each value's tile rectangle
// from `trect` (indexed by value) and its tile count into rect_out / nt_out.
int radix_sort_planned(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* k0,
                       uint32_t* v0, uint32_t* k1, uint32_t* v1, int64_t n,
                       const uint32_t* plan, int first_pass, uint32_t* counts,
                       const uint2* trect, uint32_t* nt_out, uint2* rect_out, hipStream_t s);

// Exclusive scan of ntiles in sorted-slot order and emission of instances.
size_t scan_blocks_size(int64_t n);
// Exclusive scan of the depth-sorted tile counts (nt_sorted), or with
// nt_sorted null of the tile counts of the rectangles in slot order, per block
// of 512 slots (block totals in block_sums; scanned across blocks here
// only when there are more blocks than the emission sums itself).
void launch_emit_scan(const uint32_t* nt_sorted, const uint2* trect, int64_t n_slots,
                      uint32_t* scan_local, uint32_t* block_sums, hipStream_t s);
// Writes the instances of the depth-sorted slots (rectangles in
// rect_sorted), or with sorted_slots null of the slots in their own order
// (rectangles in trect); instances at positions >= capacity are not written.
void launch_emit_write(const uint32_t* sorted_slots, const uint2* rect_sorted,
                       const uint2* trect, int64_t n_slots, int32_t n_gauss,
                       const ViewDev* views, const uint32_t* scan_local,
                       const uint32_t* block_sums, uint32_t capacity, uint32_t* inst_tile,
                       uint32_t* inst_val, hipStream_t s);

// The tile-first order: after a stable sort by tile of instances emitted in
// slot order, each tile's list (ranges) is sorted stably by its slots'
// float32 depth bits (depth_key), in LDS up to kSegMax entries and through
// `temp` (the same positions) beyond; the bits that vary come from the
// projection's counters.  Nothing is done for a failed deferred render.
constexpr int kSegMax = 4096;
void launch_tile_depth_sort(const uint2* ranges, int64_t n_tiles, const uint32_t* depth_key,
                            const Counters* counters, uint32_t* list, uint32_t* temp,
                            hipStream_t s);




// Tile ranges: ranges[tile] = [first, end) of the tile's entries in the
// tile-sorted instance list (tiles without instances keep what the caller
// filled in, normally [0, 0)).
void launch_fill_u32(uint32_t* p, int64_t n, uint32_t value, hipStream_t s);
// m: the number of instances, or with `dn` its upper bound (the count itself
// is then read on the device; the grid is planned for m_plan instances and
// loops beyond them).
void launch_ranges(const uint32_t* inst_tile, int64_t m, uint2* ranges, hipStream_t s,
                   const Counters* dn = nullptr, int64_t m_plan = 0);

struct CompositeParams {
  float log2_alpha_min;
  float t_eps;              // exponential termination threshold (<= 0: never)
  float param;              // operator parameter (c, gamma or v) for models 4..7
  float bg[3];
  int32_t lds_batch;        // list entries gathered per round: 64, 128 or 256
};
// pstate: null, or 3 float4 per pixel kept for the backward pass:
//   (L0, L1, L2, T_final), (E_k, tau_k), (U, 0) with E_k the saturating splat's
//   emission (background if none), tau_k the optical depth before it and
//   U = sum_{j<k} E_j alpha_j.
// Composite launch geometry.  schedule: NXS_SCHED_TILES, NXS_SCHED_BLOCKS,
// NXS_SCHED_QUEUE or NXS_SCHED_PERSISTENT (the last two also need `order`
// [2 n_tiles] as scratch and kSchedCounters u32 counters that are zero at
// the launch: kQueues queue counters, then the length-bucket counters; the
// persistent one sizes its grid from the CU count).
struct CompositeLaunch {
  int schedule;
  int tile_w, tile_h;
  int64_t n_tiles;
  const ViewDev* views;
  int n_views;
  const uint2* ranges;
  const uint32_t* inst_val;  // tile-sorted list of projected slots
  const float4* rec;         // the projection's records, per slot
  uint32_t* order;
  uint32_t* sched_counters;
  int n_cu;
};
constexpr int kQueueWavesPerCU = 32;
constexpr int kQueues = 8;   // one per XCD
constexpr int kSchedCounters = 64;
// The tile order the queue schedules consume (longest tile lists first);
// enqueue before launch_composite for NXS_SCHED_QUEUE and NXS_SCHED_PERSISTENT
// (does nothing for the others).
void launch_composite_order(const CompositeLaunch& L, hipStream_t s);
void launch_composite(int model, const CompositeLaunch& L, const CompositeParams& p,
                      float4* pstate, hipStream_t s);

// Path-replay backward of the composite (models 0..4): per-slot moments
// gslot[9 * slot + f], f = sums over the slot's pixels of alpha dLoss/dalpha
// times (1, dx, dy, dx^2, dx dy, dy^2) and of p dLoss/dL (r, g, b),
// accumulated with atomics (the caller zeroes gslot; launch_project_bwd turns
// them into gradients).  `order`: the forward's
// tile order (longest lists first) to walk the tiles in, or null.
void launch_composite_bwd(int model, int tile_w, int tile_h, int64_t n_tiles,
                          const ViewDev* views, int n_views, const uint2* ranges,
                          const uint32_t* inst_val, const float4* rec, const CompositeParams& p,
                          const float4* pstate, float* gslot, const uint32_t* order,
                          hipStream_t s);

// Gradients of the Gaussians' parameters from the per-slot gradients (summed
// over views; overwrites the outputs).
struct GaussGradDev {
  float* means;
  float* scales;
  float* quats;
  float* opac;
  float* sh;
};
// gslot holds each slot's moments from the composite's backward on entry and
// its dL/d(opacity, u, v, A, B, C, r, g, b) on return.
void launch_project_bwd(const GaussDev& g, const ViewDev* views, int n_views,
                        float* gslot, const GaussGradDev& out, hipStream_t s);

// Measured peaks (peaks.hip): `groups` work-groups of independent FP32 FMA
// chains, `iters` steps each (peak_fma_flops of them, out: peak_fma_out_floats
// floats); a float4 copy of n4 elements (n4 < 2^39), one per thread.
int64_t peak_fma_flops(int groups, int iters);
size_t peak_fma_out_floats(int groups);
void launch_peak_fma(float* out, int groups, int iters, hipStream_t s);
void launch_peak_copy(const float4* src, float4* dst, int64_t n4, hipStream_t s);

// Waits for the context's work, then grows its instance buffers to `need`
// instances (api.hip; a pipeline grows every lane to what one of them needed).
nxs_status grow_instance_capacity(nxs_context* ctx, uint64_t need);

}  // namespace nxs
