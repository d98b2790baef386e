// Gather of splat records into a wave's LDS, batch by batch, for the
// composite and its backward (the tile's sorted list holds projected slots;
// their records stay where the projection wrote them).
#pragma once

#include <hip/hip_fp16.h>

#include "nxs_internal.h"

namespace nxs {

// Records staged per wave: 64 x 3 float4, in list order, only the splats
// whose footprint reaches the wave's 8x8 block:
//   (du, dv, A', B')   centre relative to the tile corner (pixels), conic terms
//   (C', lo, r, g)     log2(alpha) = lo + A' dx^2 + B' dx dy + C' dy^2; emission
//   (b, slot, 0, 0)    emission; the projected slot (view * n + Gaussian)
constexpr int kStageF4 = 3 * 64;

// Per-wave constants of the staging test.
struct StageBlock {
  float cu, cv;                 // tile corner (pixels)
  float x0, x1, y0, y1;         // pixel-centre extent of the block, tile-relative
  float amin;                   // log2(alpha_min)
};

template <int TW>
__device__ __forceinline__ StageBlock stage_block(int tx, int ty, int th, int wid,
                                                  float log2_alpha_min) {
  StageBlock b;
  b.cu = (float)(tx * TW);
  b.cv = (float)(ty * th);
  const int bx = (wid % (TW / 8)) * 8, by = (wid / (TW / 8)) * 8;
  b.x0 = (float)bx + 0.5f;
  b.x1 = (float)bx + 7.5f;
  b.y0 = (float)by + 0.5f;
  b.y1 = (float)by + 7.5f;
  b.amin = log2_alpha_min;
  return b;
}

// The block's extent cut down to the rows and columns that still hold a
// running pixel (bit 8 r + c of `act` is the pixel in row r, column c of the
// block; act != 0).  A splat that reaches none of those pixels would
// composite a = 0 on every running lane, so leaving it out of a batch
// changes no result; the cut only shrinks as pixels stop.
__device__ __forceinline__ StageBlock stage_shrink(const StageBlock& b, uint64_t act) {
  uint64_t c = act | (act >> 32);
  c |= c >> 16;
  c |= c >> 8;
  const uint32_t cols = (uint32_t)c & 0xFFu;
  uint64_t r = act | (act >> 1);
  r |= r >> 2;
  r |= r >> 4;
  r &= 0x0101010101010101ull;   // bit 8 k: row k holds a running pixel
  StageBlock s = b;
  s.x0 = b.x0 + (float)__builtin_ctz(cols);
  s.x1 = b.x0 + (float)(31 - __builtin_clz(cols));
  s.y0 = b.y0 + (float)(__builtin_ctzll(r) >> 3);
  s.y1 = b.y0 + (float)((63 - __builtin_clzll(r)) >> 3);
  return s;
}

// A batch's global reads, issued ahead of their use so that they are in
// flight while earlier batches are composited: lane j takes list entry
// base + j (if below end) and its slot (two batches ahead), then the slot's
// record (one batch ahead).  Every lane reads (past the end: the list's last
// entry again), so that no branch makes a read complete early.  Callers
// fetch only for a non-empty list (end > 0); for end = 0 the index would
// still be 0, never end - 1 wrapped around.
struct StageSlot {
  uint32_t slot;
  bool valid;
};
struct StageFetch {
  uint32_t slot;
  bool valid;
  float4 r0, r1, r2;
};

__device__ __forceinline__ StageSlot stage_slot(const uint32_t* __restrict__ inst_val,
                                                uint64_t base, uint32_t end, int lane) {
  StageSlot s;
  const uint64_t j = base + (uint64_t)lane;
  s.valid = j < end;
  s.slot = inst_val[s.valid ? (uint32_t)j : (end ? end - 1 : 0u)];
  return s;
}

__device__ __forceinline__ StageFetch stage_records(const StageSlot& s,
                                                    const float4* __restrict__ rec) {
  StageFetch f;
  f.slot = s.slot;
  f.valid = s.valid;
  const float4* r = rec + 3 * (size_t)s.slot;
  f.r0 = r[0];
  f.r1 = r[1];
  f.r2 = r[2];
  return f;
}

// A fetched splat's footprint in the frame of its tile: the tile-relative
// centre ((hi - corner) is exact, then + lo), the half-extents of its
// alpha >= alpha_min box (two fp16, rounded up) and the exponent terms of
// Q = -(e - lo) >= 0, with the bound qlim: e >= log2(alpha_min) <=> Q <= qlim
// (plus 2e-3 of margin in log2 units, so that float32 rounding can keep a
// splat that no pixel needs but never drop one that some pixel needs).
struct SplatGeom {
  float du, dv, rx, ry;
  float qa, qb, qc, qlim;
};

__device__ __forceinline__ SplatGeom splat_geom(const StageFetch& f, float cu, float cv,
                                                float amin) {
  SplatGeom g;
  g.du = (f.r0.x - cu) + f.r0.y;
  g.dv = (f.r0.z - cv) + f.r0.w;
  const uint32_t hx = __float_as_uint(f.r2.w);
  g.rx = __half2float(__ushort_as_half((unsigned short)(hx & 0xFFFFu)));
  g.ry = __half2float(__ushort_as_half((unsigned short)(hx >> 16)));
  g.qa = -f.r1.x;
  g.qb = -f.r1.y;
  g.qc = -f.r1.z;
  g.qlim = f.r1.w - amin + 2e-3f;
  return g;
}

// Whether the splat can reach alpha_min somewhere on the rectangle
// [x0, x1] x [y0, y1] of pixel centres (tile relative; x0 > x1 or y0 > y1:
// an empty rectangle, never reached): its box must overlap the rectangle and
// the smallest Q over the rectangle must be within qlim.
__device__ __forceinline__ bool reach_rect(const SplatGeom& g, float x0, float x1, float y0,
                                           float y1) {
  if (g.dv - g.ry > y1 || g.dv + g.ry < y0 || g.du - g.rx > x1 || g.du + g.rx < x0) return false;
  const float xlo = x0 - g.du, xhi = x1 - g.du;   // dx range over the rectangle
  const float ylo = y0 - g.dv, yhi = y1 - g.dv;   // dy range over the rectangle
  float qmin = 0.0f;
  const bool face_x = !(xlo <= 0.0f && xhi >= 0.0f);   // the centre is left or right
  const bool face_y = !(ylo <= 0.0f && yhi >= 0.0f);   // the centre is above or below
  if (face_x || face_y) {
    // the centre is outside: Q is convex, so its minimum over the rectangle
    // lies on an edge that faces the centre (at most one in x and one in y),
    // at the edge's own minimiser clamped to the edge (hardware reciprocals:
    // a relative error of ~1e-7 in the minimiser moves Q far less than the
    // margin)
    const float qa = g.qa, qb = g.qb, qc = g.qc;
    const float ia = 0.5f * __builtin_amdgcn_rcpf(qa), ic = 0.5f * __builtin_amdgcn_rcpf(qc);
    const float X = xlo > 0.0f ? xlo : xhi;
    const float y = fminf(fmaxf(-qb * X * ic, ylo), yhi);
    const float qx = X * (qa * X + qb * y) + qc * y * y;
    const float Y = ylo > 0.0f ? ylo : yhi;
    const float x = fminf(fmaxf(-qb * Y * ia, xlo), xhi);
    const float qy = Y * (qc * Y + qb * x) + qa * x * x;
    qmin = fminf(face_x ? qx : __builtin_inff(), face_y ? qy : __builtin_inff());
  }
  return qmin <= g.qlim;
}

// LDS operations of one wave complete in order: the reads that follow see the
// wave's earlier writes without a barrier; this keeps the compiler from
// moving them
__device__ __forceinline__ void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Keeps the splats whose footprint reaches the wave's block (reach_rect over
// the block's running rows and columns) and writes their records, in list
// order, to `wlds`; returns how many.
__device__ __forceinline__ uint32_t stage_batch(const StageFetch& f, const StageBlock& b,
                                                float4* wlds) {
  bool keep = false;
  SplatGeom g{};
  if (f.valid) {
    g = splat_geom(f, b.cu, b.cv, b.amin);
    keep = reach_rect(g, b.x0, b.x1, b.y0, b.y1);
  }
  const uint64_t sel = __builtin_amdgcn_ballot_w64(keep);
  if (keep) {
    // position among the kept lanes below this one
    const uint32_t pos = __builtin_amdgcn_mbcnt_hi(
        (uint32_t)(sel >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)sel, 0u));
    wlds[3 * pos + 0] = make_float4(g.du, g.dv, f.r1.x, f.r1.y);
    wlds[3 * pos + 1] = make_float4(f.r1.z, f.r1.w, f.r2.x, f.r2.y);
    wlds[3 * pos + 2] = make_float4(f.r2.z, __uint_as_float(f.slot), 0.0f, 0.0f);
  }
  wave_lds_order();
  return (uint32_t)__builtin_popcountll(sel);
}

// Work-group -> item mapping that gives each of the 8 XCDs (which receive
// work-groups round-robin) one contiguous band of items: neighbouring tiles,
// which share Gaussians, then read their records from the same L2.
__device__ __forceinline__ uint32_t xcd_banded(uint32_t wg, uint32_t per_xcd) {
  return (wg % 8u) * per_xcd + wg / 8u;
}

}  // namespace nxs
