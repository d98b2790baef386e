// Per-tile front-to-back composite with a pluggable transmittance operator.
//
// One work-group per screen tile, one thread per pixel; each wave owns an
// 8x8 pixel block of the tile and runs on its own (no LDS, no barriers).
// The tile's splats, gathered into depth order and contiguous in HBM, are
// the same for every lane of a wave, so they are read with scalar loads into
// SGPRs: no per-lane copies, no LDS bandwidth.  A splat whose footprint box
// misses the wave's block (one bit of its record) is skipped by a scalar
// branch.  Per pixel (Sec. 4, eq. generalized_gaussian and eq. nexp_p):
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
#include "nxs_internal.h"

namespace nxs {

namespace {

// Per-pixel state and update of a Table 1 operator.  MODEL: 0 exponential,
// 1 linear, 2 quadratic c = -0.5, 3 quadratic c = +0.5, 4 quadratic with
// c = param, 5 blended (gamma = param), 6 Vicini et al. (gamma = param),
// 7 power law (v = param).  `step` composites one splat of opacity a >=
// alpha_min and returns its p; `done` is set once the pixel stops.
template <int MODEL>
struct Op {
  float S = 0.0f;      // running sum of p (T = 1 - S)
  float tau = 0.0f;    // discrete optical depth
  float T = 1.0f;      // running product of (1 - a) (exponential parts)
  float S2 = 0.0f;     // Vicini: linear part's running sum
  bool d1 = false;     // Vicini: linear part saturated
  bool d2 = false;     // Vicini: exponential part stopped

  __device__ __forceinline__ float saturate(float p, bool& done) {
    const float Sn = S + p;
    done = Sn >= 1.0f;
    p = done ? 1.0f - S : p;
    S = done ? 1.0f : Sn;
    return p;
  }
  __device__ __forceinline__ float step(float a, float param, float t_eps, bool& done) {
    if (MODEL == 0) {
      const float p = a * T;
      T = T * (1.0f - a);
      done = !(T >= t_eps) || T == 0.0f;
      return p;
    } else if (MODEL == 1) {
      return saturate(a, done);
    } else if (MODEL <= 4) {
      const float c = MODEL == 2 ? -0.5f : MODEL == 3 ? 0.5f : param;
      const float p = a * fmaf(c, tau, 1.0f);
      tau += a;
      return saturate(p, done);
    } else if (MODEL == 5) {
      const float p = a * fmaf(param, T, 1.0f - param);
      T = T * (1.0f - a);
      return saturate(p, done);
    } else if (MODEL == 6) {
      float pl = 0.0f, pe = 0.0f;
      if (!d1) {
        const float Sn = S2 + a;
        d1 = Sn >= 1.0f;
        pl = d1 ? 1.0f - S2 : a;
        S2 = d1 ? 1.0f : Sn;
      }
      if (!d2) {
        pe = a * T;
        T = T * (1.0f - a);
        d2 = !(T >= t_eps) || T == 0.0f;
      }
      done = d1 && d2;
      return fmaf(param, pe - pl, pl);
    } else {
      const float base = fmaf(param, tau, 1.0f);
      tau += a;
      const float p = base > 0.0f
                          ? a * __builtin_amdgcn_exp2f(-(1.0f + param) / param *
                                                      __builtin_amdgcn_logf(base))
                          : __builtin_inff();
      return saturate(p, done);
    }
  }
  __device__ __forceinline__ float transmittance(float param) const {
    if (MODEL == 0) return T;
    if (MODEL == 6) return fmaf(param, T - (1.0f - S2), 1.0f - S2);
    return 1.0f - S;
  }
};

template <int MODEL, int TW, int TH>
__global__ __launch_bounds__(TW* TH) void composite_kernel(
    const ViewDev* __restrict__ views, int n_views, const uint2* __restrict__ ranges,
    const float4* __restrict__ crec, CompositeParams prm) {
  static_assert(TW % 8 == 0 && TH % 8 == 0, "waves cover 8x8 blocks");
  const uint32_t tile = blockIdx.x;
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
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int bx = (wid % (TW / 8)) * 8, by = (wid / (TW / 8)) * 8;   // wave's 8x8 block
  const int lx = bx + (lane & 7), ly = by + (lane >> 3);
  const int px = tx * TW + lx, py = ty * TH + ly;
  const bool inside = px < v.width && py < v.height;
  const float fx = (float)lx + 0.5f, fy = (float)ly + 0.5f;
  const uint32_t wbit = 1u << wid;

  const uint2 rg = ranges[tile];
  const float amin = prm.log2_alpha_min;
  const float t_eps = prm.t_eps;
  const float param = prm.param;
  Op<MODEL> op;

  float L0 = 0.0f, L1 = 0.0f, L2 = 0.0f;
  int od = 0;
  bool done = !inside;

  // Batches of 64 splats: lane j reads the block bits of splat (base + j)
  // (one coalesced load); a ballot gives the wave a bitmap of the splats whose
  // footprint reaches its 8x8 block.  Those are visited in order, each one's
  // fields read with scalar loads into SGPRs (no per-lane copies, no LDS).
  const float* crf = reinterpret_cast<const float*>(crec);
  bool all_done = __builtin_amdgcn_ballot_w64(!done) == 0;
  for (uint32_t base = rg.x; base < rg.y && !all_done; base += 64) {
    const uint32_t j = base + (uint32_t)lane;
    const uint32_t bits = j < rg.y ? __float_as_uint(crf[12 * (size_t)j + 9]) : 0u;
    uint64_t rel = __builtin_amdgcn_ballot_w64((bits & wbit) != 0);
    if (rel == 0) continue;
    // up to four relevant splats per step: their scalar loads are all issued
    // before the first is composited, so the load latency overlaps the work
    do {
      uint32_t kk[4];
      int cnt = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const bool have = rel != 0;
        kk[q] = have ? base + (uint32_t)__builtin_ctzll(rel) : kk[0];
        rel = have ? rel & (rel - 1) : 0ull;
        cnt += have ? 1 : 0;
      }
      float cur[4][9];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int f = 0; f < 9; ++f) cur[q][f] = crf[12 * (size_t)kk[q] + f];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (q < cnt && !done) {
          const float dx = fx - cur[q][0], dy = fy - cur[q][1];
          const float e =
              fmaf(dx, fmaf(cur[q][2], dx, cur[q][3] * dy), fmaf(cur[q][4] * dy, dy, cur[q][5]));
          if (e >= amin) {
            const float a = __builtin_amdgcn_exp2f(e);
            const float p = op.step(a, param, t_eps, done);
            L0 = fmaf(cur[q][6], p, L0);
            L1 = fmaf(cur[q][7], p, L1);
            L2 = fmaf(cur[q][8], p, L2);
            ++od;
          }
        }
      }
      all_done = __builtin_amdgcn_ballot_w64(!done) == 0;
    } while (rel != 0 && !all_done);
  }
  if (inside) {
    const float Tf = op.transmittance(param);
    const int64_t pix = (int64_t)py * v.width + px;
    v.rgb[3 * pix + 0] = L0 + prm.bg[0] * Tf;
    v.rgb[3 * pix + 1] = L1 + prm.bg[1] * Tf;
    v.rgb[3 * pix + 2] = L2 + prm.bg[2] * Tf;
    v.trans[pix] = Tf;
    if (v.od) v.od[pix] = od;
  }
}

template <int MODEL, int TW, int TH>
void launch_t(int64_t n_tiles, const ViewDev* views, int n_views, const uint2* ranges,
              const float4* crec, const CompositeParams& p, hipStream_t s) {
  hipLaunchKernelGGL((composite_kernel<MODEL, TW, TH>), dim3((unsigned)n_tiles),
                     dim3(TW * TH), 0, s, views, n_views, ranges, crec, p);
}

template <int MODEL>
void launch_m(int tile_w, int tile_h, int64_t n_tiles, const ViewDev* views, int n_views,
              const uint2* ranges, const float4* crec, const CompositeParams& p,
              hipStream_t s) {
  if (tile_w == 8 && tile_h == 8)
    launch_t<MODEL, 8, 8>(n_tiles, views, n_views, ranges, crec, p, s);
  else if (tile_w == 32 && tile_h == 8)
    launch_t<MODEL, 32, 8>(n_tiles, views, n_views, ranges, crec, p, s);
  else
    launch_t<MODEL, 16, 16>(n_tiles, views, n_views, ranges, crec, p, s);
}

}  // namespace

void launch_composite(int model, int tile_w, int tile_h, int64_t n_tiles,
                      const ViewDev* views, int n_views, const uint2* ranges,
                      const float4* crec, const CompositeParams& p, hipStream_t s) {
  if (n_tiles <= 0) return;
  switch (model) {
#define NXS_M(M) \
  case M: launch_m<M>(tile_w, tile_h, n_tiles, views, n_views, ranges, crec, p, s); break;
    NXS_M(0) NXS_M(1) NXS_M(2) NXS_M(3) NXS_M(4) NXS_M(5) NXS_M(6) NXS_M(7)
#undef NXS_M
    default: break;
  }
}

}  // namespace nxs
