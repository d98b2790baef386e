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

template <int MODEL>
struct OpC;
template <> struct OpC<0> { static constexpr float c = 0.0f; };   // exponential
template <> struct OpC<1> { static constexpr float c = 0.0f; };   // linear
template <> struct OpC<2> { static constexpr float c = -0.5f; };  // quadratic, sublinear
template <> struct OpC<3> { static constexpr float c = 0.5f; };   // quadratic, superlinear

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
  constexpr float c = OpC<MODEL>::c;

  float L0 = 0.0f, L1 = 0.0f, L2 = 0.0f;
  float T = 1.0f;      // exponential: running product; others: 1 - S
  float S = 0.0f;      // running sum of p (non-exponential)
  float tau = 0.0f;    // discrete optical depth (quadratic)
  int od = 0;
  bool done = !inside;

  // Batches of 64 splats: lane j loads splat (base + j) into registers with
  // coalesced loads; a ballot of the block bits gives the wave a bitmap of the
  // splats whose footprint reaches its 8x8 block; those are visited in order,
  // each field broadcast from its lane into a scalar register.
  for (uint32_t base = rg.x; base < rg.y; base += 64) {
    if (__builtin_amdgcn_ballot_w64(!done) == 0) break;
    const uint32_t j = base + (uint32_t)lane;
    float4 q0 = make_float4(0.f, 0.f, 0.f, 0.f), q1 = q0, q2 = q0;
    if (j < rg.y) {
      q0 = crec[3 * (size_t)j];
      q1 = crec[3 * (size_t)j + 1];
      q2 = crec[3 * (size_t)j + 2];
    }
    uint64_t rel = __builtin_amdgcn_ballot_w64((__float_as_uint(q2.y) & wbit) != 0);
    while (rel) {
      const int k = __builtin_ctzll(rel);
      rel &= rel - 1;
      const float s_du = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(q0.x), k));
      const float s_dv = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(q0.y), k));
      const float s_A = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(q0.z), k));
      const float s_B = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(q0.w), k));
      const float s_C = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(q1.x), k));
      const float s_lo = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(q1.y), k));
      if (!done) {
        const float dx = fx - s_du, dy = fy - s_dv;
        const float e = fmaf(dx, fmaf(s_A, dx, s_B * dy), fmaf(s_C * dy, dy, s_lo));
        if (e >= amin) {
          const float a = __builtin_amdgcn_exp2f(e);
          float p;
          if (MODEL == 0) {
            p = a * T;
            T = T * (1.0f - a);
            done = !(T >= t_eps) || T == 0.0f;
          } else {
            p = (MODEL == 1) ? a : a * fmaf(c, tau, 1.0f);
            if (MODEL >= 2) tau += a;
            const float Sn = S + p;
            done = Sn >= 1.0f;
            p = done ? 1.0f - S : p;
            S = done ? 1.0f : Sn;
          }
          const float s_r = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(q1.z), k));
          const float s_g = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(q1.w), k));
          const float s_b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(q2.x), k));
          L0 = fmaf(s_r, p, L0);
          L1 = fmaf(s_g, p, L1);
          L2 = fmaf(s_b, p, L2);
          ++od;
        }
      }
      if (__builtin_amdgcn_ballot_w64(!done) == 0) break;
    }
  }
  if (inside) {
    const float Tf = (MODEL == 0) ? T : 1.0f - S;
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
    case 0: launch_m<0>(tile_w, tile_h, n_tiles, views, n_views, ranges, crec, p, s); break;
    case 1: launch_m<1>(tile_w, tile_h, n_tiles, views, n_views, ranges, crec, p, s); break;
    case 2: launch_m<2>(tile_w, tile_h, n_tiles, views, n_views, ranges, crec, p, s); break;
    default: launch_m<3>(tile_w, tile_h, n_tiles, views, n_views, ranges, crec, p, s); break;
  }
}

}  // namespace nxs
