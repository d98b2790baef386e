// Per-tile front-to-back composite with a pluggable transmittance operator.
//
// One work-group per screen tile, one thread per pixel.  The tile's splats,
// already gathered into depth order and contiguous in HBM, are staged into
// LDS in batches (coalesced loads); every pixel then walks the batch in
// order.  Per pixel (Sec. 4, eq. generalized_gaussian and eq. nexp_p):
//   alpha = aleph exp(-q/2), evaluated as exp2 of a precomputed quadratic;
//   splats with alpha < alpha_min are skipped;
//   p = alpha * T                (exponential, T <- T (1 - alpha))
//     = alpha                    (linear)
//     = alpha (1 + c tau)        (quadratic; tau <- tau + alpha)
//   if the running sum of p would reach 1, p takes the remainder, T becomes
//   exactly 0 and the pixel stops (saturation); the exponential also stops
//   after the first splat that leaves T < t_eps;
//   L += E p, overdraw += 1 for every composited splat.
// A pixel that has stopped leaves the inner loop; the work-group leaves the
// tile as soon as a block-wide vote finds every pixel stopped.
#include "nxs_internal.h"

namespace nxs {

namespace {

template <int MODEL>
struct OpC;
template <> struct OpC<0> { static constexpr float c = 0.0f; };   // exponential
template <> struct OpC<1> { static constexpr float c = 0.0f; };   // linear
template <> struct OpC<2> { static constexpr float c = -0.5f; };  // quadratic, sublinear
template <> struct OpC<3> { static constexpr float c = 0.5f; };   // quadratic, superlinear

template <int MODEL, int TW, int TH, int BATCH>
__global__ __launch_bounds__(TW* TH) void composite_kernel(
    const ViewDev* __restrict__ views, int n_views, const uint2* __restrict__ ranges,
    const float4* __restrict__ rec0, const float4* __restrict__ rec1,
    const float* __restrict__ rec2, CompositeParams prm) {
  constexpr int NT = TW * TH;
  __shared__ float4 s0[BATCH];
  __shared__ float4 s1[BATCH];
  __shared__ float s2[BATCH];

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
  const int lx = threadIdx.x % TW, ly = threadIdx.x / TW;
  const int px = tx * TW + lx, py = ty * TH + ly;
  const bool inside = px < v.width && py < v.height;
  const float fx = (float)lx + 0.5f, fy = (float)ly + 0.5f;

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

  for (uint32_t base = rg.x; base < rg.y; base += BATCH) {
    if (!__syncthreads_or(!done)) break;
    const int cnt = (int)min((uint32_t)BATCH, rg.y - base);
    for (int i = threadIdx.x; i < cnt; i += NT) {
      s0[i] = rec0[base + i];
      s1[i] = rec1[base + i];
      s2[i] = rec2[base + i];
    }
    __syncthreads();
    if (!done) {
      for (int k = 0; k < cnt; ++k) {
        const float4 g0 = s0[k];   // du, dv, A', B'
        const float4 g1 = s1[k];   // C', log2(aleph), r, g
        const float dx = fx - g0.x, dy = fy - g0.y;
        const float e = g1.y + dx * (g0.z * dx + g0.w * dy) + g1.x * dy * dy;
        if (e < amin) continue;
        const float a = __builtin_amdgcn_exp2f(e);
        float p;
        if (MODEL == 0) {
          p = a * T;
          T = T * (1.0f - a);
          if (!(T >= t_eps) || T == 0.0f) done = true;
        } else {
          p = (MODEL == 1) ? a : a * (1.0f + c * tau);
          if (MODEL >= 2) tau += a;
          const float Sn = S + p;
          if (Sn >= 1.0f) {
            p = 1.0f - S;
            S = 1.0f;
            done = true;
          } else {
            S = Sn;
          }
        }
        L0 += g1.z * p;
        L1 += g1.w * p;
        L2 += s2[k] * p;
        ++od;
        if (done) break;
      }
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
void launch_b(int64_t n_tiles, int batch, const ViewDev* views, int n_views,
              const uint2* ranges, const float4* r0, const float4* r1, const float* r2,
              const CompositeParams& p, hipStream_t s) {
  dim3 grid((unsigned)n_tiles), block(TW * TH);
  switch (batch) {
    case 128:
      hipLaunchKernelGGL((composite_kernel<MODEL, TW, TH, 128>), grid, block, 0, s, views,
                         n_views, ranges, r0, r1, r2, p);
      break;
    case 512:
      hipLaunchKernelGGL((composite_kernel<MODEL, TW, TH, 512>), grid, block, 0, s, views,
                         n_views, ranges, r0, r1, r2, p);
      break;
    default:
      hipLaunchKernelGGL((composite_kernel<MODEL, TW, TH, 256>), grid, block, 0, s, views,
                         n_views, ranges, r0, r1, r2, p);
  }
}

template <int MODEL>
void launch_m(int tile_w, int tile_h, int64_t n_tiles, const ViewDev* views, int n_views,
              const uint2* ranges, const float4* r0, const float4* r1, const float* r2,
              const CompositeParams& p, hipStream_t s) {
  if (tile_w == 8 && tile_h == 8)
    launch_b<MODEL, 8, 8>(n_tiles, p.lds_batch, views, n_views, ranges, r0, r1, r2, p, s);
  else if (tile_w == 32 && tile_h == 8)
    launch_b<MODEL, 32, 8>(n_tiles, p.lds_batch, views, n_views, ranges, r0, r1, r2, p, s);
  else
    launch_b<MODEL, 16, 16>(n_tiles, p.lds_batch, views, n_views, ranges, r0, r1, r2, p, s);
}

}  // namespace

void launch_composite(int model, int tile_w, int tile_h, int64_t n_tiles,
                      const ViewDev* views, int n_views, const uint2* ranges,
                      const float4* rec0, const float4* rec1, const float* rec2,
                      const CompositeParams& p, hipStream_t s) {
  if (n_tiles <= 0) return;
  switch (model) {
    case 0: launch_m<0>(tile_w, tile_h, n_tiles, views, n_views, ranges, rec0, rec1, rec2, p, s); break;
    case 1: launch_m<1>(tile_w, tile_h, n_tiles, views, n_views, ranges, rec0, rec1, rec2, p, s); break;
    case 2: launch_m<2>(tile_w, tile_h, n_tiles, views, n_views, ranges, rec0, rec1, rec2, p, s); break;
    default: launch_m<3>(tile_w, tile_h, n_tiles, views, n_views, ranges, rec0, rec1, rec2, p, s); break;
  }
}

}  // namespace nxs
