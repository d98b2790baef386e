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
#include "nxs_ops.h"

namespace nxs {

namespace {

template <int MODEL, int TW, int TH, bool STATE>
__global__ __launch_bounds__(TW* TH) void composite_kernel(
    const ViewDev* __restrict__ views, int n_views, const uint2* __restrict__ ranges,
    const float4* __restrict__ crec, CompositeParams prm, float4* __restrict__ pstate) {
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
  // backward state (linear and quadratic): E_k, tau_k, U
  constexpr bool kSat = STATE && MODEL >= 1 && MODEL <= 4;
  float ek0 = prm.bg[0], ek1 = prm.bg[1], ek2 = prm.bg[2], tau_s = 0.0f;
  float u0 = 0.0f, u1 = 0.0f, u2 = 0.0f;

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
            if (kSat) {
              if (done) {
                ek0 = cur[q][6];
                ek1 = cur[q][7];
                ek2 = cur[q][8];
              } else {
                u0 = fmaf(cur[q][6], a, u0);
                u1 = fmaf(cur[q][7], a, u1);
                u2 = fmaf(cur[q][8], a, u2);
                tau_s += a;
              }
            }
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
    if (STATE) {
      float4* st = pstate + 3 * (v.pix_off + pix);
      st[0] = make_float4(L0 + prm.bg[0] * Tf, L1 + prm.bg[1] * Tf, L2 + prm.bg[2] * Tf, Tf);
      st[1] = make_float4(ek0, ek1, ek2, tau_s);
      st[2] = make_float4(u0, u1, u2, 0.0f);
    }
  }
}

template <int MODEL, int TW, int TH>
void launch_t(int64_t n_tiles, const ViewDev* views, int n_views, const uint2* ranges,
              const float4* crec, const CompositeParams& p, float4* pstate, hipStream_t s) {
  if (pstate)
    hipLaunchKernelGGL((composite_kernel<MODEL, TW, TH, true>), dim3((unsigned)n_tiles),
                       dim3(TW * TH), 0, s, views, n_views, ranges, crec, p, pstate);
  else
    hipLaunchKernelGGL((composite_kernel<MODEL, TW, TH, false>), dim3((unsigned)n_tiles),
                       dim3(TW * TH), 0, s, views, n_views, ranges, crec, p, pstate);
}

template <int MODEL>
void launch_m(int tile_w, int tile_h, int64_t n_tiles, const ViewDev* views, int n_views,
              const uint2* ranges, const float4* crec, const CompositeParams& p,
              float4* pstate, hipStream_t s) {
  if (tile_w == 8 && tile_h == 8)
    launch_t<MODEL, 8, 8>(n_tiles, views, n_views, ranges, crec, p, pstate, s);
  else if (tile_w == 32 && tile_h == 8)
    launch_t<MODEL, 32, 8>(n_tiles, views, n_views, ranges, crec, p, pstate, s);
  else
    launch_t<MODEL, 16, 16>(n_tiles, views, n_views, ranges, crec, p, pstate, s);
}

}  // namespace

void launch_composite(int model, int tile_w, int tile_h, int64_t n_tiles,
                      const ViewDev* views, int n_views, const uint2* ranges,
                      const float4* crec, const CompositeParams& p, float4* pstate,
                      hipStream_t s) {
  if (n_tiles <= 0) return;
  switch (model) {
#define NXS_M(M) \
  case M: launch_m<M>(tile_w, tile_h, n_tiles, views, n_views, ranges, crec, p, pstate, s); break;
    NXS_M(0) NXS_M(1) NXS_M(2) NXS_M(3) NXS_M(4) NXS_M(5) NXS_M(6) NXS_M(7)
#undef NXS_M
    default: break;
  }
}

}  // namespace nxs
