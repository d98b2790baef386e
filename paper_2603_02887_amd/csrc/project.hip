// EWA projection, culling, tile rectangle and composite coefficients.
//
// One thread per (Gaussian, view).  Two computations live here:
//   * the tile-key recipe in IEEE float32 (depth bits and covered tiles),
//     evaluated operation by operation in a fixed order with no fused
//     multiply-add, so that which tiles a Gaussian lands in, and at which
//     depth key, is reproducible bit for bit;
//   * the footprint used by the composite (Sec. 3: alpha = aleph * K): the
//     2D covariance with 0.3 px^2 dilation and its inverse, folded into the
//     exponent coefficients of log2(alpha); the centre in FP64, so that the
//     composite's pixel offsets keep ~1e-7 px accuracy.
// The emission is the real SH expansion (degree <= 3) at the direction from
// the camera centre to the mean, plus 1/2, clamped at 0.
//
// This translation unit is compiled with -ffp-contract=off; the pragma
// below keeps the recipe uncontracted regardless.
#include <hip/hip_fp16.h>

#include "nxs_internal.h"

#include <cstring>

namespace nxs {

namespace {

constexpr int kBlock = 256;

struct KeyGeom {
  bool visible;
  uint32_t depth_bits;
  int tx0, tx1, ty0, ty1;
  float A0[3], A1[3];   // J R R_q diag(s): Sigma2D = A A^T + 0.3 I
};

__device__ __forceinline__ KeyGeom key_recipe(const float* m, const float* s,
                                              const float* q, float aleph,
                                              const ViewDev& v, float kappa2,
                                              float alpha_min, int tile_w,
                                              int tile_h) {
#pragma clang fp contract(off)
  KeyGeom out;
  out.visible = false;
  out.depth_bits = 0xFFFFFFFFu;
  out.tx0 = out.tx1 = out.ty0 = out.ty1 = -1;
  const float* R = v.R;
  float px = ((R[0] * m[0] + R[1] * m[1]) + R[2] * m[2]) + v.t[0];
  float py = ((R[3] * m[0] + R[4] * m[1]) + R[5] * m[2]) + v.t[1];
  float pz = ((R[6] * m[0] + R[7] * m[1]) + R[8] * m[2]) + v.t[2];
  if (!(pz > v.znear) || !(aleph >= alpha_min)) return out;
  float n2 = ((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3];
  if (!(n2 > 0.0f)) return out;
  float nr = __fsqrt_rn(n2);
  float w = __fdiv_rn(q[0], nr), x = __fdiv_rn(q[1], nr);
  float y = __fdiv_rn(q[2], nr), z = __fdiv_rn(q[3], nr);
  float Rq[3][3];
  Rq[0][0] = 1.0f - 2.0f * (y * y + z * z);
  Rq[0][1] = 2.0f * (x * y - w * z);
  Rq[0][2] = 2.0f * (x * z + w * y);
  Rq[1][0] = 2.0f * (x * y + w * z);
  Rq[1][1] = 1.0f - 2.0f * (x * x + z * z);
  Rq[1][2] = 2.0f * (y * z - w * x);
  Rq[2][0] = 2.0f * (x * z - w * y);
  Rq[2][1] = 2.0f * (y * z + w * x);
  Rq[2][2] = 1.0f - 2.0f * (x * x + y * y);
  float M[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) M[i][j] = Rq[i][j] * s[j];
  float G[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      G[i][j] = (R[3 * i] * M[0][j] + R[3 * i + 1] * M[1][j]) + R[3 * i + 2] * M[2][j];
  float fxx = v.fx * px, fyy = v.fy * py, zz = pz * pz;
  float j00 = __fdiv_rn(v.fx, pz), j02 = -__fdiv_rn(fxx, zz);
  float j11 = __fdiv_rn(v.fy, pz), j12 = -__fdiv_rn(fyy, zz);
  float A0[3], A1[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    A0[j] = j00 * G[0][j] + j02 * G[2][j];
    A1[j] = j11 * G[1][j] + j12 * G[2][j];
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    out.A0[j] = A0[j];
    out.A1[j] = A1[j];
  }
  float a = ((A0[0] * A0[0] + A0[1] * A0[1]) + A0[2] * A0[2]) + 0.3f;
  float c = ((A1[0] * A1[0] + A1[1] * A1[1]) + A1[2] * A1[2]) + 0.3f;
  float u = __fdiv_rn(fxx, pz) + v.cx;
  float vv = __fdiv_rn(fyy, pz) + v.cy;
  float rx = __fsqrt_rn(kappa2 * a);
  float ry = __fsqrt_rn(kappa2 * c);
  if (!(isfinite(u) && isfinite(vv) && isfinite(rx) && isfinite(ry))) return out;
  float x0 = ceilf((u - rx) - 0.5f), x1 = floorf((u + rx) - 0.5f);
  float y0 = ceilf((vv - ry) - 0.5f), y1 = floorf((vv + ry) - 0.5f);
  x0 = x0 > 0.0f ? x0 : 0.0f;
  y0 = y0 > 0.0f ? y0 : 0.0f;
  float wm1 = (float)(v.width - 1), hm1 = (float)(v.height - 1);
  x1 = x1 < wm1 ? x1 : wm1;
  y1 = y1 < hm1 ? y1 : hm1;
  if (!(x0 <= x1) || !(y0 <= y1)) return out;
  out.visible = true;
  out.depth_bits = __float_as_uint(pz);
  out.tx0 = (int)x0 / tile_w;
  out.tx1 = (int)x1 / tile_w;
  out.ty0 = (int)y0 / tile_h;
  out.ty1 = (int)y1 / tile_h;
  return out;
}

// Real SH basis without the Condon-Shortley phase; index l*l + l + m.
// `sh` points at K*3 coefficients (channel fastest) in LDS.
template <int DEG>
__device__ __forceinline__ void sh_colour(const float* sh, float dx, float dy, float dz,
                                          float rgb[3]) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  float Y[K];
  Y[0] = 0.28209479177387814f;
  if (DEG >= 1) {
    const float c1 = 0.4886025119029199f;
    Y[1] = c1 * dy;
    Y[2] = c1 * dz;
    Y[3] = c1 * dx;
  }
  if (DEG >= 2) {
    const float c2a = 1.0925484305920792f;   // sqrt(15/pi)/2
    const float c2b = 0.31539156525252005f;  // sqrt(5/pi)/4
    const float c2c = 0.5462742152960396f;   // sqrt(15/pi)/4
    Y[4] = c2a * dx * dy;
    Y[5] = c2a * dy * dz;
    Y[6] = c2b * (3.0f * dz * dz - 1.0f);
    Y[7] = c2a * dx * dz;
    Y[8] = c2c * (dx * dx - dy * dy);
  }
  if (DEG >= 3) {
    const float c3a = 0.5900435899266435f;   // sqrt(35/(2pi))/4
    const float c3b = 2.890611442640554f;    // sqrt(105/pi)/2
    const float c3c = 0.4570457994644658f;   // sqrt(21/(2pi))/4
    const float c3d = 0.3731763325901154f;   // sqrt(7/pi)/4
    const float c3e = 1.445305721320277f;    // sqrt(105/pi)/4
    Y[9] = c3a * dy * (3.0f * dx * dx - dy * dy);
    Y[10] = c3b * dx * dy * dz;
    Y[11] = c3c * dy * (5.0f * dz * dz - 1.0f);
    Y[12] = c3d * dz * (5.0f * dz * dz - 3.0f);
    Y[13] = c3c * dx * (5.0f * dz * dz - 1.0f);
    Y[14] = c3e * dz * (dx * dx - dy * dy);
    Y[15] = c3a * dx * (dx * dx - 3.0f * dy * dy);
  }
  float r = 0.5f, g = 0.5f, b = 0.5f;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    r += Y[k] * sh[3 * k + 0];
    g += Y[k] * sh[3 * k + 1];
    b += Y[k] * sh[3 * k + 2];
  }
  rgb[0] = r > 0.0f ? r : 0.0f;
  rgb[1] = g > 0.0f ? g : 0.0f;
  rgb[2] = b > 0.0f ? b : 0.0f;
}

// A wave's reduction under an associative, commutative op (every lane active):
// within each 16-lane row by four DPP row shifts (a lane whose source lies
// before its row combines the identity), then the four rows' last lanes,
// read by readlane; the result is the same on every lane.
template <typename Op>
__device__ __forceinline__ uint32_t wave_reduce_u32(uint32_t x, uint32_t identity, Op op) {
  const int id = (int)identity;
  uint32_t v = x;
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, 0x111, 0xF, 0xF, false));
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, 0x112, 0xF, 0xF, false));
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, 0x114, 0xF, 0xF, false));
  v = op(v, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)v, 0x118, 0xF, 0xF, false));
  const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)v, 15);
  const uint32_t r1 = (uint32_t)__builtin_amdgcn_readlane((int)v, 31);
  const uint32_t r2 = (uint32_t)__builtin_amdgcn_readlane((int)v, 47);
  const uint32_t r3 = (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
  return op(op(r0, r1), op(r2, r3));
}
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x) {
  return wave_reduce_u32(x, 0u, [](uint32_t a, uint32_t b) { return a + b; });
}
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
  return wave_reduce_u32(x, 0xFFFFFFFFu, [](uint32_t a, uint32_t b) { return min(a, b); });
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
  return wave_reduce_u32(x, 0u, [](uint32_t a, uint32_t b) { return max(a, b); });
}

// One work-group of NT threads folds the per-block partials into the counters
// read by the host, plans the depth sort and, for a deferred render, checks
// that the render fits what was launched for it.
constexpr int kFoldThreads = 1024;
template <int NT>
__device__ void fold_partials(const uint4* partials, int nblocks, Counters* c,
                              const DeferCheck& chk) {
  __shared__ unsigned long long s_tot[NT / 64];
  __shared__ uint32_t s_mn[NT / 64], s_mx[NT / 64];
  unsigned long long tot = 0;
  uint32_t mn = 0xFFFFFFFFu, mx = 0u;
  // rounds of kFoldLoads partials per thread, each round's loads issued
  // before the first is used
  constexpr int kFoldLoads = 4;
  for (int b0 = 0; b0 < nblocks; b0 += NT * kFoldLoads) {
    uint4 p[kFoldLoads];
#pragma unroll
    for (int q = 0; q < kFoldLoads; ++q) {
      const int b = b0 + q * NT + (int)threadIdx.x;
      p[q] = b < nblocks ? partials[b] : make_uint4(0u, 0xFFFFFFFFu, 0u, 0u);
    }
#pragma unroll
    for (int q = 0; q < kFoldLoads; ++q) {
      tot += p[q].x;
      mn = min(mn, p[q].y);
      mx = max(mx, p[q].z);
    }
  }
  // (the 64-bit total as three 32-bit wave sums that cannot overflow: its
  // high word and the two 16-bit halves of its low word)
  {
    const uint32_t lo = (uint32_t)tot;
    const uint32_t hi = wave_sum_u32((uint32_t)(tot >> 32));
    const uint32_t l1 = wave_sum_u32(lo >> 16), l0 = wave_sum_u32(lo & 0xFFFFu);
    tot = ((unsigned long long)hi << 32) + ((unsigned long long)l1 << 16) + l0;
  }
  mn = wave_min_u32(mn);
  mx = wave_max_u32(mx);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    s_tot[wid] = tot;
    s_mn[wid] = mn;
    s_mx[wid] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < NT / 64; ++w) {
      tot += s_tot[w];
      mn = min(mn, s_mn[w]);
      mx = max(mx, s_mx[w]);
    }
    c->total = tot;
    c->dmin = mn;
    c->dmax = mx;
    // the depth sort needs the bits that vary among visible depths: three
    // balanced digits of at most kMaxDigitBits in passes 1..3 when they cover
    // them (pass 0 inactive), else four in passes 0..3
    const uint32_t diff = mn <= mx ? (mn ^ mx) : 0u;
    const int nbits = diff ? 32 - __clz((int)diff) : 0;
    const int first = nbits <= 3 * kMaxDigitBits ? 1 : 0;
    int shift = 0;
    c->plan[0] = 0u;
    for (int p = first; p < kPlanPasses; ++p) {
      const int w = (nbits - shift + (kPlanPasses - p) - 1) / (kPlanPasses - p);
      c->plan[p] = (uint32_t)shift | ((uint32_t)w << 8) | kPassActive;
      shift += w;
    }
    uint32_t fail = 0u;
    if (tot > chk.capacity) fail |= kFailCapacity;
    if (chk.first_pass > first) fail |= kFailPlan;
    c->fail = fail;
    if (chk.counters_host) {
      Counters* h = chk.counters_host;
      h->total = tot;
      h->dmin = mn;
      h->dmax = mx;
      for (int p = 0; p < kPlanPasses; ++p) h->plan[p] = c->plan[p];
      h->fail = fail;
    }
    if (chk.status) {
      DeferredStatus* st = chk.status;
      st->last = tot;
      st->last_fail = fail;
      if (fail) {
        st->need = max(st->need, tot);
        st->fail |= fail;
        st->count += 1u;
      }
      if (chk.status_host) *chk.status_host = *st;
    }
    // (the host reads the pinned copies once the kernel has completed)
    if (chk.counters_host || chk.status_host) __threadfence_system();
  }
}

// One work-group projects 256 consecutive Gaussians into every view.  The
// block's SH coefficients (contiguous in HBM) are staged into LDS with
// coalesced loads, padded to an odd stride so that per-thread reads are free
// of bank conflicts; each Gaussian's inputs are read once for all views.
// ARGS: the views come as the kernel argument `va`, and work-group 0 writes
// them to the device table `views` for the kernels that follow; otherwise
// they are read from `views`.
template <int DEG, bool ARGS>
__global__ __launch_bounds__(kBlock) void project_kernel(
    GaussDev g, ViewDev* __restrict__ views, ViewArgs va, int n_views, float kappa2,
    float alpha_min, int tile_w, int tile_h, ProjDev out, uint4* __restrict__ partials,
    uint32_t* __restrict__ clear, int64_t n_clear) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  if (ARGS && blockIdx.x == 0) {
    constexpr int kWords = (int)(sizeof(ViewDev) / 4);
    static_assert(sizeof(ViewDev) % 4 == 0, "the table is copied by words");
    const uint32_t* src = reinterpret_cast<const uint32_t*>(va.v);
    uint32_t* dst = reinterpret_cast<uint32_t*>(views);
    for (int w = threadIdx.x; w < n_views * kWords; w += kBlock) dst[w] = src[w];
  }
  // the tile ranges of this render start empty (the ranges pass fills in the
  // occupied tiles)
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n_clear;
       k += (int64_t)gridDim.x * kBlock)
    clear[k] = 0u;
  constexpr int NC = 3 * K;
  // The block's SH coefficients are staged in LDS, one row per Gaussian.
  // When a Gaussian's coefficients fill whole float4s (degrees 1 and 3), a
  // row is an odd number of float4s and every access is a 16-byte one: the
  // eight lanes served together then cover all 32 banks (conflict-free both
  // ways).  Otherwise rows are an odd number of floats, accessed by float.
  constexpr bool kVec = NC % 4 == 0;
  constexpr int NC4 = NC / 4;
  constexpr int STRIDE4 = NC4 % 2 == 1 ? NC4 : NC4 + 1;   // float4s per row (kVec)
  constexpr int STRIDE = kVec ? 4 * STRIDE4 : NC + 1;    // floats per row
  __shared__ __align__(16) float s_sh[kBlock * STRIDE];
  const int base = blockIdx.x * kBlock;
  const int cnt = min(kBlock, g.n - base);
  const int i = base + threadIdx.x;
  const bool valid = i < g.n;
  float m[3] = {0, 0, 0}, s[3] = {0, 0, 0}, q[4] = {0, 0, 0, 0}, aleph = 0.0f;
  auto load_params = [&]() {
    if (valid) {
      m[0] = g.means[3 * i]; m[1] = g.means[3 * i + 1]; m[2] = g.means[3 * i + 2];
      s[0] = g.scales[3 * i]; s[1] = g.scales[3 * i + 1]; s[2] = g.scales[3 * i + 2];
      q[0] = g.quats[4 * i]; q[1] = g.quats[4 * i + 1];
      q[2] = g.quats[4 * i + 2]; q[3] = g.quats[4 * i + 3];
      aleph = g.opac[i];
    }
  };
  // With degree 2 or 3 the Gaussian's own parameters are read first, so that
  // their loads are in flight with the coefficients' rather than after the
  // staging barrier (1080p, degree 3: 73 -> 70 us); with little to stage
  // they are read after it (degree 0: 77 against 79 us).
  constexpr bool kParamsFirst = DEG >= 2;
  if (kParamsFirst) load_params();
  {
    // every load of the block's coefficients is issued before any is used
    const float* src = g.sh + (int64_t)base * NC;
    const int nf = cnt * NC;
    const bool aligned = (reinterpret_cast<uintptr_t>(src) & 15u) == 0;
    if (kVec && aligned) {
      // NC4 float4 per thread, each stored whole into its row
      const float4* src4 = reinterpret_cast<const float4*>(src);
      float4* s4 = reinterpret_cast<float4*>(s_sh);
      const int n4 = cnt * NC4;
      float4 buf[NC4 > 0 ? NC4 : 1];
#pragma unroll
      for (int r = 0; r < NC4; ++r) {
        const int f = r * kBlock + threadIdx.x;
        buf[r] = f < n4 ? src4[f] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      }
#pragma unroll
      for (int r = 0; r < NC4; ++r) {
        const int f = r * kBlock + threadIdx.x;
        if (f < n4) s4[(f / NC4) * STRIDE4 + f % NC4] = buf[r];
      }
    } else if (aligned) {
      // NC/4 float4 per thread (the region is 16-byte aligned when sh is)
      constexpr int kIter = (kBlock * NC / 4 + kBlock - 1) / kBlock;
      float4 buf[kIter];
#pragma unroll
      for (int r = 0; r < kIter; ++r) {
        const int f = 4 * (r * kBlock + threadIdx.x);
        buf[r] = f + 3 < nf ? *reinterpret_cast<const float4*>(src + f)
                            : make_float4(f < nf ? src[f] : 0.0f,
                                          f + 1 < nf ? src[f + 1] : 0.0f,
                                          f + 2 < nf ? src[f + 2] : 0.0f, 0.0f);
      }
#pragma unroll
      for (int r = 0; r < kIter; ++r) {
        const int f = 4 * (r * kBlock + threadIdx.x);
        const float vals[4] = {buf[r].x, buf[r].y, buf[r].z, buf[r].w};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int e = f + c;
          if (e < nf) {
            const int gi = e / NC, j = e - gi * NC;
            s_sh[gi * STRIDE + j] = vals[c];
          }
        }
      }
    } else {
      for (int e = threadIdx.x; e < nf; e += kBlock) {
        const int gi = e / NC, j = e - gi * NC;
        s_sh[gi * STRIDE + j] = src[e];
      }
    }
  }
  __syncthreads();
  if (!kParamsFirst) load_params();
  uint32_t nt_sum = 0, dmin = 0xFFFFFFFFu, dmax = 0u;
  for (int vi = 0; vi < n_views; ++vi) {
    if (!valid) break;
    const ViewDev& v = ARGS ? va.v[vi] : views[vi];
    const int64_t slot = (int64_t)vi * g.n + i;
    KeyGeom kg = key_recipe(m, s, q, aleph, v, kappa2, alpha_min, tile_w, tile_h);
    uint2 rect = make_uint2(0xFFFFFFFFu, 0xFFFFFFFFu);
    uint32_t nt = 0;
    if (kg.visible) {
      dmin = min(dmin, kg.depth_bits);
      dmax = max(dmax, kg.depth_bits);
      rect = make_uint2((uint32_t)kg.tx0 | ((uint32_t)kg.tx1 << 16),
                        (uint32_t)kg.ty0 | ((uint32_t)kg.ty1 << 16));
      nt = rect_tile_count(rect);
      // ---- composite footprint ----------------------------------------------
      // Sigma2D = A A^T + 0.3 I from the recipe's A (float32).  Its determinant
      // by Cauchy-Binet, |A0 x A1|^2 + 0.3 (|A0|^2 + |A1|^2) + 0.09, is a sum
      // of non-negative terms: no cancellation, however elongated the splat.
      const float* A0 = kg.A0;
      const float* A1 = kg.A1;
      const float aa = A0[0] * A0[0] + A0[1] * A0[1] + A0[2] * A0[2];
      const float cc = A1[0] * A1[0] + A1[1] * A1[1] + A1[2] * A1[2];
      const float bb = A0[0] * A1[0] + A0[1] * A1[1] + A0[2] * A1[2];
      const float x0 = A0[1] * A1[2] - A0[2] * A1[1];
      const float x1 = A0[2] * A1[0] - A0[0] * A1[2];
      const float x2 = A0[0] * A1[1] - A0[1] * A1[0];
      const float a = aa + 0.3f, c = cc + 0.3f;
      const float det = (x0 * x0 + x1 * x1 + x2 * x2) + 0.3f * (aa + cc) + 0.09f;
      const float idet = 1.0f / det;
      // log2(alpha) = log2(aleph) - (1/2) log2(e) (cA dx^2 + 2 cB dx dy + cC dy^2)
      const float kL2e = 1.4426950408889634f;
      // image-plane centre in FP64 (kept as float hi + lo for the composite)
      const double px = ((double)v.R[0] * m[0] + (double)v.R[1] * m[1]) +
                        ((double)v.R[2] * m[2] + (double)v.t[0]);
      const double py = ((double)v.R[3] * m[0] + (double)v.R[4] * m[1]) +
                        ((double)v.R[5] * m[2] + (double)v.t[1]);
      const double pz = ((double)v.R[6] * m[0] + (double)v.R[7] * m[1]) +
                        ((double)v.R[8] * m[2] + (double)v.t[2]);
      const double iz = 1.0 / pz;
      const double u = (double)v.fx * px * iz + (double)v.cx;
      const double vv = (double)v.fy * py * iz + (double)v.cy;
      const float u_hi = (float)u, v_hi = (float)vv;
      // ---- emission -------------------------------------------------------
      const float ddx = m[0] - v.campos[0], ddy = m[1] - v.campos[1],
                  ddz = m[2] - v.campos[2];
      const float idn = 1.0f / sqrtf(ddx * ddx + ddy * ddy + ddz * ddz);
      float rgb[3];
      if (kVec) {
        // the row as whole float4s, into registers
        float coef[NC];
        const float4* row = reinterpret_cast<const float4*>(s_sh) + threadIdx.x * STRIDE4;
#pragma unroll
        for (int r = 0; r < NC4; ++r) {
          const float4 c4 = row[r];
          coef[4 * r + 0] = c4.x;
          coef[4 * r + 1] = c4.y;
          coef[4 * r + 2] = c4.z;
          coef[4 * r + 3] = c4.w;
        }
        sh_colour<DEG>(coef, ddx * idn, ddy * idn, ddz * idn, rgb);
      } else {
        sh_colour<DEG>(s_sh + threadIdx.x * STRIDE, ddx * idn, ddy * idn, ddz * idn, rgb);
      }
      // half-extents of the box where alpha >= alpha_min: q <= 2 ln(aleph / alpha_min),
      // q the Mahalanobis form of Sigma2D; enlarged, rounded up (to +inf beyond the
      // fp16 range), packed as fp16
      const float lo2 = __log2f(aleph);
      const float kq = fmaxf(2.0f * 0.6931471805599453f * (lo2 - __log2f(alpha_min)), 0.0f);
      const float ex = sqrtf(kq * a) * 1.001f + 0.01f;
      const float ey = sqrtf(kq * c) * 1.001f + 0.01f;
      const uint32_t hx = (uint32_t)__half_as_ushort(__float2half_ru(ex));
      const uint32_t hy = (uint32_t)__half_as_ushort(__float2half_ru(ey));
      float4* rec = out.rec + 3 * slot;
      rec[0] = make_float4(u_hi, (float)(u - (double)u_hi), v_hi, (float)(vv - (double)v_hi));
      rec[1] = make_float4(-0.5f * kL2e * c * idet, kL2e * bb * idet,
                           -0.5f * kL2e * a * idet, lo2);
      rec[2] = make_float4(rgb[0], rgb[1], rgb[2], __uint_as_float(hx | (hy << 16)));
    }
    out.depth_key[slot] = kg.depth_bits;
    out.trect[slot] = rect;
    nt_sum += nt;
  }
  // block reductions: instance total and visible depth-bit range
  __shared__ uint32_t s_sum[kBlock / 64], s_min[kBlock / 64], s_max[kBlock / 64];
  uint32_t ws = wave_sum_u32(nt_sum), wmn = wave_min_u32(dmin), wmx = wave_max_u32(dmax);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    s_sum[wid] = ws;
    s_min[wid] = wmn;
    s_max[wid] = wmx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0, mn = 0xFFFFFFFFu, mx = 0u;
    for (int k = 0; k < kBlock / 64; ++k) {
      tot += s_sum[k];
      mn = min(mn, s_min[k]);
      mx = max(mx, s_max[k]);
    }
    // one partial per block (no same-address atomics across thousands of
    // blocks; a device-scope fence per block to let the last one fold them
    // would write back L2 each time)
    partials[blockIdx.x] = make_uint4(tot, mn, mx, 0u);
  }
}

// One work-group folds the projection's per-block partials (none for a render
// with no Gaussians) into the counters read by the host.
__global__ __launch_bounds__(kFoldThreads) void reduce_counters_kernel(
    const uint4* __restrict__ partials, int nblocks, Counters* __restrict__ c,
    DeferCheck chk) {
  fold_partials<kFoldThreads>(partials, nblocks, c, chk);
}

}  // namespace

bool launch_project(const GaussDev& g, ViewDev* views, const ViewDev* host_views, int n_views,
                    float kappa2, float alpha_min, int tile_w, int tile_h,
                    const ProjDev& out, uint4* partials, Counters* counters,
                    const DeferCheck& check, uint32_t* clear, int64_t n_clear,
                    hipStream_t s) {
  const bool any = g.n > 0 && n_views > 0;
  const int nblocks = any ? (g.n + kBlock - 1) / kBlock : 0;
  const bool args = host_views && any && n_views <= kArgViews;
  ViewArgs va;
  std::memset(&va, 0, sizeof(va));
  if (args) std::memcpy(va.v, host_views, sizeof(ViewDev) * n_views);
#define NXS_PROJECT(D)                                                                     \
  if (args)                                                                                \
    hipLaunchKernelGGL((project_kernel<D, true>), dim3(nblocks), dim3(kBlock), 0, s, g,    \
                       views, va, n_views, kappa2, alpha_min, tile_w, tile_h, out,         \
                       partials, clear, n_clear);                                          \
  else                                                                                     \
    hipLaunchKernelGGL((project_kernel<D, false>), dim3(nblocks), dim3(kBlock), 0, s, g,   \
                       views, va, n_views, kappa2, alpha_min, tile_w, tile_h, out,         \
                       partials, clear, n_clear)
  if (any) {
    switch (g.sh_degree) {
      case 0: NXS_PROJECT(0); break;
      case 1: NXS_PROJECT(1); break;
      case 2: NXS_PROJECT(2); break;
      default: NXS_PROJECT(3); break;
    }
  } else {
    launch_fill_u32(clear, n_clear, 0u, s);
  }
#undef NXS_PROJECT
  hipLaunchKernelGGL(reduce_counters_kernel, dim3(1), dim3(kFoldThreads), 0, s, partials,
                     nblocks, counters, check);
  return args || !host_views;
}

size_t project_partials_size(int n) { return (size_t)((n + kBlock - 1) / kBlock) + 1; }

}  // namespace nxs
