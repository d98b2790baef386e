// Path-replay backward of the render (models 0..4) and of the projection.
//
// composite_bwd: each wave re-walks its 8x8 block's splats front to back
// exactly as the forward did (the same records staged in LDS in the same
// order, the same float32 decisions), rebuilding each pixel's state from the start instead of
// storing anything per splat.  The adjoint of every composited splat comes
// from quantities the forward left per pixel:
//   exponential   dL/dalpha_i = T_i E_i - R_{i+1} / (1 - alpha_i), with the
//                 radiance behind the splat R_{i+1} = L - sum_{j<=i} E_j p_j
//                 (the last composited splat uses T_k (E_k - L_b));
//   linear and    dL/dalpha_i = (E_i - E_k)(1 + c tau_i) + c Theta_i,
//   quadratic     Theta_i = sum_{i<j<k} (E_j - E_k) alpha_j, rebuilt from its
//                 total U - E_k tau_k; dL/dalpha_k = 0 for the saturating
//                 splat (appendix "Adjoints": eq. generalized_gaussians_gen
//                 and the two recursions that follow it);
//   every model   dL/dE_i = p_i.
// The final transmittance rides along as a fourth channel with emission 0 and
// background 1, so dLoss/dtrans needs no separate code.  Each splat's
// per-pixel moments alpha dL/dalpha (1, dx, dy, dx^2, dx dy, dy^2) and
// p (dL/dL_rgb) are summed over the wave and added once per wave into its
// slot (dx, dy: the pixel centre relative to the splat's).
//
// project_bwd: one thread per Gaussian turns each view's slot moments into
// dL/d(opacity, centre, conic, colour) (written back to the slot) and chains
// them through the conic inverse, the EWA covariance, the perspective
// Jacobian, the rotation and scales, and the SH emission.
#include "nxs_internal.h"
#include "nxs_ops.h"
#include "nxs_stage.h"

namespace nxs {

namespace {

constexpr float kL2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;   // 1 / log2(e)

// Sum over each row of 16 lanes with DPP adds (VALU only): pairs and quads
// by quad_perm, then half-rows and rows by mirror patterns; every lane of a
// row ends with the row's total.
// (no contraction: an add of the moved value folds into one DPP add, which a
// product of the caller fused into an FMA with it would prevent)
template <int CTRL>
__device__ __forceinline__ float dpp_add(float x) {
#pragma clang fp contract(off)
  const int y = __builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, true);
  return x + __int_as_float(y);
}
__device__ __forceinline__ float quad_total(float x) {
  x = dpp_add<0xB1>(x);    // quad_perm [1,0,3,2]
  x = dpp_add<0x4E>(x);    // quad_perm [2,3,0,1]
  return x;
}

// Per-wave sums of the 9 per-pixel fields of up to kRedSplats splats at a
// time: each splat's fields are summed over lane quads (two DPP adds each)
// and the quads' first lanes write the 16 quad sums of field f to row
// 9 j + f of the wave's table (j: the splat's place among the pending ones);
// a flush has lane r add row r's 16 sums and issue its atomic.
constexpr int kRedSplats = 4;                    // 36 rows: one per lane
constexpr int kRedF4 = 9 * kRedSplats * 16 / 4;  // float4 per wave

template <int MODEL, int TW, int TH>
__global__ __launch_bounds__(TW* TH) void composite_bwd_kernel(
    const ViewDev* __restrict__ views, int n_views, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ inst_val, const float4* __restrict__ rec, CompositeParams prm,
    const float4* __restrict__ pstate, float* __restrict__ gslot, uint32_t n_tiles,
    uint32_t per_xcd, const uint32_t* __restrict__ order) {
  __shared__ float4 stage[(TW / 8) * (TH / 8) * kStageF4];
  __shared__ float4 rsum[(TW / 8) * (TH / 8) * kRedF4];   // per wave: pending quad sums
  __shared__ uint32_t rslot[(TW / 8) * (TH / 8) * kRedSplats];   // and their slots
  // the forward's order (longest tile lists first) when it made one, else
  // each XCD a contiguous band of tiles
  const uint32_t w = order ? blockIdx.x : xcd_banded(blockIdx.x, per_xcd);
  if (w >= n_tiles) return;
  const uint32_t tile = order ? order[w] : w;
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
  const int bx = (wid % (TW / 8)) * 8, by = (wid / (TW / 8)) * 8;
  const int lx = bx + (lane & 7), ly = by + (lane >> 3);
  const int px = tx * TW + lx, py = ty * TH + ly;
  const bool inside = px < v.width && py < v.height;
  const float fx = (float)lx + 0.5f, fy = (float)ly + 0.5f;
  const StageBlock sb = stage_block<TW>(tx, ty, TH, wid, prm.log2_alpha_min);
  float4* wlds = stage + wid * kStageF4;
  float* wred = reinterpret_cast<float*>(rsum + wid * kRedF4);
  uint32_t* wslot = rslot + wid * kRedSplats;
  const uint2 rg = ranges[tile];
  const float amin = prm.log2_alpha_min;
  const float t_eps = prm.t_eps;
  const float param = prm.param;
  constexpr float kc = MODEL == 2 ? -0.5f : MODEL == 3 ? 0.5f : 0.0f;
  const float c = MODEL == 4 ? param : kc;

  // upstream gradient (g0, g1, g2, gT) and what the forward left per pixel
  float g0 = 0.f, g1 = 0.f, g2 = 0.f, gT = 0.f;
  float4 s0 = make_float4(0.f, 0.f, 0.f, 1.f), s1 = make_float4(0.f, 0.f, 0.f, 0.f),
         s2 = s1;
  if (inside) {
    const int64_t pix = (int64_t)py * v.width + px;
    g0 = v.g_rgb[3 * pix + 0];
    g1 = v.g_rgb[3 * pix + 1];
    g2 = v.g_rgb[3 * pix + 2];
    gT = v.g_trans ? v.g_trans[pix] : 0.0f;
    const float4* st = pstate + 3 * (v.pix_off + pix);
    s0 = st[0];
    s1 = st[1];
    s2 = st[2];
  }
  // exponential: radiance not yet attributed, 4 channels (rgb, T)
  float R0 = s0.x, R1 = s0.y, R2 = s0.z, R3 = s0.w;
  // linear / quadratic: E_k (4 channels) and Theta (4 channels)
  const bool saturated = s0.w == 0.0f;
  const float k0 = s1.x, k1 = s1.y, k2 = s1.z, k3 = saturated ? 0.0f : 1.0f;
  float th0 = s2.x - k0 * s1.w, th1 = s2.y - k1 * s1.w, th2 = s2.z - k2 * s1.w,
        th3 = -k3 * s1.w;

  Op<MODEL> op;
  bool done = !inside;
  // running lanes; each batch is staged against the rows and columns that
  // still hold one
  uint64_t act = __builtin_amdgcn_ballot_w64(!done);
  // (an empty tile fetches nothing: its range is [0, 0) or [x, x))
  StageSlot slots{0u, false};
  StageFetch fetched{};
  if (rg.x < rg.y) {
    slots = stage_slot(inst_val, rg.x, rg.y, lane);
    fetched = stage_records(slots, rec);
    slots = stage_slot(inst_val, (uint64_t)rg.x + 64, rg.y, lane);
  }
  // the pending splats' sums: lane r < 9 pend adds row r and issues its atomic
  uint32_t pend = 0;
  auto flush = [&]() {
    wave_lds_order();
    if (lane < 9 * (int)pend) {
      const float4* q = reinterpret_cast<const float4*>(wred + 16 * lane);
      const float4 a0 = q[0], a1 = q[1], a2 = q[2], a3 = q[3];
      const float sum = ((a0.x + a0.y) + (a0.z + a0.w)) + ((a1.x + a1.y) + (a1.z + a1.w)) +
                        (((a2.x + a2.y) + (a2.z + a2.w)) + ((a3.x + a3.y) + (a3.z + a3.w)));
      const int j = (lane * 57) >> 9;   // lane / 9 for lane < 64
      atomicAdd(gslot + 9 * (size_t)wslot[j] + (lane - 9 * j), sum);
    }
    wave_lds_order();
    pend = 0;
  };
  for (uint32_t base = rg.x; base < rg.y && act != 0; base += 64) {
    const uint32_t n = stage_batch(fetched, stage_shrink(sb, act), wlds);
    fetched = stage_records(slots, rec);                              // batch base + 64
    slots = stage_slot(inst_val, (uint64_t)base + 128, rg.y, lane);   // batch base + 128
    for (uint32_t k = 0; k < n && act != 0; ++k) {
      const float4 q0 = wlds[3 * k + 0], q1 = wlds[3 * k + 1], q2 = wlds[3 * k + 2];
      const float r[10] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w, q2.x, q2.y};
      // Every lane runs the same arithmetic: a lane that has stopped, or
      // whose alpha is below alpha_min, takes a = 0 and dL/dalpha = 0, which
      // leaves its state unchanged and makes each of its terms an exact zero.
      const float dx = fx - r[0], dy = fy - r[1];
      const float e = fmaf(dx, fmaf(r[2], dx, r[3] * dy), fmaf(r[4] * dy, dy, r[5]));
      const bool contrib = !done && e >= amin;
      const float a = contrib ? __builtin_amdgcn_exp2f(e) : 0.0f;
      const float T_before = op.T, tau_before = op.tau;
      bool stops;
      const float p = op.step(a, param, t_eps, stops);
      float dalpha = 0.0f;
      if (MODEL == 0) {
        R0 -= r[6] * p;
        R1 -= r[7] * p;
        R2 -= r[8] * p;
      }
      if (contrib) {
        if (MODEL == 0) {
          if (stops) {
            dalpha = T_before * (g0 * (r[6] - prm.bg[0]) + g1 * (r[7] - prm.bg[1]) +
                                 g2 * (r[8] - prm.bg[2]) - gT);
          } else {
            // (1 - a > 0 here: a splat with a = 1 leaves T = 0 and stops the pixel)
            const float inv = __builtin_amdgcn_rcpf(1.0f - a);
            dalpha = T_before * (g0 * r[6] + g1 * r[7] + g2 * r[8]) -
                     inv * (g0 * R0 + g1 * R1 + g2 * R2 + gT * R3);
          }
        } else if (!stops) {   // the saturating splat takes the remainder: 0
          const float e0 = r[6] - k0, e1 = r[7] - k1, e2 = r[8] - k2, e3 = -k3;
          th0 -= e0 * a;
          th1 -= e1 * a;
          th2 -= e2 * a;
          th3 -= e3 * a;
          const float w = fmaf(c, tau_before, 1.0f);
          dalpha = g0 * fmaf(e0, w, c * th0) + g1 * fmaf(e1, w, c * th1) +
                   g2 * fmaf(e2, w, c * th2) + gT * fmaf(e3, w, c * th3);
        }
      }
      done = done || stops;
      // alpha = aleph exp(-q/2), q = A dx^2 + 2 B dx dy + C dy^2: with
      // da = alpha dL/dalpha a pixel adds dL/daleph = da / aleph,
      // dL/du = da (A dx + B dy), dL/dv = da (B dx + C dy) and
      // dL/d(A, B, C) = -da (dx^2 / 2, dx dy, dy^2 / 2), all linear in the
      // moments da (1, dx, dy, dx^2, dx dy, dy^2): the wave sums those, and
      // project_bwd applies the slot's aleph and conic once per slot
      const float da = dalpha * a;
      const float dax = da * dx, day = da * dy;
      if (__builtin_amdgcn_ballot_w64(contrib) != 0) {
        float t[9] = {quad_total(da),       quad_total(dax),      quad_total(day),
                      quad_total(dax * dx), quad_total(dax * dy), quad_total(day * dy),
                      quad_total(p * g0),   quad_total(p * g1),   quad_total(p * g2)};
        // (an empty statement that keeps each sum's last add here, with every
        // lane active, where it folds into one DPP add, instead of letting it
        // sink into the quad leaders' store below)
#pragma unroll
        for (int f = 0; f < 9; ++f) __asm__ volatile("" : "+v"(t[f]));
        if ((lane & 3) == 0) {
          float* row = wred + 9 * 16 * pend + (lane >> 2);
#pragma unroll
          for (int f = 0; f < 9; ++f) row[16 * f] = t[f];
        }
        if (lane == 0) wslot[pend] = __float_as_uint(r[9]);
        if (++pend == kRedSplats) flush();
      }
      act = __builtin_amdgcn_ballot_w64(!done);
    }
  }
  if (pend) flush();
}

// ------------------------------------------------------------ projection

constexpr int kBlock = 256;

// gradient of the real SH basis value Y_k at (x, y, z), as a polynomial in
// x, y, z (the caller projects it onto the sphere's tangent plane)
template <int DEG>
__device__ __forceinline__ void sh_basis_grad(float x, float y, float z, float* Y,
                                              float* gx, float* gy, float* gz) {
  constexpr int K = (DEG + 1) * (DEG + 1);
#pragma unroll
  for (int k = 0; k < K; ++k) gx[k] = gy[k] = gz[k] = 0.0f;
  Y[0] = 0.28209479177387814f;
  if (DEG >= 1) {
    const float c1 = 0.4886025119029199f;
    Y[1] = c1 * y; gy[1] = c1;
    Y[2] = c1 * z; gz[2] = c1;
    Y[3] = c1 * x; gx[3] = c1;
  }
  if (DEG >= 2) {
    const float a = 1.0925484305920792f, b = 0.31539156525252005f, cc = 0.5462742152960396f;
    Y[4] = a * x * y; gx[4] = a * y; gy[4] = a * x;
    Y[5] = a * y * z; gy[5] = a * z; gz[5] = a * y;
    Y[6] = b * (3.0f * z * z - 1.0f); gz[6] = 6.0f * b * z;
    Y[7] = a * x * z; gx[7] = a * z; gz[7] = a * x;
    Y[8] = cc * (x * x - y * y); gx[8] = 2.0f * cc * x; gy[8] = -2.0f * cc * y;
  }
  if (DEG >= 3) {
    const float c3a = 0.5900435899266435f, c3b = 2.890611442640554f,
                c3c = 0.4570457994644658f, c3d = 0.3731763325901154f,
                c3e = 1.445305721320277f;
    Y[9] = c3a * y * (3.0f * x * x - y * y);
    gx[9] = 6.0f * c3a * x * y; gy[9] = 3.0f * c3a * (x * x - y * y);
    Y[10] = c3b * x * y * z;
    gx[10] = c3b * y * z; gy[10] = c3b * x * z; gz[10] = c3b * x * y;
    Y[11] = c3c * y * (5.0f * z * z - 1.0f);
    gy[11] = c3c * (5.0f * z * z - 1.0f); gz[11] = 10.0f * c3c * y * z;
    Y[12] = c3d * z * (5.0f * z * z - 3.0f);
    gz[12] = c3d * (15.0f * z * z - 3.0f);
    Y[13] = c3c * x * (5.0f * z * z - 1.0f);
    gx[13] = c3c * (5.0f * z * z - 1.0f); gz[13] = 10.0f * c3c * x * z;
    Y[14] = c3e * z * (x * x - y * y);
    gx[14] = 2.0f * c3e * x * z; gy[14] = -2.0f * c3e * y * z; gz[14] = c3e * (x * x - y * y);
    Y[15] = c3a * x * (x * x - 3.0f * y * y);
    gx[15] = 3.0f * c3a * (x * x - y * y); gy[15] = -6.0f * c3a * x * y;
  }
}

template <int DEG>
__global__ __launch_bounds__(kBlock) void project_bwd_kernel(
    GaussDev g, const ViewDev* __restrict__ views, int n_views,
    float* __restrict__ gslot, GaussGradDev out) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= g.n) return;
  const float m[3] = {g.means[3 * i], g.means[3 * i + 1], g.means[3 * i + 2]};
  const float s[3] = {g.scales[3 * i], g.scales[3 * i + 1], g.scales[3 * i + 2]};
  const float q[4] = {g.quats[4 * i], g.quats[4 * i + 1], g.quats[4 * i + 2],
                      g.quats[4 * i + 3]};
  const float* coef = g.sh + (size_t)i * K * 3;
  // rotation of the normalised quaternion
  const float qn = sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  float gm[3] = {0.f, 0.f, 0.f}, gs[3] = {0.f, 0.f, 0.f}, gq[4] = {0.f, 0.f, 0.f, 0.f};
  float gop = 0.f;
  float gcoef[K * 3];
#pragma unroll
  for (int k = 0; k < K * 3; ++k) gcoef[k] = 0.f;
  if (!(qn > 0.0f)) {
    // culled in every view: no gradient
  } else {
    const float w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
    const float Rq[3][3] = {{1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
                            {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
                            {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
    float M[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) M[a][b] = Rq[a][b] * s[b];
    float gRq[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
    for (int vi = 0; vi < n_views; ++vi) {
      float* gsl = gslot + 9 * ((size_t)vi * g.n + i);
      // the slot's moments: alpha dL/dalpha (1, dx, dy, dx^2, dx dy, dy^2), colour
      const float m0 = gsl[0], m1 = gsl[1], m2 = gsl[2], m3 = gsl[3], m4 = gsl[4],
                  m5 = gsl[5];
      const float g_rgb[3] = {gsl[6], gsl[7], gsl[8]};
      if (m0 == 0.f && m1 == 0.f && m2 == 0.f && m3 == 0.f && m4 == 0.f && m5 == 0.f &&
          g_rgb[0] == 0.f && g_rgb[1] == 0.f && g_rgb[2] == 0.f)
        continue;   // no pixel of this view saw the Gaussian
      const ViewDev& v = views[vi];
      const float* R = v.R;
      const float pxc = R[0] * m[0] + R[1] * m[1] + R[2] * m[2] + v.t[0];
      const float pyc = R[3] * m[0] + R[4] * m[1] + R[5] * m[2] + v.t[1];
      const float pzc = R[6] * m[0] + R[7] * m[1] + R[8] * m[2] + v.t[2];
      const float iz = 1.0f / pzc, iz2 = iz * iz;
      const float j00 = v.fx * iz, j02 = -v.fx * pxc * iz2;
      const float j11 = v.fy * iz, j12 = -v.fy * pyc * iz2;
      float T[2][3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        T[0][k] = j00 * R[k] + j02 * R[6 + k];
        T[1][k] = j11 * R[3 + k] + j12 * R[6 + k];
      }
      float A[2][3];
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int b = 0; b < 3; ++b)
          A[r][b] = T[r][0] * M[0][b] + T[r][1] * M[1][b] + T[r][2] * M[2][b];
      const float a = A[0][0] * A[0][0] + A[0][1] * A[0][1] + A[0][2] * A[0][2] + 0.3f;
      const float b = A[0][0] * A[1][0] + A[0][1] * A[1][1] + A[0][2] * A[1][2];
      const float cc = A[1][0] * A[1][0] + A[1][1] * A[1][1] + A[1][2] * A[1][2] + 0.3f;
      const float idet = 1.0f / (a * cc - b * b);
      // conic K = Sigma2D^-1; dL/dSigma = -K G_K K with G_K = [[gA, gB/2], [gB/2, gC]]
      const float K00 = cc * idet, K01 = -b * idet, K11 = a * idet;
      // dL/d(opacity, u, v) and dL/d(A, B, C) of the conic q = A dx^2 + 2 B dx dy + C dy^2
      const float g_op = m0 / g.opac[i];
      const float g_u = K00 * m1 + K01 * m2, g_v = K01 * m1 + K11 * m2;
      const float gA = -0.5f * m3, gB = -m4, gC = -0.5f * m5;
      gsl[0] = g_op;
      gsl[1] = g_u;
      gsl[2] = g_v;
      gsl[3] = gA;
      gsl[4] = gB;
      gsl[5] = gC;
      const float G00 = gA, G01 = 0.5f * gB, G11 = gC;
      // (K G K) entries
      const float KG00 = K00 * G00 + K01 * G01, KG01 = K00 * G01 + K01 * G11;
      const float KG10 = K01 * G00 + K11 * G01, KG11 = K01 * G01 + K11 * G11;
      const float S00 = -(KG00 * K00 + KG01 * K01);
      const float S01 = -(KG00 * K01 + KG01 * K11);
      const float S11 = -(KG10 * K01 + KG11 * K11);
      const float ga = S00, gb = 2.0f * S01, gc = S11;
      // A rows: a = A0.A0, b = A0.A1, c = A1.A1
      float gAm[2][3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        gAm[0][k] = 2.0f * ga * A[0][k] + gb * A[1][k];
        gAm[1][k] = gb * A[0][k] + 2.0f * gc * A[1][k];
      }
      // A = T M
      float gT[2][3];
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k)
          gT[r][k] = gAm[r][0] * M[k][0] + gAm[r][1] * M[k][1] + gAm[r][2] * M[k][2];
#pragma unroll
      for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int b2 = 0; b2 < 3; ++b2) {
          const float gM = T[0][k] * gAm[0][b2] + T[1][k] * gAm[1][b2];
          gs[b2] += gM * Rq[k][b2];
          gRq[k][b2] += gM * s[b2];
        }
      // T = J R_cam
      float gj00 = 0.f, gj02 = 0.f, gj11 = 0.f, gj12 = 0.f;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        gj00 += gT[0][k] * R[k];
        gj02 += gT[0][k] * R[6 + k];
        gj11 += gT[1][k] * R[3 + k];
        gj12 += gT[1][k] * R[6 + k];
      }
      // J and the centre as functions of the camera-space mean
      const float gpx = gj02 * (-v.fx * iz2) + g_u * v.fx * iz;
      const float gpy = gj12 * (-v.fy * iz2) + g_v * v.fy * iz;
      const float gpz = gj00 * (-v.fx * iz2) + gj02 * (2.0f * v.fx * pxc * iz2 * iz) +
                        gj11 * (-v.fy * iz2) + gj12 * (2.0f * v.fy * pyc * iz2 * iz) +
                        g_u * (-v.fx * pxc * iz2) + g_v * (-v.fy * pyc * iz2);
#pragma unroll
      for (int k = 0; k < 3; ++k) gm[k] += R[k] * gpx + R[3 + k] * gpy + R[6 + k] * gpz;
      gop += g_op;
      // emission
      const float dxw = m[0] - v.campos[0], dyw = m[1] - v.campos[1], dzw = m[2] - v.campos[2];
      const float dn = sqrtf(dxw * dxw + dyw * dyw + dzw * dzw);
      const float ux = dxw / dn, uy = dyw / dn, uz = dzw / dn;
      float Y[K], Gx[K], Gy[K], Gz[K];
      sh_basis_grad<DEG>(ux, uy, uz, Y, Gx, Gy, Gz);
      float gdx = 0.f, gdy = 0.f, gdz = 0.f;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        float val = 0.5f;
#pragma unroll
        for (int k = 0; k < K; ++k) val += Y[k] * coef[3 * k + ch];
        if (!(val > 0.0f)) continue;   // clamped at 0
        const float gch = g_rgb[ch];
#pragma unroll
        for (int k = 0; k < K; ++k) {
          gcoef[3 * k + ch] += Y[k] * gch;
          gdx += gch * coef[3 * k + ch] * Gx[k];
          gdy += gch * coef[3 * k + ch] * Gy[k];
          gdz += gch * coef[3 * k + ch] * Gz[k];
        }
      }
      const float dot = ux * gdx + uy * gdy + uz * gdz;
      gm[0] += (gdx - ux * dot) / dn;
      gm[1] += (gdy - uy * dot) / dn;
      gm[2] += (gdz - uz * dot) / dn;
    }
    // rotation entries -> normalised quaternion (w, x, y, z)
    float gw = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
    gw += gRq[0][1] * (-2 * z) + gRq[0][2] * (2 * y) + gRq[1][0] * (2 * z) +
          gRq[1][2] * (-2 * x) + gRq[2][0] * (-2 * y) + gRq[2][1] * (2 * x);
    gx += gRq[0][1] * (2 * y) + gRq[0][2] * (2 * z) + gRq[1][0] * (2 * y) +
          gRq[1][1] * (-4 * x) + gRq[1][2] * (-2 * w) + gRq[2][0] * (2 * z) +
          gRq[2][1] * (2 * w) + gRq[2][2] * (-4 * x);
    gy += gRq[0][0] * (-4 * y) + gRq[0][1] * (2 * x) + gRq[0][2] * (2 * w) +
          gRq[1][0] * (2 * x) + gRq[1][2] * (2 * z) + gRq[2][0] * (-2 * w) +
          gRq[2][1] * (2 * z) + gRq[2][2] * (-4 * y);
    gz += gRq[0][0] * (-4 * z) + gRq[0][1] * (-2 * w) + gRq[0][2] * (2 * x) +
          gRq[1][0] * (2 * w) + gRq[1][1] * (-4 * z) + gRq[1][2] * (2 * y) +
          gRq[2][0] * (2 * x) + gRq[2][1] * (2 * y);
    const float qh[4] = {w, x, y, z}, gqh[4] = {gw, gx, gy, gz};
    const float dqh = qh[0] * gqh[0] + qh[1] * gqh[1] + qh[2] * gqh[2] + qh[3] * gqh[3];
#pragma unroll
    for (int k = 0; k < 4; ++k) gq[k] = (gqh[k] - qh[k] * dqh) / qn;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    out.means[3 * i + k] = gm[k];
    out.scales[3 * i + k] = gs[k];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) out.quats[4 * i + k] = gq[k];
  out.opac[i] = gop;
#pragma unroll
  for (int k = 0; k < K * 3; ++k) out.sh[(size_t)i * K * 3 + k] = gcoef[k];
}

template <int MODEL, int TW, int TH>
void bwd_t(int64_t n_tiles, const ViewDev* views, int n_views, const uint2* ranges,
           const uint32_t* inst_val, const float4* rec, const CompositeParams& p,
           const float4* pstate, float* gslot, const uint32_t* order, hipStream_t s) {
  const uint32_t per = (uint32_t)((n_tiles + 7) / 8);
  hipLaunchKernelGGL((composite_bwd_kernel<MODEL, TW, TH>), dim3(per * 8), dim3(TW * TH), 0, s,
                     views, n_views, ranges, inst_val, rec, p, pstate, gslot,
                     (uint32_t)n_tiles, per, order);
}

template <int MODEL>
void bwd_m(int tile_w, int tile_h, int64_t n_tiles, const ViewDev* views, int n_views,
           const uint2* ranges, const uint32_t* inst_val, const float4* rec,
           const CompositeParams& p, const float4* pstate, float* gslot, const uint32_t* order,
           hipStream_t s) {
  if (tile_w == 8 && tile_h == 8)
    bwd_t<MODEL, 8, 8>(n_tiles, views, n_views, ranges, inst_val, rec, p, pstate, gslot, order,
                       s);
  else if (tile_w == 32 && tile_h == 8)
    bwd_t<MODEL, 32, 8>(n_tiles, views, n_views, ranges, inst_val, rec, p, pstate, gslot, order,
                        s);
  else
    bwd_t<MODEL, 16, 16>(n_tiles, views, n_views, ranges, inst_val, rec, p, pstate, gslot,
                         order, s);
}

}  // namespace

void launch_composite_bwd(int model, int tile_w, int tile_h, int64_t n_tiles,
                          const ViewDev* views, int n_views, const uint2* ranges,
                          const uint32_t* inst_val, const float4* rec, const CompositeParams& p,
                          const float4* pstate, float* gslot, const uint32_t* order,
                          hipStream_t s) {
  if (n_tiles <= 0) return;
  switch (model) {
#define NXS_B(M)                                                                        \
  case M:                                                                               \
    bwd_m<M>(tile_w, tile_h, n_tiles, views, n_views, ranges, inst_val, rec, p, pstate, \
             gslot, order, s);                                                          \
    break;
    NXS_B(0) NXS_B(1) NXS_B(2) NXS_B(3) NXS_B(4)
#undef NXS_B
    default: break;
  }
}

void launch_project_bwd(const GaussDev& g, const ViewDev* views, int n_views,
                        float* gslot, const GaussGradDev& out, hipStream_t s) {
  if (g.n <= 0) return;
  dim3 grid((g.n + kBlock - 1) / kBlock);
  switch (g.sh_degree) {
    case 0: hipLaunchKernelGGL(project_bwd_kernel<0>, grid, dim3(kBlock), 0, s, g, views, n_views, gslot, out); break;
    case 1: hipLaunchKernelGGL(project_bwd_kernel<1>, grid, dim3(kBlock), 0, s, g, views, n_views, gslot, out); break;
    case 2: hipLaunchKernelGGL(project_bwd_kernel<2>, grid, dim3(kBlock), 0, s, g, views, n_views, gslot, out); break;
    default: hipLaunchKernelGGL(project_bwd_kernel<3>, grid, dim3(kBlock), 0, s, g, views, n_views, gslot, out); break;
  }
}

}  // namespace nxs
