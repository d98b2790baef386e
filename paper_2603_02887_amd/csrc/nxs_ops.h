// Per-pixel operator state shared by the forward composite and its
// path-replay backward (both must take identical float32 decisions).
#pragma once

#include <hip/hip_runtime.h>

namespace nxs {

// Per-pixel state and update of a Table 1 operator.  MODEL: 0 exponential,
// 1 linear, 2 quadratic c = -0.5, 3 quadratic c = +0.5, 4 quadratic with
// c = param, 5 blended (gamma = param), 6 Vicini et al. (gamma = param),
// 7 power law (v = param).
//
// `step` composites one splat of opacity a (a >= alpha_min, or a = 0 for "no
// splat": then p = 0 and the state does not change, which lets the composite
// run it on every lane without branches) and returns its p.  Whether the pixel
// has stopped is a function of the state alone (`stopped`): the running sum of
// p has reached exactly 1 (saturation: the splat that gets there takes the
// remainder, eq. nexp_p), or, for the exponential, T < t_eps.  t_eps > 0
// always: without a termination threshold the caller passes the smallest
// normal float, below which the float32 product would underflow.
template <int MODEL>
struct Op {
  float S = 0.0f;      // running sum of p (T = 1 - S)
  float tau = 0.0f;    // discrete optical depth
  float T = 1.0f;      // running product of (1 - a) (exponential parts)
  float S2 = 0.0f;     // Vicini: the linear part's running sum

  // a pixel outside the image: stopped before the first splat
  __device__ __forceinline__ void stop() {
    S = 1.0f;
    S2 = 1.0f;
    T = 0.0f;
  }
  __device__ __forceinline__ bool stopped(float t_eps) const {
    if (MODEL == 0) return !(T >= t_eps);
    if (MODEL == 6) return S2 >= 1.0f && !(T >= t_eps);
    return S >= 1.0f;
  }
  // (no contraction into FMAs in the update: the forward and its backward,
  // compiled apart, must round it identically)
  __device__ __forceinline__ float saturate(float p) {
#pragma clang fp contract(off)
    const float Sn = S + p;
    const bool sat = Sn >= 1.0f;
    p = sat ? 1.0f - S : p;
    S = sat ? 1.0f : Sn;
    return p;
  }
  __device__ __forceinline__ float step(float a, float param, float t_eps) {
#pragma clang fp contract(off)
    if (MODEL == 0) {
      const float p = a * T;
      T = T * (1.0f - a);
      return p;
    } else if (MODEL == 1) {
      return saturate(a);
    } else if (MODEL <= 4) {
      const float c = MODEL == 2 ? -0.5f : MODEL == 3 ? 0.5f : param;
      const float p = a * fmaf(c, tau, 1.0f);
      tau += a;
      return saturate(p);
    } else if (MODEL == 5) {
      const float p = a * fmaf(param, T, 1.0f - param);
      T = T * (1.0f - a);
      return saturate(p);
    } else if (MODEL == 6) {
      // each part stops on its own and then keeps its state
      const bool d1 = S2 >= 1.0f, d2 = !(T >= t_eps);
      const float Sn = S2 + a;
      const bool s1 = Sn >= 1.0f;
      const float pl = d1 ? 0.0f : (s1 ? 1.0f - S2 : a);
      S2 = d1 ? S2 : (s1 ? 1.0f : Sn);
      const float pe = d2 ? 0.0f : a * T;
      T = d2 ? T : T * (1.0f - a);
      return fmaf(param, pe - pl, pl);
    } else {
      // where 1 + v tau <= 0 the splat saturates (p = +inf), unless a = 0
      const float base = fmaf(param, tau, 1.0f);
      tau += a;
      const float p = base > 0.0f
                          ? a * __builtin_amdgcn_exp2f(-(1.0f + param) / param *
                                                      __builtin_amdgcn_logf(base))
                          : (a > 0.0f ? __builtin_inff() : 0.0f);
      return saturate(p);
    }
  }
  // the same step, also reporting whether the pixel has now stopped
  __device__ __forceinline__ float step(float a, float param, float t_eps, bool& done) {
    const float p = step(a, param, t_eps);
    done = stopped(t_eps);
    return p;
  }
  __device__ __forceinline__ float transmittance(float param) const {
#pragma clang fp contract(off)
    if (MODEL == 0) return T;
    if (MODEL == 6) return fmaf(param, T - (1.0f - S2), 1.0f - S2);
    return 1.0f - S;
  }
};

}  // namespace nxs
