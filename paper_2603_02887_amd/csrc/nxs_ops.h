// Per-pixel operator state shared by the forward composite and its
// path-replay backward (both must take identical float32 decisions).
#pragma once

#include <hip/hip_runtime.h>

namespace nxs {

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

}  // namespace nxs
