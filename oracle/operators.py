"""Discrete transmittance operators on one pixel's front-to-back sequence, FP64.

Parity: pinned.  The sequence composite reproduces the paper's printed figure
data (Sec. 4, Fig. "Transmittance comparison" dots and Fig. "Blending
comparison" (a) scan-lines) and the closed forms checked in the tests.

What is computed (Sec. 4, "Our method" and "Choosing a transmittance
function"):
  * pixel value  L0 = sum_i E_i p_i + L_b T_{N+1}          (eq. generalized_gaussian)
  * discrete transmittance  T_i = 1 - sum_{j<i} p_j
  * discrete optical depth  tau_i = sum_{j<i} alpha_j
  * p_i = the operator's formula (Table 1, last column) while the running sum
    stays below 1; the first splat k at which it would reach 1 takes the
    remainder 1 - sum_{j<k} p_j; every later splat gets 0   (eq. nexp_p)

Readings where the paper is silent (each is listed in the design notes):
  * splats with alpha < alpha_min are not composited at all: they add nothing
    to tau, T or the overdraw count (reproduces Fig. "Blending comparison" (a)
    with alpha_min = 1e-3);
  * the exponential operator, whose T never reaches 0 unless some alpha is 1,
    stops after the first splat that leaves T < t_eps (3DGS practice, 1e-4);
  * overdraw counts every composited splat, the terminating one included;
  * Vicini et al.'s operator is the lerp of the two complete discrete
    operators (linear and exponential), each with its own saturation
    (reproduces both figures);
  * the power law uses tau_i (the discrete optical depth) where Table 1
    prints tau_i without the bar, and the figure panel labelled v = -1 is
    reproduced by v = -2; when 1 + v*tau <= 0 the mother T is clamped to 0,
    so that splat saturates.
"""
from dataclasses import dataclass
import math

import numpy as np


@dataclass(frozen=True)
class Op:
    """A Table 1 operator: kind in {exponential, linear, quadratic, blended,
    vicini, powerlaw} and its one parameter (c, gamma or v)."""
    kind: str
    param: float = 0.0

    @property
    def finite_support(self):
        """True when the mother T reaches 0 at a finite optical depth."""
        if self.kind in ("exponential", "vicini"):
            return False
        if self.kind == "powerlaw":
            return self.param < 0
        if self.kind == "blended":
            return self.param < 1
        return True


EXPONENTIAL = Op("exponential")
LINEAR = Op("linear")
SUBLINEAR = Op("quadratic", -0.5)    # Sec. 5: "sublinear" is the quadratic with c = -0.5
SUPERLINEAR = Op("quadratic", 0.5)   # Sec. 5: "superlinear" is the quadratic with c = +0.5

# The library's transmittance-model ids 0..3.
MODELS = {0: EXPONENTIAL, 1: LINEAR, 2: SUBLINEAR, 3: SUPERLINEAR}
MODEL_NAMES = {0: "exponential", 1: "linear", 2: "sublinear", 3: "superlinear"}

# The nine panels of the two figures in Sec. 4.
FIGURE_OPS = {
    "powerlaw_v2": Op("powerlaw", 2.0),
    "exponential": EXPONENTIAL,
    "quadratic_c-0.5": SUBLINEAR,
    "vicini_g0.5": Op("vicini", 0.5),
    "blended_g0.5": Op("blended", 0.5),
    "linear": LINEAR,
    "quadratic_c0.5": SUPERLINEAR,
    "quadratic_c1": Op("quadratic", 1.0),
    "powerlaw_vm1": Op("powerlaw", -2.0),
}


def mother_T(op, tau):
    """Mother transmittance T(tau) of Table 1 (third column), with [x]_+ clamps."""
    tau = np.asarray(tau, np.float64)
    if op.kind == "exponential":
        return np.exp(-tau)
    if op.kind == "linear":
        return np.maximum(1.0 - tau, 0.0)
    if op.kind == "quadratic":
        return np.maximum(1.0 - tau - 0.5 * op.param * tau * tau, 0.0)
    if op.kind == "blended":
        g = op.param
        return np.maximum((1.0 - g) * (1.0 - tau) + g * np.exp(-tau), 0.0)
    if op.kind == "vicini":
        g = op.param
        return (1.0 - g) * np.maximum(1.0 - tau, 0.0) + g * np.exp(-tau)
    if op.kind == "powerlaw":
        v = op.param
        base = 1.0 + tau * v
        with np.errstate(divide="ignore", invalid="ignore"):
            out = np.where(base > 0.0, np.abs(base) ** (-1.0 / v), 0.0)
        return out
    raise ValueError(op)


def p_unsaturated(op, alpha, tau_bar, prod):
    """Table 1, last column: p_i for i < k given alpha_i, the discrete optical
    depth tau_i = sum_{j<i} alpha_j and prod = prod_{j<i} (1 - alpha_j)."""
    if op.kind == "exponential":
        return alpha * prod
    if op.kind == "linear":
        return alpha
    if op.kind == "quadratic":
        return alpha * (1.0 + op.param * tau_bar)
    if op.kind == "blended":
        g = op.param
        return alpha * (1.0 - g + g * prod)
    if op.kind == "powerlaw":
        v = op.param
        base = 1.0 + tau_bar * v
        if base <= 0.0:
            return math.inf        # mother T already clamped to 0: saturate here
        return alpha * base ** (-(1.0 + v) / v)
    raise ValueError(op)


def composite_sequence(alphas, op, emissions=None, background=None,
                       alpha_min=0.0, t_eps=None, flips=frozenset()):
    """Composite one front-to-back sequence with operator `op` (pure Python, FP64).

    alphas     per-splat opacity alpha_i = aleph_i K_i, front to back
    emissions  [N, C] per-splat emission E_i (default: zeros, 1 channel)
    background [C] L_b (default 0)
    alpha_min  splats with alpha < alpha_min are skipped entirely
    t_eps      exponential only: stop after the first splat leaving T < t_eps
               (default 0, i.e. never)
    flips      discrete decisions to take the other way, for enumerating the
               outcomes a float32 evaluation may legitimately reach at a
               boundary (module render): (i, 0) composites splat i if its
               alpha is below alpha_min and skips it otherwise; (i, 1)
               reverses whether the pixel stops after compositing splat i
               (the saturation test of eq. nexp_p, or the exponential's
               termination).  For Vicini's operator (i, 1) and (i, 2) are
               the stops of its linear and exponential parts.  Empty: the
               plain definition.

    Returns a dict:
      p      [N] p_i per input splat (0 for skipped or post-termination splats)
      T      [N+1] T_i seen before each splat, then the final transmittance
      L      [C] the pixel value L0
      od     number of composited splats (terminating one included)
      k      index of the last composited splat, or -1
      T_final  final transmittance
      p_raw  [N] the operator's formula value before the saturation clamp
             (NaN where not composited)
      done   whether the pixel stopped (later splats were not considered)
    """
    alphas = [float(a) for a in alphas]
    n = len(alphas)
    if emissions is None:
        E = np.zeros((n, 1 if background is None else np.size(background)))
    else:
        E = np.asarray(emissions, np.float64).reshape(n, -1 if n else np.size(background))
    C = E.shape[1]
    Lb = np.zeros(C) if background is None else np.asarray(background, np.float64).reshape(C)
    if op.kind == "vicini":
        return _vicini(alphas, op.param, E, Lb, alpha_min, t_eps, flips)
    t_eps = 0.0 if t_eps is None else float(t_eps)

    S = 0.0            # sum of p_j so far; T = 1 - S
    tau = 0.0          # discrete optical depth over composited splats
    prod = 1.0         # prod (1 - alpha_j) over composited splats
    T = 1.0
    L = np.zeros(C)
    p_out = np.zeros(n)
    p_raw = np.full(n, np.nan)
    T_seen = np.zeros(n + 1)
    od, k, done = 0, -1, False
    for i, a in enumerate(alphas):
        T_seen[i] = T
        if done:
            T_seen[i:] = T
            break
        if (a < alpha_min) != ((i, 0) in flips):
            continue
        flip_stop = (i, 1) in flips
        p = p_unsaturated(op, a, tau, prod)
        p_raw[i] = p
        if op.kind == "exponential":
            # sum p = 1 - prod(1 - alpha) exactly, so T is the product; it
            # reaches 0 (saturation) only where some alpha is 1
            S += p
            T = prod * (1.0 - a)
            done = (T == 0.0 or T < t_eps) != flip_stop
        elif (S + p >= 1.0) != flip_stop:    # splat i saturates: it is the k of eq. nexp_p
            p = 1.0 - S
            S, T, done = 1.0, 0.0, True
        else:
            S += p
            T = 1.0 - S
        tau += a
        prod *= (1.0 - a)
        L += E[i] * p
        p_out[i] = p
        od += 1
        k = i
    T_seen[n] = T
    L += Lb * T
    return {"p": p_out, "T": T_seen, "L": L, "od": od, "k": k, "T_final": T,
            "p_raw": p_raw, "done": done}


def _vicini(alphas, g, E, Lb, alpha_min, t_eps, flips=frozenset()):
    keep = {f for f in flips if f[1] == 0}
    lin = composite_sequence(alphas, LINEAR, E, None, alpha_min,
                             flips=keep | {f for f in flips if f[1] == 1})
    ex = composite_sequence(alphas, EXPONENTIAL, E, None, alpha_min, t_eps,
                            flips=keep | {(f[0], 1) for f in flips if f[1] == 2})
    p = (1.0 - g) * lin["p"] + g * ex["p"]
    T = (1.0 - g) * lin["T"] + g * ex["T"]
    T_final = T[-1]
    L = (1.0 - g) * lin["L"] + g * ex["L"] + Lb * T_final
    return {"p": p, "T": T, "L": L, "od": max(lin["od"], ex["od"]),
            "k": max(lin["k"], ex["k"]), "T_final": T_final,
            "p_raw": (1.0 - g) * lin["p_raw"] + g * ex["p_raw"],
            "done": lin["done"] and ex["done"], "parts": (lin, ex)}


def back_to_front(p, T, E, background):
    """Russian-roulette appendix, recursive form: L_i = E_i s_i + (1 - s_i) L_{i+1}
    with the differential extinction s_i = p_i / T_i, evaluated back to front
    from L_{N+1} = L_b.  Splats with p_i = 0 leave L unchanged.  Equals the
    front-to-back sum of eq. generalized_gaussian exactly in exact arithmetic."""
    E = np.asarray(E, np.float64)
    L = np.asarray(background, np.float64).copy()
    for i in range(len(p) - 1, -1, -1):
        if p[i] == 0.0:
            continue
        s = p[i] / T[i]
        L = E[i] * s + (1.0 - s) * L
    return L
