"""Adjoints of the discrete operators on one pixel's sequence, FP64.

Parity: pinned by FP64 central differences of operators.composite_sequence in
the tests (random sequences, saturated and unsaturated, every model below).

For the pixel value L0 = sum_i E_i p_i + L_b T (Sec. 4) and an upstream
gradient g = dLoss/dL0, return dLoss/dalpha_i and dLoss/dE_i for the splats
the forward composited (i <= k; later splats and skipped ones get zero).

Linear and quadratic: the appendix "Adjoints" rewrites the pixel value as
L0 = sum_{i<k} (E_i - E_k) p_i + E_k with E_k the saturating splat's emission,
or L_b when nothing saturates (eq. generalized_gaussians_gen), and derives
  linear     dL/dalpha_i = E_i - E_k                                   (i < k)
  quadratic  dL/dalpha_i = (E_i - E_k)(1 + c tau_i) + c Theta_i        (i < k)
             Theta_i = sum_{i<j<k} (E_j - E_k) alpha_j
with dL/dalpha_k = 0 for a saturating splat (its p is the remainder, which
does not depend on its own alpha) and dL/dE_i = p_i for every composited i.

Exponential (not derived in the paper; the standard front-to-back form):
  dL/dalpha_i = T_i E_i - R_{i+1} / (1 - alpha_i),
  R_{i+1} = sum_{i<j<=k} E_j p_j + L_b T_{k+1}   (radiance behind splat i)
and for the last composited splat k: T_k (E_k - L_b), which needs no division.
"""
import numpy as np

from . import operators as _ops


def adjoint_sequence(alphas, op, emissions, background, g, alpha_min=0.0, t_eps=None):
    """Return (dalpha [N], dE [N, C]) for upstream gradient g [C]."""
    alphas = np.asarray(alphas, np.float64)
    n = alphas.size
    E = np.asarray(emissions, np.float64).reshape(n, -1)
    C = E.shape[1]
    Lb = np.asarray(background, np.float64).reshape(C)
    g = np.asarray(g, np.float64).reshape(C)
    fwd = _ops.composite_sequence(alphas, op, E, Lb, alpha_min, t_eps)
    p, k = fwd["p"], fwd["k"]
    comp = [i for i in range(k + 1) if alphas[i] >= alpha_min]
    dE = np.zeros((n, C))
    for i in comp:
        dE[i] = p[i] * g
    dalpha = np.zeros(n)
    if not comp:
        return dalpha, dE
    saturated = fwd["T_final"] == 0.0
    if op.kind == "exponential":
        T = 1.0
        Ts = {}
        for i in comp:
            Ts[i] = T
            T *= 1.0 - alphas[i]
        T_end = T                                   # T_{k+1}
        R = Lb * T_end                              # radiance behind the last splat
        for i in reversed(comp):
            if i == comp[-1]:
                dalpha[i] = float(g @ (Ts[i] * (E[i] - Lb)))
            else:
                dalpha[i] = float(g @ (Ts[i] * E[i] - R / (1.0 - alphas[i])))
            R = R + E[i] * p[i]
        return dalpha, dE
    if op.kind not in ("linear", "quadratic"):
        raise NotImplementedError(op.kind)
    c = op.param if op.kind == "quadratic" else 0.0
    if saturated:
        last = comp[-1]
        Ek = E[last]
        before = comp[:-1]           # the i < k
    else:
        Ek = Lb
        before = comp
    # Theta_i over the composited splats strictly between i and k
    tau = 0.0
    taus = {}
    for i in comp:
        taus[i] = tau
        tau += alphas[i]
    theta = np.zeros(C)
    for i in reversed(before):
        dalpha[i] = float(g @ ((E[i] - Ek) * (1.0 + c * taus[i]) + c * theta))
        theta = theta + (E[i] - Ek) * alphas[i]
    return dalpha, dE
