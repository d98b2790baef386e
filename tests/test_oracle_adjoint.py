"""Pins of the oracle's adjoints (appendix "Adjoints") by FP64 central differences."""
import numpy as np
import pytest

from oracle import adjoint as A
from oracle import operators as O

OPS = [O.EXPONENTIAL, O.LINEAR, O.SUBLINEAR, O.SUPERLINEAR, O.Op("quadratic", 1.0),
       O.Op("quadratic", -0.25)]


def _loss(alphas, op, E, Lb, g, amin, t_eps):
    return float(g @ O.composite_sequence(alphas, op, E, Lb, amin, t_eps)["L"])


@pytest.mark.parametrize("op", OPS, ids=lambda o: f"{o.kind}{o.param}")
@pytest.mark.parametrize("seed", range(12))
def test_adjoint_matches_central_differences(op, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(3, 25))
    scale = [0.05, 0.2, 0.45][seed % 3]          # unsaturated .. saturated
    al = rng.uniform(0.01, 1.0, n) * scale * 2
    al = np.minimum(al, 0.97)
    E = rng.uniform(0, 1, (n, 3))
    Lb = rng.uniform(0, 1, 3)
    g = rng.normal(0, 1, 3)
    t_eps = 1e-4 if op.kind == "exponential" else 0.0
    da, dE = A.adjoint_sequence(al, op, E, Lb, g, 1e-3, t_eps)
    h = 1e-7
    base = O.composite_sequence(al, op, E, Lb, 1e-3, t_eps)
    for i in range(n):
        ap, am = al.copy(), al.copy()
        ap[i] += h
        am[i] -= h
        fp = O.composite_sequence(ap, op, E, Lb, 1e-3, t_eps)
        fm = O.composite_sequence(am, op, E, Lb, 1e-3, t_eps)
        if fp["k"] != base["k"] or fm["k"] != base["k"] or fp["od"] != fm["od"]:
            continue        # the step crossed a saturation / termination boundary
        fd = (float(g @ fp["L"]) - float(g @ fm["L"])) / (2 * h)
        assert abs(fd - da[i]) <= 1e-6 * max(1.0, abs(fd)), (op, i, fd, da[i])
        for ch in range(3):
            Ep, Em = E.copy(), E.copy()
            Ep[i, ch] += h
            Em[i, ch] -= h
            fd = (_loss(al, op, Ep, Lb, g, 1e-3, t_eps) - _loss(al, op, Em, Lb, g, 1e-3, t_eps)) / (2 * h)
            assert abs(fd - dE[i, ch]) <= 1e-6 * max(1.0, abs(fd))


def test_linear_adjoint_closed_form():
    """Linear, saturating at the third splat: dL/dalpha_i = E_i - E_3 for i < 3
    and 0 for the saturating splat (appendix recursion)."""
    al = [0.4, 0.4, 0.4, 0.4]
    E = np.array([[1.0], [2.0], [5.0], [7.0]])
    da, dE = A.adjoint_sequence(al, O.LINEAR, E, [0.0], [1.0])
    assert np.allclose(da, [1 - 5, 2 - 5, 0, 0])
    assert np.allclose(dE[:, 0], [0.4, 0.4, 0.2, 0.0])
