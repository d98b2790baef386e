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


@pytest.mark.parametrize("model", [0, 1, 3])
def test_slot_sums_match_central_differences(model):
    """tests/adjoint_sums.py (the per-slot sums the GPU backward is compared
    with): its opacity and colour columns equal FP64 central differences of
    the frozen-list oracle loss (tests/fd.py) in the opacity and in the DC
    SH coefficient (which moves the emission by C0 = 1/(2 sqrt(pi)) per
    unit where the emission is not clamped)."""
    import synth
    from tests import adjoint_sums, fd
    sc = synth.random_scene(21, 60, log_scale=(-1.6, 0.3), logit=(1.5, 1.0), sh_degree=1)
    cams = [synth.look_at_camera((0, 0, -3.2), width=40, height=32)]
    F = fd.FrozenLoss(sc, cams, model, seed=4)
    w_rgb, w_T = F.weights(0)
    sums = adjoint_sums.slot_sums(sc, cams[0], model, w_rgb.astype(np.float64),
                                  w_T.astype(np.float64))
    params = fd.params_of(sc)
    c0 = 0.28209479177387814
    order = np.argsort(-np.abs(sums[:, 0]))[:6]        # the most-seen Gaussians
    checked = 0
    for i in order:
        want = F.grad_element(params, "opacities", (int(i),), 1e-6)
        assert abs(sums[i, 0] - want) <= 1e-6 * max(1.0, abs(want)), (i, sums[i, 0], want)
        for ch in range(3):
            want = F.grad_element(params, "sh", (int(i), 0, ch), 1e-6) / c0
            if want != 0.0:             # (a clamped channel moves nothing)
                assert abs(sums[i, 6 + ch] - want) <= 1e-6 * max(1.0, abs(want))
                checked += 1
    assert checked >= 6
