"""Pins of the oracle's operators against the paper's printed data and closed forms.

Sec. 4: eq. generalized_gaussian, eq. nexp_p, Table 1, constraints (a)-(c) of
"Choosing a transmittance function", and the recursion of the
Russian-roulette appendix.
"""
import math

import numpy as np
import pytest

from oracle import operators as O
from tests.golden import fixtures


# ------------------------------------------------ the paper's printed figure data

@pytest.mark.parametrize("name", list(O.FIGURE_OPS))
def test_transmittance_figure_dots(name):
    """Fig. 'Transmittance comparison': 100 splats of alpha = 0.02; the blue dots
    are T_bar after every 5 splats, printed to 8 decimals."""
    dots = fixtures.transmittance_dots()[name]
    res = O.composite_sequence([0.02] * 100, O.FIGURE_OPS[name])
    for tau, want in dots:
        i = int(round(tau / 0.02))
        assert abs(res["T"][i] - want) <= 6e-9, (name, tau, res["T"][i], want)


@pytest.mark.parametrize("name", list(O.FIGURE_OPS))
def test_transmittance_figure_mother_curve(name):
    """Same figure, green curves: the mother T(tau) of Table 1, 8 decimals."""
    want = fixtures.transmittance_mother()[name]
    tau = np.arange(want.size) * 2.02 / (want.size - 1)
    got = O.mother_T(O.FIGURE_OPS[name], tau)
    assert np.abs(got - want).max() <= 6e-9


def concentric_alphas(x):
    """Fig. 'Blending comparison' (a) scene: 3 isotropic Gaussians of opacity 1
    and standard deviation 40, 60, 80 px (red front, green, blue back), centred
    on pixel 256's centre of a 512-px scan-line; pixel x sampled at x + 1/2."""
    d = (x + 0.5) - 256.5
    return [math.exp(-0.5 * d * d / (s * s)) for s in (40.0, 60.0, 80.0)]


@pytest.mark.parametrize("name", list(O.FIGURE_OPS))
def test_blending_figure_scanline(name):
    """Per-splat contributions E_i p_i and their sum, printed to 6 decimals,
    with alpha_min = 1e-3 (the reading that reproduces the figure)."""
    rows = fixtures.blending_concentric()[name]
    E = np.eye(3)
    for x, r, g, b, s in rows:
        res = O.composite_sequence(concentric_alphas(x), O.FIGURE_OPS[name], E,
                                   alpha_min=1e-3)
        got = res["p"]
        assert np.abs(got - [r, g, b]).max() <= 5.1e-7, (name, x, got, (r, g, b))
        assert abs(got.sum() - s) <= 5.1e-7


def test_blending_figure_rejects_other_cutoffs():
    """The alpha_min reading is what the figure fixes: no cutoff, and 3DGS's
    1/255, both miss printed values by far more than the print precision."""
    rows = fixtures.blending_concentric()["linear"]
    for amin in (0.0, 1.0 / 255.0):
        worst = 0.0
        for x, r, g, b, s in rows:
            p = O.composite_sequence(concentric_alphas(x), O.LINEAR, np.eye(3),
                                     alpha_min=amin)["p"]
            worst = max(worst, np.abs(p - [r, g, b]).max())
        assert worst > 1e-4


def test_exponential_front_splat_saturates_without_clamp():
    """Fig. 'Blending comparison' (a), exponential at the centre: the front
    splat of alpha 1 takes everything (no 0.99 clamp on alpha)."""
    rows = fixtures.blending_concentric()["exponential"]
    centre = rows[rows[:, 0] == 256][0]
    assert centre[1] == 1.0 and centre[2] == 0.0 and centre[3] == 0.0
    res = O.composite_sequence(concentric_alphas(256), O.EXPONENTIAL, np.eye(3),
                               alpha_min=1e-3, t_eps=1e-4)
    assert res["p"].tolist() == [1.0, 0.0, 0.0] and res["T_final"] == 0.0


# ------------------------------------------------------------- closed forms

def _random_alphas(rng, n):
    return rng.uniform(0.0, 0.6, n) * (rng.uniform(size=n) < 0.8)


@pytest.mark.parametrize("seed", range(20))
def test_closed_forms_before_saturation(seed):
    rng = np.random.default_rng(seed)
    al = _random_alphas(rng, 40) * 0.1          # stay below saturation
    tau = np.concatenate([[0.0], np.cumsum(al)])
    # linear: T_n = [1 - tau_n]_+
    lin = O.composite_sequence(al, O.LINEAR)
    assert np.allclose(lin["T"], np.maximum(1 - tau, 0), atol=1e-14)
    # exponential: T_n = prod_{j<n} (1 - alpha_j)
    ex = O.composite_sequence(al, O.EXPONENTIAL)
    prod = np.concatenate([[1.0], np.cumprod(1 - al)])
    assert np.allclose(ex["T"], prod, atol=1e-14)
    # quadratic: T_n = T(tau_n) + (c/2) sum_{j<n} alpha_j^2 until saturation
    for c in (-0.5, 0.5, 1.0):
        q = O.composite_sequence(al, O.Op("quadratic", c))
        sq = np.concatenate([[0.0], np.cumsum(al * al)])
        want = 1 - tau - 0.5 * c * tau * tau + 0.5 * c * sq
        live = want > 0
        assert np.allclose(q["T"][live], want[live], atol=1e-13)


@pytest.mark.parametrize("name", list(O.FIGURE_OPS))
@pytest.mark.parametrize("seed", range(10))
def test_invariants(name, seed):
    """Weights plus final transmittance sum to 1; T non-increasing in [0, 1];
    p_1 = alpha_1 (constraint (c)); finite-support operators reach exactly 0."""
    rng = np.random.default_rng(100 + seed)
    al = _random_alphas(rng, 60)
    op = O.FIGURE_OPS[name]
    res = O.composite_sequence(al, op)
    assert abs(res["p"].sum() + res["T_final"] - 1.0) <= 1e-12
    T = res["T"]
    assert np.all(T >= 0.0) and np.all(T <= 1.0)
    assert np.all(np.diff(T) <= 1e-15)
    first = int(np.argmax(al > 0))
    assert abs(res["p"][first] - al[first]) <= 1e-15
    if op.finite_support and al.sum() > 8.0:
        assert res["T_final"] == 0.0


def test_single_splat_pixel_value():
    """One splat: L = alpha E + (1 - alpha) L_b for every operator."""
    for op in O.FIGURE_OPS.values():
        for a in (0.001, 0.3, 0.999, 1.0):
            res = O.composite_sequence([a], op, [[0.2, 0.5, 0.9]], [0.7, 0.1, 0.3])
            assert np.allclose(res["L"], a * np.array([0.2, 0.5, 0.9])
                               + (1 - a) * np.array([0.7, 0.1, 0.3]), atol=1e-15)


def test_saturating_splat_takes_remainder():
    """eq. nexp_p: the k-th splat gets 1 - sum_{j<k} p_j and later splats 0;
    linear with alphas 0.4, 0.4, 0.4, 0.4 -> 0.4, 0.4, 0.2, 0."""
    res = O.composite_sequence([0.4] * 4, O.LINEAR)
    assert np.allclose(res["p"], [0.4, 0.4, 0.2, 0.0], atol=1e-15)
    assert res["od"] == 3 and res["k"] == 2 and res["T_final"] == 0.0
    # quadratic c = 0.5: 0.4, 0.4 (1 + 0.2) = 0.48, then the remainder 0.12
    res = O.composite_sequence([0.4] * 4, O.SUPERLINEAR)
    assert np.allclose(res["p"], [0.4, 0.48, 0.12, 0.0], atol=1e-15)
    # quadratic c = -0.5: 0.4, 0.32, 0.4 (1 - 0.4) = 0.24, then 0.04
    res = O.composite_sequence([0.4] * 4, O.SUBLINEAR)
    assert np.allclose(res["p"], [0.4, 0.32, 0.24, 0.04], atol=1e-15)


def test_alpha_min_skip_and_exponential_termination():
    res = O.composite_sequence([0.5, 0.0005, 0.5], O.LINEAR, alpha_min=1e-3)
    assert res["od"] == 2 and res["p"][1] == 0.0
    # exponential stops after the first splat that leaves T < t_eps
    res = O.composite_sequence([0.8] * 8, O.EXPONENTIAL, t_eps=1e-4)
    # T after 5 splats = 3.2e-4 (not < 1e-4), after 6 = 6.4e-5 < 1e-4
    assert res["od"] == 6 and res["p"][6] == 0.0
    res = O.composite_sequence([0.99, 0.99, 0.5], O.EXPONENTIAL, t_eps=1e-3)
    assert res["od"] == 2 and res["p"][2] == 0.0


@pytest.mark.parametrize("name", list(O.FIGURE_OPS))
@pytest.mark.parametrize("seed", range(10))
def test_back_to_front_recursion_matches(name, seed):
    """Russian-roulette appendix: the back-to-front recursion with s_i = p_i/T_i
    gives the same pixel value as the front-to-back sum."""
    rng = np.random.default_rng(200 + seed)
    n = 50
    al = _random_alphas(rng, n)
    E = rng.uniform(0, 1, (n, 3))
    Lb = rng.uniform(0, 1, 3)
    op = O.FIGURE_OPS[name]
    res = O.composite_sequence(al, op, E, Lb)
    if op.kind == "vicini":
        pytest.skip("Vicini's operator is a lerp of two complete operators, "
                    "not one sequence with its own T")
    L = O.back_to_front(res["p"], res["T"], E, Lb)
    assert np.allclose(L, res["L"], atol=1e-12)


def test_exponential_is_classic_alpha_blending():
    """Exponential operator = eq. gaussian_splatting of Sec. 3."""
    rng = np.random.default_rng(7)
    al = rng.uniform(0, 0.5, 30)
    E = rng.uniform(0, 1, (30, 3))
    Lb = np.array([0.3, 0.2, 0.1])
    res = O.composite_sequence(al, O.EXPONENTIAL, E, Lb)
    T = 1.0
    L = np.zeros(3)
    for a, e in zip(al, E):
        L += e * a * T
        T *= 1 - a
    L += Lb * T
    assert np.allclose(res["L"], L, atol=1e-14)


def test_discrete_converges_to_mother():
    """Sec. 4 Evaluation: many small splats converge to the mother T(tau)."""
    for name, op in O.FIGURE_OPS.items():
        if op.kind == "powerlaw" and op.param < 0:
            continue   # its mother T has an infinite slope where it reaches 0
        for n in (2000,):
            a = 2.0 / n
            res = O.composite_sequence([a] * n, op)
            tau = np.arange(n + 1) * a
            assert np.abs(res["T"] - O.mother_T(op, tau)).max() < 5e-3, name
