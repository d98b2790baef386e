"""Pins of the oracle's boundary flags and of the legitimate outcomes it
lists at them (oracle.render.boundary_decisions / composite_pixel).

Sec. 4 fixes a pixel's value only away from three measure-zero boundaries
that a float32 evaluation may legitimately decide the other way: an alpha at
alpha_min (the splat is composited or skipped), a running sum of p reaching
1 (eq. nexp_p: that splat saturates, or the next one does) and the
exponential's transmittance reaching t_eps (it stops there or one splat
later).  Each case below is built by hand so that the step lands just inside
or just outside the flag window, and the outcomes are written out from the
definitions (single-splat value alpha E + (1 - alpha) L_b, the remainder
1 - sum p of the saturating splat, the product form of the exponential).
"""

import numpy as np
import pytest

from oracle import operators as O
from oracle import render as R

AMIN = 1e-3
E3 = np.array([[0.9, 0.5, 0.1], [0.2, 0.7, 0.4], [0.3, 0.3, 0.8], [0.6, 0.1, 0.5]])


def _pixel(alphas, op, t_eps=None, bg=(0.0, 0.0, 0.0)):
    if t_eps is None:
        t_eps = 1e-4 if op.kind in ("exponential", "vicini") else 0.0
    n = len(alphas)
    return R.composite_pixel(list(alphas), E3[:n], op, AMIN, t_eps, np.asarray(bg, float))


def _has(outcomes, L, T, od, tol=1e-12):
    return any(np.allclose(o[0], L, atol=tol, rtol=0) and abs(o[1] - T) <= tol and o[2] == od
               for o in outcomes)


# ------------------------------------------------------------ alpha_min window

@pytest.mark.parametrize("rel,flag", [(-5e-6, True), (5e-6, True), (-2e-5, False),
                                      (2e-5, False), (0.0, True)])
@pytest.mark.parametrize("op", [O.EXPONENTIAL, O.LINEAR, O.SUBLINEAR, O.SUPERLINEAR])
def test_alpha_min_window(op, rel, flag):
    a = AMIN * (1.0 + rel)
    bg = np.array([0.25, 0.5, 0.75])
    res, outs, aa, ac = _pixel([a], op, bg=bg)
    assert aa == flag and not ac
    kept = (E3[0] * a + bg * (1.0 - a), 1.0 - a, 1)
    dropped = (bg, 1.0, 0)
    primary = kept if a >= AMIN else dropped
    assert len(outs) == (2 if flag else 1)
    assert _has(outs[:1], *primary)
    if flag:
        assert _has(outs, *(dropped if a >= AMIN else kept))


def test_alpha_min_splat_after_the_stop_is_not_flagged():
    # the linear pixel saturates at splat 2 and never considers splat 3
    res, outs, aa, ac = _pixel([0.6, 0.7, AMIN], O.LINEAR)
    assert res["od"] == 2 and not aa and not ac and len(outs) == 1
    # ... while an unsaturated pixel does consider it
    res, outs, aa, ac = _pixel([0.2, 0.3, AMIN], O.LINEAR)
    assert res["od"] == 3 and aa and len(outs) == 2


# ------------------------------------------------ exponential termination window

@pytest.mark.parametrize("delta,flag", [(5e-7, True), (-5e-7, True), (2e-6, False),
                                        (-2e-6, False)])
def test_exponential_t_eps_window(delta, flag):
    t_eps = 1e-4
    a1 = 1.0 - (t_eps + delta)           # the first step leaves T = t_eps + delta
    a2 = 0.5
    res, outs, aa, ac = _pixel([a1, a2], O.EXPONENTIAL, t_eps=t_eps)
    assert ac == flag and not aa
    T1 = 1.0 - a1
    stop1 = (E3[0] * a1, T1, 1)
    go_on = (E3[0] * a1 + E3[1] * a2 * T1, T1 * (1.0 - a2), 2)
    primary = stop1 if T1 < t_eps else go_on
    assert _has(outs[:1], *primary)
    assert len(outs) == (2 if flag else 1)
    if flag:
        assert _has(outs, *(go_on if T1 < t_eps else stop1))


def test_exponential_underflow_without_termination():
    # t_eps = 0: the FP64 product never stops, a float32 one may flush to 0 and
    # stop at any step that leaves T below 1e-30
    alphas = [1.0 - 1e-16, 1.0 - 1e-16, 0.5, 0.5]   # T: 1e-16, 1e-32, 5e-33, 2.5e-33
    res, outs, aa, ac = _pixel(alphas, O.EXPONENTIAL, t_eps=0.0)
    assert ac and not aa and res["od"] == 4
    assert len(outs) == 4 and sorted(o[2] for o in outs[1:]) == [2, 3, 4] and outs[0][2] == 4
    # the early stops keep the colour to far below any tolerance
    for L, T, od in outs:
        assert np.abs(L - res["L"]).max() < 1e-30 and T < 1e-30


# ------------------------------------------------------- saturation window (sum p)

@pytest.mark.parametrize("delta,flag", [(5e-7, True), (-5e-7, True), (3e-6, False),
                                        (-3e-6, False)])
def test_linear_saturation_window(delta, flag):
    a = [0.6, 0.4 + delta, 0.3]
    res, outs, aa, ac = _pixel(a, O.LINEAR)
    assert ac == flag and not aa
    S2 = 0.6 + a[1]
    sat2 = (E3[0] * 0.6 + E3[1] * 0.4, 0.0, 2)           # splat 2 takes 1 - 0.6
    sat3 = (E3[0] * 0.6 + E3[1] * a[1] + E3[2] * (1.0 - S2), 0.0, 3)
    primary = sat2 if S2 >= 1.0 else sat3
    assert _has(outs[:1], *primary, tol=1e-15)
    assert len(outs) == (2 if flag else 1)
    if flag:
        assert _has(outs, *(sat3 if S2 >= 1.0 else sat2), tol=1e-15)


@pytest.mark.parametrize("op", [O.SUBLINEAR, O.SUPERLINEAR, O.Op("quadratic", 1.0)])
@pytest.mark.parametrize("delta", [4e-7, -4e-7])
def test_quadratic_saturation_window(op, delta):
    c = op.param
    a1 = 0.5
    # p2 = a2 (1 + c a1) lands at 1 - a1 + delta
    a2 = (1.0 - a1 + delta) / (1.0 + c * a1)
    res, outs, aa, ac = _pixel([a1, a2, 0.2], op)
    assert ac and not aa and len(outs) == 2
    assert sorted(o[2] for o in outs) == [2, 3]
    assert res["od"] == (2 if delta > 0 else 3)
    for L, T, od in outs:
        assert abs(T) < 1e-15 or T == 0.0


def test_no_flag_far_from_boundaries():
    for op in (O.EXPONENTIAL, O.LINEAR, O.SUBLINEAR, O.SUPERLINEAR):
        res, outs, aa, ac = _pixel([0.3, 0.2, 0.1], op)
        assert not aa and not ac and len(outs) == 1


# ------------------------------------------------------------- combinations

def test_two_boundaries_enumerate_all_consistent_outcomes():
    # splat 1 at alpha_min (kept or dropped), then a linear sum landing within
    # 5e-7 of 1 only when splat 1 is kept
    a1 = AMIN * (1.0 + 4e-6)
    a2 = 0.55
    a3 = 1.0 - a1 - a2 + 3e-7
    res, outs, aa, ac = _pixel([a1, a2, a3], O.LINEAR)
    assert aa and ac
    # kept + saturates at 3; kept + not (T = -3e-7, no later splat); dropped
    assert len(outs) == 3
    assert sorted(o[2] for o in outs) == [2, 3, 3]
    dropped = [o for o in outs if o[2] == 2][0]
    assert np.allclose(dropped[0], E3[1] * a2 + E3[2] * a3) and abs(dropped[1] - (1 - a2 - a3)) < 1e-15


def test_vicini_flags_both_parts():
    op = O.Op("vicini", 0.5)
    # the linear part saturates within 5e-7 of 1 at splat 2; the exponential
    # part's T stays far from t_eps
    res, outs, aa, ac = _pixel([0.6, 0.4 + 5e-7, 0.3], op)
    assert ac and not aa and len(outs) == 2
    dec = R.boundary_decisions([0.6, 0.4 + 5e-7, 0.3], res, op, AMIN, 1e-4)
    assert dec == [(1, 1)]
    # the exponential part alone lands near t_eps: the flip key is (i, 2)
    a1 = 1.0 - (1e-4 + 5e-7)
    res, outs, aa, ac = _pixel([a1, 0.5], op)
    dec = R.boundary_decisions([a1, 0.5], res, op, AMIN, 1e-4)
    assert (0, 2) in dec and ac


def test_outcome_limit():
    # many alpha_min boundary splats: 2^n outcomes; the enumeration refuses
    # beyond its limit instead of running away
    alphas = [AMIN] * 6
    E = np.tile(E3[:1], (6, 1))
    _, outs, aa, _ = R.composite_pixel(alphas, E, O.LINEAR, AMIN, 0.0, np.zeros(3))
    assert aa and len(outs) == 64
    with pytest.raises(RuntimeError):
        R.composite_pixel(alphas, E, O.LINEAR, AMIN, 0.0, np.zeros(3), max_outcomes=10)


def test_flags_in_a_rendered_image():
    """Through render(): every flagged pixel lists its definition first and
    every unflagged pixel has no alternative outcomes."""
    import synth
    sc, cams = synth.tiny_scene(seed=1, n=512)
    ref = R.render(sc, cams[0], O.EXPONENTIAL)
    for i, outs in ref["outcomes"].items():
        assert ref["ambiguous"][i]
        assert np.allclose(outs[0][0], ref["rgb"][i]) and outs[0][1] == ref["trans"][i]
        assert outs[0][2] == ref["od"][i] and len(outs) >= 2
    assert set(ref["outcomes"]) == set(np.nonzero(ref["ambiguous"])[0].tolist())
