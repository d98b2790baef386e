"""The finite-difference helper used by the gradient tests, pinned on the CPU.

A single isotropic Gaussian on the optical axis composited with the linear
operator: one splat, no saturation (aleph < 1), so rgb = E alpha + L_b (1 -
alpha) and trans = 1 - alpha (Sec. 4, eq. generalized_gaussian with k past the
end).  Then dLoss/daleph = sum_p [w_rgb . (E - L_b) - w_T] K_p and
dLoss/dE = sum_p w_rgb alpha_p, closed forms the helper must reproduce.
"""
import math

import numpy as np

import synth
from oracle import operators as O
from oracle import project as P
from tests import fd


def _one():
    sc = synth.Scene(np.array([[0.05, -0.02, 0.0]], np.float32), np.full((1, 3), 0.1, np.float32),
                     np.array([[1, 0, 0, 0]], np.float32), np.array([0.7], np.float32),
                     np.array([[[0.3, -0.2, 0.5]]], np.float32), 0)
    cam = synth.look_at_camera((0.0, 0.0, -2.0), width=24, height=20)
    return sc, cam


def test_closed_form_opacity_and_colour():
    sc, cam = _one()
    bg = np.array([0.2, 0.1, 0.4])
    F = fd.FrozenLoss(sc, [cam], O.LINEAR, background=bg, seed=3)
    v = F.views[0]
    proj = P.project(sc, cam)
    K = np.array([P.alpha_at(proj, np.array([0]), x, y)[0] / 0.7 if ids.size else 0.0
                  for x, y, ids in zip(v["px"], v["py"], v["lists"])])
    E = proj["rgb"][0]
    want_op = float(np.sum((v["w_rgb"] @ (E - bg) - v["w_T"]) * K))
    params = fd.params_of(sc)
    got_op = F.grad_element(params, "opacities", (0,), 1e-6)
    assert abs(got_op - want_op) <= 1e-6 * max(1.0, abs(want_op))
    # colour: emission = SH_C0 * coef + 1/2 (degree 0), not clamped here
    alpha = 0.7 * K
    want_c = float(np.sum(v["w_rgb"][:, 1] * alpha)) * 0.28209479177387814
    got_c = F.grad_element(params, "sh", (0, 0, 1), 1e-6)
    assert abs(got_c - want_c) <= 1e-6 * max(1.0, abs(want_c))


def test_base_loss_matches_render():
    """At the base point the frozen loss is the weighted oracle render."""
    from oracle import render as Rn
    sc = synth.random_scene(11, 30, log_scale=(-1.8, 0.3), logit=(1.0, 1.0), sh_degree=1)
    cam = synth.look_at_camera((0.3, 0.2, -3.0), width=20, height=16)
    for op in (O.EXPONENTIAL, O.LINEAR, O.SUPERLINEAR):
        F = fd.FrozenLoss(sc, [cam], op, seed=1)
        out = Rn.render(sc, cam, op)
        v = F.views[0]
        want = float(np.sum(v["w_rgb"] * out["rgb"]) + np.sum(v["w_T"] * out["trans"]))
        assert math.isclose(F(fd.params_of(sc)), want, rel_tol=1e-12, abs_tol=1e-12)
