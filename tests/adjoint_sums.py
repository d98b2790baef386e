"""Per-slot sums of the appendix adjoints, from the FP64 oracle.

For every pixel of a view: the composited list of the per-pixel definition
(every visible Gaussian whose FP64 alpha reaches alpha_min, in (float32
depth bits, index) order), the adjoint recursions of oracle.adjoint for
dLoss/dalpha_i and dLoss/dE_i (the appendix "Adjoints"; the final
transmittance rides along as a fourth channel with emission 0 and
background 1), chained through alpha_i = aleph_i exp(-q_i / 2),
q = A dx^2 + 2 B dx dy + C dy^2 with d = pixel centre - (u, v), into

    dLoss/d(aleph, u, v, A, B, C, r, g, b)

and summed per Gaussian: the quantities the library's backward accumulates
per slot before chaining them through the projection.
"""
import numpy as np

from oracle import adjoint as _adjoint
from oracle import keys as _keys
from oracle import operators as _ops
from oracle import project as _project
from oracle import render as _render


def slot_sums(scene, cam, op, g_rgb, g_T, alpha_min=1e-3, t_eps=None,
              background=(0.0, 0.0, 0.0)):
    """g_rgb [H,W,3], g_T [H,W]: upstream gradients (zero them at ambiguous
    pixels first: see ambiguous()).  Returns [n, 9] float64."""
    if isinstance(op, int):
        op = _ops.MODELS[op]
    if t_eps is None:
        t_eps = 1e-4 if op.kind == "exponential" else 0.0
    proj = _project.project(scene, cam)
    geom = _keys.geometry(scene, cam, alpha_min)
    vis = np.nonzero(geom["visible"])[0]
    order = vis[np.lexsort((vis, geom["depth_bits"][vis]))]
    out = np.zeros((scene.n, 9))
    E = np.concatenate([proj["rgb"], np.zeros((scene.n, 1))], 1)
    Lb = np.concatenate([np.asarray(background, np.float64), [1.0]])
    for y in range(cam.height):
        for x in range(cam.width):
            g = np.concatenate([g_rgb[y, x], [g_T[y, x]]]).astype(np.float64)
            if not np.any(g) or order.size == 0:
                continue
            al = _project.alpha_at(proj, order, x, y)
            keep = al >= alpha_min
            ids, a = order[keep], al[keep]
            if ids.size == 0:
                continue
            dalpha, dE = _adjoint.adjoint_sequence(list(a), op, E[ids], Lb, g, 0.0, t_eps)
            dx = (x + 0.5) - proj["uv"][ids, 0]
            dy = (y + 0.5) - proj["uv"][ids, 1]
            A, B, C = (proj["conic"][ids, k] for k in range(3))
            da = dalpha * a                        # dLoss/dalpha * alpha
            np.add.at(out[:, 0], ids, da / proj["opacity"][ids])
            np.add.at(out[:, 1], ids, da * (A * dx + B * dy))
            np.add.at(out[:, 2], ids, da * (B * dx + C * dy))
            np.add.at(out[:, 3], ids, -0.5 * da * dx * dx)
            np.add.at(out[:, 4], ids, -da * dx * dy)
            np.add.at(out[:, 5], ids, -0.5 * da * dy * dy)
            for c in range(3):
                np.add.at(out[:, 6 + c], ids, dE[:, c])
    return out


def ambiguous(scene, cam, op, alpha_min=1e-3, t_eps=None, background=(0.0, 0.0, 0.0)):
    """[H,W] bool: pixels where float32 may legitimately take another
    discrete decision (oracle.render's flag)."""
    if isinstance(op, int):
        op = _ops.MODELS[op]
    ref = _render.render(scene, cam, op, alpha_min, t_eps, background)
    return ref["ambiguous"].reshape(cam.height, cam.width)
