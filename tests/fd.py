"""Finite differences of the FP64 oracle render for checking analytic gradients.

The render is piecewise smooth: a Gaussian enters or leaves a pixel's list
where its alpha crosses alpha_min, and two Gaussians swap where their depths
cross.  The analytic gradient is the derivative of the smooth piece the base
point lies on, so the loss here freezes those discrete decisions at the base
point: each pixel keeps the Gaussians (and their front-to-back order) that the
oracle composites there at the base parameters, and only their alphas and
emissions move with the parameters.  Saturation and the exponential's
termination stay live (they are continuous, or flagged ambiguous within 1e-6
of the cutoff, and the steps used are far smaller than that).

Loss = sum over views and pixels of w_rgb . rgb + w_T * trans, with the
weights zeroed at the pixels the oracle flags ambiguous (a float32 render may
legitimately take another discrete decision there).
"""
import numpy as np

import synth
from oracle import keys as _keys
from oracle import operators as _ops
from oracle import project as _project
from oracle import render as _render

FIELDS = ("means", "scales", "quats", "opacities", "sh")


def params_of(scene):
    return {k: np.asarray(getattr(scene, k), np.float64).copy() for k in FIELDS}


class FrozenLoss:
    def __init__(self, scene, cams, op, alpha_min=1e-3, t_eps=None, background=(0, 0, 0),
                 seed=0):
        if isinstance(op, int):
            op = _ops.MODELS[op]
        if t_eps is None:
            t_eps = 1e-4 if op.kind == "exponential" else 0.0
        self.op, self.t_eps = op, t_eps
        self.bg = np.asarray(background, np.float64)
        self.sh_degree = scene.sh_degree
        self.cams = cams
        rng = np.random.default_rng(seed)
        self.views = []
        for cam in cams:
            W, H = cam.width, cam.height
            proj = _project.project(scene, cam)
            geom = _keys.geometry(scene, cam, alpha_min)
            vis = np.nonzero(geom["visible"])[0]
            order = vis[np.lexsort((vis, geom["depth_bits"][vis]))]
            yy, xx = np.mgrid[0:H, 0:W]
            px, py = xx.ravel(), yy.ravel()
            lists = [np.zeros(0, np.int64)] * px.size
            if order.size:
                al = _project.alpha_at(proj, order[None, :], px[:, None], py[:, None])
                lists = [order[al[p] >= alpha_min] for p in range(px.size)]
            base = _render.render(scene, cam, op, alpha_min, t_eps, background)
            w_rgb = rng.normal(size=(px.size, 3))
            w_T = rng.normal(size=px.size)
            w_rgb[base["ambiguous"]] = 0.0
            w_T[base["ambiguous"]] = 0.0
            lens = np.array([l.size for l in lists], np.int64)
            self.views.append({"px": px, "py": py, "lists": lists, "w_rgb": w_rgb,
                               "pair_pix": np.repeat(np.arange(px.size), lens),
                               "pair_id": (np.concatenate(lists) if lists else
                                           np.zeros(0, np.int64)).astype(np.int64),
                               "off": np.concatenate([[0], np.cumsum(lens)]),
                               "w_T": w_T, "n_ambiguous": int(base["ambiguous"].sum()),
                               "H": H, "W": W})

    def weights(self, v):
        """Upstream gradients of view v as images: ([H,W,3], [H,W]) float32."""
        d = self.views[v]
        return (d["w_rgb"].reshape(d["H"], d["W"], 3).astype(np.float32),
                d["w_T"].reshape(d["H"], d["W"]).astype(np.float32))

    def __call__(self, params, only=None):
        """Loss at `params` (dict of float64 arrays); with `only` = a Gaussian
        index, just the pixels whose frozen list holds it (the rest of the
        loss does not depend on that Gaussian)."""
        sc = synth.Scene(params["means"], params["scales"], params["quats"],
                         params["opacities"], params["sh"], self.sh_degree)
        total = 0.0
        for cam, d in zip(self.cams, self.views):
            proj = _project.project(sc, cam)
            if only is None:
                pix = np.arange(d["px"].size)
            else:
                pix = np.unique(d["pair_pix"][d["pair_id"] == only])
            if d["pair_id"].size:
                pp, pid = d["pair_pix"], d["pair_id"]
                alpha = _project.alpha_at(proj, pid, d["px"][pp], d["py"][pp])
            for p in pix:
                lo, hi = d["off"][p], d["off"][p + 1]
                ids = d["lists"][p]
                res = _ops.composite_sequence(list(alpha[lo:hi]) if hi > lo else [], self.op,
                                              proj["rgb"][ids], self.bg, 0.0, self.t_eps)
                total += float(d["w_rgb"][p] @ res["L"]) + d["w_T"][p] * res["T_final"]
        return total

    def grad_element(self, params, field, index, h):
        """Central difference of the loss in one scalar parameter."""
        i = index[0]
        up = {k: v.copy() for k, v in params.items()}
        dn = {k: v.copy() for k, v in params.items()}
        up[field][index] += h
        dn[field][index] -= h
        return (self(up, only=i) - self(dn, only=i)) / (2.0 * h)

    def grad_direction(self, params, direction, h):
        """Central difference along a direction (dict of arrays, any subset of fields)."""
        up = {k: v + h * direction.get(k, 0.0) for k, v in params.items()}
        dn = {k: v - h * direction.get(k, 0.0) for k, v in params.items()}
        return (self(up) - self(dn)) / (2.0 * h)
