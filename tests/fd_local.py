"""Finite differences of the FP64 oracle render around single Gaussians of a
large scene, for checking analytic gradients at full workload size.

A parameter of Gaussian i changes only the pixels where i is composited, so
the loss restricted to the pixels where i reaches alpha_min has the same
derivative in that parameter as the loss over the whole image.  For those
pixels only, each pixel's list is built as in the per-pixel definition (every
visible Gaussian whose FP64 alpha reaches alpha_min, in (float32 depth bits,
index) order) and frozen at the base point; perturbed parameters then move the
alphas and emissions of the frozen lists (as in tests/fd.py).

Loss = sum over views and listed pixels of w_rgb . rgb (the caller's weights,
e.g. the signs of an L1 loss), with the pixels the oracle flags as ambiguous
given weight 0 (the caller must pass the same zeros to the GPU backward).
"""
import math

import numpy as np

import synth
from oracle import keys as _keys
from oracle import operators as _ops
from oracle import project as _project
from oracle import render as _render

ALPHA_REL = _render.ALPHA_REL


class LocalLoss:
    def __init__(self, scene, cams, op, focus, alpha_min=1e-3, t_eps=None):
        """focus: Gaussian indices whose pixels get lists."""
        if isinstance(op, int):
            op = _ops.MODELS[op]
        if t_eps is None:
            t_eps = 1e-4 if op.kind == "exponential" else 0.0
        self.op, self.t_eps, self.alpha_min = op, t_eps, alpha_min
        self.scene, self.cams = scene, cams
        self.views = []
        k2 = 2.0 * math.log(1.0 / (alpha_min * (1.0 - ALPHA_REL)))
        for cam in cams:
            proj = _project.project(scene, cam)
            geom = _keys.geometry(scene, cam, alpha_min)
            vis = np.nonzero(geom["visible"])[0]
            rank = np.full(scene.n, -1, np.int64)
            order = vis[np.lexsort((vis, geom["depth_bits"][vis]))]
            rank[order] = np.arange(order.size)
            u, v = proj["uv"][:, 0], proj["uv"][:, 1]
            with np.errstate(invalid="ignore"):
                rx = np.sqrt(k2 * proj["cov2d"][:, 0]) + 1e-6
                ry = np.sqrt(k2 * proj["cov2d"][:, 2]) + 1e-6
            # per focus Gaussian: its pixels and their frozen lists, candidates
            # taken from the Gaussians whose boxes overlap its own box
            per = {}
            for i in focus:
                if rank[i] < 0:
                    continue
                x0 = max(int(math.ceil(u[i] - rx[i] - 0.5)), 0)
                x1 = min(int(math.floor(u[i] + rx[i] - 0.5)), cam.width - 1)
                y0 = max(int(math.ceil(v[i] - ry[i] - 0.5)), 0)
                y1 = min(int(math.floor(v[i] + ry[i] - 0.5)), cam.height - 1)
                if x1 < x0 or y1 < y0:
                    continue
                yy, xx = np.mgrid[y0:y1 + 1, x0:x1 + 1]
                a = _project.alpha_at(proj, np.full(xx.size, i), xx.ravel(), yy.ravel())
                keep = a >= alpha_min * (1.0 - ALPHA_REL)
                if not keep.any():
                    continue
                px = np.stack([xx.ravel()[keep], yy.ravel()[keep]], 1).astype(np.int64)
                cand = vis[(u[vis] + rx[vis] >= x0 + 0.5) & (u[vis] - rx[vis] <= x1 + 0.5) &
                           (v[vis] + ry[vis] >= y0 + 0.5) & (v[vis] - ry[vis] <= y1 + 0.5)]
                cand = cand[np.argsort(rank[cand])]
                lists, amb = [], np.zeros(len(px), bool)
                al_all = _project.alpha_at(proj, cand[None, :], px[:, 0][:, None],
                                           px[:, 1][:, None])
                for p in range(len(px)):
                    al = al_all[p]
                    near = np.nonzero(al >= alpha_min * (1.0 - ALPHA_REL))[0]
                    # most pixels stop within their first few dozen splats: try a
                    # prefix, and the whole list only if the pixel has not stopped
                    for cut in (64, len(near)):
                        head = near[:cut]
                        res, amb[p] = _render.composite_pixel(
                            list(al[head]), proj["rgb"][cand[head]], op, alpha_min, t_eps,
                            np.zeros(3))
                        if self._stopped(res) or cut >= len(near):
                            break
                    # frozen at the base point: the splats composited there (the
                    # pixel stops at the same one under the small perturbations,
                    # except at pixels flagged ambiguous)
                    upto = near[:res["k"] + 1]
                    lists.append(cand[upto[al[upto] >= alpha_min]])
                per[int(i)] = {"px": px, "lists": lists, "ambiguous": amb}
            self.views.append(per)

    def _stopped(self, res):
        if self.op.kind == "exponential":
            return res["T_final"] < self.t_eps or res["T_final"] == 0.0
        return res["T_final"] == 0.0

    def mask_weights(self, weights):
        """Zero, in place, the given per-view [H,W,3] weights at ambiguous pixels."""
        for w, per in zip(weights, self.views):
            for d in per.values():
                for (x, y), a in zip(d["px"], d["ambiguous"]):
                    if a:
                        w[y, x] = 0.0

    def n_pixels(self, i):
        return sum(len(per[i]["px"]) for per in self.views if i in per)

    def __call__(self, params, weights, only):
        """Loss over the pixels of Gaussian `only` (the rest does not depend on it)."""
        sc = synth.Scene(params["means"], params["scales"], params["quats"],
                         params["opacities"], params["sh"], self.scene.sh_degree)
        total = 0.0
        for cam, per, w in zip(self.cams, self.views, weights):
            d = per.get(int(only))
            if d is None:
                continue
            ids_all = np.unique(np.concatenate(d["lists"]))
            proj = _project.project(sc.subset(ids_all), cam)
            for p, ids in enumerate(d["lists"]):
                loc = np.searchsorted(ids_all, ids)
                x, y = d["px"][p]
                a = _project.alpha_at(proj, loc, x, y)
                res = _ops.composite_sequence(list(a), self.op, proj["rgb"][loc], np.zeros(3),
                                              0.0, self.t_eps)
                total += float(w[y, x] @ res["L"])
        return total

    def grad_element(self, params, weights, field, index, h):
        i = index[0]
        up = {k: v.copy() for k, v in params.items()}
        dn = {k: v.copy() for k, v in params.items()}
        up[field][index] += h
        dn[field][index] -= h
        return (self(up, weights, i) - self(dn, weights, i)) / (2.0 * h)
