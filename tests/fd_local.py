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

The per-Gaussian lists and the central differences are independent of each
other, so both are computed by a pool of worker processes (started fresh,
never forked from a process that holds the GPU; they import numpy and the
oracle only).
"""
import math
import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

import synth
from oracle import keys as _keys
from oracle import operators as _ops
from oracle import project as _project
from oracle import render as _render

ALPHA_REL = _render.ALPHA_REL

# state of one worker process (set by _init)
_W = {}


def default_workers():
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _init(scene, cams, op, alpha_min, t_eps):
    _W.update(scene=scene, cams=cams, op=op, alpha_min=alpha_min, t_eps=t_eps, views=[])
    k2 = 2.0 * math.log(1.0 / (alpha_min * (1.0 - ALPHA_REL)))
    for cam in cams:
        proj = _project.project(scene, cam)
        geom = _keys.geometry(scene, cam, alpha_min)
        vis = np.nonzero(geom["visible"])[0]
        rank = np.full(scene.n, -1, np.int64)
        order = vis[np.lexsort((vis, geom["depth_bits"][vis]))]
        rank[order] = np.arange(order.size)
        with np.errstate(invalid="ignore"):
            rx = np.sqrt(k2 * proj["cov2d"][:, 0]) + 1e-6
            ry = np.sqrt(k2 * proj["cov2d"][:, 2]) + 1e-6
        _W["views"].append({"proj": proj, "vis": vis, "rank": rank, "rx": rx, "ry": ry})


def _stopped(res):
    if _W["op"].kind == "exponential":
        return res["T_final"] < _W["t_eps"] or res["T_final"] == 0.0
    return res["T_final"] == 0.0


def _build_one(i):
    """Per view: the pixels of Gaussian i, their frozen lists and ambiguity
    flags (None for a view where i reaches no pixel)."""
    op, alpha_min, t_eps = _W["op"], _W["alpha_min"], _W["t_eps"]
    out = []
    for cam, V in zip(_W["cams"], _W["views"]):
        proj, vis, rank, rx, ry = V["proj"], V["vis"], V["rank"], V["rx"], V["ry"]
        u, v = proj["uv"][:, 0], proj["uv"][:, 1]
        if rank[i] < 0:
            out.append(None)
            continue
        x0 = max(int(math.ceil(u[i] - rx[i] - 0.5)), 0)
        x1 = min(int(math.floor(u[i] + rx[i] - 0.5)), cam.width - 1)
        y0 = max(int(math.ceil(v[i] - ry[i] - 0.5)), 0)
        y1 = min(int(math.floor(v[i] + ry[i] - 0.5)), cam.height - 1)
        if x1 < x0 or y1 < y0:
            out.append(None)
            continue
        yy, xx = np.mgrid[y0:y1 + 1, x0:x1 + 1]
        a = _project.alpha_at(proj, np.full(xx.size, i), xx.ravel(), yy.ravel())
        keep = a >= alpha_min * (1.0 - ALPHA_REL)
        if not keep.any():
            out.append(None)
            continue
        px = np.stack([xx.ravel()[keep], yy.ravel()[keep]], 1).astype(np.int64)
        cand = vis[(u[vis] + rx[vis] >= x0 + 0.5) & (u[vis] - rx[vis] <= x1 + 0.5) &
                   (v[vis] + ry[vis] >= y0 + 0.5) & (v[vis] - ry[vis] <= y1 + 0.5)]
        cand = cand[np.argsort(rank[cand])]
        lists, amb = [], np.zeros(len(px), bool)
        al_all = _project.alpha_at(proj, cand[None, :], px[:, 0][:, None], px[:, 1][:, None])
        for p in range(len(px)):
            al = al_all[p]
            near = np.nonzero(al >= alpha_min * (1.0 - ALPHA_REL))[0]
            # most pixels stop within their first few dozen splats: try a
            # prefix, and the whole list only if the pixel has not stopped
            for cut in (64, len(near)):
                head = near[:cut]
                res, _, aa, ac = _render.composite_pixel(
                    list(al[head]), proj["rgb"][cand[head]], op, alpha_min, t_eps,
                    np.zeros(3))
                amb[p] = aa or ac
                if _stopped(res) or cut >= len(near):
                    break
            # frozen at the base point: the splats composited there (the pixel
            # stops at the same one under the small perturbations, except at
            # pixels flagged ambiguous)
            upto = near[:res["k"] + 1]
            lists.append(cand[upto[al[upto] >= alpha_min]])
        out.append({"px": px, "lists": lists, "ambiguous": amb})
    return out


def _local_loss(per, wts, field, index, delta):
    """Loss over the pixels of one Gaussian (per: _build_one's result; wts:
    per view, the weights at those pixels) with params[field][index] moved by
    delta."""
    sc = _W["scene"]
    i = index[0]
    total = 0.0
    for cam, d, w in zip(_W["cams"], per, wts):
        if d is None:
            continue
        ids_all = np.unique(np.concatenate(d["lists"]))
        sub = sc.subset(ids_all)
        arrs = {k: np.asarray(getattr(sub, k), np.float64).copy()
                for k in ("means", "scales", "quats", "opacities", "sh")}
        loc_i = int(np.searchsorted(ids_all, i))
        if loc_i < ids_all.size and ids_all[loc_i] == i:
            arrs[field][(loc_i,) + tuple(index[1:])] += delta
        psc = synth.Scene(arrs["means"], arrs["scales"], arrs["quats"], arrs["opacities"],
                          arrs["sh"], sc.sh_degree)
        proj = _project.project(psc, cam)
        for p, ids in enumerate(d["lists"]):
            loc = np.searchsorted(ids_all, ids)
            x, y = d["px"][p]
            a = _project.alpha_at(proj, loc, x, y)
            res = _ops.composite_sequence(list(a), _W["op"], proj["rgb"][loc], np.zeros(3),
                                          0.0, _W["t_eps"])
            total += float(w[p] @ res["L"])
    return total


def _fd_one(job):
    per, wts, field, index, h = job
    return (_local_loss(per, wts, field, index, h) -
            _local_loss(per, wts, field, index, -h)) / (2.0 * h)


class LocalLoss:
    def __init__(self, scene, cams, op, focus, alpha_min=1e-3, t_eps=None, workers=None):
        """focus: Gaussian indices whose pixels get lists."""
        if isinstance(op, int):
            op = _ops.MODELS[op]
        if t_eps is None:
            t_eps = 1e-4 if op.kind == "exponential" else 0.0
        self.op, self.t_eps, self.alpha_min = op, t_eps, alpha_min
        self.scene, self.cams = scene, cams
        self.focus = [int(i) for i in focus]
        n = workers or default_workers()
        self.pool = ProcessPoolExecutor(max_workers=n, mp_context=mp.get_context("spawn"),
                                        initializer=_init,
                                        initargs=(scene, cams, op, alpha_min, t_eps))
        per = list(self.pool.map(_build_one, self.focus))
        # views[v][i] as before: the focus Gaussian's pixels in view v
        self.per = dict(zip(self.focus, per))
        self.views = [{i: p[v] for i, p in self.per.items() if p[v] is not None}
                      for v in range(len(cams))]

    def close(self):
        self.pool.shutdown()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def mask_weights(self, weights):
        """Zero, in place, the given per-view [H,W,3] weights at ambiguous pixels."""
        for w, per in zip(weights, self.views):
            for d in per.values():
                for (x, y), a in zip(d["px"], d["ambiguous"]):
                    if a:
                        w[y, x] = 0.0

    def n_pixels(self, i):
        return sum(len(per[i]["px"]) for per in self.views if i in per)

    def grad_elements(self, weights, items):
        """Central differences for items (field, index, h), index[0] a focus
        Gaussian; weights: per view [H,W,3] arrays."""
        jobs = []
        for field, index, h in items:
            i = int(index[0])
            per = self.per[i]
            wts = [None if d is None else w[d["px"][:, 1], d["px"][:, 0]]
                   for d, w in zip(per, weights)]
            jobs.append((per, wts, field, tuple(index), h))
        return list(self.pool.map(_fd_one, jobs))
