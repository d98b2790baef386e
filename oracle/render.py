"""Plain per-pixel renderer in FP64: the definition, one pixel at a time.

Parity: pinned through its parts (operators, project, keys, each pinned in
the tests) and as a whole by the single-Gaussian closed form, the
weights-plus-transmittance identity, the back-to-front recursion and brute
force over every Gaussian on tiny scenes.

For one pixel centre (x + 1/2, y + 1/2): take every Gaussian that survives
the cull of the key recipe (module keys), evaluate alpha = aleph * K at the
centre in FP64 (module project), keep those with alpha >= alpha_min, order
them front to back by (float32 depth bits, Gaussian index) and composite them
with the chosen operator (module operators, Sec. 4 eq. generalized_gaussian
and eq. nexp_p).

To find the Gaussians that can reach alpha_min at a pixel without scanning
all of them, Gaussians are first listed per 16x16-pixel cell by their FP64
bounding box of the ellipse q <= 2 ln(1 / (alpha_min (1 - 1e-5))), which
contains every point where alpha >= alpha_min (1 - 1e-5) because aleph <= 1.
That list only prunes; it does not change any result.

Where float32 rounding may legitimately take a discrete decision the other
way than this FP64 evaluation (a considered alpha within 1e-5 relative of
alpha_min; a step whose transmittance lands within 1e-6 of the cutoff: 0
for the running-sum operators, t_eps for the exponential, or below 1e-30
where a float32 product may flush to zero), the pixel is flagged and every
outcome reachable by taking such decisions the other way is listed beside
the definition's (boundary_decisions, composite_pixel).  The renderer's
result must then match one of them (Sec. 4 fixes the result only away from
these measure-zero boundaries).
"""
import math

import numpy as np

from . import keys as _keys
from . import operators as _ops
from . import project as _project

CELL = 16
ALPHA_REL = 1e-5
CUTOFF_ABS = 1e-6
UNDERFLOW = 1e-30    # below this a float32 product of (1 - alpha) may flush to 0


def _cell_lists(proj, vis_idx, alpha_min, width, height):
    """Gaussian indices per CELL x CELL block, from FP64 bounding boxes."""
    k2 = 2.0 * math.log(1.0 / (alpha_min * (1.0 - ALPHA_REL)))
    a, c = proj["cov2d"][vis_idx, 0], proj["cov2d"][vis_idx, 2]
    u, v = proj["uv"][vis_idx, 0], proj["uv"][vis_idx, 1]
    rx, ry = np.sqrt(k2 * a) * (1 + 1e-9) + 1e-9, np.sqrt(k2 * c) * (1 + 1e-9) + 1e-9
    ncx, ncy = (width + CELL - 1) // CELL, (height + CELL - 1) // CELL
    x0 = np.clip(np.ceil(u - rx - 0.5), 0, width - 1).astype(np.int64) // CELL
    x1 = np.clip(np.floor(u + rx - 0.5), 0, width - 1).astype(np.int64) // CELL
    y0 = np.clip(np.ceil(v - ry - 0.5), 0, height - 1).astype(np.int64) // CELL
    y1 = np.clip(np.floor(v + ry - 0.5), 0, height - 1).astype(np.int64) // CELL
    ok = (np.ceil(u - rx - 0.5) <= width - 1) & (np.floor(u + rx - 0.5) >= 0) & \
         (np.ceil(v - ry - 0.5) <= height - 1) & (np.floor(v + ry - 0.5) >= 0)
    w = np.where(ok, x1 - x0 + 1, 0)
    h = np.where(ok, y1 - y0 + 1, 0)
    cnt = w * h
    gid = np.repeat(vis_idx, cnt)
    src = np.repeat(np.arange(vis_idx.size), cnt)
    first = np.cumsum(cnt) - cnt
    local = np.arange(gid.size) - first[src]
    cx = x0[src] + local % np.maximum(w[src], 1)
    cy = y0[src] + local // np.maximum(w[src], 1)
    cell = cy * ncx + cx
    order = np.argsort(cell, kind="stable")
    cell, gid = cell[order], gid[order]
    starts = np.searchsorted(cell, np.arange(ncx * ncy), "left")
    ends = np.searchsorted(cell, np.arange(ncx * ncy), "right")
    return ncx, starts, ends, gid


def boundary_decisions(alphas, res, op, alpha_min, t_eps):
    """The discrete decisions of one composited sequence that lie within
    float32 reach of their boundary, as flip keys of
    operators.composite_sequence (sorted by position in the sequence):

      (i, 0)  splat i's alpha within ALPHA_REL (relative) of alpha_min: a
              float32 alpha may keep or drop it;
      (i, 1)  the step of splat i leaves a transmittance within CUTOFF_ABS of
              the cutoff: for the running-sum operators T = 1 - sum p near 0
              (the saturation test of eq. nexp_p), for the exponential T near
              t_eps; with no termination threshold (t_eps <= UNDERFLOW) an
              exponential step that leaves T < UNDERFLOW while the sequence
              goes on, where the float32 product may flush to zero and stop;
      (i, 2)  Vicini's operator: the exponential part's (i, 1).

    Only splats the sequence reached are considered (a pixel that stopped at
    splat k never looks at splat k + 1)."""
    if op.kind == "vicini":
        lin, ex = res["parts"]
        d = set(boundary_decisions(alphas, lin, _ops.LINEAR, alpha_min, t_eps))
        for i, s in boundary_decisions(alphas, ex, _ops.EXPONENTIAL, alpha_min, t_eps):
            d.add((i, 2 if s == 1 else 0))
        return sorted(d)
    last = res["k"] if res["done"] else len(alphas) - 1
    T, p_raw = res["T"], res["p_raw"]
    out = []
    for i in range(last + 1):
        if abs(alphas[i] - alpha_min) <= ALPHA_REL * alpha_min:
            out.append((i, 0))
        if math.isnan(p_raw[i]):
            continue                   # not composited
        # transmittance this step leaves before any clamp
        t_next = T[i] - p_raw[i]
        if op.kind != "exponential":
            near = abs(t_next) <= CUTOFF_ABS
        elif t_eps is not None and t_eps > UNDERFLOW:
            near = abs(t_next - t_eps) <= CUTOFF_ABS
        else:
            near = t_next < UNDERFLOW and not (res["done"] and i == res["k"])
        if near:
            out.append((i, 1))
    return out


def composite_pixel(alphas, rgb, op, alpha_min, t_eps, background, max_outcomes=4096):
    """Composite one pixel's front-to-back list (alphas already >= alpha_min
    or near it).

    Returns (res, outcomes, amb_alpha, amb_cut): `res` is the plain
    definition (operators.composite_sequence); `outcomes` lists (L, T_final,
    od) for the definition and for every combination of boundary decisions
    taken the other way (each flipped decision within reach of float32
    rounding in the sequence that the earlier flips produce), the
    definition first; amb_alpha / amb_cut: the definition has an alpha_min
    boundary decision / a cutoff boundary decision."""
    outcomes = []

    def run(flips, after):
        r = _ops.composite_sequence(alphas, op, rgb, background, alpha_min, t_eps,
                                    flips=flips)
        outcomes.append((r["L"], r["T_final"], r["od"]))
        if len(outcomes) > max_outcomes:
            raise RuntimeError("more than %d boundary outcomes at one pixel" % max_outcomes)
        dec = boundary_decisions(alphas, r, op, alpha_min, t_eps)
        for d in dec:
            if d > after:
                run(flips | {d}, d)
        return r, dec

    res, dec = run(frozenset(), (-1, -1))
    amb_alpha = any(s == 0 for _, s in dec)
    amb_cut = any(s != 0 for _, s in dec)
    return res, outcomes, amb_alpha, amb_cut


def render(scene, cam, op, alpha_min=1e-3, t_eps=None, background=(0.0, 0.0, 0.0),
           pixels=None, proj=None, geom=None):
    """Render `pixels` (an [P,2] int array of (x, y); default: the whole image).

    op: an operators.Op (or a library model id 0..3).  t_eps defaults to 1e-4
    for the exponential (and Vicini's exponential part) and 0 otherwise.
    Returns a dict of per-pixel arrays: rgb [P,3], trans [P], od [P] (int),
    amb_alpha / amb_cut / ambiguous [P] (bool: an alpha_min boundary, a
    cutoff boundary, either), pixels [P,2]; and `outcomes`, a dict from the
    index of every flagged pixel to its list of legitimate (rgb, trans, od)
    (composite_pixel), the definition's first.
    """
    if isinstance(op, int):
        op = _ops.MODELS[op]
    if t_eps is None:
        t_eps = 1e-4 if op.kind in ("exponential", "vicini") else 0.0
    W, H = cam.width, cam.height
    if pixels is None:
        yy, xx = np.mgrid[0:H, 0:W]
        pixels = np.stack([xx.ravel(), yy.ravel()], 1)
    pixels = np.asarray(pixels, np.int64).reshape(-1, 2)
    proj = _project.project(scene, cam) if proj is None else proj
    geom = _keys.geometry(scene, cam, alpha_min) if geom is None else geom
    vis = np.nonzero(geom["visible"])[0]
    # global front-to-back order: float32 depth bits, then index
    order = vis[np.lexsort((vis, geom["depth_bits"][vis]))]
    rank = np.full(scene.n, -1, np.int64)
    rank[order] = np.arange(order.size)
    ncx, starts, ends, gid = _cell_lists(proj, vis, alpha_min, W, H)
    bg = np.asarray(background, np.float64)

    P = pixels.shape[0]
    rgb = np.zeros((P, 3))
    trans = np.zeros(P)
    od = np.zeros(P, np.int64)
    amb_alpha = np.zeros(P, bool)
    amb_cut = np.zeros(P, bool)
    outcomes = {}
    cell_of = (pixels[:, 1] // CELL) * ncx + pixels[:, 0] // CELL
    for cell in np.unique(cell_of):
        sel = np.nonzero(cell_of == cell)[0]
        cand = gid[starts[cell]:ends[cell]]
        cand = cand[np.argsort(rank[cand])]
        if cand.size:
            al = _project.alpha_at(proj, cand[None, :], pixels[sel, 0][:, None],
                                   pixels[sel, 1][:, None])
        for r, pi in enumerate(sel):
            if cand.size:
                keep = al[r] >= alpha_min * (1.0 - ALPHA_REL)
                a_p, g_p = al[r][keep], cand[keep]
            else:
                a_p, g_p = np.zeros(0), cand
            res, outs, aa, ac = composite_pixel(list(a_p), proj["rgb"][g_p], op,
                                                alpha_min, t_eps, bg)
            rgb[pi] = res["L"]
            trans[pi] = res["T_final"]
            od[pi] = res["od"]
            amb_alpha[pi], amb_cut[pi] = aa, ac
            if aa or ac:
                outcomes[pi] = outs
    return {"rgb": rgb, "trans": trans, "od": od, "amb_alpha": amb_alpha,
            "amb_cut": amb_cut, "ambiguous": amb_alpha | amb_cut,
            "outcomes": outcomes, "pixels": pixels}


def render_brute(scene, cam, op, alpha_min=1e-3, t_eps=None, background=(0.0, 0.0, 0.0)):
    """Whole image with no cell pruning: every visible Gaussian at every pixel.
    Only for tiny scenes; used to check the pruning in render()."""
    if isinstance(op, int):
        op = _ops.MODELS[op]
    if t_eps is None:
        t_eps = 1e-4 if op.kind in ("exponential", "vicini") else 0.0
    proj = _project.project(scene, cam)
    geom = _keys.geometry(scene, cam, alpha_min)
    vis = np.nonzero(geom["visible"])[0]
    order = vis[np.lexsort((vis, geom["depth_bits"][vis]))]
    W, H = cam.width, cam.height
    rgb = np.zeros((H * W, 3))
    trans = np.zeros(H * W)
    od = np.zeros(H * W, np.int64)
    for y in range(H):
        for x in range(W):
            al = _project.alpha_at(proj, order, x, y)
            res = _ops.composite_sequence(al, op, proj["rgb"][order], background,
                                          alpha_min, t_eps)
            rgb[y * W + x], trans[y * W + x], od[y * W + x] = res["L"], res["T_final"], res["od"]
    return {"rgb": rgb, "trans": trans, "od": od}
