"""Helpers shared by the GPU parity tests: run the oracle and the library on
the same seeded inputs and compare them at the stated tolerances."""
import numpy as np

from oracle import keys as okeys
from oracle import render as orender

RGB_ATOL = 1e-4      # per channel, float32 colour
TRANS_ATOL = 1e-4    # final transmittance
# At most this share of the compared pixels may take one of the oracle's
# other legitimate boundary outcomes rather than the definition's: float32
# rounding decides a boundary differently only where the FP64 value lies far
# closer to it than the flag windows (alpha within ~2e-6 relative, T within
# ~1e-9 of the cutoff), so a renderer that departs more often has a biased
# threshold, not rounding.
MAX_ALTERNATE = 0.01


def sample_pixels(cam, n, seed=0):
    rng = np.random.default_rng(seed)
    total = cam.width * cam.height
    if n >= total:
        yy, xx = np.mgrid[0:cam.height, 0:cam.width]
        return np.stack([xx.ravel(), yy.ravel()], 1)
    flat = rng.choice(total, n, replace=False)
    return np.stack([flat % cam.width, flat // cam.width], 1)


def _matches(rgb, trans, od, outcome):
    L, T, n = outcome
    return (np.all(np.abs(rgb - L) <= RGB_ATOL) and abs(trans - T) <= TRANS_ATOL
            and od == n)


def compare_view(out, scene, cam, model, pixels=None, background=(0.0, 0.0, 0.0),
                 alpha_min=1e-3, t_eps=None, max_alternate=MAX_ALTERNATE):
    """Compare one rendered view with the oracle at `pixels` (default: all).

    * colour and transmittance within 1e-4 of the definition at every pixel
      without an alpha_min boundary splat (keeping or dropping a splat of
      alpha ~1e-3 may move the colour by more);
    * overdraw equal to the definition's at every unflagged pixel;
    * at every flagged pixel, colour, transmittance (both within 1e-4) and
      overdraw (exactly) of one of the oracle's legitimate outcomes.

    Returns a dict of statistics; raises AssertionError on a mismatch."""
    ref = orender.render(scene, cam, model, alpha_min=alpha_min, t_eps=t_eps,
                         background=background, pixels=pixels)
    px = ref["pixels"]
    rgb = out["rgb"].cpu().numpy()[px[:, 1], px[:, 0]].astype(np.float64)
    trans = out["trans"].cpu().numpy()[px[:, 1], px[:, 0]].astype(np.float64)
    od = out["overdraw"].cpu().numpy()[px[:, 1], px[:, 0]]
    amb = ref["ambiguous"]
    colour_ok = ~ref["amb_alpha"]
    drgb = np.abs(rgb - ref["rgb"])[colour_ok]
    dtr = np.abs(trans - ref["trans"])[colour_ok]
    od_bad = np.nonzero((od != ref["od"]) & ~amb)[0]
    bad_flagged, alternate = [], 0
    for i, outs in ref["outcomes"].items():
        hit = [j for j, o in enumerate(outs) if _matches(rgb[i], trans[i], od[i], o)]
        if not hit:
            bad_flagged.append(i)
        elif hit[0] != 0:
            alternate += 1
    stats = {"pixels": int(px.shape[0]), "ambiguous": int(amb.sum()),
             "amb_alpha": int(ref["amb_alpha"].sum()), "amb_cut": int(ref["amb_cut"].sum()),
             "alternate": alternate,
             "max_rgb_err": float(drgb.max()) if drgb.size else 0.0,
             "max_trans_err": float(dtr.max()) if dtr.size else 0.0,
             "od_mismatch": int(od_bad.size), "mean_od": float(ref["od"].mean())}
    assert stats["max_rgb_err"] <= RGB_ATOL, stats
    assert stats["max_trans_err"] <= TRANS_ATOL, stats
    assert od_bad.size == 0, (stats, px[od_bad[:5]], od[od_bad[:5]], ref["od"][od_bad[:5]])
    if bad_flagged:
        i = bad_flagged[0]
        raise AssertionError((stats, "flagged pixels matching no legitimate outcome:",
                              len(bad_flagged), px[i], rgb[i], trans[i], od[i],
                              ref["outcomes"][i][:4]))
    assert alternate <= max_alternate * max(px.shape[0], 1), stats
    return stats


def compare_keys(renderer, scene, cams, tile_w=16, tile_h=16, alpha_min=1e-3):
    """Bit-exact comparison of the sorted instance list, tile ranges and the
    per-Gaussian depth bits / tile rectangles with the float32 key recipe."""
    ref = okeys.instances(scene, cams, alpha_min, tile_w, tile_h)
    keys, ids = renderer.instances()
    assert keys.size == ref["keys"].size, (keys.size, ref["keys"].size)
    assert np.array_equal(keys, ref["keys"])
    assert np.array_equal(ids.astype(np.int64), ref["ids"])
    rng = renderer.ranges().astype(np.int64)
    empty = ref["ranges"][:, 0] == ref["ranges"][:, 1]
    assert np.array_equal(rng[~empty], ref["ranges"][~empty])
    assert np.all(rng[empty, 0] == rng[empty, 1])      # empty tiles: any empty range
    for v, g in enumerate(ref["geoms"]):
        d, r = renderer.projection(v, scene.n)
        vis = g["visible"]
        assert np.array_equal(d[vis], g["depth_bits"][vis])
        want = np.stack([g["tx0"], g["tx1"], g["ty0"], g["ty1"]], 1)
        assert np.array_equal(r[vis], want[vis])
        assert np.all(r[~vis] == -1)
    return int(keys.size)
