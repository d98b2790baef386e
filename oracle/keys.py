"""Tile-binning key specification, replayed in IEEE float32 with NumPy.

Parity: pinned against FP64 in the tests (depth within rounding of the FP64
depth, the tile rectangle contains every pixel whose FP64 alpha reaches
alpha_min, a hand-computed on-axis example, brute force on tiny scenes).

The paper composites splats front to back ("sorted front-to-bottom", Sec. 3);
a tile rasterizer bins them into screen tiles and sorts each tile's list by
depth.  For the GPU's keys to be comparable bit for bit, which Gaussian lands
in which tile and at what depth key is fixed by the float32 recipe below: every
operation is one IEEE float32 operation rounded to nearest even, evaluated in
the order written, with no fused multiply-add.  Readings (listed in the
design notes): view-space z of the mean is the depth (one order per tile,
not the per-ray peak depth of the paper's ray tracer); ties on equal depth
bits go to the lower Gaussian index.

Recipe for one Gaussian (mean m, scales s, quaternion q = (w, x, y, z),
opacity aleph) and one camera (R row-major, t, fx, fy, cx, cy, znear, W, H),
with kappa2 = float32(2 ln(1 / alpha_min)):
  pz = ((R6*m0 + R7*m1) + R8*m2) + t2   (px, py likewise with rows 0 and 1)
  cull unless pz > znear and aleph >= alpha_min
  n2 = ((qw*qw + qx*qx) + qy*qy) + qz*qz;  cull unless n2 > 0
  nr = sqrt(n2);  w, x, y, z = qw/nr, qx/nr, qy/nr, qz/nr
  Rq = [[1 - 2*(y*y + z*z), 2*(x*y - w*z),     2*(x*z + w*y)],
        [2*(x*y + w*z),     1 - 2*(x*x + z*z), 2*(y*z - w*x)],
        [2*(x*z - w*y),     2*(y*z + w*x),     1 - 2*(x*x + y*y)]]
  M_ij = Rq_ij * s_j;   G_ij = (R_i0*M_0j + R_i1*M_1j) + R_i2*M_2j
  fxx = fx*px;  fyy = fy*py;  zz = pz*pz
  j00 = fx/pz;  j02 = -(fxx/zz);  j11 = fy/pz;  j12 = -(fyy/zz)
  A_0j = j00*G_0j + j02*G_2j;  A_1j = j11*G_1j + j12*G_2j
  a = ((A00*A00 + A01*A01) + A02*A02) + 0.3;  c likewise with row 1
  u = fxx/pz + cx;  v = fyy/pz + cy
  rx = sqrt(kappa2*a);  ry = sqrt(kappa2*c);  cull unless u, v, rx, ry finite
  x0 = max(ceil((u - rx) - 0.5), 0);  x1 = min(floor((u + rx) - 0.5), W - 1)
  y0, y1 likewise with v, ry, H;  cull unless x0 <= x1 and y0 <= y1
  tiles tx0..tx1 = x0//TW..x1//TW,  ty0..ty1 = y0//TH..y1//TH
  depth key = the float32 bit pattern of pz (positive, so monotone)
The pixel range is exactly the pixels whose centre (x + 1/2) lies within
[u - rx, u + rx]: the bounding box of the ellipse d^T Sigma2D^{-1} d <= kappa2,
outside which alpha = aleph exp(-q/2) < alpha_min since aleph <= 1.

Instances are emitted per Gaussian in index order, rows of tiles top to
bottom, left to right within a row; instance key = (global_tile << 32) |
depth_bits, global_tile = view's first tile + ty * tiles_x + tx; the sorted
list is ascending in key, then Gaussian index.
"""
import math

import numpy as np

F = np.float32


def kappa2(alpha_min):
    """float32(2 ln(1/alpha_min)): squared Mahalanobis radius of the footprint."""
    return F(2.0 * math.log(1.0 / float(alpha_min)))


def geometry(scene, cam, alpha_min=1e-3, tile_w=16, tile_h=16):
    """Float32 replay of the recipe for every Gaussian of `scene` in `cam`.

    Returns a dict of [N] arrays: visible (bool), depth (float32 pz),
    depth_bits (uint32), u, v, rx, ry (float32), x0, x1, y0, y1 (int64 pixel
    bounds, valid where visible), tx0, tx1, ty0, ty1, n_tiles (int64, 0 if
    culled).
    """
    m = np.asarray(scene.means, F)
    s = np.asarray(scene.scales, F)
    q = np.asarray(scene.quats, F)
    op = np.asarray(scene.opacities, F)
    R = np.asarray(cam.R, F).reshape(9)
    t = np.asarray(cam.t, F)
    fx, fy, cx, cy = F(cam.fx), F(cam.fy), F(cam.cx), F(cam.cy)
    znear = F(cam.znear)
    k2 = kappa2(alpha_min)
    one, two, half, dil = F(1.0), F(2.0), F(0.5), F(0.3)
    m0, m1, m2 = m[:, 0], m[:, 1], m[:, 2]

    with np.errstate(all="ignore"):
        px = ((R[0] * m0 + R[1] * m1) + R[2] * m2) + t[0]
        py = ((R[3] * m0 + R[4] * m1) + R[5] * m2) + t[1]
        pz = ((R[6] * m0 + R[7] * m1) + R[8] * m2) + t[2]
        n2 = ((q[:, 0] * q[:, 0] + q[:, 1] * q[:, 1]) + q[:, 2] * q[:, 2]) + q[:, 3] * q[:, 3]
        nr = np.sqrt(n2)
        w, x, y, z = q[:, 0] / nr, q[:, 1] / nr, q[:, 2] / nr, q[:, 3] / nr
        Rq = [[one - two * (y * y + z * z), two * (x * y - w * z), two * (x * z + w * y)],
              [two * (x * y + w * z), one - two * (x * x + z * z), two * (y * z - w * x)],
              [two * (x * z - w * y), two * (y * z + w * x), one - two * (x * x + y * y)]]
        M = [[Rq[i][j] * s[:, j] for j in range(3)] for i in range(3)]
        G = [[(R[3 * i] * M[0][j] + R[3 * i + 1] * M[1][j]) + R[3 * i + 2] * M[2][j]
              for j in range(3)] for i in range(3)]
        fxx, fyy, zz = fx * px, fy * py, pz * pz
        j00, j02 = fx / pz, -(fxx / zz)
        j11, j12 = fy / pz, -(fyy / zz)
        A0 = [j00 * G[0][j] + j02 * G[2][j] for j in range(3)]
        A1 = [j11 * G[1][j] + j12 * G[2][j] for j in range(3)]
        a = ((A0[0] * A0[0] + A0[1] * A0[1]) + A0[2] * A0[2]) + dil
        c = ((A1[0] * A1[0] + A1[1] * A1[1]) + A1[2] * A1[2]) + dil
        u = fxx / pz + cx
        v = fyy / pz + cy
        rx = np.sqrt(k2 * a)
        ry = np.sqrt(k2 * c)
        x0 = np.maximum(np.ceil((u - rx) - half), F(0.0))
        x1 = np.minimum(np.floor((u + rx) - half), F(cam.width - 1))
        y0 = np.maximum(np.ceil((v - ry) - half), F(0.0))
        y1 = np.minimum(np.floor((v + ry) - half), F(cam.height - 1))
    for arr in (px, py, pz, u, v, rx, ry, x0, x1):
        assert arr.dtype == F
    finite = np.isfinite(u) & np.isfinite(v) & np.isfinite(rx) & np.isfinite(ry)
    visible = (pz > znear) & (op >= F(alpha_min)) & (n2 > 0) & finite
    visible &= (x0 <= x1) & (y0 <= y1)
    n = m.shape[0]
    out = {"visible": visible, "depth": pz, "depth_bits": pz.view(np.uint32).copy(),
           "u": u, "v": v, "rx": rx, "ry": ry, "a": a, "c": c}
    for name, arr in (("x0", x0), ("x1", x1), ("y0", y0), ("y1", y1)):
        iv = np.zeros(n, np.int64)
        iv[visible] = arr[visible].astype(np.int64)
        out[name] = iv
    out["tx0"], out["tx1"] = out["x0"] // tile_w, out["x1"] // tile_w
    out["ty0"], out["ty1"] = out["y0"] // tile_h, out["y1"] // tile_h
    nt = (out["tx1"] - out["tx0"] + 1) * (out["ty1"] - out["ty0"] + 1)
    out["n_tiles"] = np.where(visible, nt, 0)
    return out


def tile_grid(cam, tile_w, tile_h):
    return (cam.width + tile_w - 1) // tile_w, (cam.height + tile_h - 1) // tile_h


def instances(scene, cams, alpha_min=1e-3, tile_w=16, tile_h=16):
    """Sorted (key, Gaussian index) instance list over one or more views.

    Returns dict: keys uint64 [M] ascending, ids int64 [M], ranges int64
    [total_tiles, 2] (start, end) into the sorted list, tile_offset [V+1] the
    first global tile of each view, geoms (per-view geometry dicts).
    """
    keys_all, ids_all, geoms, tile_offset = [], [], [], [0]
    for cam in cams:
        g = geometry(scene, cam, alpha_min, tile_w, tile_h)
        geoms.append(g)
        tx_n, ty_n = tile_grid(cam, tile_w, tile_h)
        base = tile_offset[-1]
        tile_offset.append(base + tx_n * ty_n)
        ids = np.repeat(np.arange(scene.n), g["n_tiles"])
        first = np.cumsum(g["n_tiles"]) - g["n_tiles"]
        local = np.arange(ids.size) - first[ids]
        wdt = (g["tx1"] - g["tx0"] + 1)[ids]
        tx = g["tx0"][ids] + local % wdt
        ty = g["ty0"][ids] + local // wdt
        tile = base + ty * tx_n + tx
        keys_all.append((tile.astype(np.uint64) << np.uint64(32))
                        | g["depth_bits"][ids].astype(np.uint64))
        ids_all.append(ids)
    keys = np.concatenate(keys_all) if keys_all else np.zeros(0, np.uint64)
    ids = np.concatenate(ids_all) if ids_all else np.zeros(0, np.int64)
    order = np.lexsort((ids, keys))
    keys, ids = keys[order], ids[order]
    total = tile_offset[-1]
    tiles = (keys >> np.uint64(32)).astype(np.int64)
    starts = np.searchsorted(tiles, np.arange(total), side="left")
    ends = np.searchsorted(tiles, np.arange(total), side="right")
    return {"keys": keys, "ids": ids, "ranges": np.stack([starts, ends], 1),
            "tile_offset": np.array(tile_offset), "geoms": geoms}
