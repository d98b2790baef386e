"""Per-Gaussian camera projection in FP64: EWA footprint, conic and emission.

Parity: pinned by closed forms in the tests (an axis-aligned Gaussian on the
optical axis, rotation/sign invariances, brute-force comparison of the
projected footprint against the exact 3D->2D marginal for small scales).

The paper defines each primitive by centre, covariance, opacity aleph and
directional emission, and its per-pixel opacity alpha = aleph * K(y) with a
Gaussian kernel K (Sec. 3).  Its ray tracer evaluates K along rays; the
rasterizing path replaces that with the standard splatting footprint, which
these readings fix (each listed in the design notes):
  * pinhole camera, OpenCV axes (x right, y down, z forward), world->camera
    p = R mu + t, pixel (x, y) sampled at its centre (x + 1/2, y + 1/2);
  * covariance Sigma = (R_q S)(R_q S)^T from the normalised quaternion
    (w, x, y, z) and the per-axis scales;
  * EWA affine projection: Sigma2D = J R Sigma R^T J^T + 0.3 I with the
    Jacobian J of the perspective map at the mean (no clamping), conic =
    Sigma2D^{-1}; K(d) = exp(-1/2 d^T conic d) for the pixel offset d;
  * emission from real SH at the direction camera centre -> mean (module sh).
"""
import numpy as np

from . import sh as _sh

DILATION = 0.3      # px^2 added to the 2D covariance's diagonal


def quat_to_rotmat(q):
    """[N,4] (w,x,y,z) -> [N,3,3] rotation matrices, after normalising q."""
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.empty((q.shape[0], 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def covariance3d(scales, quats):
    """Sigma = (R_q diag(s)) (R_q diag(s))^T, [N,3,3]."""
    M = quat_to_rotmat(quats) * np.asarray(scales, np.float64)[:, None, :]
    return M @ np.transpose(M, (0, 2, 1))


def project(scene, cam):
    """Project every Gaussian of `scene` with `cam` in FP64.

    Returns a dict of [N] / [N,k] float64 arrays:
      p_cam [N,3]  camera-space mean;   z = p_cam[:,2]
      uv    [N,2]  image-plane position of the mean in pixels
      cov2d [N,3]  (a, b, c) of Sigma2D = [[a, b], [b, c]] incl. dilation
      conic [N,3]  (A, B, C) of Sigma2D^{-1}
      rgb   [N,3]  emission E
      opacity [N]  aleph
    Culling is not applied here (see keys.visible for the cull rule).
    """
    R = np.asarray(cam.R, np.float64)
    t = np.asarray(cam.t, np.float64)
    mu = np.asarray(scene.means, np.float64)
    p = mu @ R.T + t
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    fx, fy = float(cam.fx), float(cam.fy)
    with np.errstate(divide="ignore", invalid="ignore"):
        u = fx * x / z + cam.cx
        v = fy * y / z + cam.cy
        J = np.zeros((mu.shape[0], 2, 3))
        J[:, 0, 0] = fx / z
        J[:, 0, 2] = -fx * x / (z * z)
        J[:, 1, 1] = fy / z
        J[:, 1, 2] = -fy * y / (z * z)
    Sigma = covariance3d(scene.scales, scene.quats)
    Sc = R @ Sigma @ R.T                                   # camera-space covariance
    S2 = J @ Sc @ np.transpose(J, (0, 2, 1))
    a = S2[:, 0, 0] + DILATION
    b = S2[:, 0, 1]
    c = S2[:, 1, 1] + DILATION
    det = a * c - b * b
    with np.errstate(divide="ignore", invalid="ignore"):
        conic = np.stack([c / det, -b / det, a / det], axis=1)
    d = mu - cam.center
    with np.errstate(divide="ignore", invalid="ignore"):
        d = d / np.linalg.norm(d, axis=1, keepdims=True)
    rgb = _sh.emission(scene.sh, scene.sh_degree, d)
    return {"p_cam": p, "z": z, "uv": np.stack([u, v], 1),
            "cov2d": np.stack([a, b, c], 1), "conic": conic, "rgb": rgb,
            "opacity": np.asarray(scene.opacities, np.float64)}


def alpha_at(proj, idx, px, py):
    """alpha = aleph * exp(-1/2 d^T conic d) of Gaussians `idx` at the pixel
    centres (px + 1/2, py + 1/2).  idx, px, py broadcast together."""
    dx = (np.asarray(px, np.float64) + 0.5) - proj["uv"][idx, 0]
    dy = (np.asarray(py, np.float64) + 0.5) - proj["uv"][idx, 1]
    A, B, C = proj["conic"][idx, 0], proj["conic"][idx, 1], proj["conic"][idx, 2]
    q = A * dx * dx + 2.0 * B * dx * dy + C * dy * dy
    return proj["opacity"][idx] * np.exp(-0.5 * q)
