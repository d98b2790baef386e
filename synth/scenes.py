"""Seeded synthetic Gaussian scenes and pinhole cameras.

Every array is float32 and C-contiguous, in the layout the renderer's C ABI
takes: means [N,3], scales [N,3] (> 0), quats [N,4] as (w, x, y, z),
opacities [N] in [0, 1], sh [N, (d+1)^2, 3] real SH coefficients per colour
channel.  Cameras follow the OpenCV convention: world->camera rotation R
(rows are the camera x-right, y-down, z-forward axes in world coordinates),
translation t, so that p_cam = R @ p_world + t.

The distributions stand in for the paper's workloads (NeRF-synthetic
reconstructions of <= 200k Gaussians and refined real captures of ~3.4M
Gaussians, Sec. 5); no dataset item is reproduced.
"""
from dataclasses import dataclass, field
import math

import numpy as np

# Degree-0 real SH basis value 1/(2 sqrt(pi)): only used to turn a drawn RGB
# colour into the DC coefficient that reproduces it.
_SH_C0 = 0.28209479177387814


@dataclass
class Camera:
    R: np.ndarray          # [3,3] float32, world -> camera rotation
    t: np.ndarray          # [3]   float32
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    znear: float = 0.01

    @property
    def center(self):
        """Camera centre in world coordinates (-R^T t)."""
        return -(self.R.astype(np.float64).T @ self.t.astype(np.float64))


@dataclass
class Scene:
    means: np.ndarray
    scales: np.ndarray
    quats: np.ndarray
    opacities: np.ndarray
    sh: np.ndarray
    sh_degree: int
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self):
        return int(self.means.shape[0])

    def subset(self, idx):
        idx = np.asarray(idx)
        return Scene(self.means[idx].copy(), self.scales[idx].copy(),
                     self.quats[idx].copy(), self.opacities[idx].copy(),
                     self.sh[idx].copy(), self.sh_degree, self.name + "[subset]")


def look_at_camera(eye, target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0),
                   width=128, height=128, fov_x_deg=60.0, znear=0.01):
    """Pinhole camera at `eye` looking at `target`, horizontal FOV, square pixels,
    principal point at the image centre."""
    eye = np.asarray(eye, np.float64)
    fwd = np.asarray(target, np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    down = -np.asarray(up, np.float64)
    down = down - fwd * np.dot(down, fwd)
    down /= np.linalg.norm(down)
    right = np.cross(down, fwd)
    R = np.stack([right, down, fwd]).astype(np.float32)
    t = (-(R.astype(np.float64) @ eye)).astype(np.float32)
    fx = width / (2.0 * math.tan(math.radians(fov_x_deg) / 2.0))
    return Camera(R, t, float(np.float32(fx)), float(np.float32(fx)),
                  width / 2.0, height / 2.0, int(width), int(height), znear)


def orbit_cameras(n, radius, width, height, rng=None, elevation_deg=(0.0, 0.0),
                  azimuths=None, fov_x_deg=60.0):
    """n cameras on a sphere of `radius` around the origin, looking at it."""
    cams = []
    for j in range(n):
        az = (2 * math.pi * j / n) if azimuths is None else azimuths[j]
        lo, hi = elevation_deg
        el = math.radians(lo if rng is None or lo == hi else rng.uniform(lo, hi))
        eye = radius * np.array([math.cos(el) * math.sin(az), math.sin(el),
                                 -math.cos(el) * math.cos(az)])
        w, h = (width[j], height[j]) if np.ndim(width) else (width, height)
        cams.append(look_at_camera(eye, width=w, height=h, fov_x_deg=fov_x_deg))
    return cams


def _unit_quats(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q.astype(np.float32)


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _sh(rng, n, degree, hi_std):
    k = (degree + 1) ** 2
    sh = np.zeros((n, k, 3), np.float32)
    rgb = rng.uniform(0.0, 1.0, (n, 3))
    sh[:, 0, :] = (rgb - 0.5) / _SH_C0
    if degree > 0:
        sh[:, 1:, :] = rng.normal(0.0, hi_std, (n, k - 1, 3))
    return sh


def random_scene(seed, n, mean_lo=-1.0, mean_hi=1.0, log_scale=(-3.5, 0.4),
                 logit=(0.0, 1.0), sh_degree=0, sh_hi_std=0.05, name="uniform"):
    """Means uniform in a cube, log-normal scales, uniform rotations,
    opacity = sigmoid(normal logit)."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(mean_lo, mean_hi, (n, 3)).astype(np.float32)
    scales = np.exp(rng.normal(log_scale[0], log_scale[1], (n, 3))).astype(np.float32)
    quats = _unit_quats(rng, n)
    opac = _sigmoid(rng.normal(logit[0], logit[1], n)).astype(np.float32)
    sh = _sh(rng, n, sh_degree, sh_hi_std)
    return Scene(means, scales, quats, opac, sh, sh_degree, name)


def clustered_scene(seed, n, n_clusters, log_scale, logit, sh_degree,
                    sh_hi_std=0.05, box=5.0, eig=(0.05, 1.0), name="clustered"):
    """Means from an equal-weight mixture of anisotropic Gaussian clusters:
    centres uniform in [-box, box]^3, cluster covariance R diag(lambda) R^T with
    eigenvalues log-uniform in `eig` and a uniform random rotation."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-box, box, (n_clusters, 3))
    lam = np.exp(rng.uniform(math.log(eig[0]), math.log(eig[1]), (n_clusters, 3)))
    rots = []
    for _ in range(n_clusters):
        a = rng.standard_normal((3, 3))
        qm, r = np.linalg.qr(a)
        qm = qm * np.sign(np.diag(r))
        rots.append(qm)
    rots = np.stack(rots)
    which = rng.integers(0, n_clusters, n)
    z = rng.standard_normal((n, 3)) * np.sqrt(lam[which])
    means = (centres[which] + np.einsum("nij,nj->ni", rots[which], z)).astype(np.float32)
    scales = np.exp(rng.normal(log_scale[0], log_scale[1], (n, 3))).astype(np.float32)
    quats = _unit_quats(rng, n)
    opac = _sigmoid(rng.normal(logit[0], logit[1], n)).astype(np.float32)
    sh = _sh(rng, n, sh_degree, sh_hi_std)
    return Scene(means, scales, quats, opac, sh, sh_degree, name)


# ---------------------------------------------------------------- workloads

def tiny_scene(seed=1, n=4096):
    """4,096 Gaussians in [-1,1]^3, SH degree 0, one 128x128 camera at (0,0,-3)."""
    sc = random_scene(seed, n, log_scale=(-3.5, 0.4), logit=(0.0, 1.0),
                      sh_degree=0, name="tiny")
    cam = look_at_camera((0.0, 0.0, -3.0), width=128, height=128)
    return sc, [cam]


def scene_scale(seed=2, n=1_000_000, width=1920, height=1080, eye_dist=15.0):
    """1M Gaussians from 64 clusters, SH degree 3, one 1920x1080 camera."""
    sc = clustered_scene(seed, n, 64, log_scale=(-4.5, 0.6), logit=(0.5, 1.5),
                         sh_degree=3, name="scene")
    cam = look_at_camera((0.0, 0.0, -eye_dist), width=width, height=height)
    return sc, [cam]


def diff_scene(seed=3, n=500_000, n_views=8, width=1280, height=720):
    """500k Gaussians (uniform-cube generator), 8 cameras on a radius-6 orbit."""
    sc = random_scene(seed, n, log_scale=(-3.5, 0.4), logit=(0.0, 1.0),
                      sh_degree=0, name="diff")
    cams = orbit_cameras(n_views, 6.0, width, height)
    return sc, cams


BATCH_SIZES = [(512, 512), (960, 540), (1280, 720), (1920, 1080)]


def batched_scene(seed=4, n=3_000_000, n_views=16):
    """3M Gaussians, means from a 256-cluster mixture, per-Gaussian attributes
    of the uniform-cube generator; 16 views of uneven size on a radius-15 orbit."""
    sc = clustered_scene(seed, n, 256, log_scale=(-3.5, 0.4), logit=(0.0, 1.0),
                         sh_degree=0, name="batched")
    rng = np.random.default_rng(seed + 1000)
    sizes = [BATCH_SIZES[i] for i in rng.integers(0, 4, n_views)]
    az = rng.uniform(0, 2 * math.pi, n_views)
    cams = orbit_cameras(n_views, 15.0, [s[0] for s in sizes], [s[1] for s in sizes],
                         rng=rng, elevation_deg=(-30.0, 30.0), azimuths=az)
    return sc, cams


def serving_scenes(sizes=(200_000, 500_000, 1_000_000, 3_000_000), seed0=51):
    """Resident scenes for the serving loop (uniform-cube generator)."""
    return [random_scene(seed0 + i, n, name=f"serve{n}") for i, n in enumerate(sizes)]


WORKLOADS = {
    "tiny": tiny_scene,
    "scene": scene_scale,
    "diff": diff_scene,
    "batched": batched_scene,
}
