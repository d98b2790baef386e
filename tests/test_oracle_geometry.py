"""Pins of the oracle's SH, projection, key recipe and per-pixel renderer.

Each check compares the oracle with something other than itself: SciPy's
spherical harmonics, quadrature, hand-derived closed forms, a Monte Carlo
projection of 3D samples, the paper's printed figure data rendered through
the whole 3D pipeline, and brute force over every Gaussian.
"""
import math

import numpy as np
import pytest
from scipy.special import sph_harm_y

import synth
from oracle import keys as K
from oracle import operators as O
from oracle import project as P
from oracle import render as R
from oracle import sh as SH
from tests.golden import fixtures

SH_C0 = 0.5 / math.sqrt(math.pi)


# ------------------------------------------------------------------ SH

def _real_sh_scipy(l, m, dirs):
    th = np.arccos(np.clip(dirs[:, 2], -1, 1))
    ph = np.arctan2(dirs[:, 1], dirs[:, 0])
    if m < 0:
        return math.sqrt(2) * (-1) ** m * sph_harm_y(l, -m, th, ph).imag
    if m == 0:
        return sph_harm_y(l, 0, th, ph).real
    return math.sqrt(2) * (-1) ** m * sph_harm_y(l, m, th, ph).real


def test_sh_basis_matches_scipy():
    rng = np.random.default_rng(0)
    d = rng.standard_normal((200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    B = SH.basis(3, d)
    for l in range(4):
        for m in range(-l, l + 1):
            assert np.abs(B[:, l * l + l + m] - _real_sh_scipy(l, m, d)).max() < 1e-12


def test_sh_orthonormal_by_quadrature():
    # Gauss-Legendre in cos(theta) x uniform in phi integrates degree <= 6 exactly
    xs, ws = np.polynomial.legendre.leggauss(12)
    phis = np.arange(24) * 2 * math.pi / 24
    ct, ph = np.meshgrid(xs, phis, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    w = (ws[:, None] * np.full(phis.size, 2 * math.pi / phis.size)[None, :]).ravel()
    B = SH.basis(3, d)
    G = (B * w[:, None]).T @ B
    assert np.abs(G - np.eye(16)).max() < 1e-12


def test_sh_degree0_emission_closed_form():
    d = np.array([[0.0, 0.0, 1.0], [0.6, 0.0, 0.8]])
    c = np.zeros((2, 16, 3))
    c[:, 0, :] = [[0.4, -0.2, 3.0], [0.0, 1.0, -5.0]]
    E = SH.emission(c, 3, d)
    assert np.allclose(E, np.maximum(SH_C0 * c[:, 0, :] + 0.5, 0), atol=1e-15)


# ------------------------------------------------------------ projection

def _one(mean, scale, quat=(1, 0, 0, 0), opacity=0.8, rgb=(0.25, 0.5, 0.75)):
    sh = np.zeros((1, 1, 3), np.float32)
    sh[0, 0] = (np.asarray(rgb) - 0.5) / SH_C0
    return synth.Scene(np.array([mean], np.float32), np.array([scale], np.float32),
                       np.array([quat], np.float32), np.array([opacity], np.float32),
                       sh, 0)


def test_projection_on_axis_closed_form():
    """Axis-aligned Gaussian on the optical axis at depth z: Sigma2D =
    diag(fx^2 sx^2 / z^2, fy^2 sy^2 / z^2) + 0.3 I, centred on (cx, cy)."""
    cam = synth.look_at_camera((0, 0, -3), width=64, height=48)
    sc = _one((0, 0, 0), (0.05, 0.02, 0.3))
    pr = P.project(sc, cam)
    z = 3.0
    sx, sy = float(np.float32(0.05)), float(np.float32(0.02))   # float32 inputs
    a = (cam.fx * sx / z) ** 2 + 0.3
    c = (cam.fy * sy / z) ** 2 + 0.3
    assert np.allclose(pr["cov2d"][0], [a, 0, c], rtol=1e-12, atol=1e-12)
    assert np.allclose(pr["conic"][0], [1 / a, 0, 1 / c], rtol=1e-12)
    assert np.allclose(pr["uv"][0], [cam.cx, cam.cy], atol=1e-12)
    assert np.allclose(pr["rgb"][0], [0.25, 0.5, 0.75], atol=1e-6)
    al = P.alpha_at(pr, np.array([0]), np.array([40]), np.array([30]))
    dx, dy = 40.5 - cam.cx, 30.5 - cam.cy
    assert np.allclose(al, float(np.float32(0.8)) * math.exp(-0.5 * (dx * dx / a + dy * dy / c)), rtol=1e-12)


def test_projection_invariances():
    rng = np.random.default_rng(3)
    sc, cams = synth.tiny_scene(n=64)
    cam = cams[0]
    p1 = P.project(sc, cam)
    sc2 = synth.Scene(sc.means, sc.scales, -sc.quats, sc.opacities, sc.sh, 0)
    p2 = P.project(sc2, cam)
    assert np.allclose(p1["cov2d"], p2["cov2d"], rtol=1e-12)
    iso = synth.Scene(sc.means, np.repeat(sc.scales[:, :1], 3, 1), sc.quats,
                      sc.opacities, sc.sh, 0)
    q = rng.standard_normal((64, 4)).astype(np.float32)
    iso2 = synth.Scene(sc.means, iso.scales, q, sc.opacities, sc.sh, 0)
    assert np.allclose(P.project(iso, cam)["cov2d"], P.project(iso2, cam)["cov2d"],
                       rtol=1e-10)
    # an unnormalised quaternion (exactly scaled) gives the same footprint
    sc3 = synth.Scene(sc.means, sc.scales, sc.quats * 4.0, sc.opacities, sc.sh, 0)
    assert np.allclose(p1["cov2d"], P.project(sc3, cam)["cov2d"], rtol=1e-10)


def test_projection_matches_monte_carlo_marginal():
    """For a small, off-axis, rotated Gaussian the EWA footprint (without the
    dilation) matches the covariance of projected 3D samples to first order."""
    rng = np.random.default_rng(5)
    cam = synth.look_at_camera((0.3, -0.2, -4), width=200, height=160)
    sc = _one((0.4, 0.3, 0.2), (0.004, 0.002, 0.001), quat=(0.8, 0.3, -0.4, 0.2))
    pr = P.project(sc, cam)
    Sig = P.covariance3d(sc.scales, sc.quats)[0]
    X = rng.multivariate_normal(sc.means[0].astype(np.float64), Sig, 400000)
    pc = X @ cam.R.astype(np.float64).T + cam.t.astype(np.float64)
    uv = np.stack([cam.fx * pc[:, 0] / pc[:, 2] + cam.cx,
                   cam.fy * pc[:, 1] / pc[:, 2] + cam.cy], 1)
    C = np.cov(uv.T)
    ewa = np.array([pr["cov2d"][0, 0] - 0.3, pr["cov2d"][0, 1], pr["cov2d"][0, 2] - 0.3])
    got = np.array([C[0, 0], C[0, 1], C[1, 1]])
    scale = max(abs(ewa[0]), abs(ewa[2]))
    assert np.abs(got - ewa).max() < 0.01 * scale
    # a transposed Jacobian or rotation would break this
    assert np.allclose(pr["uv"][0], uv.mean(0), atol=0.01)


# ------------------------------------------------------------- key recipe

def test_key_recipe_depth_and_rect_against_fp64():
    sc, cams = synth.tiny_scene()
    cam = cams[0]
    g = K.geometry(sc, cam)
    pr = P.project(sc, cam)
    vis = g["visible"]
    z32 = g["depth"][vis].astype(np.float64)
    z64 = pr["z"][vis]
    assert np.all(np.abs(z32 - z64) <= 4 * np.spacing(np.float32(z64)).astype(np.float64))
    u64, a64 = pr["uv"][vis, 0], pr["cov2d"][vis, 0]
    assert np.allclose(g["u"][vis], u64, rtol=1e-6, atol=1e-4)
    assert np.allclose(g["a"][vis], a64, rtol=1e-5)


def test_key_recipe_hand_example():
    """On-axis isotropic Gaussian: rx = sqrt(2 ln(1000) ((fx s/z)^2 + 0.3))."""
    cam = synth.look_at_camera((0, 0, -2), width=128, height=128)
    sc = _one((0, 0, 0), (0.05, 0.05, 0.05))
    g = K.geometry(sc, cam, tile_w=16, tile_h=16)
    a = (cam.fx * 0.05 / 2.0) ** 2 + 0.3
    r = math.sqrt(2 * math.log(1000) * a)          # ~ 10.9 px
    x0, x1 = math.ceil(64 - r - 0.5), math.floor(64 + r - 0.5)
    assert (g["x0"][0], g["x1"][0], g["y0"][0], g["y1"][0]) == (x0, x1, x0, x1)
    assert (g["tx0"][0], g["tx1"][0]) == (x0 // 16, x1 // 16)
    assert g["depth_bits"][0] == np.float32(2.0).view(np.uint32)


def test_key_recipe_culls():
    cam = synth.look_at_camera((0, 0, -2), width=64, height=64)
    behind = _one((0, 0, -2.5), (0.05,) * 3)
    faint = _one((0, 0, 0), (0.05,) * 3, opacity=5e-4)
    off = _one((10, 0, 0), (0.01,) * 3)
    zero_q = _one((0, 0, 0), (0.05,) * 3, quat=(0, 0, 0, 0))
    for sc in (behind, faint, off, zero_q):
        g = K.geometry(sc, cam)
        assert not g["visible"][0] and g["n_tiles"][0] == 0


def test_coverage_invariant():
    """Every (pixel, Gaussian) pair whose FP64 alpha reaches alpha_min (1 + 1e-5)
    lies inside that Gaussian's float32 pixel rectangle."""
    sc, cams = synth.tiny_scene()
    cam = cams[0]
    g = K.geometry(sc, cam)
    pr = P.project(sc, cam)
    yy, xx = np.mgrid[0:cam.height, 0:cam.width]
    xx, yy = xx.ravel(), yy.ravel()
    bad = 0
    for i in range(0, sc.n, 256):
        idx = np.arange(i, min(i + 256, sc.n))
        al = P.alpha_at(pr, idx[None, :], xx[:, None], yy[:, None])
        hit = al >= 1e-3 * (1 + 1e-5)
        pz = pr["z"][idx] > cam.znear
        hit &= pz[None, :]
        pi, gi = np.nonzero(hit)
        gg = idx[gi]
        inside = g["visible"][gg] & (xx[pi] >= g["x0"][gg]) & (xx[pi] <= g["x1"][gg]) \
            & (yy[pi] >= g["y0"][gg]) & (yy[pi] <= g["y1"][gg])
        bad += int((~inside).sum())
    assert bad == 0


def test_instances_sorted_and_brute_force():
    sc, cams = synth.tiny_scene(seed=11, n=300)
    cam = cams[0]
    inst = K.instances(sc, [cam], tile_w=16, tile_h=16)
    g = inst["geoms"][0]
    tx_n = (cam.width + 15) // 16
    brute = []
    for i in range(sc.n):
        if not g["visible"][i]:
            continue
        for ty in range(g["ty0"][i], g["ty1"][i] + 1):
            for tx in range(g["tx0"][i], g["tx1"][i] + 1):
                brute.append((ty * tx_n + tx, int(g["depth_bits"][i]), i))
    brute.sort()
    keys = [(t << 32) | d for t, d, _ in brute]
    assert inst["keys"].tolist() == keys
    assert inst["ids"].tolist() == [i for _, _, i in brute]
    for t in range(inst["ranges"].shape[0]):
        s, e = inst["ranges"][t]
        assert all(b[0] == t for b in brute[s:e])


# ------------------------------------------------------ whole renderer

def test_render_matches_brute_force_tiny():
    sc, cams = synth.tiny_scene(seed=21, n=96)
    cam = synth.look_at_camera((0, 0, -3), width=40, height=24)
    for model in range(4):
        a = R.render(sc, cam, model)
        b = R.render_brute(sc, cam, model)
        assert np.allclose(a["rgb"], b["rgb"], atol=1e-13)
        assert np.allclose(a["trans"], b["trans"], atol=1e-13)
        assert np.array_equal(a["od"], b["od"])


def test_render_single_gaussian_closed_form():
    cam = synth.look_at_camera((0, 0, -3), width=32, height=32)
    sc = _one((0.02, -0.01, 0.1), (0.03, 0.05, 0.02), quat=(0.9, 0.1, 0.2, 0.3))
    pr = P.project(sc, cam)
    bg = (0.1, 0.2, 0.3)
    for model in range(4):
        r = R.render(sc, cam, model, background=bg)
        px, py = r["pixels"][:, 0], r["pixels"][:, 1]
        al = P.alpha_at(pr, np.zeros(px.size, int), px, py)
        al = np.where(al >= 1e-3, al, 0.0)
        want = al[:, None] * pr["rgb"][0][None, :] + (1 - al)[:, None] * np.array(bg)
        assert np.allclose(r["rgb"], want, atol=1e-14)
        assert np.allclose(r["trans"], 1 - al, atol=1e-14)
        assert np.array_equal(r["od"], (al > 0).astype(int))


def _concentric_scene(n_splats, sigmas, opac, rgbs, fx=512.0):
    """On-axis isotropic 3D Gaussians at depths 1, 2, ...; the 3D scale is
    chosen so the projected footprint (with the 0.3 px^2 dilation) has the
    requested standard deviation in pixels."""
    means, scales, sh = [], [], []
    for i in range(n_splats):
        z = 1.0 + 0.01 * i
        s = math.sqrt(sigmas[i] ** 2 - 0.3) * z / fx
        means.append((0.0, 0.0, z))
        scales.append((s, s, s))
        sh.append([(np.asarray(rgbs[i]) - 0.5) / SH_C0])
    sc = synth.Scene(np.array(means, np.float32), np.array(scales, np.float32),
                     np.tile(np.array([[1, 0, 0, 0]], np.float32), (n_splats, 1)),
                     np.full(n_splats, opac, np.float32), np.array(sh, np.float32), 0)
    R_ = np.eye(3, dtype=np.float32)
    cam = synth.Camera(R_, np.zeros(3, np.float32), fx, fx, 256.5, 256.5, 512, 512)
    return sc, cam


def test_render_reproduces_blending_figure_through_3d_pipeline():
    """Fig. 'Blending comparison' (a) rendered as a 3D scene by the full
    oracle renderer (projection, culling, ordering, composite): the centre
    row's colour channels are the red, green and blue splat contributions."""
    sc, cam = _concentric_scene(3, (40.0, 60.0, 80.0), 1.0,
                                [(1, 0, 0), (0, 1, 0), (0, 0, 1)])
    rows = fixtures.blending_concentric()
    xs = rows["linear"][:, 0].astype(int)
    pix = np.stack([xs, np.full(xs.size, 256)], 1)
    for model, name in ((0, "exponential"), (1, "linear"), (2, "quadratic_c-0.5"),
                        (3, "quadratic_c0.5")):
        # the figure's exponential has no t_eps termination (blue shows 1.1e-5
        # behind T = 1.1e-5 at x = 252), so render it with t_eps = 0
        r = R.render(sc, cam, model, pixels=pix, t_eps=0.0)
        want = rows[name]
        # float32 inputs: the 3D scale is rounded, so allow a few 1e-7 more
        assert np.abs(r["rgb"] - want[:, 1:4]).max() < 2e-6, name


def test_render_reproduces_transmittance_figure_dots():
    """Fig. 'Transmittance comparison' dots through the full renderer: the
    centre pixel of 5j concentric splats of opacity 0.02 has T_bar = dot j."""
    dots = fixtures.transmittance_dots()
    for model, name in ((0, "exponential"), (1, "linear"), (2, "quadratic_c-0.5"),
                        (3, "quadratic_c0.5")):
        for tau, want in dots[name][1::4]:
            n = int(round(tau / 0.02))
            sc, cam = _concentric_scene(n, [3.0] * n, 0.02, [(0.5, 0.5, 0.5)] * n)
            r = R.render(sc, cam, model, t_eps=0.0, pixels=np.array([[256, 256]]))
            assert abs(r["trans"][0] - want) < 2e-7, (name, tau)


def test_render_weights_sum_identity_random_scene():
    sc, cams = synth.tiny_scene(seed=31, n=512)
    cam = cams[0]
    white = synth.Scene(sc.means, sc.scales, sc.quats, sc.opacities,
                        np.full_like(sc.sh, 0.5 / SH_C0), 0)
    for model in range(4):
        r = R.render(white, cam, model, background=(0.0, 0.0, 0.0))
        # E = 1 everywhere: L = sum p = 1 - T
        assert np.allclose(r["rgb"][:, 0], 1 - r["trans"], atol=1e-12)
        if model > 0:
            sat = r["trans"] == 0.0
            assert sat.any()
