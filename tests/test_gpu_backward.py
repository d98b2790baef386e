"""GPU path-replay backward against FP64 finite differences of the oracle.

The loss is a random weighting of every output pixel (colour and final
transmittance) over two views; its gradient with respect to every Gaussian
parameter comes from the library's backward (through the C ABI) and from
central differences of the oracle render with each pixel's discrete
decisions frozen at the base point (tests/fd.py).  Checked per element for a
handful of Gaussians (means, scales, quaternion, opacity, two SH
coefficients) and along random directions over all Gaussians for each
parameter block.

Tolerance: |g_gpu - g_fd| <= 2e-3 |g_fd| + 2e-4 * (largest |g_fd| of that
block) per element, and 2e-3 of sum |g_gpu . d| along a direction d.  The
GPU accumulates float32 per-pixel terms whose relative rounding is ~1e-6;
the FD step (1e-6) leaves truncation and FP64 round-off below 1e-7.
"""
import numpy as np
import pytest

import synth
from oracle import operators as O
from tests import fd

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

H_STEP = 1e-6


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2603_02887_amd import nxs
    r = nxs.Renderer(0)
    yield r
    r.close()


def _scene():
    sc = synth.random_scene(21, 60, log_scale=(-1.6, 0.3), logit=(1.5, 1.0), sh_degree=1)
    cams = [synth.look_at_camera((0, 0, -3.2), width=40, height=32),
            synth.look_at_camera((1.6, 0.6, -2.6), width=36, height=28)]
    return sc, cams


def _gpu_grads(R, sc, cams, F, model, **kw):
    from paper_2603_02887_amd import nxs
    g = nxs.scene_to_device(sc)
    R.render(g, cams, model=model, keep_state=True, **kw)
    w = [F.weights(v) for v in range(len(cams))]
    d_rgb = [torch.from_numpy(a).cuda() for a, _ in w]
    d_tr = [torch.from_numpy(b).cuda() for _, b in w]
    out = R.backward(g, d_rgb, d_tr)
    torch.cuda.synchronize()
    return {k: v.double().cpu().numpy() for k, v in out.items()}


CASES = [  # (library model, parameter, oracle operator, t_eps for both sides)
    (0, 0.0, O.EXPONENTIAL, -1.0),
    (0, 0.0, O.EXPONENTIAL, 0.05),          # frequent early termination
    (1, 0.0, O.LINEAR, None),
    (2, 0.0, O.SUBLINEAR, None),
    (3, 0.0, O.SUPERLINEAR, None),
    (4, 0.8, O.Op("quadratic", 0.8), None),
    (4, -0.3, O.Op("quadratic", -0.3), None),
]


@pytest.mark.parametrize("model,param,op,t_eps", CASES)
def test_gradients_match_finite_differences(R, model, param, op, t_eps):
    sc, cams = _scene()
    ot = None if t_eps is None else max(t_eps, 0.0)
    F = fd.FrozenLoss(sc, cams, op, t_eps=ot, background=(0.3, 0.1, 0.2), seed=model)
    kw = {"param": param, "background": (0.3, 0.1, 0.2)}
    if t_eps is not None:
        kw["t_eps"] = t_eps
    G = _gpu_grads(R, sc, cams, F, model, **kw)
    P = fd.params_of(sc)
    # Gaussians in the most pixels, plus a few drawn at random among the visible
    touched = np.zeros(sc.n, np.int64)
    for d in F.views:
        touched += np.bincount(d["pair_id"], minlength=sc.n)
    rng = np.random.default_rng(model + 17)
    pick = list(np.argsort(-touched)[:3]) + list(rng.choice(np.nonzero(touched)[0], 2, False))
    checks = [("means", (k,)) for k in range(3)] + [("scales", (k,)) for k in range(3)] + \
             [("quats", (k,)) for k in range(4)] + [("opacities", ())] + \
             [("sh", (0, 0)), ("sh", (3, 2))]
    worst = 0.0
    for i in pick:
        for field, sub in checks:
            idx = (int(i),) + sub
            h = H_STEP * (abs(P[field][idx]) if field == "scales" else 1.0)
            want = F.grad_element(P, field, idx, h)
            got = G[field][idx]
            scale = np.abs(G[field]).max()
            err = abs(got - want)
            worst = max(worst, err / (2e-3 * abs(want) + 2e-4 * scale + 1e-9))
            assert err <= 2e-3 * abs(want) + 2e-4 * scale + 1e-9, (field, idx, got, want)
    # directions over all Gaussians, one parameter block at a time
    for field in fd.FIELDS:
        d = rng.normal(size=P[field].shape)
        if field == "scales":
            d *= P[field]
        want = F.grad_direction(P, {field: d}, H_STEP)
        got = float(np.sum(G[field] * d))
        tol = 2e-3 * float(np.sum(np.abs(G[field] * d))) + 1e-7
        assert abs(got - want) <= tol, (field, got, want)
    print("model", model, param, "worst/tol", round(worst, 3),
          "ambiguous", [v["n_ambiguous"] for v in F.views])


def test_autograd_function_matches_direct_backward(R):
    from paper_2603_02887_amd import nxs
    sc, cams = _scene()
    g = nxs.scene_to_device(sc)
    leaves = {k: g[k].clone().requires_grad_(True)
              for k in ("means", "scales", "quats", "opacities", "sh")}
    rgbs, trs = nxs.render(R, cams, leaves["means"], leaves["scales"], leaves["quats"],
                           leaves["opacities"], leaves["sh"], model=3)
    gen = torch.Generator(device="cpu").manual_seed(5)
    w = [torch.randn(r.shape, generator=gen).cuda() for r in rgbs]
    wt = [torch.randn(t.shape, generator=gen).cuda() for t in trs]
    loss = sum((r * a).sum() for r, a in zip(rgbs, w)) + sum((t * b).sum() for t, b in zip(trs, wt))
    loss.backward()
    R.render(g, cams, model=3, keep_state=True)
    direct = R.backward(g, w, wt)
    torch.cuda.synchronize()
    # per-Gaussian sums are accumulated with float atomics in whatever order
    # the waves finish, so two runs agree to float32 rounding, not bitwise
    for k, leaf in leaves.items():
        scale = float(direct[k].abs().max())
        assert torch.allclose(leaf.grad, direct[k], rtol=1e-4, atol=1e-5 * scale), k


@pytest.mark.parametrize("model", [0, 2])
def test_backward_same_under_every_schedule(R, model):
    """The backward walks the tiles in the forward's order when the forward's
    schedule made one (queue, persistent) and in plain tile order otherwise;
    the gradients agree to float32 rounding of sums taken in another order
    (float atomics: on this scene two runs of one schedule already differ by
    up to 5e-5, and two schedules by up to 1.1e-4, of the largest gradient)."""
    from paper_2603_02887_amd import nxs
    sc = synth.scenes.clustered_scene(14, 20_000, 8, log_scale=(-3.5, 0.4), logit=(0.0, 1.0),
                                      sh_degree=1)
    rng = np.random.default_rng(3)
    sizes = [(203, 97), (64, 64), (131, 180)]
    cams = synth.orbit_cameras(len(sizes), 7.0, [w for w, _ in sizes], [h for _, h in sizes],
                               rng=rng, elevation_deg=(-30.0, 30.0),
                               azimuths=rng.uniform(0, 2 * np.pi, len(sizes)))
    g = nxs.scene_to_device(sc)
    gen = torch.Generator(device="cpu").manual_seed(9)
    w = [torch.randn((c.height, c.width, 3), generator=gen).cuda() for c in cams]
    grads = {}
    for sched in ("tiles", "blocks", "queue", "persistent"):
        R.render(g, cams, model=model, keep_state=True, schedule=sched)
        grads[sched] = {k: v.clone() for k, v in R.backward(g, w).items()}
        torch.cuda.synchronize()
    ref = grads["queue"]
    for sched, gr in grads.items():
        for k, v in gr.items():
            scale = float(ref[k].abs().max())
            assert scale > 0, k
            assert torch.allclose(v, ref[k], rtol=1e-4, atol=5e-4 * scale), (sched, k)


@pytest.mark.parametrize("model,param", [(0, 0.0), (1, 0.0), (2, 0.0), (3, 0.0), (4, 0.8)])
def test_slot_adjoints_match_the_appendix_recursions(R, model, param):
    """The backward's per-slot sums dLoss/d(aleph, u, v, A, B, C, r, g, b)
    (nxs_inspect_slot_grads) against the FP64 oracle's: per pixel the
    appendix recursions for dLoss/dalpha_i and dLoss/dE_i (oracle.adjoint)
    chained through alpha_i and summed per Gaussian (tests/adjoint_sums.py).
    Random upstream gradients on colour and transmittance, zero at the
    pixels the oracle flags; per element |got - want| <= 1e-3 |want| +
    2e-4 max|want| of the field."""
    from paper_2603_02887_amd import nxs
    from tests import adjoint_sums
    sc, cams = _scene()
    op = O.MODELS[model] if model < 4 else O.Op("quadratic", param)
    rng = np.random.default_rng(50 + model)
    g = nxs.scene_to_device(sc)
    R.render(g, cams, model=model, param=param, keep_state=True)
    d_rgb, d_tr, want = [], [], []
    for cam in cams:
        amb = adjoint_sums.ambiguous(sc, cam, op)
        w_rgb = rng.normal(size=(cam.height, cam.width, 3)).astype(np.float32)
        w_T = rng.normal(size=(cam.height, cam.width)).astype(np.float32)
        w_rgb[amb] = 0.0
        w_T[amb] = 0.0
        d_rgb.append(torch.from_numpy(w_rgb).cuda())
        d_tr.append(torch.from_numpy(w_T).cuda())
        want.append(adjoint_sums.slot_sums(sc, cam, op, w_rgb.astype(np.float64),
                                           w_T.astype(np.float64)))
    R.backward(g, d_rgb, d_tr)
    got = R.slot_grads(sc.n, len(cams)).astype(np.float64)
    want = np.stack(want)
    worst = 0.0
    for f in range(9):
        scale = np.abs(want[..., f]).max()
        assert scale > 0, f
        tol = 1e-3 * np.abs(want[..., f]) + 2e-4 * scale
        err = np.abs(got[..., f] - want[..., f])
        worst = max(worst, float((err / tol).max()))
        bad = np.argwhere(err > tol)
        assert bad.size == 0, (f, bad[:4], got[..., f][tuple(bad[:4].T)],
                               want[..., f][tuple(bad[:4].T)])
    print("model", model, param, "worst/tol", worst)


def test_autograd_survives_other_forwards(R):
    """Each differentiable render keeps its own forward state: forwards of
    other scenes and models on the same context between a render and its
    backward change nothing."""
    from paper_2603_02887_amd import nxs
    sc, cams = _scene()
    g = nxs.scene_to_device(sc)
    other = nxs.scene_to_device(synth.random_scene(9, 300, sh_degree=1))

    def grad(interleave):
        op = g["opacities"].clone().requires_grad_(True)
        rgbs, trs = nxs.render(R, cams, g["means"], g["scales"], g["quats"], op, g["sh"],
                               model=1)
        if interleave:
            R.render(other, cams, model=0)
            R.render(other, cams, model=3, keep_state=True)
        (sum(x.sum() for x in rgbs) + 0.5 * sum(t.sum() for t in trs)).backward()
        return op.grad

    a, b = grad(False), grad(True)
    torch.cuda.synchronize()
    scale = float(a.abs().max())
    assert scale > 0
    assert torch.allclose(a, b, rtol=1e-5, atol=1e-5 * scale)


def test_backward_errors(R):
    from paper_2603_02887_amd import nxs
    sc, cams = _scene()
    g = nxs.scene_to_device(sc)
    d = [torch.zeros(c.height, c.width, 3, device="cuda") for c in cams]
    R.last_state = None
    R.render(g, cams, model=0)               # no keep_state
    with pytest.raises(ValueError):
        R.backward(g, d)
    # the C ABI: a null or released state
    L = nxs.lib()
    assert L.nxs_render_backward(R._ctx, None, None, None, None, None) == -1
    R.render(g, cams, model=0, keep_state=True)
    st = R.last_state
    st.release()
    with pytest.raises(RuntimeError):
        R.backward(g, d, state=st)
    # no backward for models 5..7: their forward refuses to keep state
    for model, param in ((5, 0.5), (6, 0.5), (7, 2.0)):
        with pytest.raises(nxs.NxsError) as e:
            R.render(g, cams, model=model, param=param, keep_state=True)
        assert e.value.status == -5


def test_backward_culled_and_empty(R):
    from paper_2603_02887_amd import nxs
    cam = synth.look_at_camera((0, 0, -3), width=24, height=16)
    sc = synth.random_scene(2, 20, sh_degree=1)
    sc.means[:, 2] = -10.0                   # all behind the camera
    g = nxs.scene_to_device(sc)
    R.render(g, [cam], model=1, keep_state=True)
    out = R.backward(g, [torch.ones(16, 24, 3, device="cuda")],
                     [torch.ones(16, 24, device="cuda")])
    torch.cuda.synchronize()
    for k, v in out.items():
        assert torch.count_nonzero(v) == 0, k


# ------------------------------------------------ the differentiation workload

def _diff_workload():
    sc, cams = synth.diff_scene()
    rng = np.random.default_rng(33)
    logit = np.log(sc.opacities / (1 - sc.opacities)) + rng.normal(0, 0.1, sc.n)
    tgt = synth.Scene(sc.means + rng.normal(0, 0.01, sc.means.shape).astype(np.float32),
                      sc.scales, sc.quats, (1 / (1 + np.exp(-logit))).astype(np.float32),
                      sc.sh, sc.sh_degree)
    return sc, tgt, cams


@pytest.mark.timeout(600)
@pytest.mark.parametrize("model,op", [(0, O.EXPONENTIAL), (1, O.LINEAR), (2, O.SUBLINEAR),
                                      (3, O.SUPERLINEAR)])
def test_gradients_at_workload_size(R, model, op):
    """500,000 Gaussians, 8 views at 1280x720, per-pixel L1 loss against a
    render of the jittered scene: gradients of 64 random parameters (4 per
    Gaussian, over 16 visible Gaussians drawn among those with footprints under
    4 px in every view) against FP64 central differences (tests/fd_local.py)."""
    from oracle import project as P
    from paper_2603_02887_amd import nxs
    from tests import fd_local
    sc, tgt, cams = _diff_workload()
    g, gt = nxs.scene_to_device(sc), nxs.scene_to_device(tgt)
    target = R.render(gt, cams, model=model, overdraw=False)
    out = R.render(g, cams, model=model, overdraw=False)
    torch.cuda.synchronize()
    pix = sum(c.width * c.height for c in cams)
    w = [(torch.sign(o["rgb"] - t["rgb"]) / (3.0 * pix)).double().cpu().numpy()
         for o, t in zip(out, target)]
    # candidates: in some view, footprint under 4 px in all views
    smax, seen = np.zeros(sc.n), np.zeros(sc.n, bool)
    for c in cams:
        pr = P.project(sc, c)
        s_ = np.sqrt(np.maximum(pr["cov2d"][:, 0], pr["cov2d"][:, 2]))
        inimg = (pr["z"] > 0.1) & (pr["uv"][:, 0] > -20) & (pr["uv"][:, 0] < c.width + 20) & \
                (pr["uv"][:, 1] > -20) & (pr["uv"][:, 1] < c.height + 20)
        smax = np.where(inimg, np.maximum(smax, s_), smax)
        seen |= inimg
    # ... and visible: a nonzero opacity gradient (most Gaussians are hidden)
    R.render(g, cams, model=model, overdraw=False, keep_state=True)
    G0 = R.backward(g, [torch.from_numpy(a).float().cuda() for a in w])
    torch.cuda.synchronize()
    live = G0["opacities"].abs().cpu().numpy() > 0
    rng = np.random.default_rng(77 + model)
    focus = rng.choice(np.nonzero(seen & (smax < 4.0) & live)[0], 16, replace=False)
    params = fd.params_of(sc)
    fields = [("means", (0,)), ("means", (1,)), ("means", (2,)), ("scales", (0,)),
              ("scales", (2,)), ("quats", (1,)), ("quats", (3,)), ("opacities", ()),
              ("sh", (0, 0)), ("sh", (0, 2))]
    items = []
    for i in focus:
        for f in rng.choice(len(fields), 4, replace=False):
            field, sub = fields[f]
            idx = (int(i),) + sub
            h = H_STEP * (abs(params[field][idx]) if field == "scales" else 1.0)
            items.append((field, idx, h))
    with fd_local.LocalLoss(sc, cams, op, focus) as L:
        L.mask_weights(w)
        R.render(g, cams, model=model, overdraw=False, keep_state=True)
        G = R.backward(g, [torch.from_numpy(a).float().cuda() for a in w])
        torch.cuda.synchronize()
        G = {k: v.double().cpu().numpy() for k, v in G.items()}
        want = np.array(L.grad_elements(w, items))
    got = np.array([G[field][idx] for field, idx, _ in items])
    scale = np.abs(want).max()
    tol = 2e-3 * np.abs(want) + 2e-4 * scale
    bad = np.nonzero(np.abs(got - want) > tol)[0]
    print("params", len(got), "worst/tol", float(np.max(np.abs(got - want) / tol)),
          "nonzero", int(np.count_nonzero(want)))
    assert bad.size == 0, (bad, got[bad], want[bad])
    assert np.count_nonzero(want) >= len(want) // 2     # the check is not vacuous
