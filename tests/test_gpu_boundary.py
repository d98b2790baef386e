"""The C-ABI boundary on the GPU: forward states, deferred (non-waiting)
forwards with the device-side overflow check and its retry, and the two
sources of workspace memory (the caller's allocator, here PyTorch's caching
allocator, and the library's stream-ordered pool).

Every comparison here is bitwise: these are the same kernels on the same
inputs, and only the host's bookkeeping differs.
"""
import numpy as np
import pytest

import synth
from tests import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def nxs():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2603_02887_amd import nxs as m
    return m


def _same(a, b):
    for k in ("rgb", "trans", "overdraw"):
        if a.get(k) is not None:
            assert torch.equal(a[k], b[k]), k


def _depth_range_scene(near, far, n=3000, seed=8):
    """Gaussians whose camera-space depths span [near, far] (camera at z = -3)."""
    rng = np.random.default_rng(seed)
    sc = synth.random_scene(seed, n, sh_degree=0, log_scale=(-3.0, 0.3))
    z = rng.uniform(near, far, sc.n)
    sc.means[:, 0] = rng.uniform(-0.45, 0.45, sc.n) * z
    sc.means[:, 1] = rng.uniform(-0.45, 0.45, sc.n) * z
    sc.means[:, 2] = z - 3.0
    return sc


def test_deferred_overflow_is_reported_and_retried(nxs):
    """A context sized by a small render defers a large one: the device finds
    that the render needs more instances than the context holds, does no
    work after the emission and raises the flag; status() reports
    NXS_ECAPACITY and grows the context; the same deferred render then
    equals the render that waits, bitwise, and matches the oracle."""
    small = synth.random_scene(3, 50, sh_degree=0)
    big, cams = synth.tiny_scene(seed=1, n=4096)
    cam = cams[0]
    ref_ctx = nxs.Renderer(0)
    r = nxs.Renderer(0)
    try:
        gs, gb = nxs.scene_to_device(small), nxs.scene_to_device(big)
        ref = ref_ctx.render(gb, [cam], model=1)[0]
        r.render(gs, [cam], model=1)                       # sizes the context: ~100 instances
        out = r.render(gb, [cam], model=1, deferred=True)[0]
        with pytest.raises(nxs.NxsError) as e:
            r.status()
        assert e.value.status == -4
        torch.cuda.synchronize()
        assert torch.all(out["overdraw"] == 0)             # nothing was composited
        out = r.render(gb, [cam], model=1, deferred=True)[0]
        assert r.status() == 0
        _same(out, ref)
        parity.compare_keys(r, big, [cam])
        parity.compare_view(out, big, cam, 1, pixels=parity.sample_pixels(cam, 2000))
    finally:
        r.close()
        ref_ctx.close()


def test_deferred_depth_plan_change_is_retried(nxs):
    """After a scene whose depths vary in 25 bits the context launches three
    depth-sort passes; a deferred render of a 31-bit scene needs four, which
    the device detects: reported, retried, then bitwise equal."""
    cam = synth.look_at_camera((0, 0, -3), width=96, height=80)
    narrow, wide = _depth_range_scene(2.1, 15.0), _depth_range_scene(0.4, 60.0)
    r, ref_ctx = nxs.Renderer(0), nxs.Renderer(0)
    try:
        gn, gw = nxs.scene_to_device(narrow), nxs.scene_to_device(wide)
        ref = ref_ctx.render(gw, [cam], model=0)[0]
        r.render(gw, [cam], model=0)                  # instance capacity for both
        r.render(gn, [cam], model=0)                  # plans three passes
        r.render(gw, [cam], model=0, deferred=True)
        with pytest.raises(nxs.NxsError):
            r.status()
        out = r.render(gw, [cam], model=0, deferred=True)[0]
        assert r.status() == 0
        _same(out, ref)
        parity.compare_keys(r, wide, [cam])
    finally:
        r.close()
        ref_ctx.close()


def test_deferred_render_larger_than_expected(nxs):
    """The instance buffers hold a large render, but the context last saw a
    small one: a deferred render of the large scene launches its tile sort and
    ranges for the small count (with headroom) and their work-groups loop
    over the remaining chunks; the result equals the waiting render."""
    big = synth.random_scene(12, 20_000, sh_degree=0, log_scale=(-3.2, 0.4))
    cam = synth.look_at_camera((0.1, 0.0, -3.0), width=256, height=256)
    # the 20 nearest and 20 farthest: the same depth span (a four-pass depth
    # sort, like the large scene) in few instances
    by_depth = np.argsort(big.means[:, 2])
    small = big.subset(np.concatenate([by_depth[:20], by_depth[-20:]]))
    r, ref_ctx = nxs.Renderer(0), nxs.Renderer(0)
    try:
        gb, gs = nxs.scene_to_device(big), nxs.scene_to_device(small)
        for model in (0, 2):
            ref = ref_ctx.render(gb, [cam], model=model)[0]
            r.render(gb, [cam], model=model)        # capacity for the large scene
            m_big, _ = r.counts()
            r.render(gs, [cam], model=model)        # ... but the last count is small
            m_small, _ = r.counts()
            assert m_big > 20 * (m_small + m_small // 4 + 4096)
            out = r.render(gb, [cam], model=model, deferred=True)[0]
            assert r.status() == 0
            _same(out, ref)
        parity.compare_keys(r, big, [cam])
    finally:
        r.close()
        ref_ctx.close()


def test_deferred_pipeline_equals_waiting(nxs):
    """Many deferred renders of alternating scenes and models enqueued with
    no wait in between equal the waiting renders; status() is clean."""
    scenes = [synth.tiny_scene(seed=s, n=2000)[0] for s in (1, 2)]
    cams = synth.tiny_scene(seed=1, n=10)[1]
    r, ref_ctx = nxs.Renderer(0), nxs.Renderer(0)
    try:
        gs = [nxs.scene_to_device(s) for s in scenes]
        for g in gs:                                   # size both contexts
            r.render(g, cams, model=0)
        refs, outs = [], []
        for k in range(12):
            g, m = gs[k % 2], k % 4
            refs.append(ref_ctx.render(g, cams, model=m)[0])
            outs.append(r.render(g, cams, model=m, deferred=True)[0])
        assert r.status() == 0
        for a, b in zip(outs, refs):
            _same(a, b)
    finally:
        r.close()
        ref_ctx.close()


def test_states_are_independent(nxs):
    """Two forwards keep two states; backwards taken in any order, after
    other forwards, and repeated, agree with the backward taken at once."""
    sc1, cams = synth.tiny_scene(seed=4, n=800)
    sc2 = synth.random_scene(5, 600, sh_degree=1)
    r = nxs.Renderer(0)
    try:
        g1, g2 = nxs.scene_to_device(sc1), nxs.scene_to_device(sc2)
        d = [torch.randn(c.height, c.width, 3, device="cuda") for c in cams]
        r.render(g1, cams, model=3, keep_state=True)
        now = r.backward(g1, d)
        s1 = r.last_state
        r.render(g2, cams, model=0, keep_state=True)
        s2 = r.last_state
        r.render(g2, cams, model=1)                   # no state
        later = r.backward(g1, d, state=s1)
        again = r.backward(g1, d, state=s1)
        g2grad = r.backward(g2, d, state=s2)
        torch.cuda.synchronize()
        for k in now:
            scale = float(now[k].abs().max())
            assert scale > 0, k
            for x in (later, again):
                assert torch.allclose(x[k], now[k], rtol=1e-5, atol=1e-6 * scale), k
        assert float(g2grad["opacities"].abs().max()) > 0
        s1.release()
        s2.release()
        assert len(r._states) == 0
    finally:
        r.close()


@pytest.mark.parametrize("allocator", [None, "torch"])
def test_workspace_sources_and_streams(nxs, allocator):
    """The library's pool and PyTorch's caching allocator back the same
    renders bitwise; the workspace grows while calls alternate between two
    streams (growth frees blocks in stream order on the calling stream)."""
    r = nxs.Renderer(0, allocator=allocator)
    ref_ctx = nxs.Renderer(0, allocator=None)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    try:
        cams = synth.tiny_scene(seed=1, n=10)[1]
        outs, refs = [], []
        for k, n in enumerate((100, 1000, 3000, 8000, 500, 12000)):
            g = nxs.scene_to_device(synth.tiny_scene(seed=k, n=n)[0])
            with torch.cuda.stream(streams[k % 2]):
                outs.append(r.render(g, cams, model=k % 4)[0])
            refs.append(ref_ctx.render(g, cams, model=k % 4)[0])
        torch.cuda.synchronize()
        for a, b in zip(outs, refs):
            _same(a, b)
        assert r.workspace_bytes() > 0
        if allocator == "torch":
            assert r._alloc.bytes_held > 0               # blocks came from torch
    finally:
        r.close()
        ref_ctx.close()
