"""nxs_render_forward_noalloc through the C ABI: the render of
nxs_render_forward, bitwise, with its workspace in the library's fixed
per-device scratch; nothing allocated (the context's workspace and PyTorch's
allocator are untouched); two calls in a row, the second smaller, so that
what the first left in the scratch cannot leak into the second; a render
beyond the scratch fails cleanly."""
import ctypes

import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def nxs():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2603_02887_amd import nxs as m
    return m


def _outputs(cams):
    return [{"rgb": torch.full((c.height, c.width, 3), -1.0, device="cuda"),
             "trans": torch.full((c.height, c.width), -1.0, device="cuda"),
             "overdraw": torch.full((c.height, c.width), -1, dtype=torch.int32,
                                    device="cuda")} for c in cams]


def test_noalloc_equals_forward_twice(nxs):
    big, cams_big = synth.tiny_scene(seed=1, n=4096)
    small = synth.random_scene(7, 900, sh_degree=1)
    cams_small = [synth.look_at_camera((0.3, -0.2, -3.2), width=64, height=48),
                  synth.look_at_camera((-0.5, 0.1, -2.8), width=33, height=17)]
    r = nxs.Renderer(0)
    try:
        cases = [("4096 Gaussians, one 128x128 view, exponential", big, cams_big, 0, (16, 16)),
                 ("900 Gaussians SH1, 64x48 and 33x17 views, superlinear", small, cams_small,
                  3, (8, 8))]
        for name, sc, cams, model, tile in cases:
            print("case:", name, flush=True)
            g = nxs.scene_to_device(sc)
            ref = r.render(g, cams, model=model, tile=tile, background=(0.1, 0.2, 0.3))
            torch.cuda.synchronize()
            ws = r.workspace_bytes()
            outs = _outputs(cams)
            torch.cuda.synchronize()
            before = torch.cuda.memory_allocated()
            r.render_noalloc(g, cams, outs, model=model, tile=tile,
                             background=(0.1, 0.2, 0.3))
            torch.cuda.synchronize()
            assert torch.cuda.memory_allocated() == before
            assert r.workspace_bytes() == ws
            for a, b in zip(outs, ref):
                for k in ("rgb", "trans", "overdraw"):
                    assert torch.equal(a[k], b[k]), (name, k)
    finally:
        r.close()


def test_noalloc_rejects_what_does_not_fit(nxs):
    sc = synth.random_scene(3, 700_000, sh_degree=0)      # ~70 MB of per-slot buffers
    cam = synth.look_at_camera((0, 0, -3), width=64, height=64)
    r = nxs.Renderer(0)
    try:
        g = nxs.scene_to_device(sc)
        outs = _outputs([cam])
        print("case: 700,000 Gaussians, beyond the scratch", flush=True)
        with pytest.raises(nxs.NxsError) as e:
            r.render_noalloc(g, [cam], outs)
        assert e.value.status == -4 and "scratch" in str(e.value)
        torch.cuda.synchronize()
        assert torch.all(outs[0]["rgb"] == -1.0)           # no output was written
        # flags are refused before anything is launched
        gs = nxs._make_gaussians(g)
        carr = (nxs.Camera * 1)(nxs.make_camera(cam))
        imgs = (nxs.Image * 1)(nxs._make_image(outs[0]))
        opts = nxs._make_opts(deferred=True)
        assert r._L.nxs_render_forward_noalloc(r._ctx, ctypes.byref(gs), carr, 1,
                                               ctypes.byref(opts), imgs, None) == -1
    finally:
        r.close()
