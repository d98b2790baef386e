"""nxs_pipeline_* through the C ABI: renders dealt to several lanes (contexts on
streams of their own) equal the renders of one context bitwise, the caller's
stream sees complete outputs after a join, outputs are reused after a join,
and a deferred render that outgrew its lane is reported and then succeeds on
whichever lane takes it."""
import numpy as np
import pytest

import synth
from tests import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _same(a, b):
    for k in ("rgb", "trans", "overdraw"):
        assert torch.equal(a[k], b[k]), k


@pytest.mark.timeout(300)
def test_pipeline_equals_one_context():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2603_02887_amd import nxs
    sc, _ = synth.tiny_scene(seed=1, n=4096)
    cams = synth.orbit_cameras(3, 3.0, [128, 96, 160], [128, 64, 96],
                               rng=np.random.default_rng(5))
    g = nxs.scene_to_device(sc)
    R = nxs.Renderer(0)
    P = nxs.Pipeline(0, lanes=3)
    try:
        ref = {m: R.render(g, cams, model=m) for m in range(4)}
        torch.cuda.synchronize()
        # a waiting render on each lane sizes its workspace (a fresh lane has
        # no instance capacity for a deferred render)
        for m in range(3):
            P.render(g, cams, model=m, deferred=False)
        P.join()
        # eight renders in flight at once, distinct outputs, waiting and deferred
        print("case: 8 renders over 3 lanes", flush=True)
        outs = [P.render(g, cams, model=i % 4, deferred=(i % 2 == 0)) for i in range(8)]
        P.join()
        torch.cuda.synchronize()
        P.status()
        for i, o in enumerate(outs):
            for v in range(len(cams)):
                _same(o[v], ref[i % 4][v])
        # outputs reused after a join: the next render's writes follow it
        for o in outs:
            for v in o:
                v["rgb"].fill_(-1.0)
        stream = torch.cuda.current_stream()
        for i, o in enumerate(outs):
            P.render(g, cams, model=i % 4, outputs=o)
        P.join(stream)
        torch.cuda.synchronize()
        for i, o in enumerate(outs):
            for v in range(len(cams)):
                _same(o[v], ref[i % 4][v])
        parity.compare_view(outs[1][0], sc, cams[0], 1, pixels=parity.sample_pixels(cams[0], 200))
    finally:
        P.close()
        R.close()


@pytest.mark.timeout(300)
def test_pipeline_outgrown_render_is_reported_and_rendered_again():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2603_02887_amd import nxs
    small, _ = synth.tiny_scene(seed=1, n=512)
    big = synth.random_scene(7, 60_000, sh_degree=0, log_scale=(-2.0, 0.3))
    cam = synth.look_at_camera((0, 0, -3), width=160, height=128)
    gs, gb = nxs.scene_to_device(small), nxs.scene_to_device(big)
    R = nxs.Renderer(0)
    P = nxs.Pipeline(0, lanes=2)
    try:
        ref = R.render(gb, [cam], model=1)
        torch.cuda.synchronize()
        # both lanes sized by a small render, then the big one deferred
        for _ in range(2):
            P.render(gs, [cam], model=1, deferred=False)
        P.join()
        print("case: deferred render beyond its lane's capacity", flush=True)
        out = P.render(gb, [cam], model=1, deferred=True)
        P.join()
        torch.cuda.synchronize()
        with pytest.raises(nxs.NxsError) as e:
            P.status()
        assert e.value.status == -4
        # the next render goes to the other lane, which has grown as well
        out = P.render(gb, [cam], model=1, outputs=out, deferred=True)
        P.join()
        torch.cuda.synchronize()
        assert P.status() == 0
        _same(out[0], ref[0])
        out = P.render(gb, [cam], model=1, outputs=out, deferred=True)
        P.join()
        torch.cuda.synchronize()
        assert P.status() == 0
        _same(out[0], ref[0])
    finally:
        P.close()
        R.close()


@pytest.mark.timeout(300)
def test_pipeline_of_one_and_of_eight_lanes():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2603_02887_amd import nxs
    sc, cams = synth.tiny_scene(seed=2, n=2048)
    g = nxs.scene_to_device(sc)
    R = nxs.Renderer(0)
    try:
        ref = R.render(g, cams, model=3)
        torch.cuda.synchronize()
        for lanes in (1, 8):
            print("case: %d lane(s)" % lanes, flush=True)
            P = nxs.Pipeline(0, lanes=lanes)
            try:
                outs = [P.render(g, cams, model=3, deferred=False) for _ in range(lanes + 2)]
                P.join()
                torch.cuda.synchronize()
                assert P.status() == 0
                for o in outs:
                    _same(o[0], ref[0])
            finally:
                P.close()
    finally:
        R.close()
