"""Sorts past the chunk-size switch (16M keys), bit-exact against the oracle.

2.2M Gaussians seen by 8 small views give 17.6M projected slots (the depth
sort takes 4,096-key chunks) and about 29M tile instances (so does the tile
sort); the instance list, tile ranges and per-slot keys must equal the float32
key recipe's exactly, and sampled pixels must match the oracle render.
"""
import numpy as np
import pytest

import synth
from tests import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.timeout(600)
def test_depth_and_tile_sorts_past_16m_keys():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2603_02887_amd import nxs
    R = nxs.Renderer(0)
    try:
        sc = synth.random_scene(21, 2_200_000, sh_degree=0, log_scale=(-4.0, 0.3))
        cams = synth.orbit_cameras(8, 4.0, [96] * 8, [64] * 8, rng=np.random.default_rng(1))
        assert sc.n * len(cams) > (1 << 24)
        g = nxs.scene_to_device(sc)
        out = R.render(g, cams, model=1)
        torch.cuda.synchronize()
        m = parity.compare_keys(R, sc, cams)
        assert m > (1 << 24), m
        for v in (0, 5):
            px = parity.sample_pixels(cams[v], 400, seed=v)
            parity.compare_view(out[v], sc, cams[v], 1, pixels=px)
        print("instances", m)
    finally:
        R.close()
