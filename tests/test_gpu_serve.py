"""Serving loop (continuous batching under a workspace budget) on the GPU.

Each served request must be bitwise what rendering it alone gives, whatever
batch it was served in; the budget must split batches and turn a request that
cannot fit on its own into an NXS_ECAPACITY completion without stopping the
others.
"""
import math

import numpy as np
import pytest

import synth
from tests import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SIZES = [(64, 48), (200, 120), (96, 96), (33, 17)]


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2603_02887_amd import nxs
    r = nxs.Renderer(0)
    yield r
    r.close()


def _scenes():
    return [synth.random_scene(61, 20_000, sh_degree=0),
            synth.random_scene(62, 50_000, sh_degree=1, log_scale=(-4.0, 0.4)),
            synth.random_scene(63, 5_000, sh_degree=0, logit=(1.0, 1.0))]


def _requests(n, n_scenes, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for k in range(n):
        w, h = SIZES[rng.integers(len(SIZES))]
        r, az = rng.uniform(3, 6), rng.uniform(0, 2 * math.pi)
        el = math.radians(rng.uniform(-30, 30))
        eye = (r * math.cos(el) * math.sin(az), r * math.sin(el), -r * math.cos(el) * math.cos(az))
        reqs.append({"scene": int(rng.integers(n_scenes)), "cam": synth.look_at_camera(
            eye, width=w, height=h), "model": int(rng.integers(4)), "tag": 1000 + k})
    return reqs


def _alone(R, g, req):
    out = R.render(g, [req["cam"]], model=req["model"], overdraw=False)
    torch.cuda.synchronize()
    return out[0]


def test_mix_equals_alone(R):
    from paper_2603_02887_amd import nxs
    scenes = [nxs.scene_to_device(s) for s in _scenes()]
    S = nxs.Server(0, workspace_budget=0, max_batch_views=16, n_slots=2)
    ids = [S.add_scene(g) for g in scenes]
    reqs = _requests(48, len(scenes), seed=1)
    for q in reqs[:30]:
        S.submit(ids[q["scene"]], q["cam"], q["tag"], model=q["model"])
    done, steps, batch_sizes = {}, 0, []
    while S.pending or S.in_flight:
        res = S.step(wait=True)
        steps += 1
        batch_sizes.append(len(res))
        for tag, st, out in res:
            assert st == 0
            done[tag] = out
        if steps == 2:                # later arrivals join the queue mid-stream
            for q in reqs[30:]:
                S.submit(ids[q["scene"]], q["cam"], q["tag"], model=q["model"])
    assert len(done) == len(reqs)
    assert steps < len(reqs) and max(batch_sizes) > 1
    for q in reqs:
        ref = _alone(R, scenes[q["scene"]], q)
        assert torch.equal(done[q["tag"]]["rgb"], ref["rgb"]), q["tag"]
        assert torch.equal(done[q["tag"]]["trans"], ref["trans"]), q["tag"]
    S.close()


def test_budget_splits_and_rejects(R):
    from paper_2603_02887_amd import nxs
    small = synth.random_scene(64, 4_000, sh_degree=0)
    big = synth.random_scene(65, 400_000, sh_degree=0)
    gs, gb = nxs.scene_to_device(small), nxs.scene_to_device(big)
    budget = 12 << 20             # 12 MiB: a 400k-Gaussian render alone needs ~35 MB
    S = nxs.Server(0, workspace_budget=budget, max_batch_views=64, n_slots=2)
    i_small, i_big = S.add_scene(gs), S.add_scene(gb)
    reqs = [q for q in _requests(40, 1, seed=2)]
    for q in reqs:
        S.submit(i_small, q["cam"], q["tag"], model=q["model"])
    S.submit(i_big, reqs[0]["cam"], 7, model=0)
    results, steps = {}, 0
    while S.pending or S.in_flight:
        for tag, st, out in S.step(wait=True):
            results[tag] = (st, out)
        steps += 1
        assert S.workspace_bytes() <= budget
    assert results[7][0] == -4                       # NXS_ECAPACITY, on its own
    assert all(results[q["tag"]][0] == 0 for q in reqs)
    assert steps > 2                                 # the budget split the 40 views
    for q in reqs[:8]:
        ref = _alone(R, gs, q)
        assert torch.equal(results[q["tag"]][1]["rgb"], ref["rgb"])
    S.close()


def test_submit_errors(R):
    from paper_2603_02887_amd import nxs
    S = nxs.Server(0)
    sid = S.add_scene(nxs.scene_to_device(synth.random_scene(1, 100)))
    cam = synth.look_at_camera((0, 0, -3), width=32, height=32)
    with pytest.raises(nxs.NxsError):
        S.submit(sid + 5, cam, 1)
    with pytest.raises(nxs.NxsError):
        S.submit(sid, cam, 2, deferred=True)          # served renders take no flags
    S.submit(sid, cam, 3, model=9)                   # invalid model: fails alone
    S.submit(sid, cam, 4, model=1)
    got = {tag: st for tag, st, _ in S.drain()}
    assert got == {3: -1, 4: 0}
    assert S.step() == []
    S.close()


def test_batches_overlap_on_the_device(R):
    """Two slots: requests for two scenes start as two batches in one step,
    both in flight before either is collected; results equal renders alone."""
    from paper_2603_02887_amd import nxs
    scenes = [nxs.scene_to_device(s) for s in _scenes()[:2]]
    S = nxs.Server(0, n_slots=2)
    ids = [S.add_scene(g) for g in scenes]
    reqs = _requests(12, 2, seed=4)
    for q in reqs:
        S.submit(ids[q["scene"]], q["cam"], q["tag"], model=0)
    first = S.step(wait=False)
    started = len(reqs) - S.pending - len(first)
    assert S.in_flight == started
    # both slots took a batch: more requests started than the larger batch holds
    per_scene = max(sum(q["scene"] == k for q in reqs) for k in range(2))
    assert started + len(first) > per_scene or S.pending == 0
    done = {tag: out for tag, st, out in first + S.drain()}
    for q in reqs:
        q["model"] = 0
        assert torch.equal(done[q["tag"]]["rgb"], _alone(R, scenes[q["scene"]], q)["rgb"])
    S.close()


def test_served_results_match_the_oracle(R):
    """Served requests of mixed scene, resolution and model (two slots,
    continuous batching, deferred batches) against the FP64 oracle on
    sampled pixels, at the tolerances of every other parity test."""
    from paper_2603_02887_amd import nxs
    scs = _scenes()
    scenes = [nxs.scene_to_device(sc) for sc in scs]
    S = nxs.Server(0, n_slots=2)
    ids = [S.add_scene(g) for g in scenes]
    reqs = _requests(16, len(scenes), seed=11)
    for q in reqs:
        S.submit(ids[q["scene"]], q["cam"], q["tag"], model=q["model"], overdraw=True)
    done = {tag: (st, out) for tag, st, out in S.drain()}
    S.close()
    for q in reqs:
        st, out = done[q["tag"]]
        assert st == 0
        px = parity.sample_pixels(q["cam"], 400, seed=q["tag"])
        stats = parity.compare_view(out, scs[q["scene"]], q["cam"], q["model"], pixels=px)
        print("served", q["tag"], q["model"], stats["max_rgb_err"], stats["ambiguous"])


def test_deferred_overflow_in_a_batch_is_served_again(R):
    """One slot sized by a tiny request, then a batch that needs far more
    instances: its deferred render overflows, the batch is queued again and
    rendered waiting after the slot has grown; every result equals the
    request rendered alone."""
    from paper_2603_02887_amd import nxs
    scenes = [nxs.scene_to_device(sc) for sc in _scenes()]
    S = nxs.Server(0, n_slots=1)
    ids = [S.add_scene(g) for g in scenes]
    tiny = synth.look_at_camera((0, 0, -5), width=16, height=16)
    S.submit(ids[2], tiny, 1, model=1)
    assert [t for t, st, _ in S.drain()] == [1]
    small_ws = S.workspace_bytes()
    reqs = [q for q in _requests(12, 2, seed=21)]
    for q in reqs:
        S.submit(ids[q["scene"]], q["cam"], q["tag"], model=q["model"])
    done = {tag: (st, out) for tag, st, out in S.drain()}
    assert S.workspace_bytes() > small_ws
    for q in reqs:
        st, out = done[q["tag"]]
        assert st == 0
        assert torch.equal(out["rgb"], _alone(R, scenes[q["scene"]], q)["rgb"])
    S.close()
