"""The benchmark's stage roofline (host arithmetic only): the depth sort's pass
count from the depth-bit range, and T_roof = sum of max(bytes / BW, lane-ops /
VALU rate) per stage against the measured stage times."""
import types

import numpy as np

import bench


def _scene(z, sh_degree=3):
    n = len(z)
    means = np.zeros((n, 3), np.float32)
    means[:, 2] = z
    return types.SimpleNamespace(n=n, means=means, sh_degree=sh_degree)


def _cam(w=64, h=32):
    return types.SimpleNamespace(R=np.eye(3, dtype=np.float32), t=np.zeros(3, np.float32),
                                 znear=0.01, width=w, height=h)


def test_depth_passes_follow_the_varying_bits():
    # depths within one binade vary only in the 23 mantissa bits: three passes
    assert bench.depth_sort_passes(_scene(np.linspace(2.0, 3.9, 100)), _cam()) == 3
    # depths over many binades vary in the exponent's bits as well: four
    assert bench.depth_sort_passes(_scene(np.geomspace(0.02, 1e6, 100)), _cam()) == 4
    # Gaussians behind the near plane do not count
    z = np.concatenate([np.linspace(2.0, 3.9, 50), [-1e6, 0.001]])
    assert bench.depth_sort_passes(_scene(z), _cam()) == 3


def test_stage_roofline_sums_the_stage_bounds():
    sc, cam = _scene(np.linspace(2.0, 3.0, 1000)), _cam()
    M, T, od = 5000, 8, 40000
    st = {"project": 0.01, "depth_sort": 0.02, "emit": 0.01, "tile_sort": 0.02,
          "ranges": 0.005, "composite": 0.05}
    r = bench.stage_roofline(0, sc, cam, {"sort_order": "depth_first"}, (M, T), od, st, 0.05e-3)
    s = r["stages"]
    bw = bench.HBM_PEAK_GBS * 1e9
    assert s["project"]["bytes"] == (56 + 12 * 16) * 1000 + 60 * 1000
    assert s["tile_sort"]["bytes"] == 16 * M * 1          # 8 tiles: one 3-bit pass
    assert s["depth_sort"]["bytes"] == 16 * 1000 * 3 + 20 * 1000
    assert np.isclose(s["ranges"]["roof_ms"], (4 * M + 8 * T) / bw * 1e3)
    t_ops = od * bench.SLOTS_PER_PAIR / (bench.VALU_SLOT_PEAK_T * 1e12) * 1e3
    t_bytes = (52 * M + 20 * cam.width * cam.height) / bw * 1e3
    assert np.isclose(s["composite"]["roof_ms"], max(t_ops, t_bytes))
    assert s["composite"]["bound"] == ("alu" if t_ops > t_bytes else "hbm")
    tot = sum(v["roof_ms"] for v in s.values())
    assert np.isclose(r["roof_ms"], tot)
    assert np.isclose(r["frac"], tot / sum(st.values()))
    assert np.isclose(r["frac_throughput"], tot / 0.05)
    for k, v in s.items():
        assert np.isclose(v["frac"], v["roof_ms"] / st[k])
    # tile-first lists: the per-tile depth sort runs in the ranges stage
    r2 = bench.stage_roofline(0, sc, cam, {"sort_order": "tile_first"}, (M, T), od, st, 0.05e-3)
    assert r2["stages"]["depth_sort"]["bytes"] == 0
    assert r2["stages"]["ranges"]["bytes"] == 4 * M + 8 * T + (16 * 3 + 4) * M
