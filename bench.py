#!/usr/bin/env python3
"""Forward-render benchmark on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Workload: 1,000,000 Gaussians drawn from 64 anisotropic clusters, SH degree 3,
one 1920x1080 pinhole camera.  One step renders that frame once with each
transmittance model (exponential, linear, quadratic sublinear, quadratic
superlinear): the whole path (projection, depth sort, binning, tile sort,
tile ranges, composite with its gather) runs for every render, with the
tile shape, composite schedule and LDS batch the library's autotuner picks
for each model.  The scene is uploaded to HBM before the timed region.

The timed steps enqueue their renders back to back without waiting
(deferred renders, whose instance count is checked on the device), taking
two or three library contexts in turn, each on a stream of its own: one
render's short, latency-bound sort kernels then overlap another's projection
or composite.  Each is timed with the tuner's configuration and with the
tile schedule in its place where the tuner chose the longest-first queue
(another render in flight fills the composite's tail, so the queue's two
order kernels may not pay for themselves); the fastest is `value`.  `value` is the frame's pixels
over that time.  The same steps on one context and one stream, deferred and
waiting, are reported beside it, as is per-model throughput.  Latency is measured
separately, one render at a time, waiting for each: p50/p99 per model, with
per-stage GPU times from hipEvents the library records on the render stream
(the composite's time there, alone on the GPU, is the one the roofline uses).

Prints one JSON line: aggregate Mpix/s over all renders, per-model Mpix/s,
splats blended per second (sum of per-pixel overdraw / time), mean overdraw,
p50/p99 render latency, per-stage GPU times, the roofline of the dominant
kernel, the CPU oracle timed on a bounded pixel sample of the same frame with
a process pool over the host's cores, and the batched (16 views),
differentiation (8 views, forward + backward) and serving (four resident
scenes, continuous batching under Poisson arrivals, against one plain
launch per request) workloads.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

MODELS = ("exponential", "linear", "sublinear", "superlinear")
METRIC = "Mpix/s + splats blended/s per transmittance model; p50/p99 render latency"

# FP32 arithmetic of one composited (pixel, splat) pair, counting an FMA as 2
# flops and the exp2 as 1 (the convention of the FLOP/s peak below): offset
# 2, exponent 8, exp2 1, accumulate 6, plus the operator (exponential 3,
# linear 1, quadratic 5).
FLOPS_PER_PAIR = {0: 20, 1: 18, 2: 22, 3: 22}
# MI355X FP32 vector peak: 256 CUs x 128 FP32 lanes x 2 flops (FMA) x 2.4 GHz.
FP32_VALU_PEAK_TFLOPS = 157.2864
# VALU issue slots of one pair (an FMA is one slot, the exp2 four at quarter
# rate, plus two compares and the overdraw increment): about 24.  Reported
# against the non-packed issue rate of 256 CUs x 64 lanes x 2.4 GHz as a
# second view of the same kernel.
SLOTS_PER_PAIR = 24
VALU_SLOT_PEAK_T = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of each composite kernel on this workload (16x16 tiles,
# per schedule: the queue and the tile schedule),
# from FETCH_SIZE and WRITE_SIZE counter runs scaled by a copy kernel of known
# size (profiles/forward_hbm_traffic_scene1m_1080p.md).  They describe the
# kernel sources with this digest and are reported as null once those change.
TRAFFIC_SOURCES = ("composite.hip", "nxs_ops.h", "nxs_stage.h", "nxs_internal.h")
TRAFFIC = {"digest": "4dbd297174eaaed7865081fbd6d73b76f50b9775b3666197a56c27f04d2d49aa",
           "tile": "16x16",
           "bytes": {
               "queue": {0: 485824065, 1: 253662114, 2: 287820851, 3: 240616214},
               "tiles": {0: 225022077, 1: 131614891, 2: 145831234, 3: 127215006}}}


def measured_traffic(model, tile, schedule):
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2603_02887_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != TRAFFIC["digest"] or tile != TRAFFIC["tile"]:
        return None
    return TRAFFIC["bytes"].get(schedule, {}).get(model)


def depth_sort_passes(scene, cam):
    """Digit passes of the depth sort for this frame: three 9-bit digits when
    the float32 depth bits of the Gaussians in front of the camera vary in at
    most 27 bits, else four (the device plans from the visible ones; a few
    culled off-screen ones could only narrow the range)."""
    z = (scene.means.astype(np.float32) @ np.asarray(cam.R, np.float32)[2]
         + np.float32(cam.t[2])).astype(np.float32)
    bits = z[z > cam.znear].view(np.uint32)
    if bits.size == 0:
        return 3
    nbits = int(bits.min() ^ bits.max()).bit_length()
    return 3 if nbits <= 27 else 4


def stage_roofline(m, scene, cam, conf, counts, od, stage_ms, thr_ms):
    """T_roof = sum over stages of max(algorithmic bytes / 8 TB/s, lane-ops /
    39.3 T lane-ops/s), per stage and overall, against the stages measured
    alone and against one render's share of the throughput mode.  Algorithmic
    bytes are those this pipeline must move: S slots (one view), M tile
    instances, T tiles, P pixels; the composite's lane-ops are 24 per
    composited pair."""
    M, T = counts
    S = scene.n
    P = cam.width * cam.height
    K = (scene.sh_degree + 1) ** 2
    dpass = depth_sort_passes(scene, cam)
    tpass = -(-max(1, int(T - 1).bit_length()) // 9)
    b = {"project": (56 + 12 * K) * scene.n + 60 * S,      # inputs; record, depth, rectangle
         "depth_sort": 16 * S * dpass + 20 * S,           # passes; rectangles laid out in order
         "emit": 24 * S + 8 * M,                          # scan and slot records; instances
         "tile_sort": 16 * M * tpass,
         "ranges": 4 * M + 8 * T,
         "composite": 52 * M + 20 * P}                    # slot index + record per entry; image
    if conf["sort_order"] == "tile_first":                # per-tile depth sort in "ranges"
        b["ranges"] += (16 * dpass + 4) * M
        b["depth_sort"] = 0
    ops = {"composite": od * SLOTS_PER_PAIR}
    stages = {}
    roof_total = 0.0
    for k, ms in stage_ms.items():
        t_bytes = b.get(k, 0) / (HBM_PEAK_GBS * 1e9)
        t_ops = ops.get(k, 0) / (VALU_SLOT_PEAK_T * 1e12)
        t_roof = max(t_bytes, t_ops) * 1e3
        roof_total += t_roof
        stages[k] = {"bytes": b.get(k, 0), "lane_ops": ops.get(k, 0),
                     "bound": "alu" if t_ops > t_bytes else "hbm",
                     "roof_ms": t_roof, "measured_ms": ms,
                     "frac": t_roof / ms if ms > 0 else None}
    meas = sum(stage_ms.values())
    return {"stages": stages, "roof_ms": roof_total, "measured_ms": meas,
            "frac": roof_total / meas, "throughput_ms_per_render": thr_ms * 1e3,
            "frac_throughput": roof_total / (thr_ms * 1e3),
            "depth_sort_passes": dpass, "tile_sort_passes": tpass}


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q / 100.0
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


# CPU oracle baseline: worker processes (started fresh; they import numpy and
# the oracle only) each rebuild the seeded frame and project it once.
_CPU = {}


def _cpu_init():
    from threadpoolctl import threadpool_limits
    import synth
    from oracle import keys as okeys
    from oracle import project as oproject
    _CPU["threads"] = threadpool_limits(1)     # one thread per process
    scene, cams = synth.scene_scale()
    cam = cams[0]
    t0 = time.perf_counter()
    proj = oproject.project(scene, cam)
    geom = okeys.geometry(scene, cam)
    _CPU.update(scene=scene, cam=cam, proj=proj, geom=geom,
                setup_s=time.perf_counter() - t0)


def _cpu_setup_time(_):
    return _CPU["setup_s"]


def _cpu_chunk(job):
    """Render one chunk of pixels with one model; returns (time of a 1-pixel
    render, i.e. the per-model pruning lists; time of the chunk; pixels)."""
    from oracle import render as orender
    model, pix = job
    sc, cam, proj, geom = _CPU["scene"], _CPU["cam"], _CPU["proj"], _CPU["geom"]
    t0 = time.perf_counter()
    orender.render(sc, cam, model, pixels=pix[:1], proj=proj, geom=geom)
    t1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    orender.render(sc, cam, model, pixels=pix, proj=proj, geom=geom)
    return t1, time.perf_counter() - t0, len(pix)


def cpu_baseline(width, height, n_pixels, seed=123):
    """Time the CPU oracle on a random pixel sample of the frame, per model, on
    a pool of one process per host core (at most 16), and extrapolate to the
    full frame: set-up (projection and key replay of all Gaussians) + per-model
    pruning lists + per-pixel time x W*H / cores."""
    import multiprocessing as mp
    import platform
    from concurrent.futures import ProcessPoolExecutor
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    cpu_model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu_model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    rng = np.random.default_rng(seed)
    flat = rng.choice(width * height, n_pixels, replace=False)
    pix = np.stack([flat % width, flat // width], 1)
    chunks = np.array_split(pix, cores)
    t_all = time.perf_counter()
    frame_s = []
    with ProcessPoolExecutor(max_workers=cores, mp_context=mp.get_context("spawn"),
                             initializer=_cpu_init) as pool:
        setup = min(pool.map(_cpu_setup_time, range(cores)))
        for m in range(4):
            res = list(pool.map(_cpu_chunk, [(m, c) for c in chunks]))
            t_lists = max(r[0] for r in res)
            per_px = float(np.median([max(r[1] - r[0], 0.0) / max(r[2] - 1, 1) for r in res]))
            frame_s.append(setup + t_lists + per_px * width * height / cores)
    spent = time.perf_counter() - t_all
    mpix = 4 * width * height / sum(frame_s) / 1e6
    return {"value": mpix, "unit": "Mpix/s", "cores": cores, "kind": "oracle",
            "cpu": cpu_model,
            "sample": (f"{n_pixels} random pixels of the {width}x{height} frame per model "
                       f"(4 models), split over {cores} processes; full-frame time = set-up "
                       f"(FP64 projection and key replay of all 1M Gaussians) + per-model "
                       f"pruning lists + per-pixel time x W*H / {cores}; {spent:.1f} s wall"),
            "frame_seconds": {MODELS[m]: frame_s[m] for m in range(4)}}


def batched_views(R, torch, nxs, synth, steps, models=(0, 1, 2, 3)):
    """Multi-view batch: 3M Gaussians (256-cluster means), 16 views of uneven
    size.  Per model: one batched render of all views with the autotuned tile
    shape and schedule, the same with the default tile/schedule, and one render
    per view (16 calls), each timed over `steps` repetitions after a warm-up."""
    scene, cams = synth.batched_scene()
    g = nxs.scene_to_device(scene)
    pix = sum(c.width * c.height for c in cams)
    outs = [{"rgb": torch.empty((c.height, c.width, 3), device="cuda"),
             "trans": torch.empty((c.height, c.width), device="cuda"), "overdraw": None}
            for c in cams]
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(steps):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / steps

    res = {}
    for m in models:
        tune = R.autotune(g, cams, model=m, outputs=outs, reps=3)
        kw = {"tile": tune["tile"], "schedule": tune["schedule"],
              "lds_batch": tune["lds_batch"], "sort_order": tune["sort_order"]}
        t_tuned = timed(lambda: R.render(g, cams, model=m, outputs=outs, **kw))
        t_default = timed(lambda: R.render(g, cams, model=m, outputs=outs))
        t_per_view = timed(lambda: [R.render(g, [c], model=m, outputs=[o], **kw)
                                    for c, o in zip(cams, outs)])
        n_inst, _ = R.counts()
        res[MODELS[m]] = {"batched_ms": t_tuned, "batched_default_ms": t_default,
                          "per_view_ms": t_per_view, "mpix_per_s": pix / t_tuned / 1e3,
                          "tuned": {"tile": "%dx%d" % tune["tile"],
                                    "schedule": tune["schedule"],
                                    "lds_batch": tune["lds_batch"],
                                    "sort_order": tune["sort_order"]},
                          "speedup_vs_per_view": t_per_view / t_tuned}
    return {"workload": ("3,000,000 Gaussians (means from 256 clusters), SH degree 0, "
                         "16 views of uneven size on a radius-15 orbit"),
            "pixels": pix, "views": len(cams), "per_model": res}


SERVE_SIZES = [(512, 512), (1280, 720), (1920, 1080)]


def serving(args, torch, nxs, synth):
    """Serving workload: four resident scenes (200k, 500k, 1M, 3M Gaussians);
    each request picks a scene, an eye at radius U[3,6], azimuth U[0,2pi),
    elevation U[-30,30] deg, a resolution from SERVE_SIZES and a model, all
    uniformly.  First the saturation rate (a burst of requests all queued at
    once), then Poisson arrivals at fractions of it; latency = arrival ->
    result ready.  The burst's requests are also rendered one plain launch
    each (one nxs_render_forward per request, back to back on one context)
    for comparison.  Returns the serving block of the JSON line."""
    rng = np.random.default_rng(50)
    scenes = synth.serving_scenes()
    S = nxs.Server(0, workspace_budget=args.serve_budget_gib << 30, max_batch_views=16,
                   n_slots=args.serve_slots)
    gpu_scenes = [nxs.scene_to_device(sc) for sc in scenes]
    ids = [S.add_scene(g) for g in gpu_scenes]
    pool = {wh: [] for wh in SERVE_SIZES}

    def draw():
        w, h = SERVE_SIZES[rng.integers(len(SERVE_SIZES))]
        r, az = rng.uniform(3, 6), rng.uniform(0, 2 * math.pi)
        el = math.radians(rng.uniform(-30, 30))
        eye = (r * math.cos(el) * math.sin(az), r * math.sin(el),
               -r * math.cos(el) * math.cos(az))
        return (int(rng.integers(len(scenes))), synth.look_at_camera(eye, width=w, height=h),
                int(rng.integers(4)))

    def out_for(cam):
        free = pool[(cam.width, cam.height)]
        if free:
            return free.pop()
        return {"rgb": torch.empty((cam.height, cam.width, 3), device="cuda"),
                "trans": torch.empty((cam.height, cam.width), device="cuda"),
                "overdraw": None}

    def run(arrivals, reqs):
        """Serve requests arriving at `arrivals` (seconds from now); returns
        per-request latency (s), wall time and pixels served."""
        t0 = time.perf_counter()
        n, nxt, lat, pix = len(reqs), 0, [0.0] * len(reqs), 0
        cams = {}
        while nxt < n or S.pending or S.in_flight:
            now = time.perf_counter() - t0
            while nxt < n and arrivals[nxt] <= now:
                sc, cam, m = reqs[nxt]
                S.submit(ids[sc], cam, nxt, outputs=out_for(cam), model=m)
                cams[nxt] = cam
                nxt += 1
            # block only when every slot is busy and requests wait for one;
            # otherwise poll, so that new arrivals are admitted promptly
            res = S.step(wait=S.pending > 0)
            t_done = time.perf_counter() - t0
            for tag, st, out in res:
                if st != 0:
                    raise RuntimeError(f"request {tag} failed with status {st}")
                lat[tag] = t_done - arrivals[tag]
                cam = cams.pop(tag)
                pix += cam.width * cam.height
                pool[(cam.width, cam.height)].append(out)
            if not res and not S.pending and nxt < n:
                time.sleep(max(0.0, min(arrivals[nxt] - (time.perf_counter() - t0), 2e-4)))
        return lat, time.perf_counter() - t0, pix

    # warm-up, then the saturation rate from a burst
    run([0.0] * 32, [draw() for _ in range(32)])
    burst = [draw() for _ in range(args.serve_burst)]
    lat_b, wall_b, pix_b = run([0.0] * len(burst), burst)
    rate_sat = len(burst) / wall_b
    # the same requests, one plain launch each
    R = nxs.Renderer(0)
    outs = [out_for(cam) for _, cam, _ in burst[:8]]
    for (sc, cam, m), o in zip(burst[:8], outs):
        R.render(gpu_scenes[sc], [cam], model=m, overdraw=False, outputs=[o])
    torch.cuda.synchronize()
    for o, (_, cam, _) in zip(outs, burst[:8]):
        pool[(cam.width, cam.height)].append(o)
    t0 = time.perf_counter()
    for sc, cam, m in burst:
        o = out_for(cam)
        R.render(gpu_scenes[sc], [cam], model=m, overdraw=False, outputs=[o])
        pool[(cam.width, cam.height)].append(o)
    torch.cuda.synchronize()
    wall_plain = time.perf_counter() - t0
    R.close()
    loads = []
    for frac in args.serve_loads:
        lam = frac * rate_sat
        n = args.serve_warmup + args.serve_requests
        arr = np.cumsum(rng.exponential(1.0 / lam, n))
        reqs = [draw() for _ in range(n)]
        lat, wall, pix = run(list(arr), reqs)
        meas = lat[args.serve_warmup:]
        loads.append({"load": frac, "rate_req_per_s": lam,
                      "achieved_req_per_s": n / wall, "mpix_per_s": pix / wall / 1e6,
                      "p50_ms": percentile(meas, 50) * 1e3, "p99_ms": percentile(meas, 99) * 1e3,
                      "mean_ms": float(np.mean(meas)) * 1e3, "requests": n})
        print(f"serving load {frac}: p50 {loads[-1]['p50_ms']:.2f} ms p99 "
              f"{loads[-1]['p99_ms']:.2f} ms", file=sys.stderr, flush=True)
    S.close()
    return {"workload": ("resident scenes of 200k/500k/1M/3M Gaussians; requests uniform "
                         "over scene, pose (radius 3-6), resolution (512x512, 1280x720, "
                         "1920x1080) and the four models"),
            "slots": args.serve_slots, "workspace_budget_gib": args.serve_budget_gib,
            "max_batch_views": 16,
            "saturation": {"requests": len(burst), "req_per_s": rate_sat,
                           "mpix_per_s": pix_b / wall_b / 1e6, "wall_s": wall_b,
                           "p50_ms": percentile(lat_b, 50) * 1e3,
                           "p99_ms": percentile(lat_b, 99) * 1e3},
            "plain_launches": {"requests": len(burst), "wall_s": wall_plain,
                               "req_per_s": len(burst) / wall_plain,
                               "mpix_per_s": pix_b / wall_plain / 1e6},
            "served_vs_plain": wall_plain / wall_b,
            "poisson": loads}


def differentiation(R, torch, nxs, synth, steps, models=(0, 1, 2, 3)):
    """Differentiation workload: 500k Gaussians (uniform-cube generator), 8
    views on a radius-6 orbit at 1280x720, per-pixel L1 loss against a render
    of the same scene with means jittered by N(0, 0.01) and opacity logits by
    N(0, 0.1).  One step = forward keeping state + path-replay backward for
    means, scales, rotations, opacities and SH, all 8 views, timed with
    events on the render stream."""
    scene, cams = synth.diff_scene()
    rng = np.random.default_rng(33)
    tgt = synth.Scene(scene.means + rng.normal(0, 0.01, scene.means.shape).astype(np.float32),
                      scene.scales, scene.quats,
                      (1.0 / (1.0 + np.exp(-(np.log(scene.opacities / (1 - scene.opacities))
                                             + rng.normal(0, 0.1, scene.n))))).astype(np.float32),
                      scene.sh, scene.sh_degree)
    g, gt = nxs.scene_to_device(scene), nxs.scene_to_device(tgt)
    pix = sum(c.width * c.height for c in cams)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    res = {}
    for m in models:
        target = R.render(gt, cams, model=m, overdraw=False)
        outs = [{"rgb": torch.empty_like(t["rgb"]), "trans": torch.empty_like(t["trans"]),
                 "overdraw": None} for t in target]

        def step():
            R.render(g, cams, model=m, keep_state=True, outputs=outs)
            ev[1].record()
            d_rgb = [torch.sign(o["rgb"] - t["rgb"]) / (3.0 * pix) for o, t in zip(outs, target)]
            return R.backward(g, d_rgb)

        step()
        torch.cuda.synchronize()
        fwd, tot = [], []
        for _ in range(steps):
            ev[0].record()
            gr = step()
            ev[2].record()
            torch.cuda.synchronize()
            fwd.append(ev[0].elapsed_time(ev[1]))
            tot.append(ev[0].elapsed_time(ev[2]))
        loss = sum(float((o["rgb"] - t["rgb"]).abs().sum()) for o, t in zip(outs, target)) / (3 * pix)
        res[MODELS[m]] = {"forward_ms": float(np.median(fwd)),
                          "forward_backward_ms": float(np.median(tot)),
                          "backward_ms": float(np.median(tot) - np.median(fwd)),
                          "mpix_per_s_fwd_bwd": pix / float(np.median(tot)) / 1e3,
                          "l1_loss": loss,
                          "grad_norm_means": float(gr["means"].norm())}
    return {"workload": ("500,000 Gaussians (uniform cube), SH degree 0, 8 views on a radius-6 "
                         "orbit at 1280x720, L1 loss against a jittered-scene render"),
            "pixels": pix, "views": len(cams), "per_model": res}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[1])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--tile", default="auto",
                    help="auto: the autotuned tile shape, schedule and LDS batch per model; "
                         "or WxH with the default schedule and batch")
    ap.add_argument("--cpu-pixels", type=int, default=262144)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 16-view batched workload")
    ap.add_argument("--batched-steps", type=int, default=3)
    ap.add_argument("--no-diff", action="store_true",
                    help="skip the 8-view forward + backward workload")
    ap.add_argument("--diff-steps", type=int, default=5)
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the continuous-batching server under Poisson load")
    ap.add_argument("--serve-requests", type=int, default=500)
    ap.add_argument("--serve-warmup", type=int, default=50)
    ap.add_argument("--serve-burst", type=int, default=400)
    ap.add_argument("--serve-loads", type=float, nargs="+", default=[0.5, 1.0])
    ap.add_argument("--serve-budget-gib", type=int, default=64)
    ap.add_argument("--serve-slots", type=int, default=2)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 256 MiB device-to-device copy (untimed) so that "
                         "counter runs can scale FETCH_SIZE / WRITE_SIZE by a kernel "
                         "of known traffic")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(views and requests shard across GPUs with no exchange in the forward "
              "pass, so the multi-GPU figure is the single-GPU one times N)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2603_02887_amd import nxs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        # an elementwise kernel that reads 256 MiB and writes 256 MiB
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    scene, cams = synth.scene_scale()
    cam = cams[0]
    W, H = cam.width, cam.height
    dev = torch.device("cuda", 0)
    g = nxs.scene_to_device(scene, dev)
    R = nxs.Renderer(0)
    ctxs = [R, nxs.Renderer(0), nxs.Renderer(0)]   # up to three renders in flight
    outs = {m: R.render(g, [cam], model=m) for m in range(4)}
    # (each further context writes outputs of its own)
    ctx_outs = [outs] + [{m: c.render(g, [cam], model=m) for m in range(4)} for c in ctxs[1:]]
    torch.cuda.synchronize()
    # the render configuration per model
    if args.tile == "auto":
        cfg = {}
        for m in range(4):
            t = R.autotune(g, [cam], model=m, outputs=outs[m], reps=5)
            cfg[m] = {"tile": t["tile"], "schedule": t["schedule"], "lds_batch": t["lds_batch"],
                      "sort_order": t["sort_order"]}
    else:
        tw, th = (int(x) for x in args.tile.split("x"))
        cfg = {m: {"tile": (tw, th), "schedule": "queue", "lds_batch": 64,
                   "sort_order": "depth_first"} for m in range(4)}
    for m in range(4):
        for c, o in zip(ctxs, ctx_outs):
            c.render(g, [cam], model=m, outputs=o[m], **cfg[m])
    torch.cuda.synchronize()
    od_sum = {m: int(outs[m][0]["overdraw"].sum().item()) for m in range(4)}
    n_inst, _ = R.counts()
    # this GPU's measured FP32 FMA rate (non-packed) and copy bandwidth, beside
    # the datasheet peaks
    peaks = R.measure_peaks()

    def render(m, ci=0, deferred=True, conf=None):
        ctxs[ci].render(g, [cam], model=m, outputs=ctx_outs[ci][m], deferred=deferred,
                        **(conf or cfg)[m])

    # The tuner measures one render at a time; with several renders in flight
    # another render fills the composite's tail, so the longest-first queue
    # (two latency-bound order kernels per render) can lose to the tile
    # schedule: both sets are timed and the faster is reported
    cfg_sets = {"tuned": cfg}
    no_order = {m: dict(c, schedule="tiles") if c["schedule"] in ("queue", "persistent") else c
                for m, c in cfg.items()}
    if no_order != cfg:
        cfg_sets["tuned_tile_schedule"] = no_order
    # the tile schedule with the library's default tiles and lists for every
    # model: with renders in flight, the tuner's per-render choices (timed one
    # render at a time) need not be the fastest mix
    plain_tiles = {m: {"tile": (16, 16), "schedule": "tiles", "lds_batch": 64,
                       "sort_order": "depth_first"} for m in range(4)}
    if plain_tiles not in cfg_sets.values():
        cfg_sets["tile_schedule_16x16"] = plain_tiles
    for conf in cfg_sets.values():
        for m in range(4):
            for c, o in zip(ctxs, ctx_outs):
                c.render(g, [cam], model=m, outputs=o[m], **conf[m])
    torch.cuda.synchronize()

    # Throughput (the timed steps): each step enqueues one render per model back
    # to back, as a pipelined caller would (each model writes its own outputs)
    streams = [torch.cuda.Stream(dev) for _ in ctxs]
    turn = [0]

    def step_multi(k, conf):   # k contexts on k streams, taken in turn
        def step():
            for m in range(4):
                ci = turn[0] % k
                turn[0] += 1
                with torch.cuda.stream(streams[ci]):
                    render(m, ci, conf=conf)
        return step

    def step_one():          # one context, one stream, deferred
        for m in range(4):
            render(m)

    def step_wait():         # one context, one stream, each render waits for its count
        for m in range(4):
            render(m, deferred=False)

    def timed(step):
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        for attempt in range(3):
            t0 = time.perf_counter()
            for _ in range(args.steps):
                step()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            try:                       # every deferred render fitted its context
                for c in ctxs:
                    c.status()
                return dt
            except nxs.NxsError:       # (the contexts have grown: time it again)
                continue
        raise RuntimeError("deferred renders kept outgrowing their contexts")

    modes, mode_cfg = {}, {}
    for name, conf in cfg_sets.items():
        for k, kname in ((3, "three"), (2, "two")):
            key = f"{kname}_contexts_deferred" + ("" if name == "tuned" else "_" + name)
            modes[key] = timed(step_multi(k, conf))
            mode_cfg[key] = conf
    modes["one_context_deferred"] = timed(step_one)
    modes["one_context_waiting"] = timed(step_wait)

    # one pipeline object (nxs_pipeline_*: three lanes, renders dealt in turn,
    # joined on the caller's stream at the end of the timed steps) with each
    # configuration set
    pipe = nxs.Pipeline(0, lanes=3)
    pipe_outs = [{m: pipe.render(g, [cam], model=m, deferred=False, **cfg[m]) for m in range(4)}
                 for _ in range(3)]
    pipe.join()
    torch.cuda.synchronize()

    def step_pipe(conf):
        turn = [0]

        def step():
            for m in range(4):
                pipe.render(g, [cam], model=m, outputs=pipe_outs[turn[0] % 3][m],
                            deferred=True, **conf[m])
                turn[0] += 1
        return step

    for name, conf in cfg_sets.items():
        step = step_pipe(conf)
        for _ in range(args.warmup):
            step()
        pipe.join()
        torch.cuda.synchronize()
        for attempt in range(3):
            t0 = time.perf_counter()
            for _ in range(args.steps):
                step()
            pipe.join()                # the timed renders, complete on this stream
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            try:                       # every deferred render fitted its lane
                pipe.status()
                key = "pipeline_three_lanes" + ("" if name == "tuned" else "_" + name)
                modes[key] = dt
                mode_cfg[key] = conf
                break
            except nxs.NxsError:       # (the lanes have grown: time it again)
                continue
    pipe.close()
    best_mode = min(modes, key=modes.get)
    total = modes[best_mode]
    best_cfg = mode_cfg.get(best_mode, cfg)
    for c in ctxs[1:]:
        c.close()
    # per model, the same back-to-back throughput (one context, deferred)
    thr = {}
    for m in range(4):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            render(m)
        torch.cuda.synchronize()
        thr[m] = (time.perf_counter() - t0) / args.steps
    R.status()
    # Latency (each render waited for) and per-stage GPU times (hipEvents on the
    # render stream), outside the timed steps
    R.set_timing(True)
    lat = {m: [] for m in range(4)}
    stages = {m: [] for m in range(4)}
    counts = {}
    for _ in range(args.steps):
        for m in range(4):
            t0 = time.perf_counter()
            render(m, deferred=False)
            torch.cuda.synchronize()
            lat[m].append(time.perf_counter() - t0)
            stages[m].append(R.stage_times())
            counts[m] = R.counts()   # (instances, tiles) of this model's configuration
    R.set_timing(False)

    per_model = {}
    stage_mean = {}
    for m in range(4):
        # (medians: a render that a host hiccup delays shifts the mean)
        st = {k: float(np.median([x[k] for x in stages[m]])) for k in R.STAGES}
        stage_mean[m] = st
        per_model[MODELS[m]] = {
            "mpix_per_s": W * H / thr[m] / 1e6,
            "splats_blended_per_s": od_sum[m] / thr[m],
            "avg_overdraw": od_sum[m] / (W * H),
            "ms_per_render": thr[m] * 1e3,
            "p50_ms": percentile(lat[m], 50) * 1e3,
            "p99_ms": percentile(lat[m], 99) * 1e3,
            "stages_ms": st,
            "gpu_ms": sum(st.values()),
            "config": {"tile": "%dx%d" % cfg[m]["tile"], "schedule": cfg[m]["schedule"],
                       "lds_batch": cfg[m]["lds_batch"], "sort_order": cfg[m]["sort_order"]},
        }
    # dominant kernel: the largest stage of any model
    all_stage = {(m, k): stage_mean[m][k] for m in range(4) for k in R.STAGES}
    (dm, dk), dms = max(all_stage.items(), key=lambda kv: kv[1])
    if dk == "composite":
        flops = od_sum[dm] * FLOPS_PER_PAIR[dm]
        achieved = flops / (dms * 1e-3) / 1e12
        slots = od_sum[dm] * SLOTS_PER_PAIR / (dms * 1e-3) / 1e12
        tile = "%dx%d" % cfg[dm]["tile"]
        roofline = {"bound": "alu", "kernel": f"composite<{MODELS[dm]}>",
                    "achieved": achieved, "peak": FP32_VALU_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": achieved / FP32_VALU_PEAK_TFLOPS,
                    "traffic": (measured_traffic(dm, tile, cfg[dm]["schedule"])
                                if cfg[dm]["lds_batch"] == 64 else None),
                    "work_per_launch": {"composited_pairs": od_sum[dm],
                                        "flops_per_pair": FLOPS_PER_PAIR[dm]},
                    "valu_issue_slots": {"per_pair": SLOTS_PER_PAIR, "achieved_T_per_s": slots,
                                         "peak_T_per_s": VALU_SLOT_PEAK_T,
                                         "frac": slots / VALU_SLOT_PEAK_T},
                    "config": per_model[MODELS[dm]]["config"],
                    "avg_launch_ms": dms,
                    "measured_peak": peaks["fp32_fma_tflops"],
                    "frac_of_measured_peak": achieved / peaks["fp32_fma_tflops"]}
    else:
        roofline = {"bound": "hbm", "kernel": dk, "avg_launch_ms": dms, "achieved": None,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None, "traffic": None}

    renders = 4 * args.steps
    value = W * H * renders / total / 1e6
    stage_roof = {MODELS[m]: stage_roofline(m, scene, cam, cfg[m], counts[m], od_sum[m],
                                            stage_mean[m], total / renders)
                  for m in range(4)}
    exp_ms = per_model["exponential"]["ms_per_render"]
    for name in MODELS[1:]:
        per_model[name]["speedup_vs_exponential"] = exp_ms / per_model[name]["ms_per_render"]

    batched = None
    if not args.no_batched:
        batched = batched_views(R, torch, nxs, synth, args.batched_steps)

    diff = None
    if not args.no_diff:
        diff = differentiation(R, torch, nxs, synth, args.diff_steps)
    R.close()

    serve = None
    if not args.no_serving:
        serve = serving(args, torch, nxs, synth)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(W, H, args.cpu_pixels)

    line = {
        "metric": METRIC, "value": value, "unit": "Mpix/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": total / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": ("scene-scale forward: 1,000,000 Gaussians from 64 "
                                "anisotropic clusters, SH degree 3, one 1920x1080 camera; "
                                "one step = one render per transmittance model"),
                   "gaussians": scene.n, "width": W, "height": H,
                   "render_config": {MODELS[m]: {"tile": "%dx%d" % best_cfg[m]["tile"],
                                                 "schedule": best_cfg[m]["schedule"],
                                                 "lds_batch": best_cfg[m]["lds_batch"],
                                                 "sort_order": best_cfg[m]["sort_order"]}
                                     for m in range(4)},
                   "in_flight": best_mode, "instances": n_inst, "models": list(MODELS)},
        "throughput_modes_mpix_per_s": {k: W * H * renders / v / 1e6 for k, v in modes.items()},
        "per_model": per_model,
        "roofline": roofline,
        "stage_roofline": stage_roof,
        "measured_peaks": {"fp32_fma_tflops": peaks["fp32_fma_tflops"],
                           "copy_gbs": peaks["copy_gbs"],
                           "datasheet": {"fp32_tflops": FP32_VALU_PEAK_TFLOPS,
                                         "hbm_gbs": HBM_PEAK_GBS}},
        "cpu_baseline": cpu,
        "batched": batched,
        "differentiation": diff,
        "serving": serve,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
