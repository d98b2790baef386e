"""Python binding of libnxs (ctypes): argument marshalling only.

Every step of the render runs in the HIP library; this module checks that
tensors are on the GPU, float32 and contiguous, fills the C structs of
include/nxs.h and passes device pointers and the current HIP stream.  The
library's device workspace comes from PyTorch's caching allocator through the
allocator callbacks of nxs_create (TorchAllocator).  Loading fails loudly
when libnxs.so has not been built.
"""
import ctypes
import math
import weakref
from ctypes import POINTER, byref, c_float, c_int32, c_int64, c_uint32, c_uint64, c_void_p
from pathlib import Path

import numpy as np
import torch

LIB_PATH = Path(__file__).resolve().parent / "libnxs.so"

MODEL_IDS = {"exponential": 0, "linear": 1, "sublinear": 2, "superlinear": 3,
             "quadratic": 4, "blended": 5, "vicini": 6, "powerlaw": 7}
STATUS = {0: "NXS_OK", -1: "NXS_EINVAL", -2: "NXS_ENOMEM", -3: "NXS_EHIP",
          -4: "NXS_ECAPACITY", -5: "NXS_EUNSUPPORTED"}
SYMBOLS = ["nxs_create", "nxs_destroy", "nxs_render_forward", "nxs_render_backward",
           "nxs_state_release", "nxs_forward_status", "nxs_render_forward_noalloc",
           "nxs_autotune", "nxs_set_workspace_limit", "nxs_workspace_bytes",
           "nxs_release_workspace",
           "nxs_server_create", "nxs_server_destroy", "nxs_server_add_scene",
           "nxs_server_submit", "nxs_server_step", "nxs_server_pending",
           "nxs_server_in_flight", "nxs_server_workspace_bytes", "nxs_server_last_error",
           "nxs_last_error",
           "nxs_pipeline_create", "nxs_pipeline_destroy", "nxs_pipeline_render",
           "nxs_pipeline_join", "nxs_pipeline_status", "nxs_pipeline_last_error",
           "nxs_measure_peaks",
           "nxs_set_timing", "nxs_inspect_stage_times", "nxs_inspect_counts",
           "nxs_inspect_instances", "nxs_inspect_ranges", "nxs_inspect_projection",
           "nxs_inspect_slot_grads"]
# entry points that do not return an nxs_status
_NOT_STATUS = {"nxs_last_error": ctypes.c_char_p, "nxs_server_last_error": ctypes.c_char_p,
               "nxs_pipeline_last_error": ctypes.c_char_p,
               "nxs_server_pending": c_int32, "nxs_server_in_flight": c_int32}


class NxsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Gaussians(ctypes.Structure):
    _fields_ = [("n", c_int32), ("sh_degree", c_int32), ("means", c_void_p),
                ("scales", c_void_p), ("quats", c_void_p), ("opacities", c_void_p),
                ("sh", c_void_p)]


class Camera(ctypes.Structure):
    _fields_ = [("R", c_float * 9), ("t", c_float * 3), ("fx", c_float), ("fy", c_float),
                ("cx", c_float), ("cy", c_float), ("znear", c_float),
                ("width", c_int32), ("height", c_int32)]


class RenderOpts(ctypes.Structure):
    _fields_ = [("model", c_int32), ("background", c_float * 3), ("alpha_min", c_float),
                ("t_eps", c_float), ("tile_w", c_int32), ("tile_h", c_int32),
                ("lds_batch", c_int32), ("param", c_float), ("flags", c_int32),
                ("schedule", c_int32), ("instance_hint", c_float), ("sort_order", c_int32)]


FLAG_DEFERRED = 1


class Tuning(ctypes.Structure):
    _fields_ = [("tile_w", c_int32), ("tile_h", c_int32), ("schedule", c_int32),
                ("lds_batch", c_int32), ("sort_order", c_int32), ("ms", c_float)]


SORT_ORDERS = {"auto": 0, "depth_first": 1, "tile_first": 2}


ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, ctypes.c_size_t, c_void_p, c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_void_p, c_void_p)


SCHEDULES = {"tiles": 1, "blocks": 2, "queue": 3, "persistent": 4}


class Image(ctypes.Structure):
    _fields_ = [("rgb", c_void_p), ("trans", c_void_p), ("overdraw", c_void_p)]


class GaussiansGrad(ctypes.Structure):
    _fields_ = [("means", c_void_p), ("scales", c_void_p), ("quats", c_void_p),
                ("opacities", c_void_p), ("sh", c_void_p)]


_lib = None


def lib():
    """The loaded libnxs.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise RuntimeError(f"{LIB_PATH} not found: build it with "
                               "`python -m paper_2603_02887_amd.build`")
        L = ctypes.CDLL(str(LIB_PATH))
        L.nxs_create.argtypes = [POINTER(c_void_p), ctypes.c_int, ALLOC_FN, FREE_FN, c_void_p]
        L.nxs_destroy.argtypes = [c_void_p]
        L.nxs_render_forward.argtypes = [c_void_p, POINTER(Gaussians), POINTER(Camera), c_int32,
                                         POINTER(RenderOpts), POINTER(Image),
                                         POINTER(c_void_p), c_void_p]
        L.nxs_render_backward.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p,
                                          POINTER(GaussiansGrad), c_void_p]
        L.nxs_state_release.argtypes = [c_void_p, c_void_p, c_void_p]
        L.nxs_forward_status.argtypes = [c_void_p, POINTER(c_int64)]
        L.nxs_render_forward_noalloc.argtypes = [c_void_p, POINTER(Gaussians), POINTER(Camera),
                                                 c_int32, POINTER(RenderOpts), POINTER(Image),
                                                 c_void_p]
        L.nxs_autotune.argtypes = [c_void_p, POINTER(Gaussians), POINTER(Camera), c_int32,
                                   POINTER(RenderOpts), POINTER(Image), ctypes.c_char_p,
                                   c_int32, POINTER(Tuning), c_void_p]
        L.nxs_set_workspace_limit.argtypes = [c_void_p, ctypes.c_size_t]
        L.nxs_workspace_bytes.argtypes = [c_void_p, POINTER(ctypes.c_size_t)]
        L.nxs_release_workspace.argtypes = [c_void_p]
        L.nxs_server_create.argtypes = [ctypes.c_int, ctypes.c_size_t, c_int32, c_int32,
                                        POINTER(c_void_p)]
        L.nxs_server_destroy.argtypes = [c_void_p]
        L.nxs_server_in_flight.argtypes = [c_void_p]
        L.nxs_server_workspace_bytes.argtypes = [c_void_p, POINTER(ctypes.c_size_t)]
        L.nxs_server_add_scene.argtypes = [c_void_p, POINTER(Gaussians), POINTER(c_int32)]
        L.nxs_server_submit.argtypes = [c_void_p, c_int32, POINTER(Camera), POINTER(RenderOpts),
                                        POINTER(Image), c_int64]
        L.nxs_server_step.argtypes = [c_void_p, c_int32, c_void_p, c_void_p, c_int32,
                                      POINTER(c_int32)]
        L.nxs_server_pending.argtypes = [c_void_p]
        L.nxs_server_last_error.argtypes = [c_void_p]
        L.nxs_pipeline_create.argtypes = [POINTER(c_void_p), ctypes.c_int, c_int32, ALLOC_FN,
                                          FREE_FN, c_void_p]
        L.nxs_pipeline_destroy.argtypes = [c_void_p]
        L.nxs_pipeline_render.argtypes = [c_void_p, POINTER(Gaussians), POINTER(Camera),
                                          c_int32, POINTER(RenderOpts), POINTER(Image), c_void_p]
        L.nxs_pipeline_join.argtypes = [c_void_p, c_void_p]
        L.nxs_pipeline_status.argtypes = [c_void_p, POINTER(c_int64)]
        L.nxs_pipeline_last_error.argtypes = [c_void_p]
        L.nxs_last_error.argtypes = [c_void_p]
        L.nxs_last_error.restype = ctypes.c_char_p
        L.nxs_set_timing.argtypes = [c_void_p, c_int32]
        L.nxs_inspect_stage_times.argtypes = [c_void_p, c_void_p, c_int32]
        L.nxs_inspect_counts.argtypes = [c_void_p, POINTER(c_int64), POINTER(c_int64)]
        L.nxs_inspect_instances.argtypes = [c_void_p, c_void_p, c_void_p, c_int64]
        L.nxs_inspect_ranges.argtypes = [c_void_p, c_void_p, c_int64]
        L.nxs_inspect_projection.argtypes = [c_void_p, c_int32, c_void_p, c_void_p, c_int64]
        L.nxs_inspect_slot_grads.argtypes = [c_void_p, c_void_p, c_int64]
        for name in SYMBOLS:
            if name in _NOT_STATUS:
                getattr(L, name).restype = _NOT_STATUS[name]
            else:
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _f32(t, name, shape_tail=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float32")
    return t


def scene_to_device(scene, device="cuda"):
    """Upload a synth.Scene's arrays as contiguous float32 GPU tensors."""
    f = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
    return {"means": f(scene.means), "scales": f(scene.scales), "quats": f(scene.quats),
            "opacities": f(scene.opacities), "sh": f(scene.sh),
            "sh_degree": int(scene.sh_degree)}


def make_camera(cam):
    """C camera struct from any object with R, t, fx, fy, cx, cy, znear, width, height."""
    c = Camera()
    R = np.asarray(cam.R, np.float32).reshape(9)
    t = np.asarray(cam.t, np.float32).reshape(3)
    for k in range(9):
        c.R[k] = float(R[k])
    for k in range(3):
        c.t[k] = float(t[k])
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.znear = float(getattr(cam, "znear", 0.01))
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def _make_gaussians(g):
    n = int(g["means"].shape[0])
    gs = Gaussians()
    gs.n, gs.sh_degree = n, int(g["sh_degree"])
    if n:
        gs.means = _f32(g["means"], "means").data_ptr()
        gs.scales = _f32(g["scales"], "scales").data_ptr()
        gs.quats = _f32(g["quats"], "quats").data_ptr()
        gs.opacities = _f32(g["opacities"], "opacities").data_ptr()
        gs.sh = _f32(g["sh"], "sh").data_ptr()
        K = (gs.sh_degree + 1) ** 2
        if tuple(g["sh"].shape[1:]) != (K, 3) or tuple(g["means"].shape[1:]) != (3,):
            raise ValueError("bad Gaussian array shapes")
    return gs


def _make_outputs(device, cams, outputs, overdraw):
    if outputs is not None:
        return outputs
    outputs = []
    for c in cams:
        H, W = int(c.height), int(c.width)
        outputs.append({
            "rgb": torch.empty((H, W, 3), dtype=torch.float32, device=device),
            "trans": torch.empty((H, W), dtype=torch.float32, device=device),
            "overdraw": (torch.empty((H, W), dtype=torch.int32, device=device)
                         if overdraw else None)})
    return outputs


def _make_image(o):
    img = Image()
    img.rgb = _f32(o["rgb"], "rgb").data_ptr()
    img.trans = _f32(o["trans"], "trans").data_ptr()
    od = o.get("overdraw")
    img.overdraw = od.data_ptr() if od is not None else None
    return img


def _make_opts(model=0, background=(0.0, 0.0, 0.0), alpha_min=0.0, t_eps=0.0, tile=(16, 16),
               lds_batch=0, param=0.0, schedule=0, deferred=False, instance_hint=0.0,
               sort_order=0):
    if isinstance(model, str):
        model = MODEL_IDS[model]
    if isinstance(schedule, str):
        schedule = SCHEDULES[schedule]
    if isinstance(sort_order, str):
        sort_order = SORT_ORDERS[sort_order]
    opts = RenderOpts()
    opts.model = int(model)
    for k in range(3):
        opts.background[k] = float(background[k])
    opts.alpha_min, opts.t_eps = float(alpha_min), float(t_eps)
    opts.tile_w, opts.tile_h = int(tile[0]), int(tile[1])
    opts.lds_batch = int(lds_batch)
    opts.param = float(param)
    opts.flags = FLAG_DEFERRED if deferred else 0
    opts.schedule = int(schedule)
    opts.instance_hint = float(instance_hint)
    opts.sort_order = int(sort_order)
    return opts


def _raw_stream(stream):
    return int(stream.cuda_stream) if stream is not None else 0


class TorchAllocator:
    """Device memory for a library context from PyTorch's caching allocator
    (the nxs_alloc_fn / nxs_free_fn callbacks of nxs_create).

    A block is allocated for the stream the library names and freed the
    way the library's free promises: in stream order on the stream it names.
    Freed on the stream it was allocated for, it goes straight back to the
    cache; freed on another stream, it is held until an event recorded on
    that stream has completed."""

    def __init__(self, device):
        self.device = device
        self.blocks = {}        # pointer -> raw stream it was allocated for
        self.deferred = []      # (event, pointer) freed on another stream
        self.alloc_cb = ALLOC_FN(self._alloc)
        self.free_cb = FREE_FN(self._free)

    def _stream(self, raw):
        if raw:
            return torch.cuda.ExternalStream(raw, device=self.device)
        return torch.cuda.default_stream(self.device)

    def _reap(self):
        keep = []
        for ev, p in self.deferred:
            if ev.query():
                torch.cuda.caching_allocator_delete(p)
            else:
                keep.append((ev, p))
        self.deferred = keep

    def _alloc(self, nbytes, stream, user):
        try:
            self._reap()
            raw = int(stream or 0)
            p = torch.cuda.caching_allocator_alloc(int(nbytes), self.device.index, raw)
            self.blocks[int(p)] = raw
            return int(p)
        except Exception:      # the library reports NXS_ENOMEM
            return None

    def _free(self, ptr, stream, user):
        try:
            raw0 = self.blocks.pop(int(ptr))
            raw = int(stream or 0)
            if raw == raw0:
                torch.cuda.caching_allocator_delete(int(ptr))
            else:
                ev = torch.cuda.Event()
                ev.record(self._stream(raw))
                self.deferred.append((ev, int(ptr)))
        except Exception:
            pass

    def drain(self):
        """After the context is gone: give back what waits on events."""
        if self.deferred:
            torch.cuda.synchronize(self.device)
            for _, p in self.deferred:
                torch.cuda.caching_allocator_delete(p)
            self.deferred = []

    @property
    def bytes_held(self):
        return len(self.blocks)


class FwdState:
    """What a forward kept for its backward (an nxs_fwd_state); released when
    garbage-collected, by release(), or when its Renderer closes."""

    def __init__(self, renderer, handle, shapes):
        self._r = weakref.ref(renderer)
        self._h = handle
        self.shapes = shapes              # [(H, W)] per view
        renderer._states.add(self)

    @property
    def handle(self):
        if not self._h:
            raise RuntimeError("this forward state has been released")
        return self._h

    def release(self, stream=None):
        r = self._r()
        if self._h and r is not None and r._ctx:
            if stream is None:
                stream = torch.cuda.current_stream(r.device)
            r._L.nxs_state_release(r._ctx, self._h, c_void_p(_raw_stream(stream)))
            r._states.discard(self)
        self._h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


class Renderer:
    """A library context on one GPU; render() enqueues on the current stream.

    allocator="torch" (default): the workspace comes from PyTorch's caching
    allocator; None: from the library's own stream-ordered pool."""

    def __init__(self, device=0, allocator="torch"):
        self._L = lib()
        self._ctx = c_void_p()
        self.device = torch.device("cuda", int(device))
        self._states = weakref.WeakSet()
        self._alloc = TorchAllocator(self.device) if allocator == "torch" else None
        if self._alloc is not None:
            st = self._L.nxs_create(byref(self._ctx), int(device), self._alloc.alloc_cb,
                                    self._alloc.free_cb, None)
        else:
            st = self._L.nxs_create(byref(self._ctx), int(device), ALLOC_FN(), FREE_FN(), None)
        if st != 0:
            raise NxsError(st, "nxs_create failed")
        self.last_state = None    # the state of the last render(keep_state=True)

    def close(self):
        if self._ctx:
            self.last_state = None
            for s in list(self._states):
                s._h = None       # nxs_destroy frees them
            self._L.nxs_destroy(self._ctx)
            self._ctx = c_void_p()
            if self._alloc is not None:
                self._alloc.drain()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != 0:
            msg = self._L.nxs_last_error(self._ctx)
            raise NxsError(st, msg.decode() if msg else "")

    def _marshal(self, g, cams, model, background, alpha_min, t_eps, tile, lds_batch,
                 outputs, overdraw, param, schedule, deferred, sort_order=0,
                 instance_hint=0.0):
        gs = _make_gaussians(g)
        V = len(cams)
        carr = (Camera * V)(*[make_camera(c) for c in cams])
        outputs = _make_outputs(self.device, cams, outputs, overdraw)
        imgs = (Image * V)(*[_make_image(o) for o in outputs])
        opts = _make_opts(model, background, alpha_min, t_eps, tile, lds_batch, param,
                          schedule, deferred, instance_hint, sort_order)
        return gs, carr, V, imgs, opts, outputs

    def render(self, g, cams, model=0, background=(0.0, 0.0, 0.0), alpha_min=0.0,
               t_eps=0.0, tile=(16, 16), lds_batch=0, outputs=None, overdraw=True,
               stream=None, param=0.0, keep_state=False, schedule=0, deferred=False,
               sort_order=0, instance_hint=0.0):
        """Render the Gaussians `g` (dict of GPU tensors, see scene_to_device) in
        every camera of `cams`.  Returns a list of dicts {rgb [H,W,3], trans [H,W],
        overdraw [H,W] int32} (or fills `outputs`, a list of such dicts).
        keep_state: keep a FwdState for backward() in self.last_state.
        deferred: do not wait for the instance count (NXS_FLAG_DEFERRED); check
        the outcome with status().  sort_order: "auto", "depth_first" or
        "tile_first" (nxs_sort_order)."""
        gs, carr, V, imgs, opts, outputs = self._marshal(
            g, cams, model, background, alpha_min, t_eps, tile, lds_batch, outputs, overdraw,
            param, schedule, deferred, sort_order, instance_hint)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        h = c_void_p()
        st = self._L.nxs_render_forward(self._ctx, byref(gs), carr, V, byref(opts), imgs,
                                        byref(h) if keep_state else None,
                                        c_void_p(stream.cuda_stream))
        self._check(st)
        if keep_state:
            self.last_state = FwdState(self, h, [(int(c.height), int(c.width)) for c in cams])
        return outputs

    def render_noalloc(self, g, cams, outputs, model=0, background=(0.0, 0.0, 0.0),
                       alpha_min=0.0, t_eps=0.0, tile=(16, 16), lds_batch=0, param=0.0,
                       schedule=0, stream=None):
        """The same render through nxs_render_forward_noalloc: the library
        allocates nothing (its workspace is a fixed 64 MiB scratch per
        device); `outputs` must be given (a list of dicts as render returns)."""
        gs, carr, V, imgs, opts, outputs = self._marshal(
            g, cams, model, background, alpha_min, t_eps, tile, lds_batch, outputs, True,
            param, schedule, False)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self._check(self._L.nxs_render_forward_noalloc(self._ctx, byref(gs), carr, V,
                                                       byref(opts), imgs,
                                                       c_void_p(stream.cuda_stream)))
        return outputs

    def workspace_bytes(self):
        """Device workspace the context holds (bytes; states not counted)."""
        b = ctypes.c_size_t()
        self._check(self._L.nxs_workspace_bytes(self._ctx, byref(b)))
        return int(b.value)

    def status(self):
        """Outcome of the deferred renders since the last call (nxs_forward_status):
        raises NxsError(NXS_ECAPACITY) if any outgrew the workspace (the context
        has then grown; render them again); returns 0 otherwise."""
        need = c_int64()
        self._check(self._L.nxs_forward_status(self._ctx, byref(need)))
        return need.value

    def autotune(self, g, cams, model=0, cache_path=None, reps=5, outputs=None, stream=None,
                 background=(0.0, 0.0, 0.0), alpha_min=0.0, t_eps=0.0, param=0.0):
        """Measured best tile shape and composite schedule for this workload
        (see nxs_autotune).  Returns {"tile": (w, h), "schedule": name, "ms": t}."""
        gs, carr, V, imgs, opts, outputs = self._marshal(
            g, cams, model, background, alpha_min, t_eps, (16, 16), 0, outputs, True, param,
            False, 0)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        res = Tuning()
        path = None if cache_path is None else str(cache_path).encode()
        st = self._L.nxs_autotune(self._ctx, byref(gs), carr, V, byref(opts), imgs, path,
                                  int(reps), byref(res), c_void_p(stream.cuda_stream))
        self._check(st)
        name = {v: k for k, v in SCHEDULES.items()}[res.schedule]
        order = {v: k for k, v in SORT_ORDERS.items()}[res.sort_order]
        return {"tile": (res.tile_w, res.tile_h), "schedule": name,
                "lds_batch": int(res.lds_batch), "sort_order": order, "ms": float(res.ms)}

    def backward(self, g, dL_drgb, dL_dtrans=None, stream=None, state=None):
        """Gradients of the Gaussians (dict of tensors shaped like `g`) from the
        upstream gradients of a forward that kept its state (`state`, default
        the last render(keep_state=True)): dL_drgb a list of [H,W,3] per view,
        dL_dtrans None or a list of [H,W] (entries may be None)."""
        state = self.last_state if state is None else state
        if state is None:
            raise ValueError("no forward state: render with keep_state=True first")
        shapes = state.shapes
        V = len(dL_drgb)
        if V != len(shapes):
            raise ValueError(f"{V} upstream gradients for {len(shapes)} views")
        if dL_dtrans is not None and len(dL_dtrans) != V:
            raise ValueError("dL_dtrans needs one entry per view")
        keep = []
        for v, (H, W) in enumerate(shapes):
            t = _f32(dL_drgb[v].contiguous(), "dL_drgb")
            if tuple(t.shape) != (H, W, 3):
                raise ValueError(f"view {v}: dL_drgb must be [{H},{W},3]")
            keep.append(t)
            if dL_dtrans is not None and dL_dtrans[v] is not None:
                t = _f32(dL_dtrans[v].contiguous(), "dL_dtrans")
                if tuple(t.shape) != (H, W):
                    raise ValueError(f"view {v}: dL_dtrans must be [{H},{W}]")
                keep.append(t)
            else:
                keep.append(None)
        rgb_ptrs = (c_void_p * V)(*[keep[2 * v].data_ptr() for v in range(V)])
        tr_ptrs = None
        if dL_dtrans is not None:
            tr_ptrs = (c_void_p * V)(*[(keep[2 * v + 1].data_ptr()
                                        if keep[2 * v + 1] is not None else None)
                                       for v in range(V)])
        out = {k: torch.empty_like(g[k]) for k in ("means", "scales", "quats", "opacities", "sh")}
        gg = GaussiansGrad(out["means"].data_ptr(), out["scales"].data_ptr(),
                           out["quats"].data_ptr(), out["opacities"].data_ptr(),
                           out["sh"].data_ptr())
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        elif stream != torch.cuda.current_stream(self.device):
            for t in keep:
                if t is not None:
                    t.record_stream(stream)
        st = self._L.nxs_render_backward(self._ctx, state.handle, rgb_ptrs, tr_ptrs, byref(gg),
                                         c_void_p(stream.cuda_stream))
        self._check(st)
        return out

    # -------------------------------------------------------- inspection
    STAGES = ("project", "depth_sort", "emit", "tile_sort", "ranges", "composite")

    def measure_peaks(self, stream=None):
        """Measured FP32 FMA rate (TFLOP/s, non-packed) and copy bandwidth
        (GB/s) of this GPU (nxs_measure_peaks)."""
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        fma, copy = ctypes.c_double(0.0), ctypes.c_double(0.0)
        self._check(self._L.nxs_measure_peaks(self._ctx, byref(fma), byref(copy),
                                              c_void_p(stream.cuda_stream)))
        return {"fp32_fma_tflops": fma.value, "copy_gbs": copy.value}

    def set_timing(self, enable=True):
        self._check(self._L.nxs_set_timing(self._ctx, int(bool(enable))))

    def stage_times(self):
        """Milliseconds per stage of the last render (needs set_timing(True))."""
        ms = np.zeros(len(self.STAGES), np.float32)
        self._check(self._L.nxs_inspect_stage_times(self._ctx, ms.ctypes.data, ms.size))
        return dict(zip(self.STAGES, ms.astype(float).tolist()))

    def counts(self):
        m, t = c_int64(), c_int64()
        self._check(self._L.nxs_inspect_counts(self._ctx, byref(m), byref(t)))
        return m.value, t.value

    def instances(self):
        m, _ = self.counts()
        keys = np.zeros(max(m, 1), np.uint64)
        ids = np.zeros(max(m, 1), np.int32)
        self._check(self._L.nxs_inspect_instances(self._ctx, keys.ctypes.data,
                                                  ids.ctypes.data, keys.size))
        return keys[:m], ids[:m]

    def ranges(self):
        _, t = self.counts()
        r = np.zeros(2 * max(t, 1), np.int32)
        self._check(self._L.nxs_inspect_ranges(self._ctx, r.ctypes.data, r.size))
        return r[:2 * t].reshape(t, 2)

    def slot_grads(self, n, n_views):
        """Per-slot sums of the last backward: [n_views, n, 9] float32 with
        dLoss/d(aleph, u, v, A, B, C, r, g, b) (nxs_inspect_slot_grads)."""
        out = np.zeros(9 * max(n * n_views, 1), np.float32)
        self._check(self._L.nxs_inspect_slot_grads(self._ctx, out.ctypes.data, out.size))
        return out[:9 * n * n_views].reshape(n_views, n, 9)

    def projection(self, view, n):
        d = np.zeros(max(n, 1), np.uint32)
        r = np.zeros(4 * max(n, 1), np.int32)
        self._check(self._L.nxs_inspect_projection(self._ctx, int(view), d.ctypes.data,
                                                   r.ctypes.data, max(n, 1)))
        return d[:n], r[:4 * n].reshape(n, 4)


class Pipeline:
    """Renders dealt in turn to `lanes` contexts on streams of their own
    (nxs_pipeline_*): consecutive renders overlap on the device.  render()
    returns its outputs, complete once join() has made a stream wait for the
    lanes and that stream has reached the join; renders in flight at the same
    time need distinct outputs.  A lane has no instance buffers before its
    first render: a waiting render (deferred=False) sizes it, else status()
    reports the deferred render that outgrew it (every lane then grows, and
    the render succeeds when repeated)."""

    def __init__(self, device=0, lanes=3, allocator="torch"):
        self._L = lib()
        self._p = c_void_p()
        self.device = torch.device("cuda", int(device))
        self._alloc = TorchAllocator(self.device) if allocator == "torch" else None
        a = (self._alloc.alloc_cb, self._alloc.free_cb) if self._alloc else (ALLOC_FN(), FREE_FN())
        st = self._L.nxs_pipeline_create(byref(self._p), int(device), int(lanes), a[0], a[1], None)
        if st != 0:
            raise NxsError(st, "nxs_pipeline_create failed")

    def close(self):
        if self._p:
            self._L.nxs_pipeline_destroy(self._p)
            self._p = c_void_p()
            if self._alloc is not None:
                self._alloc.drain()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != 0:
            msg = self._L.nxs_pipeline_last_error(self._p)
            raise NxsError(st, msg.decode() if msg else "")

    def render(self, g, cams, model=0, outputs=None, stream=None, background=(0.0, 0.0, 0.0),
               alpha_min=0.0, t_eps=0.0, tile=(16, 16), lds_batch=0, overdraw=True, param=0.0,
               schedule=0, deferred=True, sort_order=0, instance_hint=0.0):
        gs = _make_gaussians(g)
        V = len(cams)
        carr = (Camera * V)(*[make_camera(c) for c in cams])
        outputs = _make_outputs(self.device, cams, outputs, overdraw)
        imgs = (Image * V)(*[_make_image(o) for o in outputs])
        opts = _make_opts(model, background, alpha_min, t_eps, tile, lds_batch, param,
                          schedule, deferred, instance_hint, sort_order)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self._check(self._L.nxs_pipeline_render(self._p, byref(gs), carr, V, byref(opts), imgs,
                                                c_void_p(stream.cuda_stream)))
        return outputs

    def join(self, stream=None):
        """Make `stream` (default: the current one) wait for every render so far."""
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self._check(self._L.nxs_pipeline_join(self._p, c_void_p(stream.cuda_stream)))

    def status(self):
        """nxs_pipeline_status: raises NxsError(NXS_ECAPACITY) if a deferred
        render outgrew its lane (render it again); returns the largest count."""
        need = c_int64()
        self._check(self._L.nxs_pipeline_status(self._p, byref(need)))
        return need.value


class Server:
    """Continuous-batching render server over resident scenes (nxs_server_*),
    with `n_slots` batches in flight at once.

    add_scene(g) keeps a scene's device arrays alive; submit() queues one view
    and returns its output images (written before a step reports the request);
    step(wait) serves and returns [(tag, status, outputs)]."""

    def __init__(self, device=0, workspace_budget=0, max_batch_views=16, n_slots=2):
        self._L = lib()
        self._s = c_void_p()
        st = self._L.nxs_server_create(int(device), int(workspace_budget), int(max_batch_views),
                                       int(n_slots), byref(self._s))
        if st != 0:
            raise NxsError(st, "nxs_server_create failed")
        self.device = torch.device("cuda", int(device))
        self._scenes = []
        self._inflight = {}
        self._cap = int(max_batch_views or 16) + int(n_slots or 2) + 8
        self._tags = (c_int64 * self._cap)()
        self._status = (c_int32 * self._cap)()

    def close(self):
        if self._s:
            self._L.nxs_server_destroy(self._s)
            self._s = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != 0:
            msg = self._L.nxs_server_last_error(self._s)
            raise NxsError(st, msg.decode() if msg else "")

    def add_scene(self, g):
        sid = c_int32()
        self._check(self._L.nxs_server_add_scene(self._s, byref(_make_gaussians(g)), byref(sid)))
        self._scenes.append(g)
        return sid.value

    def submit(self, scene, cam, tag, outputs=None, overdraw=False, **opts):
        tag = int(tag)
        if tag in self._inflight:
            raise ValueError(f"tag {tag} is already pending")
        out = _make_outputs(self.device, [cam], None if outputs is None else [outputs],
                            overdraw)[0]
        img = _make_image(out)
        self._check(self._L.nxs_server_submit(self._s, int(scene), byref(make_camera(cam)),
                                              byref(_make_opts(**opts)), byref(img), tag))
        self._inflight[tag] = out
        return out

    @property
    def pending(self):
        """Requests queued and not yet started."""
        return int(self._L.nxs_server_pending(self._s))

    @property
    def in_flight(self):
        """Requests started on a slot and not yet reported."""
        return int(self._L.nxs_server_in_flight(self._s))

    def step(self, wait=True):
        n = c_int32()
        self._check(self._L.nxs_server_step(self._s, int(bool(wait)), self._tags, self._status,
                                            self._cap, byref(n)))
        return [(int(self._tags[k]), int(self._status[k]), self._inflight.pop(int(self._tags[k])))
                for k in range(n.value)]

    def drain(self):
        """Step until nothing is pending or in flight; returns all completions."""
        done = []
        while self.pending or self.in_flight:
            done += self.step(wait=True)
        return done

    def workspace_bytes(self):
        b = ctypes.c_size_t()
        self._check(self._L.nxs_server_workspace_bytes(self._s, byref(b)))
        return int(b.value)


class RenderFunction(torch.autograd.Function):
    """Differentiable render: (means, scales, quats, opacities, sh) -> per view
    (rgb [H,W,3], trans [H,W]).  The backward is the library's path replay
    over the forward state this render kept (other renders may run between
    the two); the state is released after the backward."""

    @staticmethod
    def forward(ctx, renderer, cams, opts, means, scales, quats, opacities, sh):
        g = {"means": means.detach().contiguous(), "scales": scales.detach().contiguous(),
             "quats": quats.detach().contiguous(), "opacities": opacities.detach().contiguous(),
             "sh": sh.detach().contiguous(),
             "sh_degree": int(round(math.sqrt(sh.shape[1]))) - 1}
        outs = renderer.render(g, cams, keep_state=True, overdraw=False, **opts)
        # this forward's own state: other forwards may run before its backward
        ctx.renderer, ctx.g, ctx.state = renderer, g, renderer.last_state
        renderer.last_state = None
        ctx.shapes = [(o["rgb"].shape, o["trans"].shape) for o in outs]
        return tuple(o["rgb"] for o in outs) + tuple(o["trans"] for o in outs)

    @staticmethod
    def backward(ctx, *grads):
        r = ctx.renderer
        V = len(ctx.shapes)
        d_rgb = [gr if gr is not None else torch.zeros(sh[0], device=r.device)
                 for gr, sh in zip(grads[:V], ctx.shapes)]
        d_tr = list(grads[V:])
        if all(t is None for t in d_tr):
            d_tr = None
        gr = r.backward(ctx.g, d_rgb, d_tr, state=ctx.state)
        ctx.state.release()
        return (None, None, None, gr["means"], gr["scales"], gr["quats"], gr["opacities"],
                gr["sh"])


def render(renderer, cams, means, scales, quats, opacities, sh, **opts):
    """Differentiable multi-view render; returns (list of rgb, list of trans)."""
    out = RenderFunction.apply(renderer, list(cams), opts, means, scales, quats, opacities, sh)
    V = len(cams)
    return list(out[:V]), list(out[V:])
