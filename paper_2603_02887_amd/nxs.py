"""Python binding of libnxs (ctypes): argument marshalling only.

Every step of the render runs in the HIP library; this module checks that
tensors are on the GPU, float32 and contiguous, fills the C structs of
include/nxs.h and passes device pointers and the current HIP stream.
Loading fails loudly when libnxs.so has not been built.
"""
import ctypes
import math
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
           "nxs_last_error",
           "nxs_set_timing", "nxs_inspect_stage_times", "nxs_inspect_counts", "nxs_inspect_instances", "nxs_inspect_ranges",
           "nxs_inspect_projection"]


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
                ("lds_batch", c_int32), ("param", c_float), ("keep_state", c_int32)]


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
        L.nxs_create.argtypes = [POINTER(c_void_p), ctypes.c_int]
        L.nxs_destroy.argtypes = [c_void_p]
        L.nxs_render_forward.argtypes = [c_void_p, POINTER(Gaussians), POINTER(Camera), c_int32,
                                         POINTER(RenderOpts), POINTER(Image), c_void_p]
        L.nxs_render_backward.argtypes = [c_void_p, c_void_p, c_void_p,
                                          POINTER(GaussiansGrad), c_void_p]
        L.nxs_last_error.argtypes = [c_void_p]
        L.nxs_last_error.restype = ctypes.c_char_p
        L.nxs_set_timing.argtypes = [c_void_p, c_int32]
        L.nxs_inspect_stage_times.argtypes = [c_void_p, c_void_p, c_int32]
        L.nxs_inspect_counts.argtypes = [c_void_p, POINTER(c_int64), POINTER(c_int64)]
        L.nxs_inspect_instances.argtypes = [c_void_p, c_void_p, c_void_p, c_int64]
        L.nxs_inspect_ranges.argtypes = [c_void_p, c_void_p, c_int64]
        L.nxs_inspect_projection.argtypes = [c_void_p, c_int32, c_void_p, c_void_p, c_int64]
        for name in SYMBOLS:
            if name not in ("nxs_last_error",):
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


class Renderer:
    """A library context on one GPU; render() enqueues on the current stream."""

    def __init__(self, device=0):
        self._L = lib()
        self._ctx = c_void_p()
        st = self._L.nxs_create(byref(self._ctx), int(device))
        if st != 0:
            raise NxsError(st, "nxs_create failed")
        self.device = torch.device("cuda", int(device))
        self.generation = 0      # forwards issued on this context
        self._last_shapes = []

    def close(self):
        if self._ctx:
            self._L.nxs_destroy(self._ctx)
            self._ctx = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != 0:
            msg = self._L.nxs_last_error(self._ctx)
            raise NxsError(st, msg.decode() if msg else "")

    def render(self, g, cams, model=0, background=(0.0, 0.0, 0.0), alpha_min=0.0,
               t_eps=0.0, tile=(16, 16), lds_batch=0, outputs=None, overdraw=True,
               stream=None, param=0.0, keep_state=False):
        """Render the Gaussians `g` (dict of GPU tensors, see scene_to_device) in
        every camera of `cams`.  Returns a list of dicts {rgb [H,W,3], trans [H,W],
        overdraw [H,W] int32} (or fills `outputs`, a list of such dicts)."""
        if isinstance(model, str):
            model = MODEL_IDS[model]
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
        V = len(cams)
        carr = (Camera * V)(*[make_camera(c) for c in cams])
        if outputs is None:
            outputs = []
            for c in cams:
                H, W = int(c.height), int(c.width)
                outputs.append({
                    "rgb": torch.empty((H, W, 3), dtype=torch.float32, device=self.device),
                    "trans": torch.empty((H, W), dtype=torch.float32, device=self.device),
                    "overdraw": (torch.empty((H, W), dtype=torch.int32, device=self.device)
                                 if overdraw else None)})
        imgs = (Image * V)()
        for k, o in enumerate(outputs):
            imgs[k].rgb = _f32(o["rgb"], "rgb").data_ptr()
            imgs[k].trans = _f32(o["trans"], "trans").data_ptr()
            od = o.get("overdraw")
            imgs[k].overdraw = od.data_ptr() if od is not None else None
        opts = RenderOpts()
        opts.model = int(model)
        for k in range(3):
            opts.background[k] = float(background[k])
        opts.alpha_min, opts.t_eps = float(alpha_min), float(t_eps)
        opts.tile_w, opts.tile_h = int(tile[0]), int(tile[1])
        opts.lds_batch = int(lds_batch)
        opts.param = float(param)
        opts.keep_state = int(bool(keep_state))
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        st = self._L.nxs_render_forward(self._ctx, byref(gs), carr, V, byref(opts), imgs,
                                        c_void_p(stream.cuda_stream))
        self.generation += 1
        self._last_shapes = [(int(c.height), int(c.width)) for c in cams]
        self._check(st)
        return outputs

    def backward(self, g, dL_drgb, dL_dtrans=None, stream=None):
        """Gradients of the Gaussians (dict of tensors shaped like `g`) from the
        upstream gradients of the last forward, which had keep_state=True:
        dL_drgb a list of [H,W,3] per view, dL_dtrans None or a list of [H,W]
        (entries may be None)."""
        V = len(dL_drgb)
        if V != len(self._last_shapes):
            raise ValueError(f"{V} upstream gradients for {len(self._last_shapes)} views")
        if dL_dtrans is not None and len(dL_dtrans) != V:
            raise ValueError("dL_dtrans needs one entry per view")
        keep = []
        for v, (H, W) in enumerate(self._last_shapes):
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
        st = self._L.nxs_render_backward(self._ctx, rgb_ptrs, tr_ptrs, byref(gg),
                                         c_void_p(stream.cuda_stream))
        self._check(st)
        return out

    # -------------------------------------------------------- inspection
    STAGES = ("project", "depth_sort", "emit", "tile_sort", "gather", "composite")

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

    def projection(self, view, n):
        d = np.zeros(max(n, 1), np.uint32)
        r = np.zeros(4 * max(n, 1), np.int32)
        self._check(self._L.nxs_inspect_projection(self._ctx, int(view), d.ctypes.data,
                                                   r.ctypes.data, max(n, 1)))
        return d[:n], r[:4 * n].reshape(n, 4)


class RenderFunction(torch.autograd.Function):
    """Differentiable render: (means, scales, quats, opacities, sh) -> per view
    (rgb [H,W,3], trans [H,W]).  The backward is the library's path replay; it
    must run before the next forward on the same Renderer."""

    @staticmethod
    def forward(ctx, renderer, cams, opts, means, scales, quats, opacities, sh):
        g = {"means": means.detach().contiguous(), "scales": scales.detach().contiguous(),
             "quats": quats.detach().contiguous(), "opacities": opacities.detach().contiguous(),
             "sh": sh.detach().contiguous(),
             "sh_degree": int(round(math.sqrt(sh.shape[1]))) - 1}
        outs = renderer.render(g, cams, keep_state=True, overdraw=False, **opts)
        ctx.renderer, ctx.g, ctx.gen = renderer, g, renderer.generation
        ctx.shapes = [(o["rgb"].shape, o["trans"].shape) for o in outs]
        return tuple(o["rgb"] for o in outs) + tuple(o["trans"] for o in outs)

    @staticmethod
    def backward(ctx, *grads):
        r = ctx.renderer
        if r.generation != ctx.gen:
            raise RuntimeError("another forward ran on this Renderer since this one; "
                               "its backward state is gone")
        V = len(ctx.shapes)
        d_rgb = [gr if gr is not None else torch.zeros(sh[0], device=r.device)
                 for gr, sh in zip(grads[:V], ctx.shapes)]
        d_tr = list(grads[V:])
        if all(t is None for t in d_tr):
            d_tr = None
        gr = r.backward(ctx.g, d_rgb, d_tr)
        return (None, None, None, gr["means"], gr["scales"], gr["quats"], gr["opacities"],
                gr["sh"])


def render(renderer, cams, means, scales, quats, opacities, sh, **opts):
    """Differentiable multi-view render; returns (list of rgb, list of trans)."""
    out = RenderFunction.apply(renderer, list(cams), opts, means, scales, quats, opacities, sh)
    V = len(cams)
    return list(out[:V]), list(out[V:])
