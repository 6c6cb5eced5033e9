"""ctypes binding of the C ABI in include/rgx.h (argument marshalling only).

Every step of the path runs in librgx.so; this module converts Python
objects into the C structures and passes device pointers (torch tensors'
data_ptr) and the current HIP stream.  It raises if the library is missing:
there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("RGX_LIBRARY", os.path.join(HERE, "librgx.so"))

RGX_OK = 0
NSTAT = 16
STAT_NAMES = ("Q", "P", "samples", "segments", "closest", "box_only", "nodes", "leaves",
              "windows", "chunked", "cand", "cand_hit", "kcyc_collect", "kcyc_closest",
              "kcyc_tile", "t_end")
STAT_T_END = 15   # float bits
TOTAL_NAMES = ("rays", "Q", "P", "samples", "segments", "closest", "nodes", "box_only",
               "chunked", "inactive", "unrecorded")   # RGX_TOT_* order


class RgxError(RuntimeError):
    pass


class Gaussians(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("means", C.c_void_p),
                ("log_scales", C.c_void_p), ("quats", C.c_void_p), ("density", C.c_void_p),
                ("sh", C.c_void_p), ("n_sg", C.c_int32), ("sg", C.c_void_p)]


class BuildOpts(C.Structure):
    _fields_ = [("sigma_eps", C.c_float), ("morton_bits", C.c_int32)]


class Camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("cam_to_world", C.c_float * 12),
                ("t_near", C.c_float), ("t_far", C.c_float)]


class RenderOpts(C.Structure):
    _fields_ = [("adaptive", C.c_int32), ("dt", C.c_float), ("dt_min", C.c_float),
                ("dt_max", C.c_float), ("beta", C.c_float), ("n_s", C.c_int32),
                ("t_eps", C.c_float), ("ess", C.c_int32), ("brute_force", C.c_int32),
                ("ray_order", C.c_int32), ("tile_w", C.c_int32), ("tile_h", C.c_int32),
                ("persistent", C.c_int32), ("window_segments", C.c_int32),
                ("bg", C.c_float * 3), ("no_record", C.c_int32),
                ("no_sample_record", C.c_int32)]


class Grads(C.Structure):
    _fields_ = [("n", C.c_int64), ("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("density", C.c_void_p), ("sh", C.c_void_p), ("sg", C.c_void_p),
                ("accumulate", C.c_int32),
                ("densify", C.c_void_p), ("densify_views", C.c_void_p)]


class AdamGroup(C.Structure):
    _fields_ = [("n", C.c_int64), ("param", C.c_void_p), ("grad", C.c_void_p), ("m", C.c_void_p),
                ("v", C.c_void_p), ("lr", C.c_float)]


EXPORTS = ("rgx_create", "rgx_destroy", "rgx_build_bvh", "rgx_bvh_destroy", "rgx_bvh_size",
           "rgx_render_forward", "rgx_render_backward", "rgx_fwd_destroy", "rgx_sync_stats",
           "rgx_false_positives", "rgx_dump_hits", "rgx_bvh_debug",
           "rgx_error_flags", "rgx_set_kernel_timing", "rgx_kernel_times", "rgx_isotropic_loss",
           "rgx_isotropic_loss_noalloc", "rgx_adam_step",
           "rgx_backward_replayed", "rgx_status_string", "rgx_last_error", "rgx_set_record_limit")

KERNEL_KINDS = ("build", "forward", "backward", "finalize")   # RGX_KERN_* order

_LIB = None


def load():
    """Load librgx.so (built in-tree by build.py); raises if it is absent."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RgxError(f"{LIB_PATH} is missing: build it with paper_2509_07782_amd/build.py")
    L = C.CDLL(LIB_PATH)
    vp, st = C.c_void_p, C.c_int
    L.rgx_create.argtypes = [C.c_int, C.POINTER(vp)]
    L.rgx_create.restype = st
    L.rgx_destroy.argtypes = [vp]
    L.rgx_destroy.restype = None
    L.rgx_build_bvh.argtypes = [vp, C.POINTER(Gaussians), C.POINTER(BuildOpts), C.POINTER(vp), vp]
    L.rgx_build_bvh.restype = st
    L.rgx_bvh_destroy.argtypes = [vp]
    L.rgx_bvh_destroy.restype = None
    L.rgx_bvh_size.argtypes = [vp]
    L.rgx_bvh_size.restype = C.c_int64
    L.rgx_render_forward.argtypes = [vp, vp, C.POINTER(Camera), C.c_int32, C.POINTER(RenderOpts),
                                     vp, vp, vp, C.POINTER(vp), vp]
    L.rgx_render_forward.restype = st
    L.rgx_render_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp, C.POINTER(Grads), vp]
    L.rgx_render_backward.restype = st
    L.rgx_fwd_destroy.argtypes = [vp]
    L.rgx_fwd_destroy.restype = None
    L.rgx_sync_stats.argtypes = [vp, vp, C.POINTER(C.c_int64), vp]
    L.rgx_sync_stats.restype = st
    L.rgx_false_positives.argtypes = [vp, vp, C.POINTER(Camera), vp, C.c_int32, vp, vp, vp]
    L.rgx_false_positives.restype = st
    L.rgx_dump_hits.argtypes = [vp, vp, C.POINTER(Camera), C.POINTER(RenderOpts), vp, C.c_int32,
                                C.c_int32, vp, vp, vp, vp]
    L.rgx_dump_hits.restype = st
    L.rgx_bvh_debug.argtypes = [vp, vp, vp, vp, vp, vp, vp, C.POINTER(C.c_int64), vp]
    L.rgx_bvh_debug.restype = st
    L.rgx_error_flags.argtypes = [vp, C.POINTER(C.c_int32), vp]
    L.rgx_error_flags.restype = st
    L.rgx_isotropic_loss.argtypes = [vp, C.c_int64, vp, C.c_float, vp, vp, C.c_int32, vp]
    L.rgx_isotropic_loss.restype = st
    L.rgx_isotropic_loss_noalloc.argtypes = [vp, C.c_int64, vp, C.c_float, vp, vp, C.c_int32, vp]
    L.rgx_isotropic_loss_noalloc.restype = st
    L.rgx_adam_step.argtypes = [vp, C.POINTER(AdamGroup), C.c_int32, vp, C.c_float, C.c_float,
                                C.c_float, vp]
    L.rgx_adam_step.restype = st
    L.rgx_set_kernel_timing.argtypes = [vp, C.c_int32]
    L.rgx_set_kernel_timing.restype = st
    L.rgx_kernel_times.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int32]
    L.rgx_kernel_times.restype = st
    L.rgx_backward_replayed.argtypes = [vp]
    L.rgx_backward_replayed.restype = C.c_int32
    L.rgx_set_record_limit.argtypes = [vp, C.c_int64]
    L.rgx_set_record_limit.restype = st
    L.rgx_status_string.argtypes = [st]
    L.rgx_status_string.restype = C.c_char_p
    L.rgx_last_error.argtypes = [vp]
    L.rgx_last_error.restype = C.c_char_p
    _LIB = L
    return L


def check(rc, ctx=None, what=""):
    if rc != RGX_OK:
        L = load()
        msg = L.rgx_status_string(rc).decode()
        detail = L.rgx_last_error(ctx).decode() if ctx else ""
        raise RgxError(f"{what}: {msg} ({rc}) {detail}")


def make_camera(cam) -> Camera:
    c = Camera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    flat = [float(v) for v in __import__("numpy").asarray(cam.cam_to_world, "float32").reshape(12)]
    for i in range(12):
        c.cam_to_world[i] = flat[i]
    c.t_near, c.t_far = float(cam.t_near), float(cam.t_far)
    return c


def camera_array(cams):
    arr = (Camera * len(cams))()
    for i, cam in enumerate(cams):
        arr[i] = make_camera(cam)
    return arr


def make_opts(o) -> RenderOpts:
    r = RenderOpts()
    r.adaptive = int(bool(o.adaptive))
    r.dt, r.dt_min, r.dt_max, r.beta = o.dt, o.dt_min, o.dt_max, o.beta
    r.n_s, r.t_eps, r.ess = int(o.n_s), float(o.t_eps), int(o.ess)
    r.brute_force = int(bool(o.brute_force))
    r.ray_order = int(o.ray_order)
    r.tile_w, r.tile_h = int(o.tile_w), int(o.tile_h)
    r.persistent = int(bool(o.persistent))
    r.window_segments = int(getattr(o, "window_segments", 0))
    for i in range(3):
        r.bg[i] = float(o.bg[i])
    r.no_record = int(bool(getattr(o, "no_record", False)))
    r.no_sample_record = int(bool(getattr(o, "no_sample_record", False)))
    return r


class Context:
    """Owns an rgx_context on one HIP device."""

    def __init__(self, device: int = 0):
        L = load()
        h = C.c_void_p()
        check(L.rgx_create(int(device), C.byref(h)), None, "rgx_create")
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            load().rgx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_kernel_timing(self, enable: bool):
        check(load().rgx_set_kernel_timing(self.h, int(bool(enable))), self.h, "set_kernel_timing")

    def kernel_times(self, reset: bool = True) -> dict:
        """{kind: (total ms, launches)} of the launches recorded since timing
        was enabled (or the last reset); waits for the recorded events."""
        n = len(KERNEL_KINDS)
        ms, cnt = (C.c_double * n)(), (C.c_int64 * n)()
        check(load().rgx_kernel_times(self.h, ms, cnt, int(bool(reset))), self.h, "kernel_times")
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(KERNEL_KINDS)}

    def set_record_limit(self, max_bytes: int):
        """Caps the record pool of later forwards given a state (0: no cap)."""
        check(load().rgx_set_record_limit(self.h, int(max_bytes)), self.h, "set_record_limit")

    def backward_replayed(self) -> bool:
        """Whether the last backward replayed its forward's closest-hit results."""
        return bool(load().rgx_backward_replayed(self.h))

    def error_flags(self, stream=0) -> int:
        f = C.c_int32(0)
        check(load().rgx_error_flags(self.h, C.byref(f), C.c_void_p(stream)), self.h, "error_flags")
        return int(f.value)


class BVH:
    """Owns an rgx_bvh; rebuilt in place by build()."""

    def __init__(self, ctx: Context):
        self.ctx = ctx
        self.h = C.c_void_p()

    def build(self, means, log_scales, quats, density, sh, sh_degree, sigma_eps=0.01,
              morton_bits=21, stream=0, sg=None):
        n_sg = 0 if sg is None else int(sg.shape[1])
        g = Gaussians(int(means.shape[0]), int(sh_degree), means.data_ptr(),
                      log_scales.data_ptr(), quats.data_ptr(), density.data_ptr(), sh.data_ptr(),
                      n_sg, None if sg is None else sg.data_ptr())
        o = BuildOpts(float(sigma_eps), int(morton_bits))
        check(load().rgx_build_bvh(self.ctx.h, C.byref(g), C.byref(o), C.byref(self.h),
                                   C.c_void_p(stream)), self.ctx.h, "rgx_build_bvh")
        self.n = int(means.shape[0])
        self.sh_degree = int(sh_degree)
        self.n_sg = n_sg
        return self

    def close(self):
        if self.h:
            load().rgx_bvh_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def debug(self, stream=0):
        """Host copies of keys, perm, leaf AABBs, binary nodes, 4-wide records
        and the active count."""
        import numpy as np
        n = self.n
        keys = np.zeros(n, np.uint64)
        perm = np.zeros(n, np.int32)
        aabb = np.zeros((n, 6), np.float32)
        nodes = np.zeros((max(n - 1, 1), 16), np.float32)
        nodes4 = np.zeros((max(n - 1, 1), 36), np.float32)
        na = C.c_int64(0)
        check(load().rgx_bvh_debug(self.ctx.h, self.h, keys.ctypes.data, perm.ctypes.data,
                                   aabb.ctypes.data, nodes.ctypes.data, nodes4.ctypes.data,
                                   C.byref(na), C.c_void_p(stream)), self.ctx.h, "rgx_bvh_debug")
        return keys, perm, aabb, nodes, nodes4, int(na.value)


def isotropic_loss(ctx: Context, log_scales, r0, loss, grad, accumulate=False, stream=0):
    """Loss (device scalar) and dL/d(log_scales) of the isotropic scale loss."""
    check(load().rgx_isotropic_loss(ctx.h, int(log_scales.shape[0]), log_scales.data_ptr(),
                                    float(r0), loss.data_ptr(), grad.data_ptr(),
                                    int(bool(accumulate)), C.c_void_p(stream)),
          ctx.h, "rgx_isotropic_loss")


def isotropic_loss_noalloc(ctx: Context, log_scales, r0, loss, grad, accumulate=False, stream=0):
    """Same as isotropic_loss, through the entry point that allocates nothing
    (fixed per-device workspace)."""
    check(load().rgx_isotropic_loss_noalloc(ctx.h, int(log_scales.shape[0]), log_scales.data_ptr(),
                                            float(r0), loss.data_ptr(), grad.data_ptr(),
                                            int(bool(accumulate)), C.c_void_p(stream)),
          ctx.h, "rgx_isotropic_loss_noalloc")


class ForwardState:
    """Owns an rgx_fwd: what one forward rendered and what its searches
    found, for the matching backward.  Reused in place by later forwards."""

    def __init__(self, ctx: Context):
        self.ctx = ctx
        self.h = C.c_void_p()

    def close(self):
        if self.h:
            load().rgx_fwd_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def totals(self, stream=0) -> dict:
        """Statistics totals of the forward (it must have been given stats)."""
        out = (C.c_int64 * len(TOTAL_NAMES))()
        check(load().rgx_sync_stats(self.ctx.h, self.h, out, C.c_void_p(stream)), self.ctx.h,
              "rgx_sync_stats")
        return {k: int(out[i]) for i, k in enumerate(TOTAL_NAMES)}


def adam_step(ctx: Context, groups, step, beta1=0.9, beta2=0.999, eps=1e-15, stream=0):
    """One Adam step; groups = [(param, grad, m, v, lr)] of contiguous float32
    device tensors, step an int32 device scalar advanced by the call."""
    arr = (AdamGroup * len(groups))()
    for i, (p, g, m, v, lr) in enumerate(groups):
        arr[i] = AdamGroup(int(p.numel()), p.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(),
                           float(lr))
    check(load().rgx_adam_step(ctx.h, arr, len(groups), step.data_ptr(), float(beta1), float(beta2),
                               float(eps), C.c_void_p(stream)), ctx.h, "rgx_adam_step")


def render_forward(ctx: Context, bvh: BVH, cams, opts, out_rgb, out_T, stats=None, stream=0,
                   state: ForwardState | None = None):
    """Forward render; with `state` the forward records what its backward
    needs into it (state.h is created on first use, reused afterwards)."""
    arr = camera_array(cams)
    o = make_opts(opts)
    check(load().rgx_render_forward(ctx.h, bvh.h, arr, len(cams), C.byref(o), out_rgb.data_ptr(),
                                    out_T.data_ptr(), None if stats is None else stats.data_ptr(),
                                    None if state is None else C.byref(state.h),
                                    C.c_void_p(stream)), ctx.h, "rgx_render_forward")


def render_backward(ctx: Context, bvh: BVH, state: ForwardState, out_rgb, out_T, grad_rgb, grad_T,
                    grads, accumulate=False, stream=0, densify=None, densify_views=None):
    g = Grads(int(grads["means"].shape[0]), grads["means"].data_ptr(),
              grads["log_scales"].data_ptr(), grads["quats"].data_ptr(),
              grads["density"].data_ptr(), grads["sh"].data_ptr(),
              grads["sg"].data_ptr() if grads.get("sg") is not None else None,
              int(bool(accumulate)),
              None if densify is None else densify.data_ptr(),
              None if densify_views is None else densify_views.data_ptr())
    check(load().rgx_render_backward(ctx.h, bvh.h, state.h, out_rgb.data_ptr(), out_T.data_ptr(),
                                     grad_rgb.data_ptr(),
                                     None if grad_T is None else grad_T.data_ptr(), C.byref(g),
                                     C.c_void_p(stream)), ctx.h, "rgx_render_backward")


def false_positives(ctx: Context, bvh: BVH, cam, pix, t_end, count, stream=0):
    """Whole-ray AABB false positives of the listed pixels' rays over
    [t_near, t_end] (int32 counts into `count`)."""
    c = make_camera(cam)
    check(load().rgx_false_positives(ctx.h, bvh.h, C.byref(c), pix.data_ptr(), int(pix.numel()),
                                     t_end.data_ptr(), count.data_ptr(), C.c_void_p(stream)),
          ctx.h, "rgx_false_positives")


def dump_hits(ctx: Context, bvh: BVH, cam, opts, pix, cap, seg_a, ids, count, stream=0):
    c = make_camera(cam)
    o = make_opts(opts)
    check(load().rgx_dump_hits(ctx.h, bvh.h, C.byref(c), C.byref(o), pix.data_ptr(),
                               int(pix.numel()), int(cap), seg_a.data_ptr(), ids.data_ptr(),
                               count.data_ptr(), C.c_void_p(stream)), ctx.h, "rgx_dump_hits")
