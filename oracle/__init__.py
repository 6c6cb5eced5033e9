"""CPU FP64 oracle for Gaussian-based volume ray marching (RayGaussX).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg use this package; the GPU library never imports, links or
calls it, and it shares no code with the GPU path.

The arithmetic lives in `oracle.c` (plain C, double precision, every ray
against every Gaussian); `geometry.py` holds closed forms of Sec. 3.4 and
Supp. B.  This module is the ctypes wrapper.  Scenes are dicts of arrays as
drawn by the input generators; cameras are objects with width, height, fx,
fy, cx, cy, cam_to_world [3,4], t_near and t_far.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

N_STATS = 5
STAT_NAMES = ("Q", "P", "samples", "segments", "closest")


class _Scene(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32),
                ("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("density", C.c_void_p), ("sh", C.c_void_p), ("n_sg", C.c_int32),
                ("sg", C.c_void_p)]


class _Camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_double),
                ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("c2w", C.c_double * 12), ("t_near", C.c_double), ("t_far", C.c_double)]


class _Opts(C.Structure):
    _fields_ = [("adaptive", C.c_int32), ("dt", C.c_double), ("dt_min", C.c_double),
                ("dt_max", C.c_double), ("beta", C.c_double), ("n_s", C.c_int32),
                ("t_eps", C.c_double), ("ess", C.c_int32), ("bg", C.c_double * 3),
                ("sigma_eps", C.c_double)]


@dataclasses.dataclass
class Opts:
    """Ray-marching options (Alg. 1 inputs; Eq. 5 constants)."""
    adaptive: bool = False
    dt: float = 0.0025
    dt_min: float = 0.005
    dt_max: float = 0.02
    beta: float = 1024.0
    n_s: int = 8
    t_eps: float = 1e-4
    ess: int = 1
    bg: tuple = (0.0, 0.0, 0.0)
    sigma_eps: float = 0.01


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = C.CDLL(path)
        vp = C.c_void_p
        L.orc_render.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera), C.POINTER(_Opts), vp,
                                 C.c_int64, vp, vp, vp, vp]
        L.orc_render.restype = C.c_int
        L.orc_backward.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera), C.POINTER(_Opts), vp,
                                   C.c_int64, vp, vp, vp, vp, vp, vp, vp, vp]
        L.orc_colour.argtypes = [C.POINTER(_Scene), C.c_int64, vp, C.c_int64, vp]
        L.orc_backward.restype = C.c_int
        L.orc_hits.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera), C.POINTER(_Opts), C.c_int64,
                               vp, vp, vp, C.c_int64, vp, C.c_int64]
        L.orc_hits.restype = C.c_int64
        L.orc_sh_basis.argtypes = [C.c_int32, vp, vp]
        L.orc_rays.argtypes = [C.POINTER(_Camera), vp, C.c_int64, vp, vp]
        L.orc_gaussians.argtypes = [C.POINTER(_Scene), C.c_double, vp, vp, vp, vp]
        L.orc_density_at.argtypes = [C.POINTER(_Scene), C.c_double, C.c_int64, vp, C.c_int64, vp]
        L.orc_num_threads.restype = C.c_int
        L.orc_false_positives.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera),
                                          C.POINTER(_Opts), vp, C.c_int64, vp, vp, vp]
        L.orc_false_positives.restype = C.c_int
        L.orc_chords.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera), C.c_double, C.c_int64, vp,
                                 C.c_int64, vp, vp, vp, vp]
        _LIB = L
    return _LIB


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class _SceneHold:
    """Keeps float64 copies alive while the C structure points at them.
    A scene may carry spherical-Gaussian lobes: "sg" [n, n_sg, 7] (amplitude
    rgb, axis xyz, sharpness)."""

    def __init__(self, scene):
        self.arrs = [_f64(scene[k]) for k in ("means", "log_scales", "quats", "density", "sh")]
        n = self.arrs[0].shape[0]
        sg = scene.get("sg")
        self.sg = None if sg is None or np.size(sg) == 0 else _f64(sg).reshape(n, -1, 7)
        n_sg = 0 if self.sg is None else self.sg.shape[1]
        self.s = _Scene(n, int(scene["sh_degree"]), *[a.ctypes.data for a in self.arrs], n_sg,
                        None if self.sg is None else self.sg.ctypes.data)


def _cam(cam) -> _Camera:
    c = _Camera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    m = np.asarray(cam.cam_to_world, np.float64).reshape(12)
    for i in range(12):
        c.c2w[i] = m[i]
    c.t_near, c.t_far = float(cam.t_near), float(cam.t_far)
    return c


def _opts(o: Opts) -> _Opts:
    r = _Opts()
    r.adaptive = int(bool(o.adaptive))
    r.dt, r.dt_min, r.dt_max, r.beta = o.dt, o.dt_min, o.dt_max, o.beta
    r.n_s, r.t_eps, r.ess = int(o.n_s), float(o.t_eps), int(o.ess)
    for i in range(3):
        r.bg[i] = float(o.bg[i])
    r.sigma_eps = float(o.sigma_eps)
    return r


def num_threads() -> int:
    return int(lib().orc_num_threads())


def render(scene, cam, opts: Opts, pix=None):
    """Colour [n,3], final transmittance [n], per-ray statistics [n,5]
    (Q, P, samples, segments, closest-hit calls) and decision margin [n] of
    the listed row-major pixels (all pixels when pix is None)."""
    if pix is None:
        pix = np.arange(cam.width * cam.height, dtype=np.int64)
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    n = pix.shape[0]
    sh = _SceneHold(scene)
    rgb = np.zeros((n, 3))
    T = np.zeros(n)
    st = np.zeros((n, N_STATS), np.int64)
    mg = np.zeros(n)
    c, o = _cam(cam), _opts(opts)
    rc = lib().orc_render(C.byref(sh.s), C.byref(c), C.byref(o), pix.ctypes.data, n,
                          rgb.ctypes.data, T.ctypes.data, st.ctypes.data, mg.ctypes.data)
    if rc != 0:
        raise ValueError(f"orc_render failed ({rc})")
    return rgb, T, st, mg


def backward(scene, cam, opts: Opts, pix, grad_rgb, grad_T=None):
    """Gradients (float64, user order) of the loss whose derivatives with
    respect to the listed pixels' colour / final transmittance are given."""
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    n = pix.shape[0]
    sh = _SceneHold(scene)
    g_rgb = _f64(grad_rgb).reshape(n, 3)
    g_T = None if grad_T is None else _f64(grad_T).reshape(n)
    N = sh.arrs[0].shape[0]
    out = dict(means=np.zeros((N, 3)), log_scales=np.zeros((N, 3)), quats=np.zeros((N, 4)),
               density=np.zeros(N), sh=np.zeros(sh.arrs[4].shape))
    if sh.sg is not None:
        out["sg"] = np.zeros(sh.sg.shape)
    c, o = _cam(cam), _opts(opts)
    rc = lib().orc_backward(C.byref(sh.s), C.byref(c), C.byref(o), pix.ctypes.data, n,
                            g_rgb.ctypes.data, None if g_T is None else g_T.ctypes.data,
                            out["means"].ctypes.data, out["log_scales"].ctypes.data,
                            out["quats"].ctypes.data, out["density"].ctypes.data,
                            out["sh"].ctypes.data,
                            out["sg"].ctypes.data if "sg" in out else None)
    if rc != 0:
        raise ValueError(f"orc_backward failed ({rc})")
    return out


def hits(scene, cam, opts: Opts, pix: int, cap_segs=4096, cap_ids=1 << 20):
    """Processed segments of one ray: list of (a, dt, sorted original ids)."""
    sh = _SceneHold(scene)
    off = np.zeros(cap_segs + 1, np.int64)
    a = np.zeros(cap_segs)
    dt = np.zeros(cap_segs)
    ids = np.zeros(cap_ids, np.int64)
    c, o = _cam(cam), _opts(opts)
    ns = lib().orc_hits(C.byref(sh.s), C.byref(c), C.byref(o), int(pix), off.ctypes.data,
                        a.ctypes.data, dt.ctypes.data, cap_segs, ids.ctypes.data, cap_ids)
    if ns < 0:
        raise ValueError("orc_hits: capacity too small")
    return [(a[i], dt[i], ids[off[i]:off[i + 1]].copy()) for i in range(ns)]


def false_positives(scene, cam, opts: Opts, pix=None):
    """Per ray: the number of Gaussians whose minimal AABB meets [t_n, t_end]
    while the ellipsoid does not, the number of near-tie decisions among them,
    and t_end (where the ray's march ended)."""
    if pix is None:
        pix = np.arange(cam.width * cam.height, dtype=np.int64)
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    n = pix.shape[0]
    sh = _SceneHold(scene)
    count = np.zeros(n, np.int64)
    ties = np.zeros(n, np.int64)
    t_end = np.zeros(n)
    c, o = _cam(cam), _opts(opts)
    rc = lib().orc_false_positives(C.byref(sh.s), C.byref(c), C.byref(o), pix.ctypes.data, n,
                                   count.ctypes.data, ties.ctypes.data, t_end.ctypes.data)
    if rc != 0:
        raise ValueError(f"orc_false_positives failed ({rc})")
    return count, ties, t_end


def chords(scene, cam, sigma_eps, pix: int, ids):
    """k^2, h^2 (closest approach, local frame) and the chord [t0, t1] of the
    listed Gaussians along one pixel's ray (NaN where there is none)."""
    sh = _SceneHold(scene)
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    n = ids.shape[0]
    out = [np.zeros(n) for _ in range(4)]
    c = _cam(cam)
    lib().orc_chords(C.byref(sh.s), C.byref(c), float(sigma_eps), int(pix), ids.ctypes.data, n,
                     *[a.ctypes.data for a in out])
    return tuple(out)


def colour(scene, l: int, dirs):
    """Colour [n,3] of Gaussian l at the listed unit directions (SH sum plus
    spherical-Gaussian lobes)."""
    sh = _SceneHold(scene)
    d = _f64(dirs).reshape(-1, 3)
    out = np.zeros((d.shape[0], 3))
    lib().orc_colour(C.byref(sh.s), int(l), d.ctypes.data, d.shape[0], out.ctypes.data)
    return out


def sh_basis(deg: int, d):
    d = _f64(d).reshape(-1, 3)
    out = np.zeros((d.shape[0], 16))
    for i in range(d.shape[0]):
        lib().orc_sh_basis(deg, d[i].ctypes.data, out[i].ctypes.data)
    return out[:, : (deg + 1) ** 2]


def rays(cam, pix):
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    o = np.zeros((len(pix), 3))
    d = np.zeros((len(pix), 3))
    c = _cam(cam)
    lib().orc_rays(C.byref(c), pix.ctypes.data, len(pix), o.ctypes.data, d.ctypes.data)
    return o, d


def gaussians(scene, sigma_eps):
    """k^2, active flag, rotation matrices [N,3,3] and minimal-AABB
    half-lengths [N,3] (Supp. B)."""
    sh = _SceneHold(scene)
    N = sh.arrs[0].shape[0]
    k2 = np.zeros(N)
    act = np.zeros(N, np.int32)
    R = np.zeros((N, 3, 3))
    half = np.zeros((N, 3))
    lib().orc_gaussians(C.byref(sh.s), float(sigma_eps), k2.ctypes.data, act.ctypes.data,
                        R.ctypes.data, half.ctypes.data)
    return k2, act.astype(bool), R, half


def density_at(scene, sigma_eps, l, x):
    sh = _SceneHold(scene)
    x = _f64(x).reshape(-1, 3)
    out = np.zeros(x.shape[0])
    lib().orc_density_at(C.byref(sh.s), float(sigma_eps), int(l), x.ctypes.data, x.shape[0],
                         out.ctypes.data)
    return out
