"""Seeded synthetic scenes and cameras.

This module only draws inputs: Gaussian parameter arrays with the shapes and
value distributions of the paper's workloads, and pinhole cameras.  It holds
none of the rendering arithmetic; both the GPU path and the CPU oracle consume
what it returns.

Parameterisation (one row per Gaussian, float32):
  means       [N,3]    world-space centre mu
  log_scales  [N,3]    l, with s = exp(l) per local axis
  quats       [N,4]    unnormalised quaternion (w, x, y, z)
  density     [N]      raw density parameter sigma~ (no activation applied later)
  sh          [N,K,3]  SH coefficients, K = (deg+1)^2, per RGB channel

Cameras follow the OpenCV convention (x right, y down, z forward), world up is
+y, horizontal field of view 60 degrees, principal point at the image centre.

Workload recipes (seed = 1000 + config index, target seed = 2000 + index):
  1  1k Gaussians, means U[-1,1]^3, l ~ N(-3,0.3), SH degree 0 with colour
     U(0,1); one 64x64 view from distance 3.
  2  100k Gaussians, means from a mixture of 32 isotropic normals (sd 0.2)
     whose centres are uniform in the unit ball (points outside the unit ball
     redrawn), l ~ N(-4,0.5), SH degree 3 with coefficients N(0,0.2); one
     800x800 view from distance 3.
  3  1M Gaussians as in 2; four 1024x768 views on an orbit of radius 3.
  4  3M Gaussians: 70% the mixture of 2, 30% a shell with radius U(2,50)
     (number density ~ 1/r^2) and scale growing linearly with r; four
     1297x840 views from a radius-0.5 circle.  A "regularised" variant shrinks
     each Gaussian's log-scale spread until the rotation-invariant AABB/volume
     bound (Sec. 3.4, Eq. 7/9) is at most r0 = 10.
  5  5M Gaussians in the layout of 4; 16 views of random size in
     [256,1920] x [256,1080].
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SH_C0 = 0.28209479177387814  # value of the degree-0 real SH basis function


@dataclasses.dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    cam_to_world: np.ndarray  # [3,4] float32, columns: right, down, forward, centre
    t_near: float = 0.0
    t_far: float = 6.0

    @property
    def n_rays(self) -> int:
        return self.width * self.height


def look_at_camera(width, height, eye, target=(0.0, 0.0, 0.0), fov_deg=60.0,
                   t_near=0.0, t_far=6.0) -> Camera:
    eye = np.asarray(eye, np.float64)
    fwd = np.asarray(target, np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    up = np.array([0.0, 1.0, 0.0])
    right = np.cross(fwd, up)
    if np.linalg.norm(right) < 1e-9:          # looking straight up/down
        right = np.array([1.0, 0.0, 0.0])
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    c2w = np.stack([right, down, fwd, eye], axis=1).astype(np.float32)
    f = width / (2.0 * math.tan(math.radians(fov_deg) / 2.0))
    return Camera(int(width), int(height), float(np.float32(f)), float(np.float32(f)),
                  width / 2.0, height / 2.0, c2w, float(t_near), float(t_far))


def _random_quats(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q.astype(np.float32)


def _softplus(x):
    return np.log1p(np.exp(-np.abs(x))) + np.maximum(x, 0.0)


def _density(rng, n):
    return (10.0 * _softplus(rng.standard_normal(n))).astype(np.float32)


def _mixture_means(rng, n, n_comp=32, sd=0.2):
    # component centres uniform in the unit ball
    c = rng.standard_normal((n_comp, 3))
    c /= np.linalg.norm(c, axis=1, keepdims=True)
    c *= rng.random((n_comp, 1)) ** (1.0 / 3.0)
    out = np.empty((n, 3), np.float64)
    todo = np.arange(n)
    while todo.size:
        comp = rng.integers(0, n_comp, todo.size)
        x = c[comp] + sd * rng.standard_normal((todo.size, 3))
        ok = np.einsum("ij,ij->i", x, x) <= 1.0
        out[todo[ok]] = x[ok]
        todo = todo[~ok]
    return out


def _shell_means(rng, n, r_lo=2.0, r_hi=50.0):
    # radius uniform <=> number density proportional to 1/r^2
    r = rng.uniform(r_lo, r_hi, n)
    u = rng.standard_normal((n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    return u * r[:, None], r


def make_scene(kind: str, n: int, seed: int, sh_degree: int | None = None,
               log_scale_sd: float = 0.5, n_sg: int = 0) -> dict:
    """Draw a scene of `n` Gaussians.

    kind: "uniform" (config 1), "cluster" (configs 2-3) or "outdoor"
    (configs 4-5).  Returns float32 arrays as described in the module doc.
    n_sg > 0 adds spherical-Gaussian colour lobes "sg" [n, n_sg, 7]:
    amplitudes N(0, 0.2) per channel, axes uniform on the sphere times a
    length U(0.5, 2), sharpness U(1, 30); drawn after everything else, so
    the other arrays do not depend on n_sg.
    """
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        deg = 0 if sh_degree is None else sh_degree
        means = rng.uniform(-1.0, 1.0, (n, 3))
        log_scales = rng.normal(-3.0, 0.3, (n, 3))
    elif kind == "cluster":
        deg = 3 if sh_degree is None else sh_degree
        means = _mixture_means(rng, n)
        log_scales = rng.normal(-4.0, log_scale_sd, (n, 3))
    elif kind == "outdoor":
        deg = 3 if sh_degree is None else sh_degree
        n_in = int(round(0.7 * n))
        m_in = _mixture_means(rng, n_in)
        m_out, r = _shell_means(rng, n - n_in)
        means = np.concatenate([m_in, m_out])
        log_scales = rng.normal(-4.0, log_scale_sd, (n, 3))
        log_scales[n_in:] += np.log(r)[:, None]
    else:
        raise ValueError(f"unknown scene kind {kind!r}")
    quats = _random_quats(rng, n)
    density = _density(rng, n)
    k = (deg + 1) ** 2
    if kind == "uniform" and deg == 0:
        colour = rng.uniform(0.0, 1.0, (n, 1, 3))
        sh = colour / SH_C0
    else:
        sh = rng.normal(0.0, 0.2, (n, k, 3))
    out = dict(means=means.astype(np.float32), log_scales=log_scales.astype(np.float32),
               quats=quats, density=density, sh=sh.astype(np.float32), sh_degree=deg)
    if n_sg:
        amp = rng.normal(0.0, 0.2, (n, n_sg, 3))
        ax = rng.standard_normal((n, n_sg, 3))
        ax *= (rng.uniform(0.5, 2.0, (n, n_sg, 1)) / np.linalg.norm(ax, axis=2, keepdims=True))
        lam = rng.uniform(1.0, 30.0, (n, n_sg, 1))
        out["sg"] = np.concatenate([amp, ax, lam], axis=2).astype(np.float32)
    return out


def subset_scene(scene: dict, idx) -> dict:
    out = {k: (v[idx] if isinstance(v, np.ndarray) else v) for k, v in scene.items()}
    for k, v in out.items():
        if isinstance(v, np.ndarray):
            out[k] = np.ascontiguousarray(v)
    return out


def regularize_log_scales(log_scales: np.ndarray, r0: float = 10.0, iters: int = 40) -> np.ndarray:
    """Shrink each row's log-scale deviations about the row mean (volume kept)
    by the largest factor in [0,1] for which the rotation-invariant bound of
    Eq. 7/9, 2/(pi sqrt 3) (s1^2+s2^2+s3^2)^(3/2) / (s1 s2 s3), is <= r0.
    Bisection on the factor; the bound is monotone in it."""
    ls = log_scales.astype(np.float64)
    m = ls.mean(axis=1, keepdims=True)
    dev = ls - m

    def bound(lam):
        e = lam[:, None] * dev                    # mean term cancels in the ratio
        s2 = np.exp(2.0 * e)
        return 2.0 / (math.pi * math.sqrt(3.0)) * s2.sum(1) ** 1.5 / np.exp(e.sum(1))

    lo = np.zeros(len(ls))
    hi = np.ones(len(ls))
    ok_full = bound(hi) <= r0
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        good = bound(mid) <= r0
        lo = np.where(good, mid, lo)
        hi = np.where(good, hi, mid)
    lam = np.where(ok_full, 1.0, lo)
    return (m + lam[:, None] * dev).astype(np.float32)


# ----------------------------------------------------------------------------
# workloads


def config_cameras(config: int, seed: int | None = None) -> list[Camera]:
    if config == 1:
        return [look_at_camera(64, 64, (0.0, 0.0, 3.0))]
    if config == 2:
        return [look_at_camera(800, 800, (0.0, 0.0, 3.0))]
    if config == 3:
        cams = []
        for az in (0.0, 90.0, 180.0, 270.0):
            a = math.radians(az)
            cams.append(look_at_camera(1024, 768, (3.0 * math.sin(a), 0.0, 3.0 * math.cos(a))))
        return cams
    if config == 4:
        cams = []
        for az in (0.0, 90.0, 180.0, 270.0):
            a = math.radians(az)
            cams.append(look_at_camera(1297, 840, (0.5 * math.sin(a), 0.0, 0.5 * math.cos(a)),
                                       t_far=128.0))
        return cams
    if config == 5:
        rng = np.random.default_rng(1005 if seed is None else seed)
        cams = []
        for v in range(16):
            w = int(rng.integers(256, 1921))
            h = int(rng.integers(256, 1081))
            a = 2.0 * math.pi * v / 16.0
            cams.append(look_at_camera(w, h, (0.5 * math.sin(a), 0.0, 0.5 * math.cos(a)),
                                       t_far=128.0))
        return cams
    raise ValueError(config)


def hd_camera() -> Camera:
    """1920x1080 frame of the 1M-Gaussian scene from the first orbit camera."""
    return look_at_camera(1920, 1080, (0.0, 0.0, 3.0))


CONFIG_SCENES = {1: ("uniform", 1_000), 2: ("cluster", 100_000), 3: ("cluster", 1_000_000),
                 4: ("outdoor", 3_000_000), 5: ("outdoor", 5_000_000)}


def config_scene(config: int, n: int | None = None, regularized: bool = False,
                 log_scale_sd: float = 0.5) -> dict:
    kind, n_def = CONFIG_SCENES[config]
    sc = make_scene(kind, n_def if n is None else n, 1000 + config, log_scale_sd=log_scale_sd)
    if regularized:
        sc["log_scales"] = regularize_log_scales(sc["log_scales"])
    return sc


def target_image(config: int, n_pixels: int) -> np.ndarray:
    rng = np.random.default_rng(2000 + config)
    return rng.uniform(0.0, 1.0, (n_pixels, 3)).astype(np.float32)


def pixel_subset(cam: Camera, stride: int) -> np.ndarray:
    """Deterministic pixel subset (every stride-th pixel on both axes), as
    row-major pixel indices of the view."""
    v, u = np.meshgrid(np.arange(0, cam.height, stride), np.arange(0, cam.width, stride),
                       indexing="ij")
    return (v * cam.width + u).reshape(-1).astype(np.int64)
