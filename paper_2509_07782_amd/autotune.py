"""Autotuner for the launch knobs of the ray marcher.

The knobs -- tile shape, persistent launch and the initial depth-window
length -- only change how work is scheduled, never the arithmetic of a ray:
every candidate's image must equal the reference image bit for bit, which the
tuner checks before it times anything.  The fastest candidate is cached per
(device, CU count, Gaussian count, total rays, SH degree, mode) in memory and,
when a path is given, in a JSON file."""
from __future__ import annotations

import dataclasses
import json
import os
import time

import torch

from .render import RenderOptions, Renderer

TILES = ((8, 8), (16, 4), (4, 16), (32, 2), (64, 1))
WINDOWS = (1, 2, 4)

_CACHE: dict = {}


def cache_key(renderer: Renderer, cams, opts: RenderOptions) -> str:
    prop = torch.cuda.get_device_properties(renderer.ctx.device)
    rays = sum(c.width * c.height for c in cams)
    mode = "adaptive" if opts.adaptive else f"fixed{opts.dt:g}"
    return (f"{prop.name}|{prop.multi_processor_count}|{renderer.bvh.n}|{rays}|"
            f"{renderer.bvh.sh_degree}|{mode}|ns{opts.n_s}|ess{opts.ess}")


def _time(fn, reps):
    fn()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / reps


def tune(renderer: Renderer, cams, opts: RenderOptions, reps: int = 2,
         cache_path: str | None = None, with_backward: bool = False, params=None,
         persistent: bool | None = None):
    """Returns the fastest equivalent RenderOptions (and the timing table).
    persistent: None searches both launch forms, True / False fixes it."""
    key = cache_key(renderer, cams, opts) + f"|pers{persistent}"
    if cache_path and os.path.exists(cache_path) and key not in _CACHE:
        with open(cache_path) as fh:
            _CACHE.update(json.load(fh))
    if key in _CACHE:
        return dataclasses.replace(opts, **_CACHE[key]["knobs"]), _CACHE[key]["table"]
    ref_rgb, ref_T = renderer.forward(cams, opts)
    st = renderer.new_state() if with_backward else None
    table = []
    best = None
    for (tw, th) in TILES:
        for pers in ((False, True) if persistent is None else (bool(persistent),)):
            for win in WINDOWS:
                cand = dataclasses.replace(opts, ray_order=1, tile_w=tw, tile_h=th,
                                           persistent=pers, window_segments=win)
                rgb, T = renderer.forward(cams, cand)
                if not (torch.equal(rgb, ref_rgb) and torch.equal(T, ref_T)):
                    raise RuntimeError(f"tuning knobs changed the image: {cand}")

                def run():
                    out = renderer.forward(cams, cand, state=st if with_backward else None)
                    if with_backward:
                        g = torch.full_like(out[0], 1e-3)
                        renderer.backward(st, out[0], out[1], g, None, params)
                    return out

                t = _time(run, reps)
                knobs = dict(tile_w=tw, tile_h=th, persistent=pers, window_segments=win)
                table.append((knobs, t))
                if best is None or t < best[1]:
                    best = (knobs, t)
    if st is not None:
        st.close()
    _CACHE[key] = {"knobs": best[0], "table": [(k, t) for k, t in table]}
    if cache_path:
        with open(cache_path, "w") as fh:
            json.dump(_CACHE, fh, indent=1)
    return dataclasses.replace(opts, **best[0]), table
