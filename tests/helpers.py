"""Shared test helpers: device copies of seeded scenes, option mapping between
the GPU renderer and the oracle, and comparison utilities."""
import numpy as np

import oracle
from paper_2509_07782_amd import inputs

PARAM_KEYS = ("means", "log_scales", "quats", "density", "sh")


def f32(x):
    return float(np.float32(x))


def to_device(scene):
    import torch
    return {k: torch.from_numpy(np.ascontiguousarray(scene[k], np.float32)).cuda()
            for k in PARAM_KEYS}


def oracle_opts(o, sigma_eps=0.01):
    """Oracle options equal to the GPU's (float32-rounded) values."""
    return oracle.Opts(adaptive=bool(o.adaptive), dt=f32(o.dt), dt_min=f32(o.dt_min),
                       dt_max=f32(o.dt_max), beta=f32(o.beta), n_s=int(o.n_s),
                       t_eps=f32(o.t_eps), ess=int(o.ess), bg=tuple(f32(b) for b in o.bg),
                       sigma_eps=f32(sigma_eps))


def renderer_for(scene, sigma_eps=0.01, morton_bits=21):
    from paper_2509_07782_amd.render import Renderer
    r = Renderer(0, sigma_eps=sigma_eps, morton_bits=morton_bits)
    params = to_device(scene)
    r.build(params, scene["sh_degree"])
    return r, params


def gpu_render(r, cams, opts, stats=False):
    import torch
    out = r.forward(cams, opts, stats=stats)
    torch.cuda.synchronize()
    assert r.ctx.error_flags() == 0
    return tuple(x.cpu().numpy() for x in out)


def grad_rel_errors(g, ref):
    """Per-tensor relative L2 error and the fraction of elements within
    |d| <= 1e-3 |ref| + 1e-3 rms(ref)."""
    out = {}
    for k in PARAM_KEYS:
        a = np.asarray(g[k], np.float64).reshape(-1)
        b = np.asarray(ref[k], np.float64).reshape(-1)
        nb = np.linalg.norm(b)
        rel = np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a - b)
        rms = np.sqrt(np.mean(b * b)) if b.size else 0.0
        ok = np.abs(a - b) <= 1e-3 * np.abs(b) + 1e-3 * rms
        out[k] = (rel, ok.mean() if ok.size else 1.0)
    return out
