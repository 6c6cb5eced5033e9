"""GPU backward (re-traversal adjoint with wave-level reduction) against the
FP64 oracle adjoint, and the autograd.Function end to end."""
import numpy as np
import pytest

import oracle
from paper_2509_07782_amd import inputs

from helpers import PARAM_KEYS, grad_rel_errors, oracle_opts, renderer_for, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _opts(**kw):
    from paper_2509_07782_amd.render import RenderOptions
    return RenderOptions(**kw)


@pytest.fixture(scope="module")
def small_setup(torch_cuda):
    sc = inputs.make_scene("cluster", 3000, 31)
    cam = inputs.look_at_camera(33, 27, (0.3, 0.2, 2.6), fov_deg=40.0)
    r, params = renderer_for(sc)
    rng = np.random.default_rng(5)
    n = cam.width * cam.height
    gC = rng.standard_normal((n, 3)).astype(np.float32)
    gT = rng.standard_normal(n).astype(np.float32)
    return sc, cam, r, params, gC, gT


def _gpu_grads(torch, r, cam, o, params, gC, gT):
    rgb, T = r.forward([cam], o)
    g = r.backward([cam], o, rgb, T, torch.from_numpy(gC).cuda(),
                   None if gT is None else torch.from_numpy(gT).cuda(), params)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in g.items()}


@pytest.mark.parametrize("mode", ["fixed", "fixed_teps", "adaptive"])
def test_backward_matches_oracle(small_setup, torch_cuda, mode):
    sc, cam, r, params, gC, gT = small_setup
    if mode == "fixed":
        o = _opts(dt=0.005, ess=1, t_eps=0.0, bg=(0.2, 0.3, 0.1))
    elif mode == "fixed_teps":
        o = _opts(dt=0.005, ess=1, t_eps=1e-4)
    else:
        o = _opts(adaptive=True, ess=1, t_eps=0.0)
    g = _gpu_grads(torch_cuda, r, cam, o, params, gC, gT)
    ref = oracle.backward(sc, cam, oracle_opts(o), np.arange(cam.width * cam.height),
                          gC.astype(np.float64), gT.astype(np.float64))
    errs = grad_rel_errors(g, ref)
    for k, (rel, frac) in errs.items():
        assert rel <= 1e-3, (k, rel)
        assert frac >= 0.999, (k, frac)


@pytest.mark.parametrize("deg,ns", [(0, 2), (1, 16), (2, 1), (3, 4)])
def test_backward_sh_degrees_and_segment_sizes(torch_cuda, deg, ns):
    """Every SH degree (the SH-coefficient gradients go through the per-tile
    matrix product, masked past the degree) and segment sizes other than 8,
    against the oracle adjoint."""
    sc = inputs.make_scene("cluster", 2500, 41 + deg, sh_degree=deg)
    cam = inputs.look_at_camera(29, 23, (0.2, 0.3, 2.7), fov_deg=42.0)
    r, params = renderer_for(sc)
    rng = np.random.default_rng(9)
    n = cam.width * cam.height
    gC = rng.standard_normal((n, 3)).astype(np.float32)
    o = _opts(dt=0.005, ess=1, t_eps=1e-4, n_s=ns)
    g = _gpu_grads(torch_cuda, r, cam, o, params, gC, None)
    ref = oracle.backward(sc, cam, oracle_opts(o), np.arange(n), gC.astype(np.float64))
    assert np.size(g["sh"]) == ref["sh"].size == sc["means"].shape[0] * (deg + 1) ** 2 * 3
    errs = grad_rel_errors(g, ref)
    for k, (rel, frac) in errs.items():
        assert rel <= 1e-3, (deg, ns, k, rel)
        assert frac >= 0.999, (deg, ns, k, frac)
    r.close()


def test_closest_hit_replay(small_setup, torch_cuda):
    """A backward right after its forward replays the recorded closest-hit
    results; after a forward of other rays, or after a rebuild, it searches
    them itself.  Both give the same gradients (the same restarts)."""
    torch = torch_cuda
    sc, cam, r, params, gC, gT = small_setup
    o = _opts(adaptive=True, ess=1, t_eps=1e-4)
    other = inputs.look_at_camera(21, 17, (-0.4, 0.3, 2.5), fov_deg=40.0)
    gCt = torch.from_numpy(gC).cuda()
    rgb, T = r.forward([cam], o)
    g_rep = r.backward([cam], o, rgb, T, gCt, None, params)
    torch.cuda.synchronize()
    assert r.ctx.backward_replayed()
    r.forward([other], o)                      # the record now holds other rays
    g_own = r.backward([cam], o, rgb, T, gCt, None, params)
    torch.cuda.synchronize()
    assert not r.ctx.backward_replayed()
    for k in PARAM_KEYS:
        a, b = g_rep[k].cpu().numpy(), g_own[k].cpu().numpy()
        d = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        assert d <= 1e-5, (k, d)
    r.forward([cam], o)
    r.build(params, sc["sh_degree"], force=True)   # a new build invalidates the record
    r.backward([cam], o, rgb, T, gCt, None, params)
    torch.cuda.synchronize()
    assert not r.ctx.backward_replayed()
    # no empty-space skipping: nothing recorded, nothing replayed
    o2 = _opts(dt=0.005, ess=0)
    rgb2, T2 = r.forward([cam], o2)
    r.backward([cam], o2, rgb2, T2, gCt, None, params)
    torch.cuda.synchronize()
    assert not r.ctx.backward_replayed()


def test_window_replay_dense_chunked(torch_cuda):
    """A dense cluster whose windows overflow the 512-entry list, so segments
    run in Z chunks and some tiles may not fit their record region: the
    replayed backward (recorded chunks, earlier chunks of a segment re-read for
    pass B) equals the backward that walks the tree itself."""
    torch = torch_cuda
    sc = inputs.make_scene("cluster", 60000, 77)
    sc["log_scales"] = sc["log_scales"] + 0.8       # larger Gaussians: long lists
    cam = inputs.look_at_camera(40, 32, (0.2, 0.1, 2.4), fov_deg=35.0)
    r, params = renderer_for(sc)
    o = _opts(adaptive=True, ess=1, t_eps=1e-4, window_segments=4)
    rgb, T, st = r.forward([cam], o, stats=True)
    torch.cuda.synchronize()
    from paper_2509_07782_amd import lib
    chunked = int(st[:, lib.STAT_NAMES.index("chunked")].sum())
    assert chunked > 0
    rng = np.random.default_rng(13)
    gCt = torch.from_numpy(rng.standard_normal((cam.width * cam.height, 3)).astype(np.float32)).cuda()
    g_rep = r.backward([cam], o, rgb, T, gCt, None, params)
    torch.cuda.synchronize()
    assert r.ctx.backward_replayed()
    other = inputs.look_at_camera(16, 16, (-0.3, 0.2, 2.6), fov_deg=35.0)
    r.forward([other], o)
    g_own = r.backward([cam], o, rgb, T, gCt, None, params)
    torch.cuda.synchronize()
    assert not r.ctx.backward_replayed()
    for k in PARAM_KEYS:
        a, b = g_rep[k].cpu().numpy(), g_own[k].cpu().numpy()
        d = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        assert d <= 1e-5, (k, d)
    assert r.ctx.error_flags() == 0
    r.close()


def test_backward_bvh_equals_brute_force(small_setup, torch_cuda):
    sc, cam, r, params, gC, gT = small_setup
    a = _gpu_grads(torch_cuda, r, cam, _opts(dt=0.005, brute_force=True), params, gC, gT)
    b = _gpu_grads(torch_cuda, r, cam, _opts(dt=0.005, brute_force=False), params, gC, gT)
    for k in PARAM_KEYS:
        d = np.linalg.norm(a[k] - b[k]) / max(np.linalg.norm(a[k]), 1e-30)
        assert d <= 1e-5, (k, d)


def test_quaternion_gradient_orthogonal(small_setup, torch_cuda):
    sc, cam, r, params, gC, gT = small_setup
    g = _gpu_grads(torch_cuda, r, cam, _opts(dt=0.005), params, gC, gT)
    dots = np.einsum("ij,ij->i", g["quats"].astype(np.float64), sc["quats"].astype(np.float64))
    assert np.abs(dots).max() <= 1e-4 * np.abs(g["quats"]).max()


def test_autograd_function_l2_loss(small_setup, torch_cuda):
    """L = mean((C - C*)^2) through RayMarchFunction: gradients equal the
    oracle adjoint of the same loss."""
    torch = torch_cuda
    from paper_2509_07782_amd.render import Renderer, render
    sc, cam, _, _, _, _ = small_setup
    o = _opts(dt=0.005)
    rr = Renderer(0)
    p = {k: v.clone().requires_grad_(True) for k, v in to_device(sc).items()}
    n = cam.width * cam.height
    target = torch.from_numpy(inputs.target_image(3, n)).cuda()
    rgb, T = render(p, sc["sh_degree"], rr, [cam], o)
    loss = ((rgb - target) ** 2).mean()
    loss.backward()
    torch.cuda.synchronize()
    gC = (2.0 / (3 * n)) * (rgb.detach() - target).cpu().numpy().astype(np.float64)
    ref = oracle.backward(sc, cam, oracle_opts(o), np.arange(n), gC, None)
    g = {k: p[k].grad.cpu().numpy() for k in PARAM_KEYS}
    for k, (rel, frac) in grad_rel_errors(g, ref).items():
        assert rel <= 1e-3, (k, rel)
