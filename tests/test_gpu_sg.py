"""Spherical-Gaussian colour lobes (SH degree 2 plus 7 lobes per Gaussian,
the appearance model of the supplement's comparison with 3D-GS) on the GPU:
images and gradients of every parameter, the lobes' included, against the
FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_2509_07782_amd import inputs

from helpers import grad_rel_errors, oracle_opts

pytestmark = pytest.mark.gpu

KEYS = ("means", "log_scales", "quats", "density", "sh", "sg")


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
def sg_setup(torch_cuda):
    torch = torch_cuda
    from paper_2509_07782_amd.render import Renderer
    sc = inputs.make_scene("cluster", 3000, 91, sh_degree=2, n_sg=7)
    cam = inputs.look_at_camera(37, 29, (0.3, 0.2, 2.6), fov_deg=40.0)
    r = Renderer(0)
    params = {k: torch.from_numpy(np.ascontiguousarray(sc[k], np.float32)).cuda() for k in KEYS}
    r.build(params, 2)
    return sc, cam, r, params


@pytest.mark.parametrize("mode", ["fixed", "adaptive"])
def test_sg_forward_matches_oracle(sg_setup, torch_cuda, mode):
    sc, cam, r, params = sg_setup
    o = _opts(dt=0.005, ess=1, t_eps=1e-4) if mode == "fixed" else _opts(adaptive=True, ess=1, t_eps=1e-4)
    rgb, T = (x.cpu().numpy() for x in r.forward([cam], o))
    r.check_errors()
    orgb, oT, ost, mg = oracle.render(sc, cam, oracle_opts(o))
    assert (ost[:, 0] > 5).mean() > 0.3
    err = np.abs(rgb - orgb).max(axis=1)
    bad = err > 1e-4
    assert bad.mean() <= 0.001 and np.all(mg[bad] < 1e-6), (bad.sum(), err.max())
    # the lobes matter: the same scene without them renders differently
    no_sg = {k: v for k, v in sc.items() if k != "sg"}
    orgb0, _, _, _ = oracle.render(no_sg, cam, oracle_opts(o))
    assert np.abs(orgb0 - orgb).max() > 1e-2


@pytest.mark.parametrize("mode", ["fixed", "adaptive"])
def test_sg_backward_matches_oracle(sg_setup, torch_cuda, mode):
    torch = torch_cuda
    sc, cam, r, params = sg_setup
    o = _opts(dt=0.005, ess=1, t_eps=0.0) if mode == "fixed" else _opts(adaptive=True, ess=1, t_eps=0.0)
    n = cam.width * cam.height
    rng = np.random.default_rng(17)
    gC = rng.standard_normal((n, 3)).astype(np.float32)
    st = r.new_state()
    rgb, T = r.forward([cam], o, state=st)
    g = r.backward(st, rgb, T, torch.from_numpy(gC).cuda(), None, params)
    torch.cuda.synchronize()
    r.check_errors()
    st.close()
    got = {k: v.cpu().numpy() for k, v in g.items()}
    assert set(got) == set(KEYS)
    ref = oracle.backward(sc, cam, oracle_opts(o), np.arange(n), gC.astype(np.float64))
    errs = grad_rel_errors({k: got[k] for k in KEYS[:5]}, ref)
    for k in ("sg",):
        a = got[k].astype(np.float64).reshape(-1)
        b = ref[k].reshape(-1)
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        rms = np.sqrt(np.mean(b * b))
        frac = (np.abs(a - b) <= 1e-3 * np.abs(b) + 1e-3 * rms).mean()
        errs[k] = (rel, frac)
    for k, (rel, frac) in errs.items():
        assert rel <= 1e-3, (k, rel)
        assert frac >= 0.999, (k, frac)
    # the lobe axis gradient is orthogonal to the axis
    dots = np.einsum("lkj,lkj->lk", got["sg"][..., 3:6].astype(np.float64),
                     sc["sg"][..., 3:6].astype(np.float64))
    assert np.abs(dots).max() <= 1e-4 * np.abs(got["sg"][..., 3:6]).max()


def test_sg_autograd_and_unsupported_segment_size(sg_setup, torch_cuda):
    """The lobes are a differentiable input of the autograd.Function, and
    segment sizes other than 8 are refused for lobed scenes."""
    torch = torch_cuda
    from paper_2509_07782_amd import lib
    from paper_2509_07782_amd.render import Renderer, render
    sc, cam, _, _ = sg_setup
    rr = Renderer(0)
    p = {k: torch.from_numpy(np.ascontiguousarray(sc[k], np.float32)).cuda().requires_grad_(True)
         for k in KEYS}
    o = _opts(dt=0.005, ess=1, t_eps=0.0)
    rgb, T = render(p, 2, rr, [cam], o)
    (rgb.sum() + T.sum()).backward()
    torch.cuda.synchronize()
    n = cam.width * cam.height
    ref = oracle.backward(sc, cam, oracle_opts(o), np.arange(n), np.ones((n, 3)), np.ones(n))
    for k in KEYS:
        a = p[k].grad.cpu().numpy().astype(np.float64)
        rel = np.linalg.norm(a - ref[k]) / np.linalg.norm(ref[k])
        assert rel <= 1e-3, (k, rel)
    with pytest.raises(lib.RgxError, match="unsupported"):
        rr.forward([cam], _opts(dt=0.005, n_s=4))
    rr.check_errors()
    rr.close()
