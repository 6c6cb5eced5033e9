"""The workloads at full size: sampled pixels and gradients against the oracle,
the batched persistent launch, the hipGraph-captured training step, the
autotuner and the false-positive counts of the anisotropy study."""
import math

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


def _view_offsets(cams):
    off, out = 0, []
    for c in cams:
        out.append(off)
        off += c.width * c.height
    return out


def _check_pixels(rgb, orgb, mg, frac_bad=0.002):
    err = np.abs(rgb - orgb).max(axis=1)
    bad = err > 1e-4
    assert bad.mean() <= frac_bad, (bad.sum(), err.max())
    assert np.all(mg[bad] < 1e-5), mg[bad]
    return err


def test_config2_full_size(torch_cuda):
    """100k Gaussians, 800x800: fixed-step and adaptive pixels against the
    oracle on a stride-16 subset; Morton tiles == scanline bit for bit."""
    sc = inputs.config_scene(2)
    cam = inputs.config_cameras(2)[0]
    r, _ = renderer_for(sc)
    pix = inputs.pixel_subset(cam, 16)
    for o in (_opts(dt=0.005, ess=1, t_eps=1e-4), _opts(adaptive=True, ess=1, t_eps=1e-4)):
        rgb, T = (x.cpu().numpy() for x in r.forward([cam], o))
        orgb, oT, ost, mg = oracle.render(sc, cam, oracle_opts(o), pix)
        assert (ost[:, 0] > 0).mean() > 0.2
        _check_pixels(rgb[pix], orgb, mg)
        raster = [x.cpu().numpy() for x in r.forward([cam], _opts(**{**o.__dict__, "ray_order": 0}))]
        assert np.array_equal(raster[0], rgb) and np.array_equal(raster[1], T)


@pytest.fixture(scope="module")
def config3(torch_cuda):
    sc = inputs.config_scene(3)
    cams = inputs.config_cameras(3)
    r, params = renderer_for(sc)
    return sc, cams, r, params


def test_config3_sampled_pixels(config3):
    """1M Gaussians, 4 views 1024x768, the benchmark's sampling (adaptive,
    closest-hit restarts, T_eps 1e-4): every 64th pixel against the oracle."""
    sc, cams, r, params = config3
    o = _opts(adaptive=True, ess=1, t_eps=1e-4, persistent=True)
    rgb, T = (x.cpu().numpy() for x in r.forward(cams, o))
    for c, off in zip(cams, _view_offsets(cams)):
        pix = inputs.pixel_subset(c, 64)
        orgb, oT, ost, mg = oracle.render(sc, c, oracle_opts(o), pix)
        _check_pixels(rgb[off + pix], orgb, mg)


def test_config3_masked_gradients(config3, torch_cuda):
    """Gradients of a loss on every 64th pixel of the 4 views, full 1M scene,
    against the oracle adjoint of the same loss."""
    torch = torch_cuda
    sc, cams, r, params = config3
    o = _opts(dt=0.005, ess=1, t_eps=0.0, persistent=True)
    rgb, T = r.forward(cams, o)
    R = rgb.shape[0]
    rng = np.random.default_rng(3)
    gC = np.zeros((R, 3), np.float32)
    ref = None
    offs = _view_offsets(cams)
    for c, off in zip(cams, offs):
        pix = inputs.pixel_subset(c, 64)
        w = rng.standard_normal((len(pix), 3)).astype(np.float32)
        gC[off + pix] = w
        g = oracle.backward(sc, c, oracle_opts(o), pix, w.astype(np.float64), None)
        ref = g if ref is None else {k: ref[k] + g[k] for k in PARAM_KEYS}
    gg = r.backward(cams, o, rgb, T, torch.from_numpy(gC).cuda(), None, params)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in gg.items()}
    for k, (rel, frac) in grad_rel_errors(got, ref).items():
        assert rel <= 1e-3, (k, rel)
        assert frac >= 0.999, (k, frac)


def test_fd_4096_gaussian_subset(torch_cuda):
    """The 4096-Gaussian scene with the config-3 distributions and views:
    GPU gradients of a loss on every 32nd pixel against the oracle adjoint
    and, for a sample of parameters, central differences of the oracle."""
    torch = torch_cuda
    sc = inputs.make_scene("cluster", 4096, 1003)
    cams = inputs.config_cameras(3)
    o = _opts(dt=0.005, ess=1, t_eps=0.0)
    oo = oracle_opts(o, sigma_eps=1e-30)
    from paper_2509_07782_amd.render import Renderer
    r = Renderer(0, sigma_eps=1e-30)
    params = to_device(sc)
    r.build(params, 3)
    rgb, T = r.forward(cams, o)
    R = rgb.shape[0]
    rng = np.random.default_rng(11)
    gC = np.zeros((R, 3), np.float32)
    subs = []
    for c, off in zip(cams, _view_offsets(cams)):
        pix = inputs.pixel_subset(c, 32)
        w = rng.standard_normal((len(pix), 3)).astype(np.float32)
        gC[off + pix] = w
        subs.append((c, pix, w.astype(np.float64)))
    gg = r.backward(cams, o, rgb, T, torch.from_numpy(gC).cuda(), None, params)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy().astype(np.float64) for k, v in gg.items()}
    ref = None
    for c, pix, w in subs:
        g = oracle.backward(sc, c, oo, pix, w, None)
        ref = g if ref is None else {k: ref[k] + g[k] for k in PARAM_KEYS}
    for k, (rel, frac) in grad_rel_errors(got, ref).items():
        assert rel <= 1e-3, (k, rel)

    def loss(scene):
        tot = 0.0
        for c, pix, w in subs:
            orgb, _, _, _ = oracle.render(scene, c, oo, pix)
            tot += float(np.sum(orgb * w))
        return tot

    touched = np.nonzero(np.abs(ref["density"]) > 1e-6 * np.abs(ref["density"]).max())[0]
    picks = rng.choice(touched, size=min(6, len(touched)), replace=False)
    for l in picks:
        for k, idx in (("means", (l, 0)), ("log_scales", (l, 2)), ("quats", (l, 1)),
                       ("density", (l,)), ("sh", (l, 5, 1))):
            base = {kk: (v.astype(np.float64) if isinstance(v, np.ndarray) else v) for kk, v in sc.items()}
            h = 1e-4 * max(1.0, abs(base[k][idx]))
            base[k] = base[k].copy(); base[k][idx] += h
            lp = loss(base)
            base[k][idx] -= 2 * h
            lm = loss(base)
            fd = (lp - lm) / (2 * h)
            scale = np.abs(ref[k]).max()
            assert abs(got[k][idx] - fd) <= 2e-3 * scale + 1e-3 * abs(fd), (k, idx, got[k][idx], fd)


def test_config4_false_positives_and_parity(torch_cuda):
    """Outdoor layout (3M Gaussians, shell to r = 50, 1297x840 views from
    inside): the scale-regularised scene has fewer AABB-only leaf tests per
    ray than the unregularised one (stress log-scale spread 1.0); sampled
    pixels against the oracle."""
    cams = inputs.config_cameras(4)
    counts = {}
    for reg in (False, True):
        sc = inputs.config_scene(4, regularized=reg, log_scale_sd=1.0)
        r, _ = renderer_for(sc)
        o = _opts(adaptive=True, ess=1, t_eps=1e-4, persistent=True)
        rgb, T, st = (x.cpu().numpy() for x in r.forward(cams, o, stats=True))
        counts[reg] = st[:, 5].mean()
        if reg:
            c, off = cams[1], _view_offsets(cams)[1]
            pix = inputs.pixel_subset(c, 128)
            orgb, oT, ost, mg = oracle.render(sc, c, oracle_opts(o), pix)
            _check_pixels(rgb[off + pix], orgb, mg)
        r.close()
    assert counts[True] < counts[False], counts


def test_config5_batched_persistent_and_graph(torch_cuda):
    """5M Gaussians, 16 views of mixed size in one persistent launch: equal
    bit for bit to 16 separate plain launches; the hipGraph-captured training
    step replays to the eager step's loss and image."""
    torch = torch_cuda
    from paper_2509_07782_amd.render import TrainStep
    sc = inputs.config_scene(5)
    cams = inputs.config_cameras(5)
    r, params = renderer_for(sc)
    ob = _opts(adaptive=True, ess=1, t_eps=1e-4, persistent=True)
    op = _opts(adaptive=True, ess=1, t_eps=1e-4, persistent=False)
    rgb, T = r.forward(cams, ob)
    off = 0
    for c in cams:
        one = r.forward([c], op)
        n = c.width * c.height
        assert torch.equal(one[0], rgb[off:off + n]) and torch.equal(one[1], T[off:off + n])
        off += n
    # captured fwd + loss + bwd, replayed
    R = rgb.shape[0]
    target = torch.from_numpy(inputs.target_image(5, R)).cuda()
    p = {k: v.clone().requires_grad_(True) for k, v in params.items()}

    def loss_fn(c, t):
        return ((c - target) ** 2).mean()

    step = TrainStep(r, p, 3, cams, ob, loss_fn, lr=0.0)
    eager_rgb, _ = r.forward(cams, ob)
    eager_loss = float(((eager_rgb - target) ** 2).mean())
    for rep in range(3):
        loss = float(step.replay())
        torch.cuda.synchronize()
        assert torch.equal(step.rgb, eager_rgb)
        assert abs(loss - eager_loss) <= 1e-6 * abs(eager_loss)
        _ = r.forward([cams[0]], op)        # eager work between replays
        torch.cuda.synchronize()
    g0 = {k: v.clone() for k, v in step.grads.items()}
    step.replay()
    torch.cuda.synchronize()
    for k in PARAM_KEYS:
        d = (step.grads[k] - g0[k]).norm() / max(float(g0[k].norm()), 1e-30)
        assert d <= 1e-5, (k, float(d))


def test_autotuner_keeps_images(torch_cuda):
    from paper_2509_07782_amd import autotune
    sc = inputs.make_scene("cluster", 30000, 41)
    cams = [inputs.look_at_camera(160, 120, (0.2, 0.1, 2.9))]
    r, _ = renderer_for(sc)
    o = _opts(adaptive=True, ess=1)
    best, table = autotune.tune(r, cams, o, reps=1)
    assert len(table) == len(autotune.TILES) * 2 * len(autotune.WINDOWS)
    a = r.forward(cams, o)
    b = r.forward(cams, best)
    assert all(bool((x == y).all()) for x, y in zip(a, b))


@pytest.mark.parametrize("case", ["single", "pair", "inactive", "inside", "near_far", "bg"])
def test_edge_cases(torch_cuda, case):
    sc = inputs.make_scene("cluster", 2000, 51)
    cam = inputs.look_at_camera(19, 13, (0.2, 0.1, 2.7), fov_deg=40.0)
    o = _opts(dt=0.005, ess=1, t_eps=1e-4)
    if case == "single":
        sc = inputs.subset_scene(sc, [0])
        sc["means"][0] = [0.0, 0.0, 0.0]
        sc["log_scales"][0] = [-1.5, -1.8, -1.2]
    elif case == "pair":
        sc = inputs.subset_scene(sc, [0, 1])
        sc["means"][:] = [[0.05, 0.0, 0.0], [-0.05, 0.02, 0.1]]
        sc["log_scales"][:] = -1.6
    elif case == "inactive":
        sc["density"][:] = 0.001
    elif case == "inside":
        cam = inputs.look_at_camera(19, 13, (0.0, 0.0, 0.05), target=(0.0, 0.0, -1.0))
        sc["log_scales"][:10] += 2.5
    elif case == "near_far":
        cam = inputs.look_at_camera(19, 13, (0.2, 0.1, 2.7), fov_deg=40.0, t_near=2.5, t_far=3.1)
    elif case == "bg":
        o = _opts(dt=0.005, ess=2, t_eps=1e-4, bg=(0.3, 0.6, 0.9))
    r, _ = renderer_for(sc)
    rgb, T = (x.cpu().numpy() for x in r.forward([cam], o))
    orgb, oT, _, _ = oracle.render(sc, cam, oracle_opts(o))
    assert np.abs(rgb - orgb).max() <= 1e-4
    assert np.abs(T - oT).max() <= 1e-4
    if case == "inactive":
        assert np.all(T == 1.0)


@pytest.mark.parametrize("deg,ns", [(1, 4), (2, 16), (3, 1), (0, 2)])
def test_sh_degrees_and_segment_sizes(torch_cuda, deg, ns):
    sc = inputs.make_scene("cluster", 4000, 61, sh_degree=deg)
    cam = inputs.look_at_camera(23, 17, (0.1, 0.3, 2.8), fov_deg=45.0)
    o = _opts(dt=0.005, ess=1, t_eps=1e-4, n_s=ns)
    r, _ = renderer_for(sc)
    rgb, T = (x.cpu().numpy() for x in r.forward([cam], o))
    orgb, oT, _, mg = oracle.render(sc, cam, oracle_opts(o))
    assert np.abs(rgb - orgb).max() <= 1e-4


def test_segment_size_invariance_gpu(torch_cuda):
    """Fixed step, T_eps = 0: N_s does not change which samples exist; the
    GPU images agree to rounding for N_s = 2, 4, 8, 16."""
    sc = inputs.make_scene("cluster", 8000, 71)
    cam = inputs.look_at_camera(31, 29, (0.3, 0.1, 2.8))
    r, _ = renderer_for(sc)
    ref = None
    for ns in (2, 4, 8, 16):
        rgb, T = (x.cpu().numpy() for x in r.forward([cam], _opts(dt=0.005, t_eps=0.0, n_s=ns)))
        if ref is None:
            ref = rgb
        d = np.abs(rgb - ref).max(axis=1)
        # a sample on an ellipsoid boundary may be counted by q <= k^2 yet fall
        # outside the rounded chord of a neighbouring segment: <= sigma_eps*dt
        assert d.max() <= 1e-4 and (d <= 2e-6).mean() >= 0.999
