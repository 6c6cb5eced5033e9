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


def _check_pixels(rgb, orgb, mg, frac_bad=0.001):
    """Every pixel within 1e-4 of the oracle, except rays whose oracle
    decisions had a near tie (margin below 1e-6: an inclusion, termination
    or emptiness decision); those stay below 0.1 % of the rays."""
    err = np.abs(rgb - orgb).max(axis=1)
    bad = err > 1e-4
    assert bad.mean() <= frac_bad, (bad.sum(), err.max())
    assert np.all(mg[bad] < 1e-6), mg[bad]
    return err


def test_config2_full_size(torch_cuda):
    """100k Gaussians, 800x800: fixed-step and adaptive pixels against the
    oracle on every second pixel of every second row; Morton tiles ==
    scanline bit for bit."""
    sc = inputs.config_scene(2)
    cam = inputs.config_cameras(2)[0]
    r, _ = renderer_for(sc)
    pix = inputs.pixel_subset(cam, 2)
    for o in (_opts(dt=0.005, ess=1, t_eps=1e-4), _opts(adaptive=True, ess=1, t_eps=1e-4)):
        rgb, T = (x.cpu().numpy() for x in r.forward([cam], o))
        orgb, oT, ost, mg = oracle.render(sc, cam, oracle_opts(o), pix)
        assert (ost[:, 0] > 0).mean() > 0.2
        _check_pixels(rgb[pix], orgb, mg)
        raster = [x.cpu().numpy() for x in r.forward([cam], _opts(**{**o.__dict__, "ray_order": 0}))]
        assert np.array_equal(raster[0], rgb) and np.array_equal(raster[1], T)
    assert r.ctx.error_flags() == 0


@pytest.fixture(scope="module")
def config3(torch_cuda):
    sc = inputs.config_scene(3)
    cams = inputs.config_cameras(3)
    r, params = renderer_for(sc)
    return sc, cams, r, params


def test_config3_benchmark_mode_pixels_and_gradients(config3, torch_cuda):
    """1M Gaussians, 4 views 1024x768, in the benchmark's mode (adaptive
    steps, closest-hit restarts, T_eps 1e-4, persistent launch, the forward's
    searches recorded and replayed by the backward): every 16th pixel of
    every 16th row of every view against the oracle, and the gradients of a
    loss on those pixels against the oracle adjoint of the same loss."""
    torch = torch_cuda
    sc, cams, r, params = config3
    o = _opts(adaptive=True, ess=1, t_eps=1e-4, persistent=True)
    st = r.new_state()
    rgb, T = r.forward(cams, o, state=st)
    rgb_np = rgb.cpu().numpy()
    R = rgb.shape[0]
    rng = np.random.default_rng(3)
    gC = np.zeros((R, 3), np.float32)
    ref = None
    oo = oracle_opts(o)
    for c, off in zip(cams, _view_offsets(cams)):
        pix = inputs.pixel_subset(c, 16)
        orgb, oT, ost, mg = oracle.render(sc, c, oo, pix)
        _check_pixels(rgb_np[off + pix], orgb, mg)
        w = rng.standard_normal((len(pix), 3)).astype(np.float32)
        gC[off + pix] = w
        g = oracle.backward(sc, c, oo, pix, w.astype(np.float64), None)
        ref = g if ref is None else {k: ref[k] + g[k] for k in PARAM_KEYS}
    gg = r.backward(st, rgb, T, torch.from_numpy(gC).cuda(), None, params)
    torch.cuda.synchronize()
    assert r.ctx.backward_replayed()
    assert r.ctx.error_flags() == 0
    st.close()
    got = {k: v.cpu().numpy() for k, v in gg.items()}
    for k, (rel, frac) in grad_rel_errors(got, ref).items():
        assert rel <= 1e-3, (k, rel)
        assert frac >= 0.999, (k, frac)


def test_config3_fixed_step_masked_gradients(config3, torch_cuda):
    """Fixed step, T_eps 0 (no near ties at all): gradients of a loss on
    every 64th pixel of the 4 views against the oracle adjoint."""
    torch = torch_cuda
    sc, cams, r, params = config3
    o = _opts(dt=0.005, ess=1, t_eps=0.0, persistent=True)
    st = r.new_state()
    rgb, T = r.forward(cams, o, state=st)
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
    gg = r.backward(st, rgb, T, torch.from_numpy(gC).cuda(), None, params)
    torch.cuda.synchronize()
    assert r.ctx.error_flags() == 0
    st.close()
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
    st = r.new_state()
    rgb, T = r.forward(cams, o, state=st)
    R = rgb.shape[0]
    rng = np.random.default_rng(11)
    gC = np.zeros((R, 3), np.float32)
    subs = []
    for c, off in zip(cams, _view_offsets(cams)):
        pix = inputs.pixel_subset(c, 32)
        w = rng.standard_normal((len(pix), 3)).astype(np.float32)
        gC[off + pix] = w
        subs.append((c, pix, w.astype(np.float64)))
    gg = r.backward(st, rgb, T, torch.from_numpy(gC).cuda(), None, params)
    torch.cuda.synchronize()
    assert r.ctx.error_flags() == 0
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
            # the oracle adjoint against FP64 differences, element by element
            assert abs(ref[k][idx] - fd) <= 1e-3 * abs(fd) + 1e-6 * np.abs(ref[k]).max(), \
                (k, idx, ref[k][idx], fd)
            # the GPU against FP64 differences: 1e-3 relative on entries that
            # are not tiny next to the tensor's largest
            if abs(fd) >= 1e-2 * np.abs(ref[k]).max():
                assert abs(got[k][idx] - fd) <= 1e-3 * abs(fd), (k, idx, got[k][idx], fd)
            else:
                assert abs(got[k][idx] - fd) <= 1e-5 * np.abs(ref[k]).max(), (k, idx, got[k][idx], fd)


def test_config4_false_positives_and_parity(torch_cuda):
    """Outdoor layout (3M Gaussians, shell to r = 50, 1297x840 views from
    inside), stress log-scale spread 1.0.  Whole-ray AABB false positives
    (Sec. 3.4, Eq. 6) on every 16th pixel of every 16th row: the GPU count
    equals the oracle's up to each ray's near ties, and the scale-regularised
    scene has fewer per ray than the unregularised one.  Pixels of the
    regularised scene on the same subset of every view against the oracle."""
    torch = torch_cuda
    from paper_2509_07782_amd import lib
    cams = inputs.config_cameras(4)
    fp = {}
    o = _opts(adaptive=True, ess=1, t_eps=1e-4, persistent=True)
    oo = oracle_opts(o)
    for reg in (False, True):
        sc = inputs.config_scene(4, regularized=reg, log_scale_sd=1.0)
        r, _ = renderer_for(sc)
        rgb, T, st = r.forward(cams, o, stats=True)
        t_end = st[:, lib.STAT_T_END].contiguous().view(torch.float32)
        rgb = rgb.cpu().numpy()
        counts = []
        for vi, (c, off) in enumerate(zip(cams, _view_offsets(cams))):
            pix = inputs.pixel_subset(c, 16)
            pix_t = torch.from_numpy(pix.astype(np.int32)).cuda()
            te = t_end[off + pix_t.long()].contiguous()
            cnt = r.false_positives(c, pix_t, te).cpu().numpy().astype(np.int64)
            counts.append(cnt)
            if vi == 0:
                ocnt, oties, ot_end = oracle.false_positives(sc, c, oo, pix)
                same_end = np.abs(te.cpu().numpy() - ot_end) <= 1e-5 * np.maximum(1.0, ot_end)
                assert same_end.mean() >= 0.99
                d = np.abs(cnt - ocnt)[same_end]
                assert np.all(d <= oties[same_end]), d.max()
                assert (d == 0).mean() >= 0.98
            if reg:
                orgb, oT, ost, mg = oracle.render(sc, c, oo, pix)
                _check_pixels(rgb[off + pix], orgb, mg)
        fp[reg] = float(np.concatenate(counts).mean())
        assert r.ctx.error_flags() == 0
        r.close()
    print(f"whole-ray AABB false positives per ray: unregularised {fp[False]:.1f}, "
          f"regularised {fp[True]:.1f}")
    assert fp[True] < fp[False], fp


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
    # every 32nd pixel of every 32nd row of the 16 views against the oracle
    rgb_np = rgb.cpu().numpy()
    oo = oracle_opts(ob)
    got, want, margins = [], [], []
    for c, off in zip(cams, _view_offsets(cams)):
        pix = inputs.pixel_subset(c, 32)
        orgb, oT, ost, mg = oracle.render(sc, c, oo, pix)
        got.append(rgb_np[off + pix])
        want.append(orgb)
        margins.append(mg)
    _check_pixels(np.concatenate(got), np.concatenate(want), np.concatenate(margins))
    assert sum(len(m) for m in margins) > 10000
    assert r.ctx.error_flags() == 0
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
    r.check_errors()


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
    r.check_errors()


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
    r.check_errors()
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
