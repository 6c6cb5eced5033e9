"""Densification statistic (Sec. 3.5, Eq. 12) fused into the backward: for
each view v, alpha_v |dL_v/dmu| with alpha_v = |mu - o_v| / f_v, summed over
views, and the number of views with a non-zero mean gradient -- against the
same quantities formed from the FP64 oracle's per-view adjoints."""
import numpy as np
import pytest

import oracle
from oracle import geometry
from paper_2509_07782_amd import inputs
from paper_2509_07782_amd.render import RenderOptions
from helpers import PARAM_KEYS, grad_rel_errors, oracle_opts, renderer_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _cams8():
    """Eight views around the cluster at different distances and sizes."""
    cams = []
    for i in range(8):
        az = 2.0 * np.pi * i / 8.0
        rad = 2.6 + 0.25 * i
        pos = (rad * np.sin(az), 0.4 * np.cos(3 * az), rad * np.cos(az))
        cams.append(inputs.look_at_camera(23 + 3 * i, 19 + 2 * (i % 3), pos, fov_deg=50.0))
    return cams


def test_densification_statistic_matches_oracle(torch_cuda):
    """Eight views; the first view's loss is scaled by 1e3, so a later view's
    mean gradient is tiny next to the running sum: each view's statistic is
    taken from that view's slots alone, so it keeps full precision."""
    torch = torch_cuda
    sc = inputs.make_scene("cluster", 2000, 11, sh_degree=3)
    cams = _cams8()
    o = RenderOptions(dt=0.005, ess=1, t_eps=0.0)
    r, params = renderer_for(sc)
    st = r.new_state()
    rgb, T = r.forward(cams, o, state=st)
    R = rgb.shape[0]
    rng = np.random.default_rng(5)
    gC = rng.normal(0.0, 1.0, (R, 3)).astype(np.float32)
    m0 = cams[0].width * cams[0].height
    gC[:m0] *= 1e3
    gCt = torch.from_numpy(gC).cuda()
    n = sc["means"].shape[0]
    dens = torch.zeros(n, device="cuda")
    views = torch.zeros(n, device="cuda", dtype=torch.int32)
    g_dens = r.backward(st, rgb, T, gCt, None, params, dens, views)
    g_plain = r.backward(st, rgb, T, gCt, None, params)
    torch.cuda.synchronize()
    assert r.ctx.error_flags() == 0
    # marching the views one at a time leaves the gradients unchanged (up to
    # the order of FP32 atomics)
    errs = grad_rel_errors({k: g_dens[k].cpu().numpy() for k in PARAM_KEYS},
                           {k: g_plain[k].cpu().numpy() for k in PARAM_KEYS})
    for k, (rel, frac) in errs.items():
        assert rel <= 1e-5, (k, rel)
    # oracle: per-view adjoints of the loss restricted to that view, then Eq. 12
    gmu, origins, focals = [], [], []
    off = 0
    for cam in cams:
        m = cam.width * cam.height
        g = oracle.backward(sc, cam, oracle_opts(o), np.arange(m), gC[off:off + m].astype(np.float64))
        off += m
        gmu.append(g["means"])
        origins.append(np.asarray(cam.cam_to_world, np.float64).reshape(3, 4)[:, 3])
        focals.append(float(cam.fx))
    gmu = np.stack(gmu)
    # every later view's statistic is compared on its own as well
    for v_i in range(1, len(cams)):
        one = torch.zeros(n, device="cuda")
        one_v = torch.zeros(n, device="cuda", dtype=torch.int32)
        st1 = r.new_state()
        rgb1, T1 = r.forward([cams[v_i]], o, state=st1)
        lo = sum(c.width * c.height for c in cams[:v_i])
        r.backward(st1, rgb1, T1, gCt[lo:lo + cams[v_i].width * cams[v_i].height].contiguous(),
                   None, params, one, one_v)
        st1.close()
        ref1, _ = geometry.densification_statistic(sc["means"], gmu[v_i:v_i + 1],
                                                   origins[v_i:v_i + 1], focals[v_i:v_i + 1])
        d1 = one.cpu().numpy().astype(np.float64)
        assert np.linalg.norm(d1 - ref1) <= 1e-3 * np.linalg.norm(ref1), v_i
    ref, ref_views = geometry.densification_statistic(sc["means"], gmu, origins, focals)
    d = dens.cpu().numpy().astype(np.float64)
    v = views.cpu().numpy()
    assert (ref_views > 0).mean() > 0.2
    assert np.linalg.norm(d - ref) <= 1e-3 * np.linalg.norm(ref)
    rms = np.sqrt(np.mean(ref * ref))
    assert (np.abs(d - ref) <= 1e-3 * np.abs(ref) + 1e-3 * rms).mean() >= 0.999
    # the contribution of the views after the first: the sum minus the first
    # view's own statistic, against the oracle's
    first, _ = geometry.densification_statistic(sc["means"], gmu[:1], origins[:1], focals[:1])
    rest_ref = ref - first
    st0 = r.new_state()
    rgb0, T0 = r.forward([cams[0]], o, state=st0)
    d0 = torch.zeros(n, device="cuda")
    v0 = torch.zeros(n, device="cuda", dtype=torch.int32)
    r.backward(st0, rgb0, T0, gCt[:m0].contiguous(), None, params, d0, v0)
    st0.close()
    rest = d - d0.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(rest - rest_ref) <= 2e-3 * np.linalg.norm(rest_ref) + 1e-3 * np.linalg.norm(ref) * 1e-3
    # view counts: equal wherever the oracle gradient is not vanishingly small
    clear = (ref == 0) | (ref > 1e-6 * ref.max())
    assert (v[clear] == ref_views[clear]).mean() >= 0.999
    # running sums: a second call adds the same amounts again
    r.backward(st, rgb, T, gCt, None, params, dens, views)
    torch.cuda.synchronize()
    assert np.allclose(dens.cpu().numpy(), 2 * d, rtol=1e-5, atol=1e-12)
    assert np.array_equal(views.cpu().numpy(), 2 * v)
    st.close()
    r.close()
