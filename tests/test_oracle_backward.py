"""Pins of the oracle's adjoint against FP64 central finite differences of the
oracle's own forward, a Taylor-remainder test, a closed-form derivative and the
quaternion-normalisation invariant.  The sample schedule and the truncation
boundary are piecewise constant in the parameters; the FD checks use settings
where no discrete decision flips (or detect flips and skip)."""
import math

import numpy as np
import pytest

import oracle
from paper_2509_07782_amd import inputs

KEYS = ("means", "log_scales", "quats", "density", "sh")


def tiny_scene(seed=0, n=5, deg=3, spread=0.12, ls=-2.6):
    rng = np.random.default_rng(seed)
    K = (deg + 1) ** 2
    return dict(means=rng.uniform(-spread, spread, (n, 3)),
                log_scales=ls + 0.3 * rng.standard_normal((n, 3)),
                quats=rng.standard_normal((n, 4)),
                density=rng.uniform(5.0, 30.0, n),
                sh=rng.normal(0.0, 0.5, (n, K, 3)), sh_degree=deg)


def loss_weights(n_rays, seed=1):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n_rays, 3)), rng.standard_normal(n_rays)


def loss(sc, cam, op, gC, gT):
    rgb, T, _, _ = oracle.render(sc, cam, op)
    return float(np.sum(rgb * gC) + np.sum(T * gT))


def fd_grad(sc, cam, op, gC, gT, key, idx, h):
    p = sc[key].copy()
    sp = dict(sc)
    v0 = p[idx]
    p[idx] = v0 + h
    sp[key] = p
    lp = loss(sp, cam, op, gC, gT)
    p = p.copy()
    p[idx] = v0 - h
    sp[key] = p
    lm = loss(sp, cam, op, gC, gT)
    return (lp - lm) / (2 * h)


CAM = inputs.look_at_camera(5, 4, (0.05, 0.03, 1.5), fov_deg=12.0)


@pytest.mark.parametrize("ess,teps,bg", [(1, 0.0, (0.0, 0.0, 0.0)), (0, 0.0, (0.3, 0.1, 0.7)),
                                         (2, 0.0, (0.2, 0.2, 0.2))])
def test_adjoint_matches_central_differences(ess, teps, bg):
    sc = tiny_scene()
    op = oracle.Opts(dt=0.004, n_s=8, ess=ess, t_eps=teps, sigma_eps=1e-30, bg=bg)
    n = CAM.width * CAM.height
    gC, gT = loss_weights(n)
    pix = np.arange(n)
    g = oracle.backward(sc, CAM, op, pix, gC, gT)
    rgb, T, st, _ = oracle.render(sc, CAM, op)
    assert (st[:, 0] >= 2).mean() > 0.5          # rays meet several Gaussians
    for key in KEYS:
        fd = np.zeros_like(sc[key])
        for idx in np.ndindex(*sc[key].shape):
            h = 1e-6 * max(1.0, abs(sc[key][idx]))
            fd[idx] = fd_grad(sc, CAM, op, gC, gT, key, idx, h)
        err = np.abs(g[key] - fd)
        scale = np.abs(fd).max()
        assert scale > 0
        assert err.max() <= 1e-6 * scale + 1e-8, (key, err.max(), scale)


def test_adjoint_with_truncation_and_termination():
    """sigma_eps = 0.01 (truncated ellipsoids) and T_eps > 0: central
    differences at two step sizes; parameters whose two estimates disagree
    (a sample crossed an ellipsoid boundary) are skipped, and few may be."""
    sc = tiny_scene(seed=3, n=8, spread=0.06)
    op = oracle.Opts(dt=0.004, n_s=8, ess=1, t_eps=1e-3, sigma_eps=0.01)
    n = CAM.width * CAM.height
    gC, gT = loss_weights(n, seed=4)
    g = oracle.backward(sc, CAM, op, np.arange(n), gC, gT)
    checked = skipped = 0
    for key in KEYS:
        scale = np.abs(g[key]).max()
        for idx in np.ndindex(*sc[key].shape):
            h = 1e-7 * max(1.0, abs(sc[key][idx]))
            f1 = fd_grad(sc, CAM, op, gC, gT, key, idx, h)
            f2 = fd_grad(sc, CAM, op, gC, gT, key, idx, h / 2)
            if abs(f1 - f2) > 1e-5 * scale + 1e-7:
                skipped += 1
                continue
            checked += 1
            assert abs(g[key][idx] - f2) <= 1e-5 * scale + 1e-7, (key, idx, g[key][idx], f2)
    assert skipped <= 0.03 * (checked + skipped), (checked, skipped)


def test_taylor_remainder_is_second_order():
    sc = tiny_scene(seed=5)
    op = oracle.Opts(dt=0.004, ess=1, t_eps=0.0, sigma_eps=1e-30, bg=(0.1, 0.2, 0.3))
    n = CAM.width * CAM.height
    gC, gT = loss_weights(n, seed=6)
    g = oracle.backward(sc, CAM, op, np.arange(n), gC, gT)
    rng = np.random.default_rng(7)
    v = {k: rng.standard_normal(sc[k].shape) for k in KEYS}
    L0 = loss(sc, CAM, op, gC, gT)
    gv = sum(float(np.sum(g[k] * v[k])) for k in KEYS)
    errs = []
    for h in (1e-2, 5e-3, 2.5e-3):
        sp = dict(sc)
        for k in KEYS:
            sp[k] = sc[k] + h * v[k]
        errs.append(abs(loss(sp, CAM, op, gC, gT) - L0 - h * gv))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.0 < r1 < 5.0 and 3.0 < r2 < 5.0, errs


def test_quaternion_gradient_orthogonal_to_quaternion():
    """R depends on q/|q| only, so dL/dq is orthogonal to q."""
    sc = tiny_scene(seed=8)
    op = oracle.Opts(dt=0.004, ess=1, t_eps=0.0, sigma_eps=0.01)
    n = CAM.width * CAM.height
    gC, gT = loss_weights(n, seed=9)
    g = oracle.backward(sc, CAM, op, np.arange(n), gC, gT)
    dots = np.einsum("ij,ij->i", g["quats"], sc["quats"])
    assert np.abs(dots).max() <= 1e-12 * np.abs(g["quats"]).max() * np.abs(sc["quats"]).max()
    assert np.abs(g["quats"]).max() > 0


def test_density_gradient_closed_form_single_gaussian():
    """C = c (1 - e^{-sigma I}), T = e^{-sigma I} for one Gaussian, so
    dC/dsigma = c I e^{-sigma I} and dT/dsigma = -I e^{-sigma I}."""
    Y0 = 0.5 / math.sqrt(math.pi)
    c = np.array([0.2, 0.5, 0.9])
    sc = dict(means=np.array([[0.02, -0.01, 0.05]]), log_scales=np.array([[-2.2, -2.7, -2.4]]),
              quats=np.array([[0.9, 0.2, -0.3, 0.1]]), density=np.array([12.0]),
              sh=(c / Y0).reshape(1, 1, 3), sh_degree=0)
    cam = inputs.look_at_camera(1, 1, (0.0, 0.0, 3.0))
    op = oracle.Opts(dt=0.002, ess=1, t_eps=0.0, sigma_eps=1e-30)
    _, T, _, _ = oracle.render(sc, cam, op)
    I = -math.log(T[0]) / 12.0
    gC = np.array([[1.0, -2.0, 0.5]])
    g = oracle.backward(sc, cam, op, [0], gC, np.array([0.7]))
    ref = float(gC[0] @ c) * I * math.exp(-12.0 * I) - 0.7 * I * math.exp(-12.0 * I)
    np.testing.assert_allclose(g["density"][0], ref, rtol=1e-9)
