"""Pins of the oracle's per-Gaussian geometry, SH basis, rays and closed forms.

Each check compares the oracle with something other than itself: a library
routine (scipy), a different formula for the same quantity (Hamilton product,
pinhole projection), Monte-Carlo sampling, or values fixed by the paper.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy.special import sph_harm_y

import oracle
from oracle import geometry
from paper_2509_07782_amd import inputs

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def _unit(rng, n):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def test_sh_basis_matches_scipy():
    """Real SH with the Condon-Shortley phase from scipy's complex Y_l^m."""
    rng = np.random.default_rng(0)
    d = _unit(rng, 200)
    Y = oracle.sh_basis(3, d)
    theta = np.arccos(np.clip(d[:, 2], -1, 1))
    phi = np.arctan2(d[:, 1], d[:, 0])
    for l in range(4):
        for m in range(-l, l + 1):
            c = sph_harm_y(l, abs(m), theta, phi)
            if m == 0:
                ref = c.real
            elif m > 0:
                ref = math.sqrt(2) * c.real
            else:
                ref = math.sqrt(2) * c.imag
            np.testing.assert_allclose(Y[:, l * l + l + m], ref, atol=1e-12)


def test_sh_basis_orthonormal():
    """Gauss-Legendre in cos(theta) x uniform azimuth integrates Y_i Y_j exactly."""
    xg, wg = np.polynomial.legendre.leggauss(16)
    nphi = 32
    phi = (np.arange(nphi) + 0.5) * 2 * math.pi / nphi
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    w = (wg[:, None] * np.full(nphi, 2 * math.pi / nphi)[None, :]).reshape(-1)
    Y = oracle.sh_basis(3, d)
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_low_order_signs():
    """Degree-1 functions are -c*y, c*z, -c*x with c = sqrt(3/(4 pi))."""
    c = math.sqrt(3 / (4 * math.pi))
    for d in ([1, 0, 0], [0, 1, 0], [0, 0, 1]):
        Y = oracle.sh_basis(1, np.array(d, float))[0]
        np.testing.assert_allclose(Y[1:], [-c * d[1], c * d[2], -c * d[0]], atol=1e-14)
        assert abs(Y[0] - 0.5 / math.sqrt(math.pi)) < 1e-15


def _scene_one(mu, ls, q, sig, deg=0):
    k = (deg + 1) ** 2
    return dict(means=np.array([mu], np.float64), log_scales=np.array([ls], np.float64),
                quats=np.array([q], np.float64), density=np.array([sig], np.float64),
                sh=np.ones((1, k, 3)), sh_degree=deg)


def test_rotation_matches_hamilton_product_and_scipy():
    rng = np.random.default_rng(1)
    sc = inputs.make_scene("uniform", 64, 5)
    _, act, R, _ = oracle.gaussians(sc, 0.01)
    q = sc["quats"].astype(np.float64)
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    Rs = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()
    np.testing.assert_allclose(R[act], Rs[act], atol=1e-12)

    def hmul(a, b):
        w1, x1, y1, z1 = a
        w2, x2, y2, z2 = b
        return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                         w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])

    for i in np.nonzero(act)[0][:10]:
        v = rng.standard_normal(3)
        qc = q[i] * np.array([1, -1, -1, -1])
        rv = hmul(hmul(q[i], np.r_[0.0, v]), qc)[1:]
        np.testing.assert_allclose(R[i] @ v, rv, atol=1e-12)
        assert abs(np.linalg.det(R[i]) - 1) < 1e-12


def test_level_set_and_truncation():
    """k^2 = 2 ln(sigma~/sigma_eps): the truncated density is sigma~ at the
    centre, sigma_eps on the ellipsoid and zero outside (Supp. B)."""
    sig, eps = 7.0, 0.01
    sc = _scene_one([0.1, -0.2, 0.3], [-2.0, -2.5, -1.5], [0.3, -0.5, 0.2, 0.7], sig)
    k2, act, R, half = oracle.gaussians(sc, eps)
    assert act[0] and abs(k2[0] - 2 * math.log(sig / eps)) < 1e-12
    mu = sc["means"][0]
    s = np.exp(sc["log_scales"][0])
    k = math.sqrt(k2[0])
    u = _unit(np.random.default_rng(2), 50)
    Rs = Rotation.from_quat(np.array(sc["quats"][0])[[1, 2, 3, 0]]).as_matrix()
    inside = mu + (u * (k * s * (1 - 1e-9))) @ Rs.T
    outside = mu + (u * (k * s * (1 + 1e-9))) @ Rs.T
    np.testing.assert_allclose(oracle.density_at(sc, eps, 0, inside), eps, rtol=1e-7)
    assert np.all(oracle.density_at(sc, eps, 0, outside) == 0)
    assert abs(oracle.density_at(sc, eps, 0, mu[None])[0] - sig) < 1e-12


def test_inactive_gaussians():
    sc = _scene_one([0, 0, 0], [-2, -2, -2], [1, 0, 0, 0], 0.005)
    assert not oracle.gaussians(sc, 0.01)[1][0]          # sigma~ <= sigma_eps
    sc = _scene_one([0, 0, 0], [-2, -2, -2], [0, 0, 0, 0], 5.0)
    assert not oracle.gaussians(sc, 0.01)[1][0]          # zero quaternion
    sc = _scene_one([np.nan, 0, 0], [-2, -2, -2], [1, 0, 0, 0], 5.0)
    assert not oracle.gaussians(sc, 0.01)[1][0]          # NaN parameter


def test_aabb_half_lengths_are_extreme_points():
    """L_i = k sqrt(sum_j r_ij^2 s_j^2) is the maximum of |x_i - mu_i| over the
    ellipsoid (Supp. B, minimal AABB): attained at the Cauchy-Schwarz point and
    never exceeded by sampled surface points."""
    rng = np.random.default_rng(3)
    sc = inputs.make_scene("cluster", 20, 7)
    k2, act, R, half = oracle.gaussians(sc, 0.01)
    u = _unit(rng, 200_000)
    for i in range(20):
        s = np.exp(sc["log_scales"][i].astype(np.float64))
        k = math.sqrt(k2[i])
        ext = np.abs((u * (k * s)) @ R[i].T).max(axis=0)
        assert np.all(ext <= half[i] * (1 + 1e-12))
        np.testing.assert_allclose(ext, half[i], rtol=2e-4)
        for ax in range(3):
            a = R[i][ax] * k * s
            ustar = a / np.linalg.norm(a)
            np.testing.assert_allclose(abs((R[i] @ (ustar * k * s))[ax]), half[i][ax], rtol=1e-12)


def test_volume_ratio_monte_carlo_and_bound():
    """Eq. 6 (exact ratio) against Monte Carlo, and Eq. 7 (bound) above it."""
    rng = np.random.default_rng(4)
    sc = inputs.make_scene("cluster", 6, 8, log_scale_sd=0.8)
    k2, act, R, half = oracle.gaussians(sc, 0.01)
    for i in range(6):
        s = np.exp(sc["log_scales"][i].astype(np.float64))
        r = geometry.aabb_volume_ratio(R[i], s)
        # the oracle's AABB half-lengths give the same ratio
        vol_e = 4 * math.pi / 3 * k2[i] ** 1.5 * np.prod(s)
        np.testing.assert_allclose(np.prod(2 * half[i]) / vol_e, r, rtol=1e-12)
        x = rng.uniform(-1, 1, (400_000, 3)) * half[i]
        z = (x @ R[i]) / (math.sqrt(k2[i]) * s)
        frac = np.mean(np.sum(z * z, 1) <= 1)
        assert abs(1 / frac - r) / r < 0.02
        assert r <= geometry.ratio_bound(s) * (1 + 1e-12)


def test_volume_ratio_golden_sphere_and_equality():
    assert abs(geometry.aabb_volume_ratio(np.eye(3), [0.3, 0.3, 0.3]) - GOLD["volume_ratio"]["sphere"]) < 1e-14
    assert abs(geometry.ratio_bound([2.0, 2.0, 2.0]) - GOLD["volume_ratio"]["sphere"]) < 1e-14
    # equal half-lengths without a sphere: s^2 = (1,1,4) and third column (1,1,1)/sqrt3
    c3 = np.ones(3) / math.sqrt(3)
    c1 = np.array([1.0, -1.0, 0.0]) / math.sqrt(2)
    c2 = np.cross(c3, c1)
    R = np.stack([c1, c2, c3], axis=1)
    s = np.array([1.0, 1.0, 2.0])
    np.testing.assert_allclose(geometry.aabb_volume_ratio(R, s), geometry.ratio_bound(s), rtol=1e-12)
    assert geometry.ratio_bound(s) > GOLD["volume_ratio"]["sphere"]


def test_isotropic_loss_zero_iff_bound_below_r0():
    ls = np.log(np.array([[1.0, 1.0, 1.0], [1.0, 1.0, 30.0]]))
    r = geometry.ratio_bound(np.exp(ls))
    assert r[0] < 10 < r[1]
    assert geometry.isotropic_loss(ls[:1]) == 0.0
    np.testing.assert_allclose(geometry.isotropic_loss(ls), (r[1] - 10) / 2)


def test_adaptive_step_golden():
    g = GOLD["adaptive_step"]
    for d, T, dt in g["cases"]:
        v = geometry.adaptive_step(d, T, g["dt_min"], g["dt_max"], g["beta"])
        assert abs(v - dt) < 1e-15, (d, T, v, dt)


def test_regularized_scene_meets_bound():
    sc = inputs.make_scene("outdoor", 4000, 11, log_scale_sd=1.0)
    reg = inputs.regularize_log_scales(sc["log_scales"])
    rb = geometry.ratio_bound(np.exp(reg.astype(np.float64)))
    assert rb.max() <= 10.0 * (1 + 1e-5)
    # volume (sum of log-scales) preserved, already-good rows untouched
    np.testing.assert_allclose(reg.sum(1), sc["log_scales"].sum(1), atol=1e-4)
    good = geometry.ratio_bound(np.exp(sc["log_scales"].astype(np.float64))) <= 10
    np.testing.assert_allclose(reg[good], sc["log_scales"][good], atol=1e-6)
    assert (~good).sum() > 100


def test_rays_reproject_to_pixel_centres():
    """Inverse check of ray generation: o + t d projects to the pixel centre."""
    cam = inputs.look_at_camera(37, 23, (0.4, -0.3, 2.5), target=(0.1, 0.2, -0.1))
    pix = np.arange(37 * 23)
    o, d = oracle.rays(cam, pix)
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1, atol=1e-14)
    c2w = cam.cam_to_world.astype(np.float64)
    Rc, tc = c2w[:, :3], c2w[:, 3]
    np.testing.assert_allclose(o, np.broadcast_to(tc, o.shape))
    xc = (o + 4.0 * d - tc) @ Rc                  # world -> camera (R orthonormal)
    u = cam.fx * xc[:, 0] / xc[:, 2] + cam.cx
    v = cam.fy * xc[:, 1] / xc[:, 2] + cam.cy
    # Rc is orthonormal to float32 precision only
    np.testing.assert_allclose(u, pix % 37 + 0.5, atol=1e-4)
    np.testing.assert_allclose(v, pix // 37 + 0.5, atol=1e-4)
    assert np.all(xc[:, 2] > 0)


def test_densification_weight_is_projected_gradient():
    """Supp. (densification criterion and the projected mean): for a loss that
    depends on mu only through its projection mu_P = o + f (mu - o)/|mu - o|
    onto the sphere of radius f about the camera, the gradient along that
    sphere has norm (r/f)|grad_mu L|, r = |mu - o|.  The oracle's per-view
    weight alpha |grad_mu L| must equal that norm (autograd, FP64)."""
    import torch
    rng = np.random.default_rng(3)
    V, N = 3, 64
    o = rng.normal(0.0, 2.0, (V, 3))
    f = rng.uniform(300.0, 1500.0, V)
    mu = rng.normal(0.0, 3.0, (N, 3))
    w = torch.tensor(rng.normal(0.0, 1.0, (N, 3)), dtype=torch.float64)
    grads, proj_norms = [], []
    for v in range(V):
        ov = torch.tensor(o[v])

        def h(p):   # any smooth function of the projected point
            q = (p - ov) / f[v]
            return (torch.sin(q * w) * q.roll(1, dims=1)).sum() + (q[:, 0] * q[:, 2] ** 2).sum()

        m = torch.tensor(mu, requires_grad=True)
        d = m - ov
        P = ov + f[v] * d / d.norm(dim=1, keepdim=True)
        h(P).backward()
        grads.append(m.grad.numpy().copy())
        p = P.detach().clone().requires_grad_(True)
        h(p).backward()
        u = (d / d.norm(dim=1, keepdim=True)).detach()
        gp = p.grad - (p.grad * u).sum(dim=1, keepdim=True) * u     # tangential part
        proj_norms.append(gp.norm(dim=1).numpy())
        # the assumption of the derivation holds here: no radial component
        assert np.abs((m.grad * u).sum(dim=1).numpy()).max() <= 1e-12 * m.grad.norm().item() + 1e-300
    tot, views = geometry.densification_statistic(mu, np.stack(grads), o, f)
    assert np.allclose(tot, np.sum(proj_norms, axis=0), rtol=1e-12, atol=0.0)
    assert np.array_equal(views, np.full(N, V))
    # a view in which a Gaussian gets no gradient adds nothing and is not counted
    g0 = np.stack(grads)
    g0[1, :10] = 0.0
    tot0, views0 = geometry.densification_statistic(mu, g0, o, f)
    assert np.array_equal(views0[:10], np.full(10, V - 1))
    assert np.allclose(tot0[:10], proj_norms[0][:10] + proj_norms[2][:10], rtol=1e-12)
