"""Pins of the oracle's spherical-Gaussian colour lobes (the 9 SH + 7 SG
appearance model of the supplement's comparison with 3D-GS): the lobe's
integral over the sphere in closed form, invariance under a common rotation
and under the axis length, and the adjoint of the lobe parameters against
FP64 central differences of the rendered image."""
import math

import numpy as np
from scipy.spatial.transform import Rotation

import oracle
from paper_2509_07782_amd import inputs


def lobe_scene(amp, axis, lam, sh_degree=2):
    k = (sh_degree + 1) ** 2
    return dict(means=np.zeros((1, 3)), log_scales=np.full((1, 3), -1.0),
                quats=np.array([[1.0, 0, 0, 0]]), density=np.array([10.0]),
                sh=np.zeros((1, k, 3)), sh_degree=sh_degree,
                sg=np.array([[list(amp) + list(axis) + [lam]]], np.float64))


def sphere_quadrature(n_theta=96, n_phi=192):
    """Directions and weights of a product rule on the unit sphere:
    Gauss-Legendre in cos(theta), uniform in phi."""
    x, w = np.polynomial.legendre.leggauss(n_theta)
    phi = (np.arange(n_phi) + 0.5) * 2 * math.pi / n_phi
    ct, ph = np.meshgrid(x, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    dirs = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    wts = (w[:, None] * np.full(n_phi, 2 * math.pi / n_phi)[None, :]).reshape(-1)
    return dirs, wts


def test_lobe_integral_over_the_sphere():
    """int exp(lambda (u.d - 1)) dd = 2 pi (1 - exp(-2 lambda)) / lambda, for
    any axis direction and length."""
    dirs, wts = sphere_quadrature()
    for lam, axis in ((0.7, (0, 0, 1)), (5.0, (0.3, -0.2, 0.9)), (23.0, (-2.0, 1.0, 0.5))):
        sc = lobe_scene((1.0, 2.0, -0.5), axis, lam)
        col = oracle.colour(sc, 0, dirs)
        want = 2 * math.pi * (1 - math.exp(-2 * lam)) / lam
        got = (col * wts[:, None]).sum(0)
        np.testing.assert_allclose(got, np.array([1.0, 2.0, -0.5]) * want, rtol=1e-9)
        # the peak value is the amplitude, at the axis direction
        u = np.asarray(axis, float) / np.linalg.norm(axis)
        np.testing.assert_allclose(oracle.colour(sc, 0, u[None])[0], [1.0, 2.0, -0.5], rtol=1e-12)


def test_lobes_rotate_with_the_axis_and_ignore_its_length():
    rng = np.random.default_rng(3)
    R = Rotation.random(random_state=4).as_matrix()
    sc = inputs.make_scene("cluster", 3, 7, sh_degree=0, n_sg=7)
    sc = {k: (v.astype(np.float64) if isinstance(v, np.ndarray) else v) for k, v in sc.items()}
    sc["sh"][:] = 0.0
    d = rng.standard_normal((50, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rot = dict(sc)
    rot["sg"] = sc["sg"].copy()
    rot["sg"][..., 3:6] = sc["sg"][..., 3:6] @ R.T * 3.7
    a = oracle.colour(sc, 1, d)
    b = oracle.colour(rot, 1, d @ R.T)
    np.testing.assert_allclose(a, b, rtol=1e-11, atol=1e-13)


def test_lobe_adjoint_against_central_differences():
    """Gradients of a weighted sum of pixels with respect to every lobe
    parameter of a small SH-degree-2 + 7-lobe scene, against FP64 central
    differences of the oracle render; the axis gradient is orthogonal to the
    axis (the colour sees only its direction)."""
    sc = inputs.make_scene("cluster", 40, 11, sh_degree=2, n_sg=7)
    sc = {k: (v.astype(np.float64) if isinstance(v, np.ndarray) else v) for k, v in sc.items()}
    sc["log_scales"] += 1.5
    cam = inputs.look_at_camera(9, 7, (0.2, 0.1, 2.8), fov_deg=40.0)
    op = oracle.Opts(dt=0.01, ess=1, t_eps=0.0, sigma_eps=1e-30)
    n = cam.width * cam.height
    rng = np.random.default_rng(5)
    wC = rng.standard_normal((n, 3))
    pix = np.arange(n)
    g = oracle.backward(sc, cam, op, pix, wC)
    assert g["sg"].shape == sc["sg"].shape
    dots = np.einsum("lkj,lkj->lk", g["sg"][..., 3:6], sc["sg"][..., 3:6])
    assert np.abs(dots).max() <= 1e-10 * np.abs(g["sg"]).max()

    def loss(s):
        rgb, _, _, _ = oracle.render(s, cam, op, pix)
        return float((rgb * wC).sum())

    big = np.argsort(-np.abs(g["density"]))[:4]
    checked = 0
    for l in big:
        for k in (0, 3, 6):
            for e in range(7):
                h = 1e-6 * max(1.0, abs(sc["sg"][l, k, e]))
                sp = dict(sc); sp["sg"] = sc["sg"].copy(); sp["sg"][l, k, e] += h
                sm = dict(sc); sm["sg"] = sc["sg"].copy(); sm["sg"][l, k, e] -= h
                fd = (loss(sp) - loss(sm)) / (2 * h)
                assert abs(g["sg"][l, k, e] - fd) <= 1e-6 * abs(fd) + 1e-9 * np.abs(g["sg"]).max(), \
                    (l, k, e, g["sg"][l, k, e], fd)
                checked += 1
    assert checked == 84
    # the lobes enter the other gradients too: the density gradient moves
    # when the amplitudes do
    s2 = dict(sc); s2["sg"] = sc["sg"].copy(); s2["sg"][..., :3] *= 2.0
    g2 = oracle.backward(s2, cam, op, pix, wC)
    assert np.abs(g2["density"] - g["density"]).max() > 1e-6 * np.abs(g["density"]).max()
