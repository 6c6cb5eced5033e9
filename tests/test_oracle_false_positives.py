"""Pins of the oracle's whole-ray false-positive count (Sec. 3.4, Eq. 6; the
minimal AABB of Supp. B): a Gaussian counts when its minimal axis-aligned box
meets the ray over [t_n, t_end] while its truncation ellipsoid does not, t_end
being where the march ended (Algorithm 1).  Spheres have the cube of side 2
rho as minimal box, so rays near a cube's edge give known counts; a rotated
ellipsoid's box comes from surface sampling (extreme points), its ray test
from the minimum of the quadratic form along the ray."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from paper_2509_07782_amd import inputs

Y0 = 0.5 / math.sqrt(math.pi)
SIG, SE = 50.0, 0.01
K = math.sqrt(2.0 * math.log(SIG / SE))


def ray_view(x, y, t_far=6.0):
    # one ray from (x, y, 3) along -z
    return inputs.look_at_camera(1, 1, (x, y, 3.0), target=(x, y, 0.0), t_near=0.0, t_far=t_far)


def scene(means, scales, quats):
    n = len(means)
    return dict(means=np.array(means, np.float64), log_scales=np.log(np.array(scales, np.float64)),
                quats=np.array(quats, np.float64), density=np.full(n, SIG),
                sh=np.full((n, 1, 3), 0.5 / Y0), sh_degree=0)


OPTS = oracle.Opts(dt=0.01, n_s=8, ess=0, t_eps=0.0, sigma_eps=SE)


def count(sc, cam, opts=OPTS):
    c, ties, t_end = oracle.false_positives(sc, cam, opts)
    return int(c[0]), int(ties[0]), float(t_end[0])


@pytest.mark.parametrize("x,y,t_far,expect", [
    (0.9, 0.9, 6.0, 1),     # inside the cube's shadow, outside the sphere's
    (0.5, 0.5, 6.0, 0),     # through the sphere
    (1.1, 0.0, 6.0, 0),     # beside the cube
    (0.9, 0.9, 1.5, 0),     # the cube lies beyond t_end = t_far
    (0.6, 0.0, 3.0 - 0.9, 1),   # t_end between the cube's face and the sphere's chord
    (0.6, 0.0, 3.0 - 0.7, 0),   # t_end past the start of the chord (3 - 0.8 rho)
])
def test_sphere_and_its_cube(x, y, t_far, expect):
    rho = 1.0
    s = rho / K
    sc = scene([[0.0, 0.0, 0.0]], [[s, s, s]], [[1.0, 0.0, 0.0, 0.0]])
    c, ties, t_end = count(sc, ray_view(x * rho, y * rho, t_far))
    assert t_end == pytest.approx(t_far)
    assert ties == 0
    assert c == expect


def test_counts_add_over_gaussians_and_skip_inactive():
    rho = 0.2
    s = rho / K
    corners = [[0.9 * rho * sx + 2.5 * i, 0.9 * rho * sy, -0.5 * i] for i, (sx, sy) in
               enumerate([(1, 1), (-1, 1), (1, -1), (-1, -1)])]
    # sphere i sits 2.5 i along x; the ray at x = 2.5 i passes its cube's corner
    total = 0
    for i, m in enumerate(corners):
        sc = scene(corners, [[s, s, s]] * 4, [[1.0, 0.0, 0.0, 0.0]] * 4)
        c, _, _ = count(sc, ray_view(2.5 * i, 0.0))
        total += c
    assert total == 4
    # the same four spheres on one ray's line, one of them inactive
    means = [[0.9 * rho, 0.9 * rho, z] for z in (1.0, 0.0, -1.0, -2.0)]
    sc = scene(means, [[s, s, s]] * 4, [[1.0, 0.0, 0.0, 0.0]] * 4)
    assert count(sc, ray_view(0.0, 0.0))[0] == 4
    sc["density"][2] = SE / 2.0
    assert count(sc, ray_view(0.0, 0.0))[0] == 3


def test_t_end_is_where_termination_stopped_the_march():
    """Constant medium, fixed grid: the march stops at the first segment
    start with T <= T_eps; a cube-only sphere before that point counts, one
    past it does not."""
    dt, ns, sig = 0.01, 8, 0.8
    dS = dt * ns
    T5 = math.exp(-5 * sig * dS)
    rho = 0.05
    s = rho / K
    sc = dict(means=np.array([[0.0, 0.0, 0.0], [0.9 * rho, 0.9 * rho, 3.0 - 0.2],
                              [0.9 * rho, 0.9 * rho, 3.0 - 0.6]]),
              log_scales=np.log(np.array([[1e9] * 3, [s] * 3, [s] * 3])),
              quats=np.tile([1.0, 0.0, 0.0, 0.0], (3, 1)), density=np.array([sig, SIG, SIG]),
              sh=np.full((3, 1, 3), 0.5 / Y0), sh_degree=0)
    op = oracle.Opts(dt=dt, n_s=ns, ess=0, t_eps=T5 * 1.001, sigma_eps=SE)
    c, _, t_end = count(sc, ray_view(0.0, 0.0), op)
    assert t_end == pytest.approx(5 * dS, rel=1e-12)
    assert c == 1          # the sphere at t = 0.2 (< 0.4) counts, the one at 0.6 does not


def test_rotated_ellipsoid_box_from_extreme_points():
    """A rotated, elongated ellipsoid: the ray along z at y = 0.99 L_y (L_y
    the box half-length found from surface points) meets the box but, by the
    minimum of q along the ray, not the ellipsoid -- counted once; the box of
    the transposed rotation would be narrower and miss it."""
    sc_s = np.array([0.30, 0.05, 0.08])
    rot = Rotation.from_euler("zyx", [0.5, 0.5, 0.5])
    q = rot.as_quat()[[3, 0, 1, 2]]
    Rm = rot.as_matrix()
    u = np.random.default_rng(1).standard_normal((200000, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    pts = (u * (K * sc_s)) @ Rm.T
    L = np.abs(pts).max(axis=0)
    L_wrong = K * np.sqrt((Rm.T ** 2) @ (sc_s ** 2))
    assert L_wrong[1] < 0.97 * L[1]
    Si = Rm @ np.diag(sc_s ** -2.0) @ Rm.T
    y0 = 0.99 * L[1]
    # minimum over z of q(x0, y0, z) along the ray at (x0, y0)
    x_miss = None
    for x0 in np.linspace(-0.9 * L[0], 0.9 * L[0], 73):
        e = np.array([x0, y0, 0.0])
        qmin = e @ Si @ e - (Si[2] @ e) ** 2 / Si[2, 2]
        if qmin > K * K * 1.01:
            x_miss = x0
            break
    assert x_miss is not None
    sc = scene([[0.0, 0.0, 0.0]], [sc_s], [q])
    c, ties, _ = count(sc, ray_view(x_miss, y0))
    assert ties == 0 and c == 1
