"""Pins of the oracle's decision margin: the smallest relative distance of any
discrete decision of a ray to its threshold -- a sample's inclusion q <= k^2
(Sec. 3.1, truncated Gaussians), the termination test T > T_eps at a segment
start (Alg. 1) and, where restarts are not snapped to the segment grid, a
segment's emptiness (Alg. 1 with the closest-hit skip of Eq. 4).  The GPU
parity tests excuse only pixels whose rays had such a near tie, so each kind of
margin is checked here on a ray built to sit at a known distance from its
threshold; spheres on the axis of a 1x1 view make every chord a closed form
(centre distance -/+ s k)."""
import math

import numpy as np
import pytest

import oracle
from paper_2509_07782_amd import inputs

Y0 = 0.5 / math.sqrt(math.pi)
EYE_Z = 3.0


def axis_view(t_far=6.0):
    # one ray: o = (0, 0, 3), d = (0, 0, -1) exactly
    return inputs.look_at_camera(1, 1, (0.0, 0.0, EYE_Z), t_near=0.0, t_far=t_far)


def spheres(centres_t, radii, sig, sigma_eps):
    """Isotropic Gaussians centred on the ray at distances centres_t whose
    truncation spheres (q <= k^2) have the given radii."""
    k = math.sqrt(2.0 * math.log(sig / sigma_eps))
    n = len(centres_t)
    return dict(means=np.array([[0.0, 0.0, EYE_Z - t] for t in centres_t]),
                log_scales=np.array([[math.log(r / k)] * 3 for r in radii]),
                quats=np.tile([1.0, 0.0, 0.0, 0.0], (n, 1)),
                density=np.full(n, sig),
                sh=np.full((n, 1, 3), 0.5 / Y0), sh_degree=0)


@pytest.mark.parametrize("eps", [1e-3, 1e-7, -1e-6])
def test_inclusion_margin(eps):
    """A sample at q = k^2 (1 + eps): the margin is |eps|.  The sphere's far
    end sits half a step from its nearest samples, so no other decision is
    closer."""
    dt, j, m = 0.01, 200, 20
    sig, se = 50.0, 0.01
    rho = (m + 0.5) * dt / 2.0           # 2 rho = (m + 1/2) dt
    t_j = (j + 0.5) * dt                 # a sample of the fixed grid (t_n = 0)
    t_c = t_j + rho * math.sqrt(1.0 + eps)
    sc = spheres([t_c], [rho], sig, se)
    op = oracle.Opts(dt=dt, n_s=8, ess=0, t_eps=0.0, sigma_eps=se)
    _, _, st, mg = oracle.render(sc, axis_view(), op)
    assert st[0, 0] == 1
    assert abs(mg[0] / abs(eps) - 1.0) < 1e-4, (mg[0], eps)


@pytest.mark.parametrize("eps", [1e-5, -1e-5, 3e-3])
def test_termination_margin(eps):
    """Constant medium: the transmittance at the start of segment 5 is
    exp(-5 sigma N_s dt); with T_eps = that value times (1 + eps) the margin
    is |eps| / (1 + eps), and the march ends at segment 5 (eps > 0) or 6."""
    dt, ns, sig = 0.01, 8, 0.8
    sc = dict(means=np.array([[0.0, 0.0, 0.0]]), log_scales=np.array([[20.7] * 3]),
              quats=np.array([[1.0, 0.0, 0.0, 0.0]]), density=np.array([sig]),
              sh=np.full((1, 1, 3), 0.5 / Y0), sh_degree=0)
    T5 = math.exp(-5 * sig * ns * dt)
    op = oracle.Opts(dt=dt, n_s=ns, ess=0, t_eps=T5 * (1.0 + eps), sigma_eps=1e-30)
    _, T, st, mg = oracle.render(sc, axis_view(), op)
    assert abs(mg[0] / (abs(eps) / (1.0 + eps)) - 1.0) < 1e-4, (mg[0], eps)
    stop = 5 if eps > 0 else 6
    assert st[0, 3] == stop
    np.testing.assert_allclose(T[0], math.exp(-stop * sig * ns * dt), rtol=1e-9)


@pytest.mark.parametrize("eps", [1e-8, -1e-8, 2e-4])
def test_emptiness_margin(eps):
    """Restarts at the closest hit itself (ess = 2): sphere A starts the
    march, its chord spans 2.5 segments, and segment 3 (the first after it) is
    empty unless sphere B begins before that segment's end b3.  With B's chord
    starting at b3 (1 + eps) the margin is |eps| (b3 > 1)."""
    dt, ns = 0.01, 8
    dS = ns * dt
    sig, se = 50.0, 0.01
    rho_a = 1.25 * dS
    t_a = 2.0
    a0 = t_a - rho_a
    b3 = a0 + 4 * dS
    rho_b = 1.25 * dS
    t_b = b3 * (1.0 + eps) + rho_b
    sc = spheres([t_a, t_b], [rho_a, rho_b], sig, se)
    op = oracle.Opts(dt=dt, n_s=ns, ess=2, t_eps=0.0, sigma_eps=se)
    _, _, st, mg = oracle.render(sc, axis_view(), op)
    assert st[0, 0] == 2
    assert abs(mg[0] / abs(eps) - 1.0) < 1e-4, (mg[0], eps)
    # closest-hit queries: the first one, one after each empty segment (the
    # last finds nothing behind B).  With B in segment 3 (eps < 0) there is
    # no empty segment between A and B.
    assert st[0, 4] == (2 if eps < 0 else 3)


def test_margin_without_ties():
    """A ray whose decisions are all far from their thresholds has a margin
    of the order of the step over the radius; a ray that meets nothing has no
    decision at all (infinite margin)."""
    dt, sig, se = 0.01, 50.0, 0.01
    sc = spheres([2.0], [0.1], sig, se)     # samples 0.005 inside either end
    op = oracle.Opts(dt=dt, n_s=8, ess=0, t_eps=0.0, sigma_eps=se)
    _, _, _, mg = oracle.render(sc, axis_view(), op)
    assert 0.05 < mg[0] < 0.2
    far = spheres([2.0], [0.1], sig, se)
    far["means"][0, 0] = 5.0                # off the ray
    _, _, st, mg = oracle.render(far, axis_view(), op)
    assert st[0, 0] == 0 and math.isinf(mg[0])
