"""Closed forms of the anisotropy analysis and the adaptive step (FP64 numpy).

TEST INFRASTRUCTURE ONLY (see the package docstring).

  aabb_volume_ratio  Vol(AABB(E)) / Vol(E) = (6/pi) sqrt(prod_i sum_j r_ij^2 s_j^2) / (s1 s2 s3)
                     (Sec. 3.4, Eq. 6; Supp. B, derivation of the ratio)
  ratio_bound        2/(pi sqrt 3) (s1^2+s2^2+s3^2)^(3/2) / (s1 s2 s3)
                     (Sec. 3.4, Eq. 7 and Eq. 9; Supp. B, upper bound)
  isotropic_loss     mean over Gaussians of max(r_max, r0) - r0 (Sec. 3.4, Eq. 8)
  adaptive_step      min(max(d/beta, dt_min) * T^(-1/3), dt_max) (Sec. 3.2, Eq. 5; the
                     segment is N_S times this)
  densification_statistic
                     per Gaussian: sum over views of alpha_v |grad_mu L_v| with
                     alpha_v = |mu - o_v| / f_v, and the number of views whose gradient
                     is non-zero (Sec. 3.5, Eq. 12; the ratio of the two is the average
                     the criterion thresholds)
"""
from __future__ import annotations

import math

import numpy as np


def aabb_volume_ratio(R, s):
    R = np.asarray(R, np.float64)
    s = np.asarray(s, np.float64)
    l = np.einsum("...ij,...j->...i", R * R, s * s)
    return 6.0 / math.pi * np.sqrt(np.prod(l, axis=-1)) / np.prod(s, axis=-1)


def ratio_bound(s):
    s = np.asarray(s, np.float64)
    return 2.0 / (math.pi * math.sqrt(3.0)) * np.sum(s * s, axis=-1) ** 1.5 / np.prod(s, axis=-1)


def isotropic_loss(log_scales, r0=10.0):
    r = ratio_bound(np.exp(np.asarray(log_scales, np.float64)))
    return float(np.mean(np.maximum(r, r0) - r0))


def adaptive_step(d, T, dt_min=0.005, dt_max=0.02, beta=1024.0):
    d = np.asarray(d, np.float64)
    T = np.asarray(T, np.float64)
    with np.errstate(divide="ignore"):
        v = np.maximum(d / beta, dt_min) * T ** (-1.0 / 3.0)
    return np.minimum(v, dt_max)


def densification_statistic(means, grads_mu, origins, focals):
    """means [N,3]; grads_mu [V,N,3] the per-view gradients of the loss with
    respect to the means; origins [V,3] camera centres; focals [V] focal
    lengths in pixels.  Returns (sum [N], views [N])."""
    mu = np.asarray(means, np.float64)
    g = np.asarray(grads_mu, np.float64)
    o = np.asarray(origins, np.float64)
    f = np.asarray(focals, np.float64)
    total = np.zeros(mu.shape[0])
    views = np.zeros(mu.shape[0], np.int64)
    for v in range(g.shape[0]):
        gn = np.linalg.norm(g[v], axis=1)
        alpha = np.linalg.norm(mu - o[v], axis=1) / f[v]
        total += alpha * gn
        views += gn > 0
    return total, views
