"""Patch maps F^(j): (0,1)^3 -> patch (oracle, test infrastructure only).

Section 2 assumes every patch is the image of the unit cube under a regular
map F^(j).  Two families are used by the workloads:

* boxes: F is affine, F(xi) = x_lo + diag(h) * (idx + xi);
* the annulus: direction 0 is the azimuth, represented per sector by one
  rational quadratic arc (weights 1, cos(half-angle), 1) that reproduces the
  circle exactly; radius and height are affine.

``patch_map(problem, patch, xi)`` returns physical points ``(n,3)`` and the
Jacobian ``DF (n,3,3)`` with ``DF[:, a, b] = d x_a / d xi_b``.
"""
from __future__ import annotations

import numpy as np

from workloads.problem import GEOM_ANNULUS, GEOM_BOX, patch_coords


def _box_map(prob, pidx, xi):
    P = prob.patches
    c = patch_coords(pidx, P)
    g = prob.geom_params
    lo = np.array([g[0], g[2], g[4]])
    hi = np.array([g[1], g[3], g[5]])
    h = (hi - lo) / np.array(P, dtype=np.float64)
    x = lo[None, :] + h[None, :] * (np.array(c)[None, :] + xi)
    DF = np.zeros((xi.shape[0], 3, 3))
    for a in range(3):
        DF[:, a, a] = h[a]
    return x, DF


def _arc(theta0, dtheta, s):
    """Rational quadratic arc of the unit circle over [theta0, theta0+dtheta]."""
    half = 0.5 * dtheta
    w1 = np.cos(half)
    P0 = np.array([np.cos(theta0), np.sin(theta0)])
    P2 = np.array([np.cos(theta0 + dtheta), np.sin(theta0 + dtheta)])
    mid = theta0 + half
    P1 = np.array([np.cos(mid), np.sin(mid)]) / w1
    B = np.stack([(1 - s) ** 2, 2 * s * (1 - s), s ** 2], axis=1)
    dB = np.stack([-2 * (1 - s), 2 - 4 * s, 2 * s], axis=1)
    w = np.array([1.0, w1, 1.0])
    Pw = np.stack([P0, P1, P2]) * w[:, None]  # (3,2)
    num = B @ Pw
    dnum = dB @ Pw
    W = B @ w
    dW = dB @ w
    c = num / W[:, None]
    dc = (dnum * W[:, None] - num * dW[:, None]) / (W ** 2)[:, None]
    return c, dc


def _annulus_map(prob, pidx, xi):
    P = prob.patches
    i, j, k = patch_coords(pidx, P)
    g = prob.geom_params
    z0, z1 = g[0], g[1]
    radii = g[2:2 + P[1] + 1]
    dtheta = 2.0 * np.pi / P[0]
    c, dc = _arc(i * dtheta, dtheta, xi[:, 0])
    r = radii[j] + xi[:, 1] * (radii[j + 1] - radii[j])
    hz = (z1 - z0) / P[2]
    z = z0 + (k + xi[:, 2]) * hz
    x = np.stack([r * c[:, 0], r * c[:, 1], z], axis=1)
    DF = np.zeros((xi.shape[0], 3, 3))
    DF[:, 0, 0] = r * dc[:, 0]
    DF[:, 1, 0] = r * dc[:, 1]
    DF[:, 0, 1] = (radii[j + 1] - radii[j]) * c[:, 0]
    DF[:, 1, 1] = (radii[j + 1] - radii[j]) * c[:, 1]
    DF[:, 2, 2] = hz
    return x, DF


def patch_map(prob, pidx, xi):
    xi = np.asarray(xi, dtype=np.float64)
    if prob.geom_kind == GEOM_BOX:
        return _box_map(prob, pidx, xi)
    if prob.geom_kind == GEOM_ANNULUS:
        return _annulus_map(prob, pidx, xi)
    raise ValueError("unknown geometry kind")
