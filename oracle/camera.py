"""Projection function and its Jacobian blocks (oracle; paper Sec. 5.1).

The paper's projection is p(X_j, P_i) = Phi_i(c_i R(r_i)(X_j - C_i)), with
Phi_i dividing by the third coordinate and then applying radial distortion.
Read with the focal length applied after the division (otherwise it would
cancel) and with two radial coefficients, the model evaluated here is

    x   = R(r) (X - C)                       world -> camera, R from angle-axis r
    pi  = (x1 / x3, x2 / x3)                 division by the third coordinate
    rho2 = |pi|^2,  d = 1 + k1 rho2 + k2 rho2^2
    u   = f d pi + (cx, cy)                  principal point fixed, not a parameter

R(r) is the Rodrigues map of the rotation ("Euler") vector r.  Every function
is written over an abstract number type so that it runs on float64 arrays,
on complex arrays (used by the complex-step pin) and on forward-mode duals
(used here for the Jacobian).
"""
from __future__ import annotations

import numpy as np

from . import dual
from .dual import Dual

SMALL_ANGLE2 = 1e-10  # below this squared angle the Rodrigues coefficients use series


def rotate(r, v):
    """R(r) v for 3-vectors given as tuples of components (Rodrigues)."""
    r0, r1, r2 = r
    th2 = r0 * r0 + r1 * r1 + r2 * r2
    small = dual.real(th2) < SMALL_ANGLE2
    safe2 = dual.where(small, 1.0, th2)
    th = dual.sqrt(safe2)
    a_big = dual.sin(th) / th
    b_big = (1.0 - dual.cos(th)) / safe2
    a_small = 1.0 - th2 / 6.0 + th2 * th2 / 120.0
    b_small = 0.5 - th2 / 24.0 + th2 * th2 / 720.0
    a = dual.where(small, a_small, a_big)
    b = dual.where(small, b_small, b_big)
    v0, v1, v2 = v
    # w = r x v,  r x (r x v)
    w0 = r1 * v2 - r2 * v1
    w1 = r2 * v0 - r0 * v2
    w2 = r0 * v1 - r1 * v0
    z0 = r1 * w2 - r2 * w1
    z1 = r2 * w0 - r0 * w2
    z2 = r0 * w1 - r1 * w0
    return (v0 + a * w0 + b * z0, v1 + a * w1 + b * z1, v2 + a * w2 + b * z2)


def project(cam, X, principal=(320.0, 240.0)):
    """Image coordinates of point X in camera cam (both component tuples)."""
    r = cam[0:3]
    C = cam[3:6]
    f, k1, k2 = cam[6], cam[7], cam[8]
    x = rotate(r, (X[0] - C[0], X[1] - C[1], X[2] - C[2]))
    px = x[0] / x[2]
    py = x[1] / x[2]
    rho2 = px * px + py * py
    d = 1.0 + k1 * rho2 + k2 * rho2 * rho2
    return (f * d * px + principal[0], f * d * py + principal[1])


def jacobians(cams: np.ndarray, pts: np.ndarray, obs_cam: np.ndarray, obs_pt: np.ndarray):
    """Per-observation Jacobian blocks by forward-mode dual numbers.

    Returns J_P of shape (t, 2, 9), the derivative of the two image
    coordinates with respect to the observing camera's parameters in the
    order (r, C, f, k1, k2), and J_X of shape (t, 2, 3), the derivative with
    respect to the observed point (the nonzero blocks of the sparse J of
    Sec. 5.1).
    """
    k = 12
    c = cams[obs_cam]
    x = pts[obs_pt]
    cam = tuple(Dual.variable(c[:, a], a, k) for a in range(9))
    X = tuple(Dual.variable(x[:, a], 9 + a, k) for a in range(3))
    u, v = project(cam, X)
    J = np.stack([u.d, v.d], axis=1)  # (t, 2, 12)
    return np.ascontiguousarray(J[:, :, :9]), np.ascontiguousarray(J[:, :, 9:])


def project_values(cams, pts, obs_cam, obs_pt):
    """Plain float64 projections u_hat (t, 2)."""
    c = cams[obs_cam]
    x = pts[obs_pt]
    u, v = project(tuple(c[:, a] for a in range(9)), tuple(x[:, a] for a in range(3)))
    return np.stack([u, v], axis=1)
