"""Similarity nullspace H of the Jacobian (oracle; paper Sec. 5.1).

A similarity q = [T, s, mu] (translation, rotation, scale) leaves every
projection unchanged, so H = d(theta)/dq spans the null space of J.  Its
blocks, in the paper's column order [T | s | mu] and sign convention, are

    camera i, rotation rows r_i   [0   H_r_i   0  ]
    camera i, centre rows C_i     [I   [C_i]x  C_i]
    camera i, intrinsics f,k1,k2  [0   0       0  ]
    point j                       [I   [X_j]x  X_j]

where [v]x is the cross-product matrix.  The rotation block H_r_i depends on
the rotation parametrisation; the paper obtains it from J H = 0: restricted
to the rows of camera i, J_r H_r_i = B, with B the product of the remaining
Jacobian columns and (minus) the corresponding known rows of H.  This module
solves that system for each camera by least squares over all of the camera's
observation rows (the system is consistent, so the solution is exact).
"""
from __future__ import annotations

import numpy as np


def skew(v):
    """Cross-product matrices [v]x for v of shape (..., 3)."""
    v = np.asarray(v, dtype=np.float64)
    z = np.zeros(v.shape[:-1])
    return np.stack([np.stack([z, -v[..., 2], v[..., 1]], -1),
                     np.stack([v[..., 2], z, -v[..., 0]], -1),
                     np.stack([-v[..., 1], v[..., 0], z], -1)], -2)


def rotation_blocks(cams, pts, obs_cam, obs_pt, JP, JX):
    """H_r_i (n, 3, 3) from J_r H_r = B, camera by camera."""
    n = cams.shape[0]
    order = np.argsort(obs_cam, kind="stable")
    bounds = np.searchsorted(obs_cam[order], np.arange(n + 1))
    Hr = np.zeros((n, 3, 3))
    for i in range(n):
        o = order[bounds[i]:bounds[i + 1]]
        Jr = JP[o, :, 0:3].reshape(-1, 3)
        # known rows of H in the rotation columns: [C_i]x for the centre,
        # [X_j]x for the points, zero for the intrinsics
        B = -(JP[o, :, 3:6] @ skew(cams[i, 3:6]) + JX[o] @ skew(pts[obs_pt[o]])).reshape(-1, 3)
        Hr[i] = np.linalg.lstsq(Jr, B, rcond=None)[0]
    return Hr


def camera_rows(cams, Hr) -> np.ndarray:
    """H_c: the 9n x 7 camera part of H."""
    n = cams.shape[0]
    Hc = np.zeros((9 * n, 7))
    for i in range(n):
        C = cams[i, 3:6]
        Hc[9 * i:9 * i + 3, 3:6] = Hr[i]
        Hc[9 * i + 3:9 * i + 6, 0:3] = np.eye(3)
        Hc[9 * i + 3:9 * i + 6, 3:6] = skew(C)
        Hc[9 * i + 3:9 * i + 6, 6] = C
    return Hc


def point_rows(pts) -> np.ndarray:
    """H_p: the 3m x 7 point part of H."""
    m = pts.shape[0]
    Hp = np.zeros((3 * m, 7))
    for j in range(m):
        Hp[3 * j:3 * j + 3, 0:3] = np.eye(3)
        Hp[3 * j:3 * j + 3, 3:6] = skew(pts[j])
        Hp[3 * j:3 * j + 3, 6] = pts[j]
    return Hp
