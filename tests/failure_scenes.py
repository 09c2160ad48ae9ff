"""Scenes that break one input rule each, shared by the oracle's and the
library's error tests (test helper)."""
from __future__ import annotations

import numpy as np
from scipy.spatial.transform import Rotation

import scenegen as sg


def behind_camera():
    """A point moved to the mirror image of itself through the centre of one
    of its cameras: it lies behind that camera.  Returns the scene and the set
    of observations whose point is behind their camera (third coordinate of
    R(r)(X - C) not positive, rotations from SciPy)."""
    s = sg.tiny_circle(23)
    o = 4
    i, j = int(s.obs_cam[o]), int(s.obs_pt[o])
    pts = s.pts.copy()
    pts[j] = 2.0 * s.cams[i, 3:6] - s.pts[j]
    scene = sg.Scene(s.cams, pts, s.obs_cam.copy(), s.obs_pt.copy())
    x = Rotation.from_rotvec(s.cams[s.obs_cam, :3]).apply(pts[s.obs_pt] - s.cams[s.obs_cam, 3:6])
    bad = set(np.flatnonzero(x[:, 2] <= 0).tolist())
    assert o in bad
    return scene, bad


def coincident_centres():
    """A point seen only by two cameras at the same centre (a copy of one of
    its cameras): no depth information, its 3 x 3 block is singular.
    Returns the scene and the point."""
    s = sg.tiny_circle(17)
    j = int(s.obs_pt[0])
    o = np.flatnonzero(s.obs_pt == j)
    c0, c1 = s.obs_cam[o[0]], s.obs_cam[o[1]]
    keep = (s.obs_pt != j) | np.isin(np.arange(s.n_obs), o[:2])
    n = s.n_cams
    cams = np.vstack([s.cams, s.cams[c0]])  # camera n: a copy of c0 at the same centre
    oc = s.obs_cam[keep].copy()
    op = s.obs_pt[keep].copy()
    oc[(op == j) & (oc == c1)] = n
    # one more observation ties the copy to the scene otherwise
    scene = sg.Scene(cams, s.pts, np.append(oc, n).astype(np.int32),
                     np.append(op, (j + 1) % s.n_pts).astype(np.int32))
    return scene, j


def absurd_size(n_cams=400_000):
    """A chain of n_cams cameras, each point seen by two neighbours: valid
    input, but its 9 n x 9 n camera matrix (about 1e14 bytes for the default)
    exceeds any device."""
    t = np.arange(n_cams, dtype=np.float64)
    cams = np.zeros((n_cams, 9))
    cams[:, 3] = t  # centres along x, looking along +z (identity rotation)
    cams[:, 6] = 1000.0
    m = n_cams - 1
    pts = np.column_stack([np.arange(m) + 0.5, np.zeros(m), np.full(m, 10.0)])
    oc = np.concatenate([np.arange(m), np.arange(1, n_cams)]).astype(np.int32)
    op = np.concatenate([np.arange(m), np.arange(m)]).astype(np.int32)
    return sg.Scene(cams, pts, oc, op)
