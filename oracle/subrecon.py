"""Sub-reconstruction covariance (oracle; test infrastructure only).

Sec. 6: a camera's covariance can be evaluated from a sub-reconstruction of
the cameras and points around it; each evaluation bounds the covariance of
the whole reconstruction from above, the bound tightens as the
sub-reconstruction grows, and decomposing the reconstruction several times
and keeping the covariance with the smallest trace improves it.

Here a decomposition is given as a group id per camera.  A group's
sub-reconstruction holds its cameras, the points observed by at least two of
them and those observations; it is solved exactly (Z^+ on its own gauge),
and every camera keeps, over the decompositions, the block with the smallest
trace.
"""
from __future__ import annotations

import numpy as np

from .pipeline import camera_covariance


def subscene(scene, members):
    """The sub-reconstruction of the cameras ``members`` (parent ids, in this order)."""
    import scenegen
    members = np.asarray(members)
    local = np.full(scene.n_cams, -1)
    local[members] = np.arange(members.size)
    inside = local[scene.obs_cam] >= 0
    cnt = np.bincount(scene.obs_pt[inside], minlength=scene.n_pts)
    keep_pt = np.flatnonzero(cnt >= 2)
    lp = np.full(scene.n_pts, -1)
    lp[keep_pt] = np.arange(keep_pt.size)
    sel = np.flatnonzero(inside & (lp[scene.obs_pt] >= 0))
    info = None if scene.obs_info is None else scene.obs_info[sel]
    return scenegen.Scene(scene.cams[members], scene.pts[keep_pt],
                          local[scene.obs_cam[sel]].astype(np.int32),
                          lp[scene.obs_pt[sel]].astype(np.int32), info)


def candidates(scene, groups):
    """(n_decomp, n, 9, 9): each camera's block from its group in every decomposition."""
    groups = np.atleast_2d(groups)
    out = np.zeros((groups.shape[0], scene.n_cams, 9, 9))
    for d, g in enumerate(groups):
        for gid in np.unique(g):
            members = np.flatnonzero(g == gid)
            out[d, members] = camera_covariance(subscene(scene, members))["blocks"]
    return out


def camera_covariance_min_trace(scene, groups):
    """Blocks (n, 9, 9) with the smallest trace over the decompositions, and
    the decomposition chosen for every camera."""
    cand = candidates(scene, groups)
    tr = np.trace(cand, axis1=2, axis2=3)
    chosen = np.argmin(tr, axis=0)
    return cand[chosen, np.arange(scene.n_cams)], chosen
