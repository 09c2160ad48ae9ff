"""Incremental covariance update on adding observations or a camera
(oracle; test infrastructure only).

Sec. 6 adds observations to a reconstruction: their information adds to M,
the update propagates to the Schur complement Z, and by the Woodbury
identity the covariance can only decrease.  The printed identity is garbled
(Z_i stands where Z_i^-1 belongs and the observations' own covariance is
dropped); the identity it stands for is

    (Z + J^T Omega J)^-1 = Z^-1 - Z^-1 J^T (Omega^-1 + J Z^-1 J^T)^-1 J Z^-1.

What the update must reproduce has a plain definition, the covariance of the
extended reconstruction computed from scratch (``recompute``):

* observations of existing points by existing cameras: Z'^+ of the extended
  scene (its gauge basis H_c is unchanged);
* a new camera observing existing points: the whole camera covariance of the
  extended scene in the gauge that holds the similarity of the old cameras
  fixed, i.e. the symmetric reflexive generalised inverse of Z' with null
  space [H_c; 0] (the new camera's rows zero), built as for the points in
  ``points``: (Z' + T T^T)^-1 - H' (T^T H')^-1 (H'^T T)^-1 H'^T with
  T = [H_c; 0] and H' the extended scene's camera rows.  Its old-camera block
  is the old cameras' covariance after the camera is added, the new block
  the new camera's covariance, the off-diagonal block their cross-covariance.

``woodbury`` follows the paper's route.  A new observation o of point j
(image rows J_c,o on its camera, J_x,o on the point, information Lambda_o)
acts on the cameras, once the point is eliminated from the old system (which
leaves x_j = -V_j^-1 W_j^T c plus an error of covariance V_j^-1), as the
observation

    Jt_o = J_c,o - J_x,o V_j^-1 W_j^T        (nonzero on j's old cameras and o's camera)

with error covariance Lambda_o^-1 + J_x,o V_j^-1 J_x,o^T, the new
observations of one point sharing the V_j^-1 term (Omega^-1 is block
diagonal over points).  Jt H_c = 0, so Z^+ itself follows the identity:
with S = Omega^-1 + Jt Z^+ Jt^T,

    Z'^+ = Z^+ - Z^+ Jt^T S^-1 Jt Z^+.

A new camera enters through its own Jacobian blocks J_n (columns of the
stacked rows) with a flat prior; eliminating it gives

    old cameras:  Z^+ - Z^+ Jt^T (S^-1 - S^-1 J_n C_n J_n^T S^-1) Jt Z^+,
    new camera:   C_n = (J_n^T S^-1 J_n)^-1,
    cross:        -Z^+ Jt^T S^-1 J_n C_n.
"""
from __future__ import annotations

import numpy as np

import scenegen

from . import camera, nullspace, schur
from .pipeline import camera_covariance


def extended_scene(scene, new_cam, new_pt, new_info=None, cam_new=None):
    """The scene with the observations (new_cam[k], new_pt[k]) appended and,
    when cam_new (9 parameters) is given, a new camera of index n_cams."""
    new_cam = np.asarray(new_cam, np.int32)
    new_pt = np.asarray(new_pt, np.int32)
    cams = scene.cams if cam_new is None else np.vstack([scene.cams, np.asarray(cam_new)[None]])
    info = None
    if scene.obs_info is not None or new_info is not None:
        old = scene.obs_info if scene.obs_info is not None else np.tile([1.0, 0.0, 1.0], (scene.n_obs, 1))
        add = new_info if new_info is not None else np.tile([1.0, 0.0, 1.0], (new_cam.size, 1))
        info = np.vstack([old, add])
    return scenegen.Scene(cams, scene.pts, np.concatenate([scene.obs_cam, new_cam]).astype(np.int32),
                          np.concatenate([scene.obs_pt, new_pt]).astype(np.int32), info)


def _camera_rows(scene):
    oc, op = scene.obs_cam.astype(np.int64), scene.obs_pt.astype(np.int64)
    JP, JX = camera.jacobians(scene.cams, scene.pts, oc, op)
    Hr = nullspace.rotation_blocks(scene.cams, scene.pts, oc, op, JP, JX)
    return nullspace.camera_rows(scene.cams, Hr)


def recompute(scene, new_cam, new_pt, new_info=None, cam_new=None):
    """Definition: (old-camera block N x N, new camera block 9 x 9 or None,
    cross-covariance N x 9 or None) of the extended scene."""
    ext = extended_scene(scene, new_cam, new_pt, new_info, cam_new)
    N = 9 * scene.n_cams
    if cam_new is None:
        return camera_covariance(ext, full=True)["full"], None, None
    out = camera_covariance(ext, keep=True)
    Z = out["Z"]
    H = _camera_rows(ext)
    T = H.copy()
    T[N:] = 0.0
    TH = T.T @ H
    Sig = np.linalg.inv(Z + T @ T.T) - H @ np.linalg.inv(TH) @ np.linalg.inv(TH.T) @ H.T
    Sig = 0.5 * (Sig + Sig.T)
    return Sig[:N, :N], Sig[N:, N:], Sig[:N, N:]


def effective_rows(scene, new_cam, new_pt, new_info=None, cam_new=None):
    """Jt (2k x N), J_n (2k x 9, zero rows for old cameras' observations) and
    Omega^-1 (2k x 2k) of the new observations, in their given order."""
    new_cam = np.asarray(new_cam, np.int64)
    new_pt = np.asarray(new_pt, np.int64)
    n, m, k = scene.n_cams, scene.n_pts, new_cam.size
    N = 9 * n
    oc, op = scene.obs_cam.astype(np.int64), scene.obs_pt.astype(np.int64)
    JP, JX = camera.jacobians(scene.cams, scene.pts, oc, op)
    Lam = schur.information_blocks(scene.obs_info, oc.size)
    U, V, W = schur.normal_blocks(JP, JX, Lam, oc, op, n, m)
    Vinv = np.linalg.inv(V)
    cams = scene.cams if cam_new is None else np.vstack([scene.cams, np.asarray(cam_new)[None]])
    jp, jx = camera.jacobians(cams, scene.pts, new_cam, new_pt)
    lam = schur.information_blocks(new_info, k)
    Jt = np.zeros((2 * k, N))
    Jn = np.zeros((2 * k, 9))
    Oinv = np.zeros((2 * k, 2 * k))
    for a in range(k):
        j = new_pt[a]
        r = slice(2 * a, 2 * a + 2)
        if new_cam[a] < n:
            Jt[r, 9 * new_cam[a]:9 * new_cam[a] + 9] += jp[a]
        else:
            Jn[r] = jp[a]
        for o in np.flatnonzero(op == j):   # - J_x V_j^-1 W_o^T on camera oc[o]
            Jt[r, 9 * oc[o]:9 * oc[o] + 9] -= jx[a] @ Vinv[j] @ W[o].T
        Oinv[r, r] = np.linalg.inv(lam[a])
        for b in range(k):                  # the shared error of point j
            if new_pt[b] == j:
                Oinv[r, 2 * b:2 * b + 2] += jx[a] @ Vinv[j] @ jx[b].T
    return Jt, Jn, 0.5 * (Oinv + Oinv.T)


def woodbury(scene, new_cam, new_pt, new_info=None, cam_new=None, Zp=None):
    """The update route, from the old Z^+ (computed when not given)."""
    if Zp is None:
        Zp = camera_covariance(scene, full=True)["full"]
    Jt, Jn, Oinv = effective_rows(scene, new_cam, new_pt, new_info, cam_new)
    S = Oinv + Jt @ Zp @ Jt.T
    Sinv = np.linalg.inv(S)
    B = Zp @ Jt.T
    if cam_new is None:
        X = Zp - B @ Sinv @ B.T
        return 0.5 * (X + X.T), None, None
    Cn = np.linalg.inv(Jn.T @ Sinv @ Jn)
    G = Sinv - Sinv @ Jn @ Cn @ Jn.T @ Sinv
    X = Zp - B @ G @ B.T
    return 0.5 * (X + X.T), 0.5 * (Cn + Cn.T), -B @ Sinv @ Jn @ Cn
