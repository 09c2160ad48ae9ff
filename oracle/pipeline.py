"""End-to-end oracle: reconstruction in, per-camera 9x9 covariance blocks out.

Steps, in the paper's order (Sec. 4 problem formulation, Sec. 5 solution):

1. check the inputs (the same rules the library enforces, listed in
   ``validate``);
2. Jacobian blocks J_P, J_X of every observation (Sec. 5.1, projection);
3. normal-equation blocks U, V, W (Sec. 4) and the point-block inverses;
4. Z = U - W V^-1 W^T (Sec. 5.2, Schur complement of the point block);
5. nullspace camera rows H_c with the rotation block from J_r H_r = B
   (Sec. 5.1) and an orthonormal basis Q of range(H_c);
6. Z^+ = (Z + a Q Q^T)^-1 - Q Q^T / a with Jacobi conditioning (Sec. 4 gauge,
   Sec. 5.2 conditioning), keeping the diagonal 9x9 blocks.
"""
from __future__ import annotations

import numpy as np

from . import camera, covariance, nullspace, schur


class OracleError(Exception):
    """Input or numerical failure, with the same categories as the library:
    ``EINVAL`` (malformed input), ``EPOINT`` (a point that cannot be
    eliminated), ``EGAUGE`` (the regularised matrix is not positive definite,
    i.e. the null space is not exactly the 7-dimensional similarity gauge)."""

    def __init__(self, kind: str, message: str, index: int = -1):
        super().__init__(f"{kind}: {message}")
        self.kind = kind
        self.index = index


def validate(cams, pts, obs_cam, obs_pt, obs_info=None) -> None:
    """Input rules:

    * at least 2 cameras, 1 point and 1 observation; cameras (n, 9), points (m, 3);
    * camera and point indices in range; all values finite;
    * information blocks, when given, positive definite;
    * no camera observes the same point twice;
    * every point has at least two observations;
    * every observed point lies in front of the observing camera.
    """
    cams = np.asarray(cams)
    pts = np.asarray(pts)
    if cams.ndim != 2 or cams.shape[1] != 9 or pts.ndim != 2 or pts.shape[1] != 3:
        raise OracleError("EINVAL", "bad array shapes")
    n, m, t = cams.shape[0], pts.shape[0], np.asarray(obs_cam).size
    if n < 2 or m < 1 or t < 1 or np.asarray(obs_pt).size != t:
        raise OracleError("EINVAL", "bad sizes")
    if np.any((obs_cam < 0) | (obs_cam >= n)) or np.any((obs_pt < 0) | (obs_pt >= m)):
        raise OracleError("EINVAL", "index out of range")
    if not (np.all(np.isfinite(cams)) and np.all(np.isfinite(pts))):
        raise OracleError("EINVAL", "non-finite parameter")
    if obs_info is not None:
        a, b, c = obs_info[:, 0], obs_info[:, 1], obs_info[:, 2]
        if not np.all(np.isfinite(obs_info)) or np.any(a <= 0) or np.any(a * c - b * b <= 0):
            raise OracleError("EINVAL", "information block not positive definite")
    key = np.asarray(obs_pt, np.int64) * n + np.asarray(obs_cam, np.int64)
    if np.unique(key).size != t:
        raise OracleError("EINVAL", "duplicate observation")
    cnt = np.bincount(obs_pt, minlength=m)
    if np.any(cnt < 2):
        j = int(np.flatnonzero(cnt < 2)[0])
        raise OracleError("EPOINT", "point with fewer than two observations", j)
    d = pts[obs_pt] - cams[obs_cam, 3:6]
    x = camera.rotate(tuple(cams[obs_cam, a] for a in range(3)), (d[:, 0], d[:, 1], d[:, 2]))
    if np.any(x[2] <= 0):
        o = int(np.flatnonzero(x[2] <= 0)[0])
        raise OracleError("EINVAL", "point behind camera", o)


def camera_covariance(scene, alpha=None, cameras=None, full=False, keep=False):
    """Per-camera covariance blocks Z^+_ii of a ``scenegen.Scene``.

    ``cameras`` restricts the output to a subset (triangular solves only);
    ``full`` also returns the whole Z^+; ``keep`` returns the intermediate
    quantities (J, Z, H_c, Q, alpha) for the stage-wise tests.
    """
    cams, pts = scene.cams, scene.pts
    oc, op = scene.obs_cam.astype(np.int64), scene.obs_pt.astype(np.int64)
    validate(cams, pts, oc, op, scene.obs_info)
    n, m = cams.shape[0], pts.shape[0]
    JP, JX = camera.jacobians(cams, pts, oc, op)
    Lam = schur.information_blocks(scene.obs_info, oc.size)
    U, V, W = schur.normal_blocks(JP, JX, Lam, oc, op, n, m)
    Vinv, bad = schur.point_block_inverses(V)
    if bad:
        raise OracleError("EPOINT", "degenerate point block", int(bad[0]))
    Z = schur.reduced_camera_matrix(U, W, Vinv, oc, op, n, m)
    Hr = nullspace.rotation_blocks(cams, pts, oc, op, JP, JX)
    Hc = nullspace.camera_rows(cams, Hr)
    Q = covariance.orthonormal_basis(Hc)
    if alpha is None:
        alpha = covariance.balanced_alpha(Z, Q)
    out = {"alpha": alpha}
    try:
        if full:
            S = covariance.pseudo_inverse(Z, Q, alpha)
            out["full"] = S
            blocks = covariance.camera_blocks(S)
            if cameras is not None:
                blocks = blocks[np.asarray(cameras)]
        else:
            blocks = covariance.pseudo_inverse_blocks(Z, Q, alpha, cameras)
    except np.linalg.LinAlgError as e:
        raise OracleError("EGAUGE", f"regularised camera matrix not positive definite ({e})")
    out["blocks"] = blocks
    if keep:
        out.update(JP=JP, JX=JX, U=U, V=V, W=W, Vinv=Vinv, Z=Z, Hr=Hr, Hc=Hc, Q=Q)
    return out
