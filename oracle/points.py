"""Point covariances and the whole camera covariance (oracle; test
infrastructure only).

Sec. 5.2 removes the points by block inversion.  With the camera/point
partition M = [[U, W], [W^T, V]] and Z = U - W V^-1 W^T,

    M = L diag(Z, V) L^T,   L = [[I, W V^-1], [0, I]],

so for any generalised inverse Z^g of Z the matrix
L^-T diag(Z^g, V^-1) L^-1 is a generalised inverse of M.  Its camera block is
Z^g and the 3 x 3 block of point j is

    V_j^-1 + V_j^-1 W_j^T Z^g W_j V_j^-1,

W_j being the columns of W that belong to point j (nonzero only in the rows
of the cameras that observe it).  Two gauges:

* camera gauge (the library's default contract): Z^g = Z^+.  The result is
  the symmetric reflexive generalised inverse of M whose null space is
  spanned by T = [H_c; 0], the similarity directions with the points held
  fixed.  ``dense(.., "camera")`` builds it from that characterisation: for
  any T with T^T H nonsingular, (M + T T^T)^-1 - H (T^T H)^-1 (H^T T)^-1 H^T
  (H = [H_c; H_p] the full nullspace).
* paper gauge (Sec. 4): M^+ itself.  Eliminating the points with the
  constraint term H B H^T added (as for the camera block, B -> infinity)
  gives the point block of M^+ as

      V_j^-1 - V_j^-1 H_p,j F^-1 H_p,j^T V_j^-1 + E_j^T (M^+)_cc E_j,
      E_j = (W_j + G F^-1 H_p,j^T) V_j^-1,

  with G = H_c - W V^-1 H_p and F = H_p^T V^-1 H_p as in ``paper_gauge``.
  ``dense(.., "paper")`` builds M^+ from the textbook identity for a
  symmetric M whose null space is range(H):
  M^+ = (M + H H^T)^-1 - H (H^T H)^-1 (H^T H)^-1 H^T (the same formula with
  T = H).  The eigendecomposition with the seven smallest eigenvalues dropped
  is the literal definition but resolves the small eigenvectors only to
  about 1e-4 on these scenes; the tests check the four Penrose conditions
  instead.

``structured`` follows the block-inversion route and works at any size the
dense N x N camera inverse fits; ``dense`` only for small scenes.
"""
from __future__ import annotations

import numpy as np

from . import camera, nullspace, paper_gauge, schur
from .pipeline import camera_covariance, validate

GAUGES = ("camera", "paper")


def _normal(scene):
    oc, op = scene.obs_cam.astype(np.int64), scene.obs_pt.astype(np.int64)
    validate(scene.cams, scene.pts, oc, op, scene.obs_info)
    n, m = scene.n_cams, scene.n_pts
    JP, JX = camera.jacobians(scene.cams, scene.pts, oc, op)
    Lam = schur.information_blocks(scene.obs_info, oc.size)
    U, V, W = schur.normal_blocks(JP, JX, Lam, oc, op, n, m)
    return oc, op, n, m, JP, JX, Lam, U, V, W


def structured(scene, gauge="camera", select=None):
    """Whole camera covariance (N x N) and point blocks (m, 3, 3) by the
    block-inversion route; ``select`` (point indices) restricts the point
    blocks to those points, in that order."""
    if gauge not in GAUGES:
        raise ValueError(gauge)
    oc, op, n, m, JP, JX, Lam, U, V, W = _normal(scene)
    N = 9 * n
    Vinv = np.linalg.inv(V)
    if gauge == "camera":
        X = camera_covariance(scene, full=True)["full"]
    else:
        _, X = paper_gauge.camera_blocks(scene, full=True)
        _, G, F = paper_gauge.structured_matrix(scene)
        Hp = nullspace.point_rows(scene.pts).reshape(m, 3, 7)
        Finv = np.linalg.inv(F)
    sel = np.arange(m) if select is None else np.asarray(select)
    pts = np.zeros((sel.size, 3, 3))
    track = [[] for _ in range(m)]
    for o in range(oc.size):
        track[op[o]].append(o)
    for out_i, j in enumerate(sel):
        Wj = np.zeros((N, 3))  # the columns of W of point j
        for o in track[j]:
            Wj[9 * oc[o]:9 * oc[o] + 9] = W[o]
        if gauge == "camera":
            A = Wj @ Vinv[j]
            C = Vinv[j] + A.T @ X @ A
        else:
            E = (Wj + G @ Finv @ Hp[j].T) @ Vinv[j]
            K = Vinv[j] @ Hp[j] @ Finv @ Hp[j].T @ Vinv[j]
            C = Vinv[j] - K + E.T @ X @ E
        pts[out_i] = 0.5 * (C + C.T)
    return 0.5 * (X + X.T), pts


def dense_information(scene):
    """The dense M (camera rows first) and the full nullspace H = [H_c; H_p]."""
    oc, op, n, m, JP, JX, Lam, U, V, W = _normal(scene)
    t = oc.size
    J = np.zeros((2 * t, 9 * n + 3 * m))
    for o in range(t):
        J[2 * o:2 * o + 2, 9 * oc[o]:9 * oc[o] + 9] = JP[o]
        J[2 * o:2 * o + 2, 9 * n + 3 * op[o]:9 * n + 3 * op[o] + 3] = JX[o]
    Lfull = np.zeros((2 * t, 2 * t))
    for o in range(t):
        Lfull[2 * o:2 * o + 2, 2 * o:2 * o + 2] = Lam[o]
    M = J.T @ Lfull @ J
    Hr = nullspace.rotation_blocks(scene.cams, scene.pts, oc, op, JP, JX)
    H = np.vstack([nullspace.camera_rows(scene.cams, Hr), nullspace.point_rows(scene.pts)])
    return 0.5 * (M + M.T), H


def dense(scene, gauge="camera"):
    """Whole covariance of cameras and points from the dense M (small
    scenes): returns the camera block (N x N), the point blocks (m, 3, 3) and
    the whole matrix."""
    if gauge not in GAUGES:
        raise ValueError(gauge)
    M, H = dense_information(scene)
    N, m = 9 * scene.n_cams, scene.n_pts
    T = H.copy()
    if gauge == "camera":
        T[N:] = 0.0
    TH = T.T @ H
    Sig = np.linalg.inv(M + T @ T.T) - H @ np.linalg.inv(TH) @ np.linalg.inv(TH.T) @ H.T
    Sig = 0.5 * (Sig + Sig.T)
    pts = np.stack([Sig[N + 3 * j:N + 3 * j + 3, N + 3 * j:N + 3 * j + 3] for j in range(m)])
    return Sig[:N, :N], pts, Sig
