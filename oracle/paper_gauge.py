"""The paper's own gauge: the camera block of M^+ (oracle; test infrastructure).

Sec. 4 removes the similarity freedom with constraints on the *whole*
parameter vector (cameras and points): the covariance is the Moore-Penrose
inverse M^+ of the full information matrix M = J^T Sigma_u^-1 J, and the
camera covariance is its camera block (M^+)_cc.  Sec. 5.2 evaluates it by a
block inversion that eliminates the points.  This differs from the reduced
camera matrix's own inverse Z^+ (the library's default contract) only in the
gauge: Z^+ = P_c (M^+)_cc P_c with P_c the projector onto the complement of
range(H_c).

Two routes, independent of each other:

* ``camera_blocks_dense`` -- the definition, for small scenes: the dense M,
  M^+ from its eigendecomposition with the seven smallest eigenvalues
  dropped, its camera block.
* ``camera_blocks`` -- the points eliminated with the full nullspace
  H = [H_c; H_p].  For any positive definite 7 x 7 matrix B,
  (M + H B H^T)^-1 = M^+ + H (H^T H)^-1 B^-1 (H^T H)^-1 H^T, and eliminating
  the points (Woodbury on the point block V + H_p B H_p^T) gives the camera
  block of the left side as S^-1 with

      S = Z + G (B^-1 + F)^-1 G^T,   G = H_c - W V^-1 H_p,   F = H_p^T V^-1 H_p.

  As B grows the second term on the right vanishes, so exactly

      (M^+)_cc = (Z + G F^-1 G^T)^-1,

  a positive definite matrix (H_p has full column rank).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import camera, covariance, nullspace, schur
from .pipeline import validate


def _pieces(scene):
    cams, pts = scene.cams, scene.pts
    oc, op = scene.obs_cam.astype(np.int64), scene.obs_pt.astype(np.int64)
    validate(cams, pts, oc, op, scene.obs_info)
    n, m = cams.shape[0], pts.shape[0]
    JP, JX = camera.jacobians(cams, pts, oc, op)
    Lam = schur.information_blocks(scene.obs_info, oc.size)
    U, V, W = schur.normal_blocks(JP, JX, Lam, oc, op, n, m)
    return oc, op, n, m, JP, JX, Lam, U, V, W


def structured_matrix(scene):
    """S = Z + G F^-1 G^T (the inverse of (M^+)_cc), and G, F."""
    oc, op, n, m, JP, JX, Lam, U, V, W = _pieces(scene)
    Vinv = np.linalg.inv(V)
    Z = schur.reduced_camera_matrix(U, W, Vinv, oc, op, n, m)
    Hr = nullspace.rotation_blocks(scene.cams, scene.pts, oc, op, JP, JX)
    Hc = nullspace.camera_rows(scene.cams, Hr)
    Hp = nullspace.point_rows(scene.pts).reshape(m, 3, 7)
    F = np.einsum("jak,jab,jbl->kl", Hp, Vinv, Hp)
    WVH = np.zeros((n, 9, 7))
    np.add.at(WVH, oc, W @ Vinv[op] @ Hp[op])
    G = Hc - WVH.reshape(9 * n, 7)
    S = Z + G @ np.linalg.solve(F, G.T)
    return 0.5 * (S + S.T), G, F


def camera_blocks(scene, full=False):
    """(M^+)_cc blocks (n, 9, 9), through S = Z + G F^-1 G^T."""
    S, _, _ = structured_matrix(scene)
    c = sla.cho_factor(S, lower=True)
    N = S.shape[0]
    if full:
        X = sla.cho_solve(c, np.eye(N))
        return covariance.camera_blocks(X), X
    blocks = np.zeros((N // 9, 9, 9))
    for i in range(N // 9):
        E = np.zeros((N, 9))
        E[9 * i:9 * i + 9] = np.eye(9)
        blocks[i] = sla.cho_solve(c, E)[9 * i:9 * i + 9]
    return blocks


def camera_blocks_dense(scene):
    """(M^+)_cc by definition: dense M, eigendecomposition, seven smallest
    eigenvalues dropped (small scenes only)."""
    oc, op, n, m, JP, JX, Lam, U, V, W = _pieces(scene)
    t = oc.size
    J = np.zeros((2 * t, 9 * n + 3 * m))
    for o in range(t):
        J[2 * o:2 * o + 2, 9 * oc[o]:9 * oc[o] + 9] = JP[o]
        J[2 * o:2 * o + 2, 9 * n + 3 * op[o]:9 * n + 3 * op[o] + 3] = JX[o]
    L = sla.block_diag(*Lam)
    M = J.T @ L @ J
    lam, Q = np.linalg.eigh(0.5 * (M + M.T))
    Qr, lr = Q[:, 7:], lam[7:]
    Mp = (Qr / lr) @ Qr.T
    return covariance.camera_blocks(Mp[:9 * n, :9 * n]), Mp[:9 * n, :9 * n]
