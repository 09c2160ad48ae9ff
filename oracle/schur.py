"""Normal-equation blocks and the reduced camera matrix (oracle).

Sec. 4 defines the normal equations M = J^T Sigma_u^-1 J with a block-diagonal
Sigma_u of 2x2 blocks.  Ordering cameras before points (Sec. 5.1), M splits
into a camera block U (block diagonal, one 9x9 block per camera), a point
block V (block diagonal, one 3x3 block per point, the A_p of Sec. 5.2) and the
coupling W.  Sec. 5.2 eliminates the points with a block inversion, which
leaves the Schur complement of the point block,

    Z = U - W V^-1 W^T,

a 9n x 9n symmetric positive semi-definite matrix whose null space is the
camera part of the similarity nullspace.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def information_blocks(obs_info, t: int) -> np.ndarray:
    """Per-observation 2x2 information Sigma_u^-1 (identity when absent)."""
    if obs_info is None:
        return np.broadcast_to(np.eye(2), (t, 2, 2)).copy()
    a, b, c = obs_info[:, 0], obs_info[:, 1], obs_info[:, 2]
    return np.stack([np.stack([a, b], -1), np.stack([b, c], -1)], -2)


def normal_blocks(JP, JX, Lam, obs_cam, obs_pt, n: int, m: int):
    """U (n,9,9), V (m,3,3) and the per-observation coupling W_o (t,9,3).

    Each observation o = (i, j) contributes J_P^T L J_P to U_i, J_X^T L J_X to
    V_j and J_P^T L J_X to the (i, j) block of W.
    """
    LJP = Lam @ JP
    LJX = Lam @ JX
    U = np.zeros((n, 9, 9))
    np.add.at(U, obs_cam, np.transpose(JP, (0, 2, 1)) @ LJP)
    V = np.zeros((m, 3, 3))
    np.add.at(V, obs_pt, np.transpose(JX, (0, 2, 1)) @ LJX)
    W = np.transpose(JP, (0, 2, 1)) @ LJX
    return U, V, W


POINT_PIVOT_REL = 1e-14


def point_block_inverses(V):
    """V_j^-1 for every point, with the degenerate-point check.

    A point block is rejected (returned in ``bad``) when its Cholesky factor
    does not exist or its smallest squared pivot falls below
    ``POINT_PIVOT_REL`` times the trace.
    """
    m = V.shape[0]
    try:  # all blocks at once when every factor exists
        L = np.linalg.cholesky(V)
        piv2 = np.min(np.diagonal(L, axis1=1, axis2=2), axis=1) ** 2
        bad = list(np.flatnonzero(piv2 <= POINT_PIVOT_REL * np.trace(V, axis1=1, axis2=2)))
        if not bad:
            Li = np.linalg.inv(L)
            return np.transpose(Li, (0, 2, 1)) @ Li, []
    except np.linalg.LinAlgError:
        pass
    bad = []
    Vinv = np.zeros_like(V)
    for j in range(m):
        try:
            L = np.linalg.cholesky(V[j])
        except np.linalg.LinAlgError:
            bad.append(j)
            continue
        if np.min(np.diag(L)) ** 2 <= POINT_PIVOT_REL * np.trace(V[j]):
            bad.append(j)
            continue
        Li = np.linalg.inv(L)
        Vinv[j] = Li.T @ Li
    return Vinv, bad


def reduced_camera_matrix(U, W, Vinv, obs_cam, obs_pt, n: int, m: int) -> np.ndarray:
    """Dense Z = U - W V^-1 W^T using sparse products (Sec. 5.2)."""
    t = obs_cam.size
    ar9 = np.arange(9)
    ar3 = np.arange(3)
    rows = (9 * obs_cam[:, None, None] + ar9[None, :, None]) * np.ones((1, 1, 3), np.int64)
    cols = (3 * obs_pt[:, None, None] + ar3[None, None, :]) * np.ones((1, 9, 1), np.int64)
    Wm = sp.csr_matrix((W.reshape(-1), (rows.reshape(-1), cols.reshape(-1))), shape=(9 * n, 3 * m))
    vr = (3 * np.arange(m)[:, None, None] + ar3[None, :, None]) * np.ones((1, 1, 3), np.int64)
    vc = (3 * np.arange(m)[:, None, None] + ar3[None, None, :]) * np.ones((1, 3, 1), np.int64)
    Vm = sp.csr_matrix((Vinv.reshape(-1), (vr.reshape(-1), vc.reshape(-1))), shape=(3 * m, 3 * m))
    Z = -(Wm @ Vm @ Wm.T).toarray()
    for i in range(n):
        Z[9 * i:9 * i + 9, 9 * i:9 * i + 9] += U[i]
    del t
    return Z
