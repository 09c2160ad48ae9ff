"""Moore-Penrose camera covariance (oracle).

Sec. 4: the information matrix is rank deficient by the seven similarity
degrees of freedom, and the natural (inner) covariance is its Moore-Penrose
inverse, obtained through constraints H^T dtheta = 0 with H the nullspace.
Restricted to the cameras, the reduced camera matrix Z is symmetric positive
semi-definite with null space range(H_c).  With Q an orthonormal basis of
range(H_c) and any a > 0, Z + a Q Q^T is positive definite and

    Z^+ = (Z + a Q Q^T)^-1 - Q Q^T / a,

because Z + a Q Q^T acts as Z on range(Z) and as a on range(Q).

Sec. 5.2 conditions the matrix to be inverted with diagonal scalings before
inverting; here that is the Jacobi scaling S = diag(A)^-1/2 of the positive
definite A = Z + a Q Q^T, with A^-1 = S (S A S)^-1 S exactly.

The weight a only balances the spectrum of A; every a > 0 gives the same
Z^+.  ``balanced_alpha`` picks a = 7 / sum_k |S_Z q_k|^2 with S_Z = diag(Z)^-1/2,
so that the gauge directions of the scaled matrix have unit average size.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def orthonormal_basis(Hc: np.ndarray) -> np.ndarray:
    """Q with orthonormal columns spanning range(H_c) (Householder QR)."""
    Q, _ = np.linalg.qr(Hc)
    return Q


def balanced_alpha(Z: np.ndarray, Q: np.ndarray) -> float:
    dz = np.diag(Z)
    return float(Q.shape[1] / np.sum(Q * Q / dz[:, None]))


def _scaled_factor(Z, Q, alpha):
    A = Z + alpha * (Q @ Q.T)
    dA = np.diag(A)
    if not np.all(dA > 0):
        raise np.linalg.LinAlgError("non-positive diagonal")
    s = 1.0 / np.sqrt(dA)
    As = A * s[:, None] * s[None, :]
    c = sla.cho_factor(As, lower=True, check_finite=True)
    return c, s


def pseudo_inverse(Z: np.ndarray, Q: np.ndarray, alpha: float | None = None) -> np.ndarray:
    """Full Z^+ (N x N).  Raises ``np.linalg.LinAlgError`` when A is not PD."""
    if alpha is None:
        alpha = balanced_alpha(Z, Q)
    c, s = _scaled_factor(Z, Q, alpha)
    inv = sla.cho_solve(c, np.eye(Z.shape[0]))
    return inv * s[:, None] * s[None, :] - (Q @ Q.T) / alpha


def pseudo_inverse_blocks(Z, Q, alpha=None, cameras=None) -> np.ndarray:
    """Diagonal 9x9 blocks of Z^+ for the selected cameras (all by default),
    from triangular solves with the Cholesky factor only."""
    if alpha is None:
        alpha = balanced_alpha(Z, Q)
    n = Z.shape[0] // 9
    cameras = np.arange(n) if cameras is None else np.asarray(cameras)
    c, s = _scaled_factor(Z, Q, alpha)
    out = np.zeros((cameras.size, 9, 9))
    for k, i in enumerate(cameras):
        E = np.zeros((Z.shape[0], 9))
        E[9 * i:9 * i + 9] = np.eye(9)
        X = sla.cho_solve(c, E)[9 * i:9 * i + 9]
        si = s[9 * i:9 * i + 9]
        Qi = Q[9 * i:9 * i + 9]
        out[k] = X * si[:, None] * si[None, :] - (Qi @ Qi.T) / alpha
    return out


def camera_blocks(S: np.ndarray) -> np.ndarray:
    """(n, 9, 9) diagonal blocks of a 9n x 9n matrix."""
    n = S.shape[0] // 9
    return np.stack([S[9 * i:9 * i + 9, 9 * i:9 * i + 9] for i in range(n)])
