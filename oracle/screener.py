"""Learned-screener reference (oracle; test infrastructure only).

The screener predicts a camera's 9x9 covariance from cheap per-camera
features, for fast screening of reconstructions.  Screening cameras by their
uncertainty, e.g. to drop mostly unconstrained ones before bundle adjustment,
is one of the uses the paper motivates (Sec. 1).  The network itself is not
part of the paper; the exact covariance (Sec. 5) is its training label and
the reference for its error.

Everything here is plain FP64 numpy, written for checking, not speed:

* ``camera_features``  55 values per camera:
    - 45: the diagonal block Z_ii of the reduced camera matrix (Sec. 5.2),
      Z_ii = U_i - sum over camera i's observations o of W_o V_j^-1 W_o^T,
      as log10 of its 9 diagonal entries and its 36 correlations
      Z_ab / sqrt(Z_aa Z_bb), in row-major upper-triangular order;
    - 8: log(1 + count) of the camera's observations whose track length falls
      in the bins 2, 3, 4, 5, 6-7, 8-10, 11-15, >= 16;
    - 1: the mean over the camera's observations of the largest angle (rad)
      between its viewing ray to the point and the ray of any other camera of
      that point's track;
    - 1: log(1 + number of other cameras that share a point with it).
* ``zii_from_features`` / ``block_scale``: Z_ii rebuilt from its 45
  features, and b = sqrt(diag((Z_ii)^-1)), the standard deviations of the
  block-diagonal estimate (its correlation matrix taken with a ridge of 1e-6),
  which set each camera's label scale D = s b;
* ``label_moments`` / ``standardise``: the labels' robust location and
  spread (median, scaled median absolute deviation) and the clipped
  standardised labels;
  ``label_scale``: s_a = sqrt of the lower median over a training set of the
  variance ratio Sigma_aa / b_a^2.
* ``log_cholesky`` / ``from_log_cholesky``: Sigma~ = D^-1 Sigma D^-1 = L L^T,
  parameters (log L_aa on the diagonal, L_ab below it) in row-major
  lower-triangular order; D one 9-vector, or one per camera.
* ``mlp_forward`` / ``mlp_backward``: 55 -> 256 -> 256 -> 256 -> 45, ReLU
  between layers, linear output, mean squared error over batch and outputs.
  Parameters are one flat vector: for each layer W (out x in, row-major)
  then b (out).
* ``adam_step``: Adam with bias correction.

``mlp_forward`` and ``mlp_backward`` also run in a ``bf16`` mode that rounds
every product operand (layer input, weights, output gradient) and every stored
hidden activation to bfloat16 and accumulates in FP64.  A network whose
products run in BF16 decides each ReLU on a pre-activation computed from
rounded operands; near zero that decision can differ from the FP64 one and
reroute a whole unit's gradient, so gradients of a BF16 network are compared
with this mode, in which the decisions are taken in the same precision.
"""
from __future__ import annotations

import numpy as np

from . import camera, schur

LAYERS = (55, 256, 256, 256, 45)
N_FEATURES = LAYERS[0]
N_OUT = LAYERS[-1]
TRACK_BINS = (2, 3, 4, 5, 6, 8, 11, 16)  # lower edges; the last bin is open


def param_count(layers=LAYERS) -> int:
    return sum(o * i + o for i, o in zip(layers[:-1], layers[1:]))


def split_params(p, layers=LAYERS):
    """Views (W_l, b_l) of the flat parameter vector."""
    out, k = [], 0
    for i, o in zip(layers[:-1], layers[1:]):
        W = p[k:k + o * i].reshape(o, i)
        k += o * i
        b = p[k:k + o]
        k += o
        out.append((W, b))
    assert k == p.size
    return out


# ---------------------------------------------------------------------------
# features
# ---------------------------------------------------------------------------

def z_diagonal_blocks(scene) -> np.ndarray:
    """Z_ii for every camera, straight from its observations' terms."""
    oc, op = scene.obs_cam.astype(np.int64), scene.obs_pt.astype(np.int64)
    n, m = scene.n_cams, scene.n_pts
    JP, JX = camera.jacobians(scene.cams, scene.pts, oc, op)
    Lam = schur.information_blocks(scene.obs_info, oc.size)
    U, V, W = schur.normal_blocks(JP, JX, Lam, oc, op, n, m)
    Z = U.copy()
    Vinv = np.linalg.inv(V)
    for o in range(oc.size):
        Z[oc[o]] -= W[o] @ Vinv[op[o]] @ W[o].T
    return Z


def track_bin(length: int) -> int:
    b = 0
    for k, lo in enumerate(TRACK_BINS):
        if length >= lo:
            b = k
    return b


def camera_features(scene) -> np.ndarray:
    n = scene.n_cams
    oc, op = scene.obs_cam.astype(np.int64), scene.obs_pt.astype(np.int64)
    F = np.zeros((n, N_FEATURES))
    Zd = z_diagonal_blocks(scene)
    for i in range(n):
        d = np.diag(Zd[i])
        k = 0
        for a in range(9):
            for b in range(a, 9):
                F[i, k] = np.log10(d[a]) if a == b else Zd[i, a, b] / np.sqrt(d[a] * d[b])
                k += 1
    track = {}
    for o in range(oc.size):
        track.setdefault(int(op[o]), []).append(int(oc[o]))
    hist = np.zeros((n, 8))
    ang_sum = np.zeros(n)
    cnt = np.zeros(n)
    covis = [set() for _ in range(n)]
    C = scene.cams[:, 3:6]
    for j, cams_j in track.items():
        X = scene.pts[j]
        rays = {c: (X - C[c]) / np.linalg.norm(X - C[c]) for c in cams_j}
        for c in cams_j:
            hist[c, track_bin(len(cams_j))] += 1
            best = 0.0
            for c2 in cams_j:
                if c2 != c:
                    best = max(best, float(np.arccos(np.clip(rays[c] @ rays[c2], -1.0, 1.0))))
                    covis[c].add(c2)
            ang_sum[c] += best
            cnt[c] += 1
    F[:, 45:53] = np.log1p(hist)
    F[:, 53] = ang_sum / np.maximum(cnt, 1)
    F[:, 54] = np.log1p([len(s) for s in covis])
    return F


# ---------------------------------------------------------------------------
# covariance <-> log-Cholesky parameters
# ---------------------------------------------------------------------------

def zii_from_features(F: np.ndarray) -> np.ndarray:
    """(k, >= 45) features -> (k, 9, 9) Z_ii: the diagonal from its log10, the
    off-diagonal entries from the correlations times sqrt(Z_aa Z_bb)."""
    F = np.asarray(F, np.float64)
    Z = np.zeros((F.shape[0], 9, 9))
    d = np.zeros((F.shape[0], 9))
    k = 0
    for a in range(9):
        for b in range(a, 9):
            if a == b:
                d[:, a] = 10.0 ** F[:, k]
            k += 1
    k = 0
    for a in range(9):
        for b in range(a, 9):
            Z[:, a, b] = Z[:, b, a] = d[:, a] if a == b else F[:, k] * np.sqrt(d[:, a] * d[:, b])
            k += 1
    return Z


SCALE_RIDGE = 1e-6


def block_scale(F: np.ndarray) -> np.ndarray:
    """(k, 9): b_a = sqrt(((Z_ii)^-1)_aa), Z_ii rebuilt from the features,
    with SCALE_RIDGE added to the diagonal of its correlation matrix C
    (Z_ii = diag(d)^1/2 C diag(d)^1/2, so ((Z_ii)^-1)_aa = (C^-1)_aa / d_a):
    the features hold C rounded to FP32, which the ridge keeps positive
    definite."""
    Z = zii_from_features(F)
    d = np.diagonal(Z, axis1=1, axis2=2)
    C = Z / np.sqrt(d[:, :, None] * d[:, None, :]) + SCALE_RIDGE * np.eye(9)
    return np.sqrt(np.diagonal(np.linalg.inv(C), axis1=1, axis2=2) / d)


def label_scale(S: np.ndarray, F: np.ndarray) -> np.ndarray:
    """(9,): per parameter a, the square root of the lower median (the value
    of rank (k - 1) / 2 ascending) of Sigma_aa / b_a^2 over the k blocks."""
    r = np.sort(np.diagonal(S, axis1=1, axis2=2) / block_scale(F) ** 2, axis=0)
    return np.sqrt(r[(S.shape[0] - 1) // 2])


LABEL_CLIP = 6.0


def label_moments(P: np.ndarray):
    """Per column of the (k, 45) label parameters: the lower median m (rank
    (k - 1) / 2) and 1.4826 times the lower median of |P - m| (the median
    absolute deviation scaled to a normal distribution's standard deviation),
    at least 1e-6."""
    r = (P.shape[0] - 1) // 2
    m = np.sort(P, axis=0)[r]
    mad = np.sort(np.abs(P - m), axis=0)[r]
    return m, np.maximum(1.4826 * mad, 1e-6)


def standardise(P: np.ndarray, center, spread) -> np.ndarray:
    """Training labels: (P - center) / spread clipped to +-LABEL_CLIP."""
    return np.clip((P - center) / spread, -LABEL_CLIP, LABEL_CLIP)


def _per_block(D: np.ndarray, k: int) -> np.ndarray:
    D = np.asarray(D, np.float64)
    return np.broadcast_to(D, (k, 9)) if D.ndim == 1 else D


def log_cholesky(S: np.ndarray, D: np.ndarray) -> np.ndarray:
    """(k, 9, 9) covariances -> (k, 45) parameters of D^-1 S D^-1 (D: (9,) or
    (k, 9))."""
    D = _per_block(D, S.shape[0])
    St = S / (D[:, :, None] * D[:, None, :])
    L = np.linalg.cholesky(St)
    out = np.zeros((S.shape[0], N_OUT))
    k = 0
    for a in range(9):
        for b in range(a + 1):
            out[:, k] = np.log(L[:, a, a]) if a == b else L[:, a, b]
            k += 1
    return out


def from_log_cholesky(P: np.ndarray, D: np.ndarray) -> np.ndarray:
    """(k, 45) parameters -> (k, 9, 9) covariances D L L^T D."""
    D = _per_block(D, P.shape[0])
    L = np.zeros((P.shape[0], 9, 9))
    k = 0
    for a in range(9):
        for b in range(a + 1):
            L[:, a, b] = np.exp(P[:, k]) if a == b else P[:, k]
            k += 1
    St = L @ np.transpose(L, (0, 2, 1))
    return St * (D[:, :, None] * D[:, None, :])


# ---------------------------------------------------------------------------
# MLP, loss, Adam
# ---------------------------------------------------------------------------

def bf16(a) -> np.ndarray:
    """Round to bfloat16 (the top 16 bits of an IEEE float32; round to
    nearest, ties to even), returned as float64."""
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def mlp_forward(p, x, bf16_ops=False):
    """Returns the output and the list of layer inputs (for the backward pass)."""
    r = bf16 if bf16_ops else (lambda a: a)
    h = np.asarray(x, np.float64)
    inputs = []
    layers = split_params(p)
    for li, (W, b) in enumerate(layers):
        h = r(h)
        inputs.append(h)
        a = h @ r(W).T + b
        h = np.maximum(a, 0.0) if li + 1 < len(layers) else a
    return h, inputs


def mse(y, t) -> float:
    return float(np.mean((y - t) ** 2))


def mlp_backward(p, x, t, bf16_ops=False):
    """Loss and its gradient with respect to the flat parameter vector."""
    r = bf16 if bf16_ops else (lambda a: a)
    y, inputs = mlp_forward(p, x, bf16_ops)
    loss = mse(y, t)
    g = np.zeros_like(p)
    gl = split_params(g)
    layers = split_params(p)
    dy = 2.0 * (y - t) / y.size
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        h = inputs[li]
        gl[li][1][...] = dy.sum(axis=0)
        dy = r(dy)
        gl[li][0][...] = dy.T @ h
        if li > 0:
            dh = dy @ r(W)
            dy = r(dh * (h > 0))  # h = relu(a): d relu / d a = [a > 0] = [h > 0]
    return loss, g


ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8


def adam_step(p, g, m, v, step: int, lr: float):
    """One Adam update (step counts from 1); returns new (p, m, v)."""
    m = ADAM_B1 * m + (1 - ADAM_B1) * g
    v = ADAM_B2 * v + (1 - ADAM_B2) * g * g
    mh = m / (1 - ADAM_B1 ** step)
    vh = v / (1 - ADAM_B2 ** step)
    return p - lr * mh / (np.sqrt(vh) + ADAM_EPS), m, v
