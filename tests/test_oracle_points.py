"""Pins of the point-covariance oracle (Sec. 5.2 block inversion, both gauges).

The block-inversion route (``points.structured``) is checked against the
dense characterisations (``points.dense``): the camera gauge as the
symmetric reflexive generalised inverse of M with null space [H_c; 0], the
paper gauge as the Moore-Penrose inverse, whose four defining conditions are
checked directly, and against an eigendecomposition (the literal definition,
looser: its small eigenvectors are resolved only to about 1e-4 at the
conditioning of these scenes).  The two gauges are tied by M^+ = P G P for
any generalised inverse G of M and P the orthogonal projector off range(H).
All on the CPU.
"""
import numpy as np
import pytest

import scenegen as sg
from oracle import points
from oracle.pipeline import camera_covariance

SCENES = [lambda: sg.tiny_circle(0, n=6, m=60), lambda: sg.tiny_circle(1, n=6, m=60, with_info=True),
          lambda: sg.tiny_circle(2)]


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rel_blocks(a, b):
    return float(np.max(np.linalg.norm(a - b, axis=(1, 2)) / np.linalg.norm(b, axis=(1, 2))))


@pytest.mark.parametrize("maker", SCENES)
@pytest.mark.parametrize("gauge", points.GAUGES)
def test_block_inversion_matches_dense(maker, gauge):
    s = maker()
    Xs, Ps = points.structured(s, gauge)
    Xd, Pd, _ = points.dense(s, gauge)
    assert rel(Xs, Xd) < 1e-9
    assert rel_blocks(Ps, Pd) < 1e-9


@pytest.mark.parametrize("maker", SCENES[:2])
def test_paper_gauge_is_moore_penrose(maker):
    s = maker()
    M, H = points.dense_information(s)
    _, _, G = points.dense(s, "paper")
    nm, ng = np.linalg.norm(M), np.linalg.norm(G)
    assert np.linalg.norm(M @ G @ M - M) < 1e-9 * nm
    assert np.linalg.norm(G @ M @ G - G) < 1e-9 * ng
    # M G is the orthogonal projector off range(H); M + H H^T has a condition
    # number near 1e10 here, so its symmetry holds to about eps * 1e10
    MG = M @ G
    assert np.linalg.norm(MG - MG.T) < 1e-7 * np.linalg.norm(MG)
    P = np.eye(H.shape[0]) - H @ np.linalg.solve(H.T @ H, H.T)
    assert np.linalg.norm(MG - P) < 1e-7 * np.linalg.norm(P)
    assert np.linalg.norm(G @ H) < 1e-10 * ng * np.linalg.norm(H)


@pytest.mark.parametrize("maker", SCENES[:2])
def test_camera_gauge_characterisation(maker):
    """Reflexive generalised inverse of M (so of M's rank), null space
    [H_c; 0], camera block Z^+ (the library's camera covariance)."""
    s = maker()
    M, H = points.dense_information(s)
    N = 9 * s.n_cams
    Xd, _, G = points.dense(s, "camera")
    nm, ng = np.linalg.norm(M), np.linalg.norm(G)
    assert np.linalg.norm(M @ G @ M - M) < 1e-9 * nm
    assert np.linalg.norm(G @ M @ G - G) < 1e-9 * ng
    T = np.zeros_like(H)
    T[:N] = H[:N]
    assert np.linalg.norm(G @ T) < 1e-10 * ng * np.linalg.norm(T)
    assert rel(Xd, camera_covariance(s, full=True)["full"]) < 1e-9


@pytest.mark.parametrize("maker", SCENES[:2])
def test_projector_links_the_gauges(maker):
    s = maker()
    _, H = points.dense_information(s)
    _, _, Gc = points.dense(s, "camera")
    _, _, Gp = points.dense(s, "paper")
    P = np.eye(H.shape[0]) - H @ np.linalg.solve(H.T @ H, H.T)
    assert rel(P @ Gc @ P, Gp) < 1e-9


def test_eigendecomposition_definition():
    """The literal definition (eigenvectors of the nonzero eigenvalues)."""
    s = SCENES[0]()
    M, _ = points.dense_information(s)
    N = 9 * s.n_cams
    lam, Q = np.linalg.eigh(M)
    G = (Q[:, 7:] / lam[7:]) @ Q[:, 7:].T
    Xs, Ps = points.structured(s, "paper")
    Pe = np.stack([G[N + 3 * j:N + 3 * j + 3, N + 3 * j:N + 3 * j + 3] for j in range(s.n_pts)])
    assert rel(Xs, G[:N, :N]) < 1e-4
    assert rel_blocks(Ps, Pe) < 1e-3


@pytest.mark.parametrize("maker", SCENES)
def test_camera_uncertainty_only_adds(maker):
    """Camera gauge: the point block minus V_j^-1 (the point's covariance
    with the cameras known) is positive semi-definite."""
    s = maker()
    out = camera_covariance(s, keep=True)
    _, P = points.structured(s, "camera")
    for j in range(s.n_pts):
        lam = np.linalg.eigvalsh(P[j] - out["Vinv"][j])
        assert lam.min() > -1e-9 * np.abs(P[j]).max()


def test_known_camera_part_is_triangulation_covariance():
    """With the cameras known a point's covariance is that of its
    least-squares triangulation, pinv(J) pinv(J)^T over its stacked J_X rows
    (unit information): the V_j^-1 both routes start from."""
    s = SCENES[0]()
    out = camera_covariance(s, keep=True)
    JX = out["JX"]
    op = s.obs_pt.astype(np.int64)
    for j in range(3):
        rows = np.concatenate([JX[o] for o in np.flatnonzero(op == j)])
        # least-squares triangulation covariance (J^T J)^-1 with unit information
        ref = np.linalg.pinv(rows) @ np.linalg.pinv(rows).T
        assert rel(out["Vinv"][j], ref) < 1e-10


# planted mistakes in the point oracle must make the pins above fail

def test_planted_gauge_sign_in_G_is_caught(monkeypatch):
    from oracle import paper_gauge
    orig = paper_gauge.structured_matrix

    def bad(scene):
        S, G, F = orig(scene)
        return S, -G, F

    monkeypatch.setattr(paper_gauge, "structured_matrix", bad)
    with pytest.raises(AssertionError):
        test_block_inversion_matches_dense(SCENES[0], "paper")


def test_planted_dropped_gauge_term_in_camera_block_is_caught(monkeypatch):
    from oracle import covariance

    def bad(Z, Q, alpha=None):
        c, s = covariance._scaled_factor(Z, Q, alpha if alpha is not None else
                                         covariance.balanced_alpha(Z, Q))
        import scipy.linalg as sla
        X = sla.cho_solve(c, np.eye(Z.shape[0]))
        return X * s[:, None] * s[None, :]   # (Z + a QQ^T)^-1 without - QQ^T / a

    monkeypatch.setattr(covariance, "pseudo_inverse", bad)
    with pytest.raises(AssertionError):
        test_block_inversion_matches_dense(SCENES[0], "camera")


def test_planted_wrong_point_rows_are_caught(monkeypatch):
    from oracle import nullspace
    orig = nullspace.point_rows
    # a sign error in the rotation columns [X]x of the point rows
    def bad(pts):
        H = orig(pts).copy()
        H[:, 3:6] *= -1.0
        return H

    monkeypatch.setattr(nullspace, "point_rows", bad)
    with pytest.raises(AssertionError):
        test_paper_gauge_is_moore_penrose(SCENES[0])
