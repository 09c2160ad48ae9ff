"""Pins of the FP64 oracle against facts fixed by the paper or by mathematics.

Each test checks an oracle stage against something other than the oracle
itself: a library routine for a textbook special case, complex-step
derivatives, a dense brute-force assembly, the null-space condition J H = 0,
the closed-form SO(3) inverse right Jacobian, SVD and multiprecision
pseudo-inverses (the paper's ground-truth procedure), Penrose conditions,
gauge-invariant sub-blocks, Loewner monotonicity and matrices with a known
spectrum.
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import scenegen as sg
from oracle import camera, covariance, nullspace, schur
from oracle.pipeline import OracleError, camera_covariance


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def block_rel(a_blocks, b_blocks):
    return max(np.linalg.norm(a - b) / np.linalg.norm(b) for a, b in zip(a_blocks, b_blocks))


def dense_jacobian(scene, JP, JX):
    n, m, t = scene.n_cams, scene.n_pts, scene.n_obs
    J = np.zeros((2 * t, 9 * n + 3 * m))
    for o in range(t):
        i, j = scene.obs_cam[o], scene.obs_pt[o]
        J[2 * o:2 * o + 2, 9 * i:9 * i + 9] = JP[o]
        J[2 * o:2 * o + 2, 9 * n + 3 * j:9 * n + 3 * j + 3] = JX[o]
    return J


def dense_information(scene):
    t = scene.n_obs
    L = np.eye(2 * t)
    if scene.obs_info is not None:
        for o in range(t):
            a, b, c = scene.obs_info[o]
            L[2 * o:2 * o + 2, 2 * o:2 * o + 2] = [[a, b], [b, c]]
    return L


def so3_right_jacobian_inverse(phi):
    """Textbook closed form of J_r(phi)^-1 for SO(3) (angle-axis phi)."""
    th = np.linalg.norm(phi)
    P = nullspace.skew(phi)
    c = 1.0 / th ** 2 - (1.0 + np.cos(th)) / (2.0 * th * np.sin(th))
    return np.eye(3) + 0.5 * P + c * (P @ P)


# ---------------------------------------------------------------------------
# projection model and Jacobians
# ---------------------------------------------------------------------------

def test_rotation_matches_library():
    rng = np.random.default_rng(1)
    r = rng.normal(size=(200, 3)) * rng.uniform(0, 3, (200, 1))
    r[:5] *= 1e-7  # exercise the series branch
    v = rng.normal(size=(200, 3))
    got = np.stack(camera.rotate(tuple(r.T), tuple(v.T)), 1)
    ref = Rotation.from_rotvec(r).apply(v)
    assert np.abs(got - ref).max() < 1e-14 * 10


def test_projection_hand_value():
    # r = 0, C = 0, f = 1000, k1 = 0.1, k2 = 0.01, X = (1, 2, 4):
    # pi = (0.25, 0.5), rho2 = 0.3125, d = 1 + 0.03125 + 0.0009765625
    cams = np.array([[0, 0, 0, 0, 0, 0, 1000.0, 0.1, 0.01]])
    pts = np.array([[1.0, 2.0, 4.0]])
    u = camera.project_values(cams, pts, np.array([0]), np.array([0]))
    d = 1.0322265625
    assert np.allclose(u[0], [1000 * d * 0.25 + 320, 1000 * d * 0.5 + 240], rtol=0, atol=1e-12)


def complex_step_jacobians(scene, h=1e-30):
    c = scene.cams[scene.obs_cam].astype(complex)
    x = scene.pts[scene.obs_pt].astype(complex)
    t = scene.n_obs
    J = np.zeros((t, 2, 12))
    for k in range(12):
        cc, xx = c.copy(), x.copy()
        if k < 9:
            cc[:, k] += 1j * h
        else:
            xx[:, k - 9] += 1j * h
        u, v = camera.project(tuple(cc.T), tuple(xx.T))
        J[:, 0, k] = np.imag(u) / h
        J[:, 1, k] = np.imag(v) / h
    return J[:, :, :9], J[:, :, 9:]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_jacobian_complex_step(seed):
    s = sg.tiny_circle(seed)
    JP, JX = camera.jacobians(s.cams, s.pts, s.obs_cam, s.obs_pt)
    cP, cX = complex_step_jacobians(s)
    scale = np.abs(cP).max(axis=(0, 1))
    assert np.all(np.abs(JP - cP).max(axis=(0, 1)) <= 1e-13 * scale)
    assert np.abs(JX - cX).max() <= 1e-13 * np.abs(cX).max()


def test_jacobian_centre_is_minus_point():
    s = sg.tiny_circle(4)
    JP, JX = camera.jacobians(s.cams, s.pts, s.obs_cam, s.obs_pt)
    assert np.array_equal(JP[:, :, 3:6], -JX)


# ---------------------------------------------------------------------------
# reduced camera matrix
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("with_info", [False, True])
def test_schur_complement_brute_force(with_info):
    s = sg.tiny_circle(5, with_info=with_info)
    out = camera_covariance(s, keep=True)
    J = dense_jacobian(s, out["JP"], out["JX"])
    M = J.T @ dense_information(s) @ J
    Nc = 9 * s.n_cams
    Mcc, Mcp, Mpp = M[:Nc, :Nc], M[:Nc, Nc:], M[Nc:, Nc:]
    Zb = Mcc - Mcp @ np.linalg.solve(Mpp, Mcp.T)
    assert rel(out["Z"], Zb) < 1e-11
    assert np.array_equal(out["Z"], out["Z"].T) or rel(out["Z"], out["Z"].T) < 1e-15


def test_reduced_matrix_null_space_and_rank():
    s = sg.tiny_circle(6)
    out = camera_covariance(s, keep=True)
    Z, Hc = out["Z"], out["Hc"]
    assert np.abs(Z @ Hc).max() <= 1e-14 * np.abs(Z).max() * np.abs(Hc).max()
    ev = np.sort(np.abs(np.linalg.eigvalsh(Z))) / np.abs(Z).max()
    assert ev[6] < 1e-14 and ev[7] > 1e-12  # exactly seven gauge directions


# ---------------------------------------------------------------------------
# nullspace
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 7])
def test_jacobian_times_nullspace_is_zero(seed):
    s = sg.tiny_circle(seed)
    out = camera_covariance(s, keep=True)
    J = dense_jacobian(s, out["JP"], out["JX"])
    H = np.vstack([out["Hc"], nullspace.point_rows(s.pts)])
    assert np.linalg.matrix_rank(H) == 7
    assert np.abs(J @ H).max() <= 1e-13 * np.abs(J).max() * np.abs(H).max()


def test_rotation_block_closed_form():
    s = sg.tiny_circle(8)
    out = camera_covariance(s, keep=True)
    for i in range(s.n_cams):
        ref = so3_right_jacobian_inverse(s.cams[i, :3])
        assert np.abs(out["Hr"][i] - ref).max() < 1e-12


# ---------------------------------------------------------------------------
# Moore-Penrose covariance
# ---------------------------------------------------------------------------

def svd_pinv(A, nullity=7):
    """The paper's ground-truth procedure: SVD, last seven singular values zeroed."""
    U, sv, Vt = np.linalg.svd(A)
    inv = np.zeros_like(sv)
    inv[:-nullity] = 1.0 / sv[:-nullity]
    return (Vt.T * inv) @ U.T


@pytest.mark.parametrize("seed", range(5))
def test_covariance_matches_svd_pinv(seed):
    s = sg.tiny_circle(seed)
    out = camera_covariance(s, keep=True)
    P = svd_pinv(out["Z"])
    assert block_rel(out["blocks"], covariance.camera_blocks(P)) < 1e-5


def test_covariance_matches_multiprecision_pinv():
    mp = pytest.importorskip("mpmath")
    s = sg.tiny_circle(3, n=6, m=24)
    out = camera_covariance(s, keep=True)
    Z = out["Z"]
    N = Z.shape[0]
    mp.mp.dps = 40
    E, V = mp.eigsy(mp.matrix(Z.tolist()))
    ev = np.array([float(e) for e in E])
    order = np.argsort(np.abs(ev))
    D = mp.zeros(N, N)
    for k in order[7:]:
        D[int(k), int(k)] = 1 / E[int(k)]
    P = np.array((V * D * V.T).tolist(), dtype=float)
    assert block_rel(out["blocks"], covariance.camera_blocks(P)) < 1e-9


def test_penrose_conditions_and_gauge():
    s = sg.tiny_circle(9)
    out = camera_covariance(s, full=True, keep=True)
    Z, S, Hc = out["Z"], out["full"], out["Hc"]
    assert rel(Z @ S @ Z, Z) < 1e-8
    assert rel(S @ Z @ S, S) < 1e-8
    ZS = Z @ S
    assert rel(ZS, ZS.T) < 1e-8
    assert rel(S, S.T) < 1e-12
    assert np.abs(S @ Hc).max() <= 1e-9 * np.abs(S).max() * np.abs(Hc).max()
    ev = np.linalg.eigvalsh(0.5 * (S + S.T))
    assert ev.min() > -1e-9 * ev.max()


def test_alpha_does_not_change_result():
    s = sg.tiny_circle(10)
    a = camera_covariance(s, keep=True)
    b = camera_covariance(s, alpha=a["alpha"] * 37.0)
    assert block_rel(b["blocks"], a["blocks"]) < 1e-7


def test_blocks_by_solves_equal_full_inverse():
    s = sg.tiny_circle(11)
    a = camera_covariance(s, full=True)
    b = camera_covariance(s)
    assert block_rel(b["blocks"], a["blocks"]) < 1e-10


def test_known_spectrum():
    """Z = B diag(lam) B^T with a prescribed null space: Z^+ = B diag(1/lam) B^T."""
    rng = np.random.default_rng(12)
    N = 90
    for kappa in [1e2, 1e4, 1e6, 1e8]:
        B, _ = np.linalg.qr(rng.normal(size=(N, N)))
        lam = np.geomspace(1.0, 1.0 / kappa, N - 7) * 1e3
        R = B[:, :N - 7]
        Q0 = B[:, N - 7:]
        Z = (R * lam) @ R.T
        Z = 0.5 * (Z + Z.T)
        ref = (R / lam) @ R.T
        # a non-orthonormal basis of the null space, orthonormalised by the oracle
        Hc = Q0 @ rng.normal(size=(7, 7))
        Q = covariance.orthonormal_basis(Hc)
        got = covariance.pseudo_inverse(Z, Q)
        assert rel(got, ref) < 1e-15 * kappa * 50


def test_intrinsics_blocks_are_gauge_invariant():
    """The (f, k1, k2) sub-blocks equal those of a plain Cholesky inverse of Z
    with seven gauge parameters deleted (any g-inverse projects to Z^+)."""
    s = sg.tiny_circle(13)
    out = camera_covariance(s, full=True, keep=True)
    Z = out["Z"]
    fixed = [0, 1, 2, 3, 4, 5, 9 + 3]  # camera 0's r and C, camera 1's C_x
    keep = np.setdiff1d(np.arange(Z.shape[0]), fixed)
    Zr = Z[np.ix_(keep, keep)]
    L = np.linalg.cholesky(Zr)
    Li = np.linalg.inv(L)
    G = np.zeros_like(Z)
    G[np.ix_(keep, keep)] = Li.T @ Li
    intr = np.concatenate([np.arange(9 * i + 6, 9 * i + 9) for i in range(s.n_cams)])
    assert rel(out["full"][np.ix_(intr, intr)], G[np.ix_(intr, intr)]) < 1e-8


def test_similarity_transform_leaves_intrinsics_unchanged():
    s = sg.tiny_circle(14)
    rng = np.random.default_rng(14)
    Rs = Rotation.from_rotvec(rng.normal(size=3))
    mu, T = 2.7, rng.normal(size=3) * 5
    s2 = sg.Scene(s.cams.copy(), mu * Rs.apply(s.pts) + T, s.obs_cam, s.obs_pt)
    s2.cams[:, 3:6] = mu * Rs.apply(s.cams[:, 3:6]) + T
    s2.cams[:, 0:3] = (Rotation.from_rotvec(s.cams[:, 0:3]) * Rs.inv()).as_rotvec()
    a = camera_covariance(s)["blocks"]
    b = camera_covariance(s2)["blocks"]
    assert block_rel(b[:, 6:, 6:], a[:, 6:, 6:]) < 1e-8
    assert block_rel(b, a) > 1e-4  # the pose blocks do depend on the gauge


def test_fewer_points_never_decrease_covariance():
    """Removing points removes PSD terms from Z with the null space unchanged,
    so Z^+ can only grow in the Loewner order (the paper's sub-reconstruction
    bound)."""
    s = sg.tiny_circle(15, m=300)
    rng = np.random.default_rng(15)
    keep = rng.uniform(size=s.n_pts) > 0.25
    a = camera_covariance(s, full=True)["full"]
    b = camera_covariance(s.subset_points(keep), full=True)["full"]
    ev = np.linalg.eigvalsh(0.5 * ((b - a) + (b - a).T))
    assert ev.min() > -1e-9 * np.abs(a).max()
    assert ev.max() > 0


def test_paper_route_through_full_information_matrix():
    """The paper's ground truth: M^+ of the full information matrix by SVD
    (seven singular values zeroed).  Its camera block is the same covariance
    in the all-parameter gauge; projecting it onto the complement of range(H_c)
    gives Z^+."""
    s = sg.tiny_circle(16)
    out = camera_covariance(s, full=True, keep=True)
    J = dense_jacobian(s, out["JP"], out["JX"])
    M = J.T @ J
    Nc = 9 * s.n_cams
    Mp = svd_pinv(M)[:Nc, :Nc]
    Pc = np.eye(Nc) - out["Q"] @ out["Q"].T
    assert block_rel(covariance.camera_blocks(Pc @ Mp @ Pc), out["blocks"]) < 1e-5


# ---------------------------------------------------------------------------
# input checks
# ---------------------------------------------------------------------------

def test_input_errors():
    s = sg.tiny_circle(17)
    bad = sg.Scene(s.cams, s.pts, s.obs_cam.copy(), s.obs_pt.copy())
    bad.obs_cam[3] = s.n_cams
    with pytest.raises(OracleError) as e:
        camera_covariance(bad)
    assert e.value.kind == "EINVAL"

    dup = sg.Scene(s.cams, s.pts, np.append(s.obs_cam, s.obs_cam[0]), np.append(s.obs_pt, s.obs_pt[0]))
    with pytest.raises(OracleError) as e:
        camera_covariance(dup)
    assert e.value.kind == "EINVAL"

    # a point seen once
    j = int(s.obs_pt[0])
    sel = (s.obs_pt != j) | (np.arange(s.n_obs) == 0)
    lone = sg.Scene(s.cams, s.pts, s.obs_cam[sel], s.obs_pt[sel])
    with pytest.raises(OracleError) as e:
        camera_covariance(lone)
    assert e.value.kind == "EPOINT" and e.value.index == j

    # a point seen by two cameras at the same centre has no depth information
    from failure_scenes import behind_camera, coincident_centres
    deg, j2 = coincident_centres()
    with pytest.raises(OracleError) as e:
        camera_covariance(deg)
    assert e.value.kind == "EPOINT" and e.value.index == j2

    # a point behind a camera that observes it: the first such observation
    behind, bad = behind_camera()
    with pytest.raises(OracleError) as e:
        camera_covariance(behind)
    assert e.value.kind == "EINVAL" and e.value.index == min(bad)

    # two disconnected halves: nullity 14, A is not positive definite
    a = sg.tiny_circle(18, n=5, m=60)
    b = sg.tiny_circle(19, n=5, m=60)
    two = sg.Scene(np.vstack([a.cams, b.cams]), np.vstack([a.pts, b.pts]),
                   np.concatenate([a.obs_cam, b.obs_cam + 5]).astype(np.int32),
                   np.concatenate([a.obs_pt, b.obs_pt + 60]).astype(np.int32))
    with pytest.raises(OracleError) as e:
        camera_covariance(two)
    assert e.value.kind == "EGAUGE"
