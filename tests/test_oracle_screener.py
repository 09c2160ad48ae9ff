"""Pins of the screener oracle (CPU): features, label scale, log-Cholesky, MLP, Adam."""
import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

import scenegen as sg
from oracle import screener
from oracle.pipeline import camera_covariance as oracle_cov


def test_z_diagonal_blocks_match_the_dense_schur_complement():
    s = sg.tiny_circle(3, with_info=True)
    Zd = screener.z_diagonal_blocks(s)
    Z = oracle_cov(s, keep=True)["Z"]
    for i in range(s.n_cams):
        blk = Z[9 * i:9 * i + 9, 9 * i:9 * i + 9]
        assert np.abs(Zd[i] - blk).max() <= 1e-12 * np.abs(blk).max()


def test_features_track_histogram_and_covisibility_brute_force():
    s = sg.spiral_slab(4, n=20, m=600)
    F = screener.camera_features(s)
    tl = np.bincount(s.obs_pt, minlength=s.n_pts)[s.obs_pt]
    edges = np.array(screener.TRACK_BINS)
    for i in range(s.n_cams):
        lens = tl[s.obs_cam == i]
        counts = [np.sum((lens >= lo) & (lens < hi)) for lo, hi in zip(edges, list(edges[1:]) + [10 ** 9])]
        assert np.allclose(F[i, 45:53], np.log1p(counts))
    A = np.zeros((s.n_cams, s.n_pts))
    A[s.obs_cam, s.obs_pt] = 1
    co = (A @ A.T) > 0
    np.fill_diagonal(co, False)
    assert np.allclose(F[:, 54], np.log1p(co.sum(axis=1)))
    # Z-block part: unit diagonal correlations are excluded, |corr| <= 1
    iu = [k for k, (a, b) in enumerate((a, b) for a in range(9) for b in range(a, 9)) if a != b]
    assert np.all(np.abs(F[:, iu]) <= 1 + 1e-12)


def test_triangulation_angle_hand_example():
    """Two cameras at (+-1, 0, 0) looking along +y, one point at (0, 1, 0):
    the rays meet at a right angle."""
    rows = np.array([[1.0, 0, 0], [0, 0, -1.0], [0, 1.0, 0]])  # camera z axis = world +y
    r = Rotation.from_matrix(rows).as_rotvec()
    cams = np.array([[*r, -1.0, 0, 0, 1000.0, 0, 0], [*r, 1.0, 0, 0, 1000.0, 0, 0]])
    pts = np.array([[0.0, 1.0, 0.0], [0.2, 2.0, 0.3]])
    s = sg.Scene(cams, pts, np.array([0, 1, 0, 1], np.int32), np.array([0, 0, 1, 1], np.int32))
    with np.errstate(all="ignore"):
        F = screener.camera_features(s)
    second = np.arccos(np.dot(pts[1] - cams[0, 3:6], pts[1] - cams[1, 3:6])
                       / np.linalg.norm(pts[1] - cams[0, 3:6]) / np.linalg.norm(pts[1] - cams[1, 3:6]))
    assert F[0, 53] == pytest.approx(0.5 * (np.pi / 2 + second), rel=1e-12)
    assert F[1, 53] == pytest.approx(F[0, 53], rel=1e-12)
    assert np.allclose(F[:, 54], np.log(2.0))
    assert np.allclose(F[:, 45], np.log(3.0)) and np.allclose(F[:, 46:53], 0.0)


def test_log_cholesky_closed_form_and_round_trip():
    D = np.linspace(0.5, 2.0, 9)
    s = np.linspace(1.0, 3.0, 9)
    S = np.diag((D * s) ** 2)[None]
    P = screener.log_cholesky(S, D)
    diag_idx = [a * (a + 1) // 2 + a for a in range(9)]
    assert np.allclose(P[0, diag_idx], np.log(s), atol=1e-14)
    assert np.allclose(np.delete(P[0], diag_idx), 0.0, atol=1e-14)
    rng = np.random.default_rng(0)
    A = rng.normal(size=(5, 9, 9))
    S = A @ np.transpose(A, (0, 2, 1)) + 0.1 * np.eye(9)
    back = screener.from_log_cholesky(screener.log_cholesky(S, D), D)
    assert np.abs(back - S).max() <= 1e-12 * np.abs(S).max()


def test_zii_from_features_inverts_the_feature_definition():
    """Z_ii rebuilt from the 45 features equals the block the features were
    taken from (itself pinned to the dense Schur complement)."""
    s = sg.spiral_slab(4, n=20, m=600)
    Zd = screener.z_diagonal_blocks(s)
    back = screener.zii_from_features(screener.camera_features(s))
    assert np.abs(back - Zd).max() <= 1e-12 * np.abs(Zd).max()


def features_of(Z):
    """The 45 Z_ii features of (k, 9, 9) blocks, by their definition."""
    out = []
    for a in range(9):
        for b in range(a, 9):
            out.append(np.log10(Z[:, a, a]) if a == b
                       else Z[:, a, b] / np.sqrt(Z[:, a, a] * Z[:, b, b]))
    return np.stack(out, 1)


def test_block_scale_closed_form_with_one_coupled_pair():
    """A block coupling only parameters 2 and 5 with correlation rho: with the
    ridge r on the correlation matrix, ((C + r I)^-1)_22 = (1 + r) /
    ((1 + r)^2 - rho^2) (the 2x2 inverse), the others 1 / (1 + r); b_a is the
    square root over Z_aa.  A singular block (rho = 1) stays finite."""
    d = np.linspace(0.5, 40.0, 9)
    r = screener.SCALE_RIDGE
    for rho in (0.8, 1.0):
        Z = np.diag(d)[None].copy()
        Z[0, 2, 5] = Z[0, 5, 2] = rho * np.sqrt(d[2] * d[5])
        b = screener.block_scale(features_of(Z))[0]
        want = 1.0 / np.sqrt((1 + r) * d)
        c22 = (1 + r) / ((1 + r) ** 2 - rho ** 2)
        want[2] = np.sqrt(c22 / d[2])
        want[5] = np.sqrt(c22 / d[5])
        assert np.allclose(b, want, rtol=1e-9), rho
    # an uncoupled block: b_a = 1 / sqrt((1 + r) Z_aa)
    b = screener.block_scale(features_of(np.diag(d)[None]))[0]
    assert np.allclose(b, 1.0 / np.sqrt((1 + r) * d), rtol=1e-13)


def test_label_scale_is_the_lower_median_of_the_variance_ratios():
    """Four cameras with Z_ii = I: the scale is the square root of the
    second-smallest variance ratio per parameter (rank (4 - 1) // 2 = 1)."""
    var = np.array([[4.0] * 9, [1.0] * 9, [9.0] * 9, [16.0] * 9])
    var[:, 3] = [25.0, 36.0, 49.0, 64.0]
    S = np.stack([np.diag(v) for v in var])
    F = features_of(np.broadcast_to(np.eye(9), (4, 9, 9)).copy())
    s = screener.label_scale(S, F)
    want = np.full(9, 2.0)
    want[3] = 6.0
    ridge = np.sqrt(1.0 + screener.SCALE_RIDGE)  # b = 1 / sqrt(1 + ridge) for Z_ii = I
    assert np.allclose(s, want * ridge, rtol=1e-14)
    # with Z_ii = 4 I, b halves and the ratios grow by 4
    F4 = features_of(np.broadcast_to(4.0 * np.eye(9), (4, 9, 9)).copy())
    assert np.allclose(screener.label_scale(S, F4), 2.0 * want * ridge, rtol=1e-14)


def test_label_moments_hand_values_and_a_normal_sample():
    """Lower median and scaled median absolute deviation: hand values for odd
    and even counts (one outlier does not move them), ~sigma on a normal
    sample; the standardised labels are clipped at +-6."""
    P = np.array([[1.0, 1.0], [2.0, 2.0], [3.0, 3.0], [4.0, 4.0], [100.0, -50.0]])
    m, s = screener.label_moments(P)
    assert np.array_equal(m, [3.0, 2.0])        # ranks (5 - 1) // 2 = 2
    assert np.allclose(s, [1.4826, 1.4826 * 1.0])  # |P - m| sorted: [0 1 1 2 97], [0 1 1 2 52]
    m4, s4 = screener.label_moments(P[:4])
    assert np.array_equal(m4, [2.0, 2.0]) and np.allclose(s4, 1.4826)
    rng = np.random.default_rng(5)
    x = rng.normal(3.0, 2.5, size=(200_001, 1))
    mx, sx = screener.label_moments(x)
    assert abs(mx[0] - 3.0) < 0.02 and abs(sx[0] / 2.5 - 1.0) < 0.01
    z = screener.standardise(np.array([[-100.0], [0.5], [100.0]]), np.array([0.0]), np.array([0.5]))
    assert np.array_equal(z[:, 0], [-6.0, 1.0, 6.0])


def test_log_cholesky_per_camera_scale():
    """Per-camera D: a diagonal block D_i^2 s^2 maps to log s and zeros, and
    the round trip holds block by block."""
    rng = np.random.default_rng(3)
    D = rng.uniform(0.1, 10.0, (4, 9))
    s = np.linspace(1.0, 3.0, 9)
    S = np.stack([np.diag((D[i] * s) ** 2) for i in range(4)])
    P = screener.log_cholesky(S, D)
    diag_idx = [a * (a + 1) // 2 + a for a in range(9)]
    assert np.allclose(P[:, diag_idx], np.log(s)[None], atol=1e-13)
    assert np.allclose(np.delete(P, diag_idx, axis=1), 0.0, atol=1e-13)
    A = rng.normal(size=(4, 9, 9))
    S = A @ np.transpose(A, (0, 2, 1)) + 0.1 * np.eye(9)
    back = screener.from_log_cholesky(screener.log_cholesky(S, D), D)
    assert np.abs(back - S).max() <= 1e-12 * np.abs(S).max()


def torch_mlp(p):
    mods = []
    for li, (W, b) in enumerate(screener.split_params(p)):
        lin = torch.nn.Linear(W.shape[1], W.shape[0]).double()
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(W))
            lin.bias.copy_(torch.from_numpy(b))
        mods.append(lin)
        if li + 1 < 4:
            mods.append(torch.nn.ReLU())
    return torch.nn.Sequential(*mods)


def test_mlp_forward_and_backward_match_torch_autograd():
    p = sg.mlp_init(5)
    p[200:300] += 0.05  # some nonzero biases
    assert p.size == screener.param_count() == 157485
    rng = np.random.default_rng(1)
    x, t = rng.normal(size=(33, 55)), rng.normal(size=(33, 45))
    y, _ = screener.mlp_forward(p, x)
    net = torch_mlp(p)
    yt = net(torch.from_numpy(x))
    assert np.abs(y - yt.detach().numpy()).max() <= 1e-12 * np.abs(y).max()
    loss, g = screener.mlp_backward(p, x, t)
    lt = torch.mean((yt - torch.from_numpy(t)) ** 2)
    lt.backward()
    gt = np.concatenate([np.concatenate([m.weight.grad.numpy().ravel(), m.bias.grad.numpy()])
                         for m in net if isinstance(m, torch.nn.Linear)])
    assert loss == pytest.approx(lt.item(), rel=1e-13)
    assert np.abs(g - gt).max() <= 1e-12 * np.abs(gt).max()


def test_mlp_backward_central_differences():
    p = sg.mlp_init(6)
    rng = np.random.default_rng(2)
    x, t = rng.normal(size=(7, 55)), rng.normal(size=(7, 45))
    _, g = screener.mlp_backward(p, x, t)
    idx = rng.choice(p.size, 40, replace=False)
    idx = np.concatenate([idx, [0, p.size - 1, 55 * 256 + 3]])  # W1, last bias, b1
    h = 1e-6
    for k in idx:
        e = np.zeros_like(p)
        e[k] = h
        fd = (screener.mse(screener.mlp_forward(p + e, x)[0], t)
              - screener.mse(screener.mlp_forward(p - e, x)[0], t)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])) + 1e-9, k


def test_adam_first_steps_closed_form():
    g = np.array([0.5, -2.0, 1e-3])
    p0 = np.array([1.0, 2.0, 3.0])
    p1, m, v = screener.adam_step(p0, g, np.zeros(3), np.zeros(3), 1, 0.01)
    # first step: bias-corrected moments are g and g^2
    assert np.allclose(p1, p0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    # second step with the same gradient: again the moments are g and g^2
    p2, _, _ = screener.adam_step(p1, g, m, v, 2, 0.01)
    assert np.allclose(p2, p1 - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-14)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(3)
    a = np.concatenate([rng.normal(size=1000) * 10.0 ** rng.integers(-20, 20, 1000),
                        [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -1.0 - 2.0 ** -8, 0.0, 1.0]])
    ref = torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(screener.bf16(a), ref)
    assert screener.bf16([1.0 + 2.0 ** -8])[0] == 1.0          # tie to even (down)
    assert screener.bf16([1.0 + 3 * 2.0 ** -8])[0] == 1.0 + 2.0 ** -6  # tie to even (up)


def test_bf16_mode_exact_on_representable_networks():
    """Weights in {-1, 0, 1} with one nonzero per row after the first layer,
    inputs in {0, 1}, integer biases: every value stays a small integer, which
    bfloat16 holds exactly, so the BF16 mode must equal the FP64 one."""
    rng = np.random.default_rng(8)
    p = np.zeros(screener.param_count())
    for li, (W, b) in enumerate(screener.split_params(p)):
        if li == 0:
            W[...] = rng.integers(-1, 2, W.shape)
        else:
            W[np.arange(W.shape[0]), rng.integers(0, W.shape[1], W.shape[0])] = rng.choice([-1.0, 1.0], W.shape[0])
        b[...] = rng.integers(-2, 3, b.shape)
    x = rng.integers(0, 2, (16, 55)).astype(np.float64)
    y64, _ = screener.mlp_forward(p, x)
    y16, _ = screener.mlp_forward(p, x, bf16_ops=True)
    assert np.abs(y64).max() < 256 and np.array_equal(y16, y64)


def test_bf16_mode_gradient_within_rounding_when_no_relu_can_flip():
    """All weights and inputs positive: every pre-activation is positive, no
    ReLU decision can change, and the BF16-mode gradient differs from the
    pinned FP64 gradient only by operand rounding."""
    p = np.abs(sg.mlp_init(7)) * 0.3
    rng = np.random.default_rng(4)
    x, t = np.abs(rng.normal(size=(64, 55))), rng.normal(size=(64, 45))
    y64, _ = screener.mlp_forward(p, x)
    y16, _ = screener.mlp_forward(p, x, bf16_ops=True)
    assert np.linalg.norm(y16 - y64) / np.linalg.norm(y64) < 1e-2
    _, g64 = screener.mlp_backward(p, x, t)
    _, g16 = screener.mlp_backward(p, x, t, bf16_ops=True)
    for (W1, b1), (W2, b2) in zip(screener.split_params(g16), screener.split_params(g64)):
        assert np.linalg.norm(W1 - W2) / np.linalg.norm(W2) < 2e-2
        assert np.linalg.norm(b1 - b2) / np.linalg.norm(b2) < 2e-2
