"""Pins of the paper-gauge oracle, (M^+)_cc (CPU).

The structured route (points eliminated with the full nullspace) is checked
against the definition (eigendecomposition of the dense M with seven
eigenvalues dropped), and against the already pinned Z^+ through the gauge
relation Z^+ = P_c (M^+)_cc P_c."""
import numpy as np
import pytest

import scenegen as sg
from oracle import covariance, paper_gauge as pg
from oracle.pipeline import camera_covariance


def rel(a, b):
    return max(np.linalg.norm(x - y) / np.linalg.norm(y) for x, y in zip(a, b))


@pytest.mark.parametrize("maker", [lambda: sg.tiny_circle(0), lambda: sg.tiny_circle(3, with_info=True),
                                   lambda: sg.tiny_circle(5, n=8, m=150)])
def test_structured_route_matches_the_definition(maker):
    s = maker()
    a = pg.camera_blocks(s)
    b, _ = pg.camera_blocks_dense(s)
    assert rel(a, b) < 2e-6


@pytest.mark.parametrize("maker", [lambda: sg.tiny_circle(1), lambda: sg.tiny_circle(2, with_info=True),
                                   lambda: sg.spiral_slab(4, n=20, m=600)])
def test_projection_onto_the_camera_gauge_gives_z_plus(maker):
    s = maker()
    blocks, X = pg.camera_blocks(s, full=True)
    ref = camera_covariance(s, keep=True)
    P = np.eye(X.shape[0]) - ref["Q"] @ ref["Q"].T
    assert rel(covariance.camera_blocks(P @ X @ P), ref["blocks"]) < 1e-9
    # the intrinsics sub-blocks do not depend on the gauge; the pose blocks do
    assert rel(blocks[:, 6:, 6:], ref["blocks"][:, 6:, 6:]) < 1e-9
    assert rel(blocks, ref["blocks"]) > 1e-4


def test_structured_matrix_is_positive_definite_and_not_gauge_free():
    s = sg.tiny_circle(6)
    S, G, F = pg.structured_matrix(s)
    assert np.linalg.eigvalsh(S).min() > 0
    assert np.linalg.eigvalsh(F).min() > 0
    ref = camera_covariance(s, full=True, keep=True)
    Hc, Zp = ref["Hc"], ref["full"]
    X = np.linalg.inv(S)
    # Z^+ annihilates range(H_c); the paper's (M^+)_cc does not
    assert np.linalg.norm(X @ Hc) > 1e6 * np.linalg.norm(Zp @ Hc)
