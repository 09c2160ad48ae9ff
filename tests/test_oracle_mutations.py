"""Planted mistakes in the oracle must make its pins fail.

Each test patches one oracle step with a plausible error (a dropped term, a
wrong sign, a transposed operand, a wrong exponent) and checks that the pin
covering that step rejects it.  All of this runs on the CPU.
"""
import numpy as np
import pytest

from oracle import camera, covariance, nullspace, schur
import test_oracle_pins as pins
from oracle.pipeline import OracleError


def test_wrong_sign_in_centre_rows_breaks_JH(monkeypatch):
    orig = nullspace.camera_rows

    def bad(cams, Hr):
        H = orig(cams, Hr)
        for i in range(cams.shape[0]):
            H[9 * i + 3:9 * i + 6, 3:6] *= -1.0
        return H

    monkeypatch.setattr(nullspace, "camera_rows", bad)
    with pytest.raises(AssertionError):
        pins.test_jacobian_times_nullspace_is_zero(0)


def test_transposed_rotation_block_breaks_closed_form(monkeypatch):
    orig = nullspace.rotation_blocks
    monkeypatch.setattr(nullspace, "rotation_blocks",
                        lambda *a: np.transpose(orig(*a), (0, 2, 1)))
    with pytest.raises(AssertionError):
        pins.test_rotation_block_closed_form()


def test_dropped_camera_block_breaks_brute_force(monkeypatch):
    orig = schur.reduced_camera_matrix

    def bad(U, W, Vinv, oc, op, n, m):
        return orig(np.zeros_like(U), W, Vinv, oc, op, n, m)

    monkeypatch.setattr(schur, "reduced_camera_matrix", bad)
    # the pipeline looks the function up at run time; the pin fails either by
    # its assertion or because the broken Z is no longer positive semi-definite
    with pytest.raises((AssertionError, OracleError)):
        pins.test_schur_complement_brute_force(False)


def test_ignored_information_breaks_brute_force(monkeypatch):
    monkeypatch.setattr(schur, "information_blocks",
                        lambda info, t: np.broadcast_to(np.eye(2), (t, 2, 2)).copy())
    with pytest.raises(AssertionError):
        pins.test_schur_complement_brute_force(True)


def test_wrong_gauge_sign_in_blocks_breaks_block_pin(monkeypatch):
    orig = covariance.pseudo_inverse_blocks

    def bad(Z, Q, alpha=None, cameras=None):
        a = covariance.balanced_alpha(Z, Q) if alpha is None else alpha
        out = orig(Z, Q, a, cameras)
        n = Z.shape[0] // 9
        cams = np.arange(n) if cameras is None else np.asarray(cameras)
        for k, i in enumerate(cams):
            Qi = Q[9 * i:9 * i + 9]
            out[k] += 2.0 * (Qi @ Qi.T) / a  # + instead of - for the gauge term
        return out

    monkeypatch.setattr(covariance, "pseudo_inverse_blocks", bad)
    # the gauge term is small next to the focal-length variance, so the
    # Frobenius-relative SVD pin cannot see it; the block/full comparison can
    with pytest.raises(AssertionError):
        pins.test_blocks_by_solves_equal_full_inverse()


def test_wrong_gauge_sign_breaks_gauge_condition(monkeypatch):
    orig = covariance.pseudo_inverse

    def bad(Z, Q, alpha=None):
        a = covariance.balanced_alpha(Z, Q) if alpha is None else alpha
        return orig(Z, Q, a) + 2.0 * (Q @ Q.T) / a

    monkeypatch.setattr(covariance, "pseudo_inverse", bad)
    with pytest.raises(AssertionError):
        pins.test_penrose_conditions_and_gauge()


def test_wrong_distortion_exponent_breaks_hand_value(monkeypatch):
    def bad_project(cam, X, principal=(320.0, 240.0)):
        r, C = cam[0:3], cam[3:6]
        f, k1, k2 = cam[6], cam[7], cam[8]
        x = camera.rotate(r, (X[0] - C[0], X[1] - C[1], X[2] - C[2]))
        px, py = x[0] / x[2], x[1] / x[2]
        rho2 = px * px + py * py
        d = 1.0 + k1 * rho2 + k2 * rho2  # rho^2 where rho^4 belongs
        return (f * d * px + principal[0], f * d * py + principal[1])

    monkeypatch.setattr(camera, "project", bad_project)
    with pytest.raises(AssertionError):
        pins.test_projection_hand_value()


def test_unscaled_inverse_breaks_known_spectrum(monkeypatch):
    def bad(Z, Q, alpha=None):
        a = covariance.balanced_alpha(Z, Q) if alpha is None else alpha
        return np.linalg.inv(Z + a * Q @ Q.T)  # gauge term never removed

    monkeypatch.setattr(covariance, "pseudo_inverse", bad)
    with pytest.raises(AssertionError):
        pins.test_known_spectrum()
