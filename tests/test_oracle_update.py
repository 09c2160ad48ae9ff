"""Pins of the incremental-update oracle (Sec. 6, the Woodbury identity in
its corrected form).

The update route (``update.woodbury``: effective observation rows on the
cameras, their error covariance, the identity on Z^+) must equal the
definition, the extended reconstruction recomputed from scratch
(``update.recompute``), for added observations and for a new camera; the
covariance of the old cameras can only decrease (Loewner order); two batches
equal one; the identity as printed (the information matrix where its inverse
belongs, the observations' covariance dropped) fails.  All on the CPU.
"""
import numpy as np
import pytest

import scenegen as sg
from oracle import update
from oracle.pipeline import camera_covariance

SCENES = [lambda: sg.tiny_circle(0), lambda: sg.tiny_circle(1, with_info=True),
          lambda: sg.spiral_slab(5, n=60, m=3000)]


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("maker", SCENES)
@pytest.mark.parametrize("new_camera", [False, True])
def test_woodbury_matches_recompute(maker, new_camera):
    s = maker()
    add = sg.additions(s, 3, 12, new_camera=new_camera)
    Xr, Cr, Kr = update.recompute(s, *add)
    Xw, Cw, Kw = update.woodbury(s, *add)
    assert rel(Xw, Xr) < 1e-8
    if new_camera:
        assert rel(Cw, Cr) < 1e-8 and rel(Kw, Kr) < 1e-8


@pytest.mark.parametrize("new_camera", [False, True])
def test_covariance_only_decreases(new_camera):
    s = SCENES[1]()
    Zp = camera_covariance(s, full=True)["full"]
    X, _, _ = update.woodbury(s, *sg.additions(s, 4, 10, new_camera=new_camera), Zp=Zp)
    lam = np.linalg.eigvalsh(Zp - X)
    assert lam.min() > -1e-10 * np.abs(Zp).max()
    assert np.trace(X) < np.trace(Zp)


def test_two_batches_equal_one():
    s = SCENES[0]()
    cam, pt, info, _ = sg.additions(s, 5, 16)
    X_all, _, _ = update.woodbury(s, cam, pt, info)
    X1, _, _ = update.woodbury(s, cam[:7], pt[:7], info)
    s1 = update.extended_scene(s, cam[:7], pt[:7], info)
    X2, _, _ = update.woodbury(s1, cam[7:], pt[7:], info, Zp=X1)
    assert rel(X2, X_all) < 1e-9


def test_several_observations_of_one_point_share_its_error():
    """New observations of the same point are correlated through the point's
    own uncertainty V_j^-1; dropping that term must break the agreement."""
    s = SCENES[0]()
    j = int(s.obs_pt[0])
    have = set(s.obs_cam[s.obs_pt == j].tolist())
    cams = [c for c in range(s.n_cams) if c not in have][:3]
    cam, pt = np.asarray(cams, np.int32), np.full(len(cams), j, np.int32)
    Xr, _, _ = update.recompute(s, cam, pt)
    Xw, _, _ = update.woodbury(s, cam, pt)
    assert rel(Xw, Xr) < 1e-8


def test_printed_form_fails(monkeypatch):
    """The identity as printed, with the information Z where Z^+ belongs and
    the observations' covariance replaced by I, does not give the update."""
    s = SCENES[0]()
    add = sg.additions(s, 6, 8)
    out = camera_covariance(s, keep=True)
    Xr, _, _ = update.recompute(s, *add)
    Xg, _, _ = update.woodbury(s, *add, Zp=out["Z"])
    assert rel(Xg, Xr) > 1e-2


def test_planted_dropped_shared_error_is_caught(monkeypatch):
    orig = update.effective_rows

    def bad(scene, new_cam, new_pt, new_info=None, cam_new=None):
        Jt, Jn, Oinv = orig(scene, new_cam, new_pt, new_info, cam_new)
        k = Oinv.shape[0] // 2
        keep = np.zeros_like(Oinv)
        for a in range(k):   # only the observations' own covariance
            keep[2 * a:2 * a + 2, 2 * a:2 * a + 2] = np.linalg.inv(
                update.schur.information_blocks(new_info, k)[a])
        return Jt, Jn, keep

    monkeypatch.setattr(update, "effective_rows", bad)
    with pytest.raises(AssertionError):
        test_woodbury_matches_recompute(SCENES[0], False)
