"""The parity scenes are well posed in FP64.

A 1e-6 relative bar between two FP64 implementations only means something
when rounding in FP64 moves the exact covariance far less than that.  The
oracle alone measures it: the same scene with its observations permuted
changes only the order of every sum (Schur scatter, normal equations), so the
difference of the two oracle results is the rounding sensitivity of the
scene.  Every recipe the parity tests use must stay below 1e-8.
"""
import numpy as np
import pytest

import scenegen as sg
from oracle.pipeline import camera_covariance as oracle_cov


def rounding_sensitivity(scene, seed=1):
    p = np.random.default_rng(seed).permutation(scene.n_obs)
    info = None if scene.obs_info is None else scene.obs_info[p]
    shuffled = sg.Scene(scene.cams, scene.pts, scene.obs_cam[p], scene.obs_pt[p], info)
    a, b = oracle_cov(scene)["blocks"], oracle_cov(shuffled)["blocks"]
    return max(np.linalg.norm(x - y) / np.linalg.norm(y) for x, y in zip(a, b))


@pytest.mark.parametrize("maker", [
    lambda: sg.tiny_circle(0),
    lambda: sg.tiny_circle(2, with_info=True),
    lambda: sg.spiral_slab(11, n=37, m=2000),
    lambda: sg.spiral_slab(13, n=60, m=3000),
    lambda: sg.batch_scenes(seed=3000, count=8, lo=20, hi=70)[5],
    lambda: sg.batch_scenes(count=1, lo=20, hi=21)[0],
    lambda: sg.clustered(3, n_clusters=3, per_cluster=40, m=6000),
    lambda: sg.clustered(4, n_clusters=4, per_cluster=30, m=5000, with_info=True),
])
def test_parity_scenes_are_well_conditioned(maker):
    s = maker()
    assert rounding_sensitivity(s) < 1e-8


def test_observations_lie_in_the_image():
    """Spiral observations project inside the 640 x 480 frame (visibility model)."""
    from oracle import camera
    s = sg.spiral_slab(3, n=40, m=2000)
    u = np.asarray(camera.project_values(s.cams, s.pts, s.obs_cam, s.obs_pt))
    inside = (u[:, 0] >= 0) & (u[:, 0] <= 640) & (u[:, 1] >= 0) & (u[:, 1] <= 480)
    assert inside.mean() > 0.99
    tl = np.bincount(s.obs_pt)
    assert tl.min() >= 2


def test_clustered_observations_lie_in_the_image():
    """Clustered scenes use the same visibility model; their far points have
    a near-zero baseline (ill-conditioned but accepted point blocks)."""
    from oracle import camera, schur
    s = sg.clustered(5, n_clusters=3, per_cluster=40, m=6000)
    u = np.asarray(camera.project_values(s.cams, s.pts, s.obs_cam, s.obs_pt))
    inside = (u[:, 0] >= 0) & (u[:, 0] <= 640) & (u[:, 1] >= 0) & (u[:, 1] <= 480)
    assert inside.mean() > 0.99
    far = np.linalg.norm(s.pts, axis=1) > 500
    assert 0.02 < far.mean() < 0.08
    oc, op = s.obs_cam.astype(np.int64), s.obs_pt.astype(np.int64)
    JP, JX = camera.jacobians(s.cams, s.pts, oc, op)
    _, V, _ = schur.normal_blocks(JP, JX, schur.information_blocks(None, oc.size), oc, op,
                                  s.n_cams, s.n_pts)
    cond = np.linalg.cond(V)
    assert cond[far].min() > 100 * np.median(cond[~far])
