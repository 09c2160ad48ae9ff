"""Pins of the sub-reconstruction oracle (CPU)."""
import numpy as np

import scenegen as sg
from oracle import subrecon
from oracle.pipeline import camera_covariance


def test_one_group_is_the_whole_reconstruction():
    s = sg.tiny_circle(30)
    blocks, chosen = subrecon.camera_covariance_min_trace(s, np.zeros((1, s.n_cams), np.int32))
    ref = camera_covariance(s)["blocks"]
    assert np.abs(blocks - ref).max() <= 1e-9 * np.abs(ref).max()
    assert np.all(chosen == 0)


def test_sub_reconstructions_bound_the_intrinsics_from_above():
    """Sec. 6: fewer cameras and points carry less information, so every
    sub-reconstruction's covariance of the gauge-free intrinsics (f, k1, k2)
    is at least the whole reconstruction's in the Loewner order."""
    s = sg.spiral_slab(31, n=40, m=2500)
    full = camera_covariance(s)["blocks"][:, 6:, 6:]
    g = sg.view_graph_partition(s, 12, seed=1)
    cand = subrecon.candidates(s, g)[0][:, 6:, 6:]
    for c in range(s.n_cams):
        diff = cand[c] - full[c]
        ev = np.linalg.eigvalsh(0.5 * (diff + diff.T))
        assert ev.min() >= -1e-9 * np.abs(full[c]).max(), (c, ev.min())


def test_min_trace_choice_and_partition_properties():
    s = sg.spiral_slab(32, n=50, m=3000)
    groups = np.stack([sg.view_graph_partition(s, 15, seed=d) for d in range(3)])
    for g in groups:
        sizes = np.bincount(g)
        assert sizes.min() >= 2 and g.max() + 1 == sizes.size
    blocks, chosen = subrecon.camera_covariance_min_trace(s, groups)
    cand = subrecon.candidates(s, groups)
    tr = np.trace(cand, axis1=2, axis2=3)
    assert np.all(np.trace(blocks, axis1=1, axis2=2) <= tr.min(axis=0) * (1 + 1e-12))
    assert np.array_equal(blocks, cand[chosen, np.arange(s.n_cams)])


def test_partition_groups_determine_their_cameras():
    """Every camera of a group sees at least 10 points with another camera of
    its group, and every group has at least two cameras."""
    from oracle.subrecon import subscene
    s = sg.spiral_slab(0)
    for k, seed in ((100, 0), (25, 10)):
        g = sg.view_graph_partition(s, k, seed=seed)
        assert np.bincount(g).min() >= 2
        for gid in range(g.max() + 1):
            sub = subscene(s, np.flatnonzero(g == gid))
            assert np.bincount(sub.obs_cam, minlength=sub.n_cams).min() >= 10, (k, gid)
