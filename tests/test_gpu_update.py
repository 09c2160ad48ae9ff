"""GPU parity of the incremental update (``ucov_update_covariance``, Sec. 6
Woodbury identity) against the oracle's definition: the extended
reconstruction recomputed from scratch.

Tolerances as for the camera covariance: per 9 x 9 block relative Frobenius
error <= 1e-6 and scaled error |dX_rc| / sqrt(X_rr X_cc) <= 1e-5 over the
whole matrix; the new camera's block and its cross-covariance <= 1e-6 in
relative Frobenius norm.
"""
import numpy as np
import pytest

import scenegen as sg
from oracle import update

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ucov():
    import torch
    import paper_1808_02414_amd as u
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ctx = u.Context(0)
    yield u, ctx
    ctx.close()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def camera_errors(got, ref):
    n = ref.shape[0] // 9
    fro = max(rel(got[9 * i:9 * i + 9, 9 * i:9 * i + 9], ref[9 * i:9 * i + 9, 9 * i:9 * i + 9])
              for i in range(n))
    d = np.sqrt(np.diag(ref))
    return fro, float(np.max(np.abs(got - ref) / np.outer(d, d)))


def device_additions(add):
    import torch
    cam, pt, info, cam_new = add
    t = lambda a, dt: None if a is None else torch.as_tensor(np.ascontiguousarray(a), dtype=dt).cuda()  # noqa: E731
    return t(cam, torch.int32), t(pt, torch.int32), t(info, torch.float64), t(cam_new, torch.float64)


def run_update(u, ctx, s, add):
    d = u.DeviceScene.from_scene(s)
    cam_cov, _, _ = ctx.full_covariance(d, points=False)
    return ctx.update_covariance(d, cam_cov, *device_additions(add))


MAKERS = [lambda: sg.tiny_circle(3), lambda: sg.tiny_circle(4, with_info=True),
          lambda: sg.spiral_slab(5, n=60, m=3000)]


@pytest.mark.parametrize("maker", MAKERS)
@pytest.mark.parametrize("new_camera,k", [(False, 1), (False, 12), (False, 40), (True, 12)])
def test_update_matches_recompute(ucov, maker, new_camera, k):
    u, ctx = ucov
    s = maker()
    add = sg.additions(s, 11, k, new_camera=new_camera)
    print(f"update {s.name} n={s.n_cams} new_camera={new_camera} k={add[0].size}", flush=True)
    X, Cn, Kx, rep = run_update(u, ctx, s, add)
    Xr, Cr, Kr = update.recompute(s, *add)
    fro, scaled = camera_errors(X.cpu().numpy(), Xr)
    print(f"  fro {fro:.2e} scaled {scaled:.2e}")
    assert fro < 1e-6 and scaled < 1e-5, (fro, scaled)
    if new_camera:
        ec, ek = rel(Cn.cpu().numpy(), Cr), rel(Kx.cpu().numpy(), Kr)
        print(f"  new camera {ec:.2e} cross {ek:.2e}")
        assert ec < 1e-6 and ek < 1e-6, (ec, ek)


def test_two_updates_equal_one(ucov):
    import torch
    u, ctx = ucov
    s = sg.tiny_circle(12)
    cam, pt, info, _ = sg.additions(s, 13, 20)
    d = u.DeviceScene.from_scene(s)
    X0, _, _ = ctx.full_covariance(d, points=False)
    X_all = X0.clone()
    ctx.update_covariance(d, X_all, *device_additions((cam, pt, info, None))[:2])
    X_two = X0.clone()
    ctx.update_covariance(d, X_two, *device_additions((cam[:9], pt[:9], None, None))[:2])
    s1 = update.extended_scene(s, cam[:9], pt[:9])
    d1 = u.DeviceScene.from_scene(s1)
    ctx.update_covariance(d1, X_two, *device_additions((cam[9:], pt[9:], None, None))[:2])
    assert rel(X_two.cpu().numpy(), X_all.cpu().numpy()) < 1e-9
    assert float(torch.trace(X_all)) < float(torch.trace(X0))


def test_rejects_bad_additions(ucov):
    import torch
    from paper_1808_02414_amd import _binding as B
    u, ctx = ucov
    s = sg.tiny_circle(14)
    d = u.DeviceScene.from_scene(s)
    X, _, _ = ctx.full_covariance(d, points=False)
    X0 = X.clone()
    i32 = lambda a: torch.as_tensor(np.asarray(a, np.int32)).cuda()  # noqa: E731
    c0, p0 = int(s.obs_cam[0]), int(s.obs_pt[0])
    cases = [([c0], [p0]),                      # the camera already sees the point
             ([s.n_cams], [p0]),                # new camera index without a new camera
             ([0], [s.n_pts]),                  # point out of range
             ([1, 1], [p0, p0])]                # duplicate within the new observations
    for cam, pt in cases:
        with pytest.raises(u.UcovError) as e:
            ctx.update_covariance(d, X, i32(cam), i32(pt))
        assert e.value.code == B.EINVAL, (cam, pt)
    # a failed call leaves the covariance untouched
    assert torch.equal(X, X0)


def test_undetermined_new_camera(ucov):
    """A new camera with three observations (six rows for nine parameters)
    is not determined: UCOV_EGAUGE, and the input covariance is untouched."""
    import torch
    from paper_1808_02414_amd import _binding as B
    u, ctx = ucov
    s = sg.tiny_circle(15)
    d = u.DeviceScene.from_scene(s)
    X, _, _ = ctx.full_covariance(d, points=False)
    X0 = X.clone()
    cam, pt, info, cam_new = sg.additions(s, 16, 3, new_camera=True)
    assert cam.size == 3
    with pytest.raises(u.UcovError) as e:
        ctx.update_covariance(d, X, *device_additions((cam, pt, info, cam_new)))
    assert e.value.code == B.EGAUGE
    assert torch.equal(X, X0)


@pytest.mark.parametrize("new_camera,k", [(False, 200), (True, 150)])
def test_update_full_size(ucov, new_camera, k):
    """The 500-camera spiral: 200 new observations, or a new camera with up to
    150, against the recomputed extended reconstruction; the update's time
    beside a whole-covariance recomputation on the GPU."""
    import torch
    u, ctx = ucov
    s = sg.spiral_slab(0)
    add = sg.additions(s, 21, k, new_camera=new_camera)
    print(f"update spiral 500 new_camera={new_camera} k={add[0].size}", flush=True)
    d = u.DeviceScene.from_scene(s)
    X, _, _ = ctx.full_covariance(d, points=False)
    dev_add = device_additions(add)
    torch.cuda.synchronize()
    X, Cn, Kx, rep = ctx.update_covariance(d, X, *dev_add)
    ext = u.DeviceScene.from_scene(update.extended_scene(s, *add))
    _, _, rep_full = ctx.full_covariance(ext, points=False)
    print(f"  update: rows {rep['ms_schur']:.2f} ms, Woodbury {rep['ms_inverse']:.2f} ms; "
          f"recompute dense stage {rep_full['ms_inverse']:.2f} ms", flush=True)
    Xr, Cr, Kr = update.recompute(s, *add)
    fro, scaled = camera_errors(X.cpu().numpy(), Xr)
    print(f"  fro {fro:.2e} scaled {scaled:.2e}")
    assert fro < 1e-6 and scaled < 1e-5, (fro, scaled)
    if new_camera:
        assert rel(Cn.cpu().numpy(), Cr) < 1e-6 and rel(Kx.cpu().numpy(), Kr) < 1e-6
