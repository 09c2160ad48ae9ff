"""GPU parity: the HIP path (through the C-ABI) against the FP64 CPU oracle.

Tolerance: per-camera-block relative Frobenius error <= 1e-6 for the
covariance (the contract); intermediate stages, which involve no inverse of
an ill-conditioned matrix, are compared far tighter.  A scaled metric
|dS_lm| / sqrt(S_ll S_mm) is checked as well, since the Frobenius norm of a
block is dominated by its focal-length variance.
"""
import numpy as np
import pytest

import scenegen as sg
from oracle import camera, covariance
from oracle.pipeline import camera_covariance as oracle_cov

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ucov():
    import torch
    import paper_1808_02414_amd as u
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ctx = u.Context(0)
    yield u, ctx
    ctx.close()


def block_errors(got, ref):
    fro = max(np.linalg.norm(g - r) / np.linalg.norm(r) for g, r in zip(got, ref))
    d = np.sqrt(np.abs(np.diagonal(ref, axis1=1, axis2=2)))
    scaled = np.max(np.abs(got - ref) / (d[:, :, None] * d[:, None, :]))
    return fro, scaled


def dev(u, scene):
    return u.DeviceScene.from_scene(scene, "cuda:0")


@pytest.mark.parametrize("seed,with_info", [(0, False), (1, True), (2, False)])
def test_jacobians(ucov, seed, with_info):
    u, ctx = ucov
    s = sg.tiny_circle(seed, with_info=with_info)
    print(f"jacobians seed={seed} info={with_info}", flush=True)
    jp, jx = ctx.jacobians(dev(u, s))
    JP, JX = camera.jacobians(s.cams, s.pts, s.obs_cam, s.obs_pt)
    jp, jx = jp.cpu().numpy(), jx.cpu().numpy()
    scale = np.abs(JP).max(axis=(0, 1))
    assert np.all(np.abs(jp - JP).max(axis=(0, 1)) <= 1e-12 * scale)
    assert np.abs(jx - JX).max() <= 1e-12 * np.abs(JX).max()


@pytest.mark.parametrize("maker", [lambda: sg.tiny_circle(3), lambda: sg.tiny_circle(4, with_info=True),
                                   lambda: sg.spiral_slab(5, n=60, m=3000)])
def test_reduced_camera_matrix(ucov, maker):
    u, ctx = ucov
    s = maker()
    print(f"Z {s.name} n={s.n_cams}", flush=True)
    z, rep = ctx.reduced_camera_matrix(dev(u, s))
    z = z.cpu().numpy()
    ref = oracle_cov(s, keep=True)
    Z = ref["Z"]
    assert np.linalg.norm(z - Z) / np.linalg.norm(Z) < 1e-12
    assert np.array_equal(z, z.T)
    # per entry, scaled by the diagonal (the parameter types differ by orders
    # of magnitude, so a whole-matrix norm would hide a wrong rotation or
    # distortion entry; reordering the oracle's sums moves this by ~4e-15)
    d = np.sqrt(np.diag(Z))
    assert np.max(np.abs(z - Z) / np.outer(d, d)) < 1e-12
    # per 9 x 9 camera-pair block: empty blocks exactly zero, the others to
    # a relative Frobenius 1e-11 (reordering: ~2e-15)
    n = s.n_cams
    zb = z.reshape(n, 9, n, 9).transpose(0, 2, 1, 3)
    Zb = Z.reshape(n, 9, n, 9).transpose(0, 2, 1, 3)
    nrm = np.linalg.norm(Zb, axis=(2, 3))
    assert np.all(zb[nrm == 0] == 0)
    rel = np.linalg.norm(zb - Zb, axis=(2, 3))[nrm > 0] / nrm[nrm > 0]
    assert rel.max() < 1e-11, rel.max()
    Hc = ref["Hc"]
    assert np.abs(z @ Hc).max() <= 1e-13 * np.abs(z).max() * np.abs(Hc).max()


@pytest.mark.parametrize("maker", [lambda: sg.tiny_circle(6), lambda: sg.spiral_slab(7, n=80, m=4000)])
def test_gauge_basis(ucov, maker):
    u, ctx = ucov
    s = maker()
    print(f"gauge {s.name} n={s.n_cams}", flush=True)
    hc, q = ctx.gauge_basis(dev(u, s))
    hc, q = hc.cpu().numpy(), q.cpu().numpy()
    ref = oracle_cov(s, keep=True)
    assert np.abs(hc - ref["Hc"]).max() <= 1e-10 * np.abs(ref["Hc"]).max()
    assert np.abs(q.T @ q - np.eye(7)).max() < 1e-13
    P, Pr = q @ q.T, ref["Q"] @ ref["Q"].T
    assert np.abs(P - Pr).max() < 1e-12


@pytest.mark.parametrize("N,kappa", [(90, 1e3), (576, 1e6), (1161, 1e8), (2007, 1e5)])
def test_pinv_known_spectrum(ucov, N, kappa):
    """Dense stage alone on Z = B diag(lam) B^T with a prescribed null space."""
    import torch
    u, ctx = ucov
    print(f"pinv N={N} kappa={kappa:g}", flush=True)
    rng = np.random.default_rng(N)
    B, _ = np.linalg.qr(rng.normal(size=(N, N)))
    lam = np.geomspace(1.0, 1.0 / kappa, N - 7)
    R, Q0 = B[:, :N - 7], B[:, N - 7:]
    Z = (R * lam) @ R.T
    Z = 0.5 * (Z + Z.T)
    ref = covariance.camera_blocks((R / lam) @ R.T)
    got, rep = ctx.pinv_blocks(torch.from_numpy(Z).cuda(), torch.from_numpy(Q0.copy()).cuda())
    fro, scaled = block_errors(got.cpu().numpy(), ref)
    assert fro < 1e-15 * kappa * 100, (fro, scaled)


@pytest.mark.parametrize("seed,with_info", [(0, False), (1, False), (2, True), (3, False)])
def test_covariance_tiny(ucov, seed, with_info):
    u, ctx = ucov
    s = sg.tiny_circle(seed, with_info=with_info)
    print(f"covariance tiny seed={seed}", flush=True)
    got, rep = ctx.camera_covariance(dev(u, s))
    ref = oracle_cov(s)["blocks"]
    fro, scaled = block_errors(got.cpu().numpy(), ref)
    assert fro < 1e-6 and scaled < 1e-5, (fro, scaled)


@pytest.mark.parametrize("n,m", [(37, 2000), (150, 15000)])
def test_covariance_ragged(ucov, n, m):
    """Several tiles with a ragged tail (9n not a multiple of the tile)."""
    u, ctx = ucov
    s = sg.spiral_slab(11, n=n, m=m)
    print(f"covariance spiral n={n}", flush=True)
    got, rep = ctx.camera_covariance(dev(u, s))
    ref = oracle_cov(s)["blocks"]
    fro, scaled = block_errors(got.cpu().numpy(), ref)
    assert fro < 1e-6 and scaled < 1e-5, (fro, scaled)


def smallest_scenes():
    """Two and three cameras of a circle seeing every point (the smallest
    connected scenes).  Two cameras whose optical axes meet are degenerate
    for two unknown focal lengths, so the two-camera scene tilts both."""
    from scipy.spatial.transform import Rotation
    base = sg.tiny_circle(31, n=10, m=150)
    out = []
    for n in (2, 3):
        cams = base.cams[:n].copy()
        if n == 2:
            cams[1, :3] = (Rotation.from_rotvec([0.0, 0.0, 0.12]) * Rotation.from_rotvec(cams[1, :3])).as_rotvec()
            cams[0, :3] = (Rotation.from_rotvec([0.08, 0.0, 0.0]) * Rotation.from_rotvec(cams[0, :3])).as_rotvec()
        oc = np.tile(np.arange(n), base.n_pts).astype(np.int32)
        op = np.repeat(np.arange(base.n_pts), n).astype(np.int32)
        out.append(sg.Scene(cams, base.pts, oc, op))
    return out


@pytest.mark.parametrize("which", [0, 1])
def test_covariance_smallest_scenes(ucov, which):
    u, ctx = ucov
    s = smallest_scenes()[which]
    print(f"covariance smallest scene n={s.n_cams}", flush=True)
    got, _ = ctx.camera_covariance(dev(u, s))
    fro, scaled = block_errors(got.cpu().numpy(), oracle_cov(s)["blocks"])
    assert fro < 1e-6 and scaled < 1e-5, (fro, scaled)


def test_covariance_exact_tile_multiple(ucov):
    """64 cameras: 9n = 576 is a multiple of the 64 tile, so no padding."""
    u, ctx = ucov
    s = sg.tiny_circle(21, n=64, m=3000, track=(3, 6))
    print("covariance n=64 (no padding)", flush=True)
    got, _ = ctx.camera_covariance(dev(u, s))
    fro, scaled = block_errors(got.cpu().numpy(), oracle_cov(s)["blocks"])
    assert fro < 1e-6 and scaled < 1e-5, (fro, scaled)


def test_rejects_too_small_inputs(ucov):
    u, ctx = ucov
    s = sg.tiny_circle(22)
    one = sg.Scene(s.cams[:1], s.pts, np.zeros(s.n_pts, np.int32), np.arange(s.n_pts, dtype=np.int32))
    with pytest.raises(u.UcovError) as e:
        ctx.camera_covariance(dev(u, one))
    assert e.value.kind == "EINVAL"
    empty = sg.Scene(s.cams, s.pts, np.zeros(0, np.int32), np.zeros(0, np.int32))
    with pytest.raises(u.UcovError) as e:
        ctx.camera_covariance(dev(u, empty))
    assert e.value.kind == "EINVAL"


def test_tune_dense_then_covariance(ucov):
    """The tile-schedule tuning picks one of its candidates and the
    covariance computed with it still matches the oracle."""
    u, ctx = ucov
    s = sg.spiral_slab(13, n=150, m=15000)
    th, ms = ctx.tune_dense(9 * s.n_cams)
    print(f"tuned threshold {th} ({ms:.3f} ms)", flush=True)
    assert th in (0, 256, 1024, 4096, 1 << 40) and ms > 0.0
    got, _ = ctx.camera_covariance(dev(u, s))
    fro, scaled = block_errors(got.cpu().numpy(), oracle_cov(s)["blocks"])
    assert fro < 1e-6 and scaled < 1e-5, (fro, scaled)
    with pytest.raises(u.UcovError):
        ctx.tune_dense(0)


def test_covariance_full_medium_scene(ucov):
    """The 500-camera spiral scene (Z 4500 x 4500), every block."""
    u, ctx = ucov
    s = sg.spiral_slab(0)
    print("covariance spiral n=500", flush=True)
    got, rep = ctx.camera_covariance(dev(u, s))
    ref = oracle_cov(s)["blocks"]
    fro, scaled = block_errors(got.cpu().numpy(), ref)
    print(f"  fro {fro:.3e} scaled {scaled:.3e} report {rep}")
    assert fro < 1e-6, (fro, scaled)


def test_host_pointers(ucov):
    """UCOV_HOST_PTRS: a scene in host memory and host output give the device
    path's blocks bit for bit; the flag is refused where only device pointers
    are taken."""
    import ctypes
    import torch
    u, ctx = ucov
    s = sg.spiral_slab(15, n=70, m=4000, with_info=True)
    host, rep = ctx.camera_covariance_host(s)
    dev_out, _ = ctx.camera_covariance(dev(u, s))
    assert np.array_equal(host, dev_out.cpu().numpy())
    assert block_errors(host, oracle_cov(s)["blocks"])[0] < 1e-6
    from paper_1808_02414_amd import _binding as b
    d = dev(u, sg.tiny_circle(3))
    arr = (b.Scene * 1)(d.struct())
    out = torch.empty((10, 9, 9), dtype=torch.float64, device="cuda")
    opt = b.Options(b.FP64, 0, 0.0, 0.0, b.GAUGE_CAMERA, b.HOST_PTRS)
    rep = b.Report()
    rc = ctx.lib.ucov_camera_covariance_batched(ctx.h, 1, arr, ctypes.byref(opt), out.data_ptr(),
                                                None, ctypes.byref(rep))
    assert rc == b.EINVAL


@pytest.mark.parametrize("gauge", ["camera", "paper"])
def test_repeat_calls_bitwise_equal(ucov, gauge):
    """Repeated calls give the same bits: the camera-pair bins are filled in a
    fixed order and every floating-point sum runs in a fixed order."""
    u, ctx = ucov
    g = u.GAUGE_CAMERA if gauge == "camera" else u.GAUGE_PAPER
    s = sg.spiral_slab(12, n=140, m=9000)
    d = dev(u, s)
    a, _ = ctx.camera_covariance(d, gauge=g)
    a = a.cpu().numpy()
    small = dev(u, sg.tiny_circle(1))
    ctx.camera_covariance(small, gauge=g)  # a smaller call in between reuses the workspace
    for _ in range(3):
        b, _ = ctx.camera_covariance(d, gauge=g)
        assert np.array_equal(b.cpu().numpy(), a)
    z1, _ = ctx.reduced_camera_matrix(d)
    z2, _ = ctx.reduced_camera_matrix(d)
    assert np.array_equal(z1.cpu().numpy(), z2.cpu().numpy())


def test_errors(ucov):
    u, ctx = ucov
    s = sg.tiny_circle(17)
    bad = sg.Scene(s.cams, s.pts, s.obs_cam.copy(), s.obs_pt.copy())
    bad.obs_cam[3] = s.n_cams
    with pytest.raises(u.UcovError) as e:
        ctx.camera_covariance(dev(u, bad))
    assert e.value.kind == "EINVAL"

    dup = sg.Scene(s.cams, s.pts, np.append(s.obs_cam, s.obs_cam[0]).astype(np.int32),
                   np.append(s.obs_pt, s.obs_pt[0]).astype(np.int32))
    with pytest.raises(u.UcovError) as e:
        ctx.camera_covariance(dev(u, dup))
    assert e.value.kind == "EINVAL"

    j = int(s.obs_pt[0])
    sel = (s.obs_pt != j) | (np.arange(s.n_obs) == 0)
    lone = sg.Scene(s.cams, s.pts, s.obs_cam[sel], s.obs_pt[sel])
    with pytest.raises(u.UcovError) as e:
        ctx.camera_covariance(dev(u, lone))
    assert e.value.kind == "EPOINT" and e.value.index == j

    a = sg.tiny_circle(18, n=5, m=60)
    b = sg.tiny_circle(19, n=5, m=60)
    two = sg.Scene(np.vstack([a.cams, b.cams]), np.vstack([a.pts, b.pts]),
                   np.concatenate([a.obs_cam, b.obs_cam + 5]).astype(np.int32),
                   np.concatenate([a.obs_pt, b.obs_pt + 60]).astype(np.int32))
    with pytest.raises(u.UcovError) as e:
        ctx.camera_covariance(dev(u, two))
    assert e.value.kind == "EGAUGE"

    # a point behind one of its cameras: EINVAL naming one such observation
    from failure_scenes import absurd_size, behind_camera, coincident_centres
    behind, bad_obs = behind_camera()
    with pytest.raises(u.UcovError) as e:
        ctx.camera_covariance(dev(u, behind))
    assert e.value.kind == "EINVAL" and e.value.index in bad_obs

    # a point seen only from two coincident centres: EPOINT naming the point
    deg, jd = coincident_centres()
    with pytest.raises(u.UcovError) as e:
        ctx.camera_covariance(dev(u, deg))
    assert e.value.kind == "EPOINT" and e.value.index == jd

    # a scene whose camera matrix cannot fit the device: ENOMEM before any launch
    huge = absurd_size()
    with pytest.raises(u.UcovError) as e:
        ctx.camera_covariance(dev(u, huge))
    assert e.value.kind == "ENOMEM"

    # the context still works after errors
    got, _ = ctx.camera_covariance(dev(u, s))
    ref = oracle_cov(s)["blocks"]
    assert block_errors(got.cpu().numpy(), ref)[0] < 1e-6


@pytest.mark.parametrize("prec", ["FP32_NS", "BF16X_NS"])
@pytest.mark.parametrize("maker", [lambda: sg.tiny_circle(5), lambda: sg.spiral_slab(13, n=150, m=15000),
                                   lambda: sg.spiral_slab(0)])
def test_covariance_mixed_precision(ucov, maker, prec):
    """FP32 MFMA initial inverse + Newton-Schulz with FP64 residuals, the
    corrections on FP32 MFMA or from split-BF16 products."""
    u, ctx = ucov
    s = maker()
    print(f"mixed {prec} {s.name} n={s.n_cams}", flush=True)
    got, rep = ctx.camera_covariance(dev(u, s), precision=getattr(u, prec))
    ref = oracle_cov(s)["blocks"]
    got = got.cpu().numpy()
    fro, scaled = block_errors(got, ref)
    print(f"  ns_iters {rep['ns_iters']} residual {rep['ns_residual']:.2e} fro {fro:.2e} scaled {scaled:.2e}")
    assert rep["ns_iters"] >= 1 and rep["ns_residual"] <= 1e-10
    assert fro < 1e-6 and scaled < 1e-5, (fro, scaled)
    # and against the FP64 GPU path
    f64, _ = ctx.camera_covariance(dev(u, s))
    fro64, _ = block_errors(got, f64.cpu().numpy())
    assert fro64 < 1e-6, fro64


@pytest.mark.parametrize("prec", ["FP32_NS", "BF16X_NS"])
@pytest.mark.parametrize("N,kappa", [(576, 1e3), (1161, 1e5)])
def test_pinv_known_spectrum_mixed(ucov, N, kappa, prec):
    import torch
    u, ctx = ucov
    rng = np.random.default_rng(N + 1)
    B, _ = np.linalg.qr(rng.normal(size=(N, N)))
    lam = np.geomspace(1.0, 1.0 / kappa, N - 7)
    R, Q0 = B[:, :N - 7], B[:, N - 7:]
    Z = (R * lam) @ R.T
    Z = 0.5 * (Z + Z.T)
    ref = covariance.camera_blocks((R / lam) @ R.T)
    got, rep = ctx.pinv_blocks(torch.from_numpy(Z).cuda(), torch.from_numpy(Q0.copy()).cuda(),
                               precision=getattr(u, prec))
    fro, scaled = block_errors(got.cpu().numpy(), ref)
    assert fro < 1e-15 * kappa * 1000, (fro, rep)


def bound_exponents(a, axis):
    """Per row (axis 1) or column (axis 0): the e with max |a| < 2^e."""
    mx = np.abs(a).max(axis=axis)
    e = np.zeros(mx.shape, np.int64)
    nz = mx > 0
    e[nz] = np.frexp(mx[nz])[1]  # mx = f 2^e with f in [0.5, 1)
    return e, nz


@pytest.mark.parametrize("n,seed", [(64, 1), (576, 2), (1152, 3), (8256, 4)])
def test_split_bf16_product(ucov, n, seed):
    """The split-BF16 correction x += x r alone against the FP64 product, on
    matrices whose rows (of x) and columns (of r) span six orders of
    magnitude: every entry within the slices' bound 2^(e_m + f_c - 8 S) n
    (2^e_m, 2^f_c bounding row m of x and column c of r; S = 3 slices up to
    n = 8192, 4 beyond), and far inside what one BF16 rounding of the
    operands gives.  Beyond n = 2048 the reference is formed for 64 sampled
    rows."""
    import torch
    u, ctx = ucov
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, n)) * 10.0 ** rng.uniform(-3, 3, n)[:, None]
    R = rng.normal(size=(n, n)) * 1e-4 * 10.0 ** rng.uniform(-3, 3, n)[None, :]
    X[5] = 0.0   # an all-zero row and column
    R[:, 7] = 0.0
    rows = np.arange(n) if n <= 2048 else np.unique(np.r_[5, rng.choice(n, 63, replace=False)])
    ref = X[rows] + X[rows] @ R
    t = torch.from_numpy(X.T.copy()).cuda()  # row-major storage of the column-major X
    ctx.split_bf16_update(t, torch.from_numpy(R.T.copy()).cuda())
    got = t.cpu().numpy().T[rows]
    S = 3 if n <= 8192 else 4
    ex, _ = bound_exponents(X, 1)
    er, _ = bound_exponents(R, 0)
    bound = n * np.ldexp(1.0, ex[rows][:, None] + er[None, :] - 8 * S)
    err = np.abs(got - ref)
    print(f"  n={n}: max err / bound {np.max(err / bound):.3f}", flush=True)
    assert np.all(err <= bound)
    k5 = int(np.flatnonzero(rows == 5)[0])
    assert np.all(got[k5] == 0.0) and np.array_equal(got[:, 7], X[rows, 7])
    # one BF16 rounding of the operands (8 significant bits) is far worse
    bf = lambda a: torch.from_numpy(a).float().bfloat16().double().numpy()  # noqa: E731
    err_bf16 = np.abs(X[rows] + bf(X[rows]) @ bf(R) - ref)
    assert np.median(err) < 1e-4 * np.median(err_bf16)


def test_mixed_precision_reports_no_convergence(ucov):
    """max_iter = 1 with a tolerance the first step cannot reach: ENOCONV."""
    u, ctx = ucov
    s = sg.spiral_slab(14, n=60, m=4000)
    with pytest.raises(u.UcovError) as e:
        ctx.camera_covariance(dev(u, s), precision=u.FP32_NS, max_iter=1, tol=1e-30)
    assert e.value.kind == "ENOCONV"
