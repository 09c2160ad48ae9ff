"""GPU parity of the paper's gauge, (M^+)_cc, against its FP64 oracle.

The GPU evaluates (Z + G F^-1 G^T)^-1 with the same kernels as the default
gauge (the rank-7 term in place of a Q Q^T, no final subtraction); the
oracle's structured route is itself pinned to the definition on the dense M
and to Z^+ by projection (tests/test_oracle_paper_gauge.py).  Bar: 1e-6
relative Frobenius error per camera block, as for Z^+."""
import numpy as np
import pytest

import scenegen as sg
from oracle import paper_gauge as pg

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


@pytest.mark.parametrize("maker", [lambda: sg.tiny_circle(0), lambda: sg.tiny_circle(2, with_info=True),
                                   lambda: sg.spiral_slab(7, n=60, m=3000),
                                   lambda: sg.spiral_slab(9, n=150, m=15000)])
def test_paper_gauge_matches_oracle(ucov, maker):
    u, ctx = ucov
    s = maker()
    print(f"paper gauge {s.name} n={s.n_cams}", flush=True)
    got, rep = ctx.camera_covariance(u.DeviceScene.from_scene(s), gauge=u.GAUGE_PAPER)
    ref = pg.camera_blocks(s)
    fro, scaled = block_errors(got.cpu().numpy(), ref)
    print(f"  fro {fro:.2e} scaled {scaled:.2e}")
    assert fro < 1e-6 and scaled < 1e-5, (fro, scaled)
    assert rep["alpha"] == 1.0


def test_paper_gauge_full_medium_scene(ucov):
    u, ctx = ucov
    s = sg.spiral_slab(0)
    print("paper gauge spiral n=500", flush=True)
    got, _ = ctx.camera_covariance(u.DeviceScene.from_scene(s), gauge=u.GAUGE_PAPER)
    ref, _ = pg.camera_blocks(s, full=True)
    fro, scaled = block_errors(got.cpu().numpy(), ref)
    print(f"  fro {fro:.2e} scaled {scaled:.2e}")
    assert fro < 1e-6, (fro, scaled)


@pytest.mark.parametrize("prec", ["FP32_NS", "BF16X_NS"])
@pytest.mark.parametrize("maker", [lambda: sg.tiny_circle(4), lambda: sg.spiral_slab(8, n=60, m=3000)])
def test_paper_gauge_mixed_precision(ucov, maker, prec):
    u, ctx = ucov
    s = maker()
    got, rep = ctx.camera_covariance(u.DeviceScene.from_scene(s), gauge=u.GAUGE_PAPER,
                                     precision=getattr(u, prec))
    fro, scaled = block_errors(got.cpu().numpy(), pg.camera_blocks(s))
    assert rep["ns_residual"] <= 1e-10 and fro < 1e-6, (fro, rep)


def test_gauges_share_the_intrinsics_blocks(ucov):
    """Both gauges are exact; the intrinsics (f, k1, k2) blocks do not depend
    on the gauge, the pose blocks do."""
    u, ctx = ucov
    d = u.DeviceScene.from_scene(sg.spiral_slab(10, n=80, m=4000))
    a = ctx.camera_covariance(d)[0].cpu().numpy()
    b = ctx.camera_covariance(d, gauge=u.GAUGE_PAPER)[0].cpu().numpy()
    assert block_errors(b[:, 6:, 6:], a[:, 6:, 6:])[0] < 1e-8
    assert block_errors(b, a)[0] > 1e-4


def test_batched_rejects_the_paper_gauge(ucov):
    import ctypes
    u, ctx = ucov
    from paper_1808_02414_amd import _binding as b
    d = u.DeviceScene.from_scene(sg.tiny_circle(3))
    arr = (b.Scene * 1)(d.struct())
    out = ctx.torch.empty((10, 9, 9), dtype=ctx.torch.float64, device="cuda")
    opt = b.Options(b.FP64, 0, 0.0, 0.0, b.GAUGE_PAPER)
    rc = ctx.lib.ucov_camera_covariance_batched(ctx.h, 1, arr, ctypes.byref(opt), out.data_ptr(),
                                                None, None)
    assert rc == b.EINVAL
