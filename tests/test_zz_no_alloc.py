"""The allocation-free entry point (ucov_camera_covariance_noalloc) against
ucov_camera_covariance: two calls in a row, the second on a smaller scene,
each to the parity bar (per-block relative Frobenius 1e-6; both run the same
kernels, so they agree to rounding), no change in the device's free memory
across the calls, and a scene beyond the static scratch rejected cleanly."""
import numpy as np
import pytest

import scenegen as sg

pytestmark = pytest.mark.gpu


def block_errors(got, ref):
    fro = max(np.linalg.norm(g - r) / np.linalg.norm(r) for g, r in zip(got, ref))
    d = np.sqrt(np.abs(np.diagonal(ref, axis1=1, axis2=2)))
    return fro, float(np.max(np.abs(got - ref) / (d[:, :, None] * d[:, None, :])))


def test_noalloc_matches_workspace_path():
    import torch
    import paper_1808_02414_amd as u
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    scenes = [sg.spiral_slab(12, n=120, m=12000), sg.tiny_circle(1)]
    devs = [u.DeviceScene.from_scene(s) for s in scenes]
    ref_ctx = u.Context(0)
    refs = [ref_ctx.camera_covariance(d)[0].cpu().numpy() for d in devs]
    ref_paper = ref_ctx.camera_covariance(devs[1], gauge=u.GAUGE_PAPER)[0].cpu().numpy()
    ref_ctx.close()
    outs = [torch.empty((s.n_cams, 9, 9), dtype=torch.float64, device="cuda:0") for s in scenes]
    out_paper = torch.empty_like(outs[1])
    ctx = u.Context(0)  # a fresh context: no workspace of its own
    # no other context may be collected (and free its memory) meanwhile
    import gc
    gc.collect()
    gc.disable()
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for k, (s, d, out, ref) in enumerate(zip(scenes, devs, outs, refs)):
        print(f"noalloc call {k}: n={s.n_cams} t={s.n_obs}", flush=True)
        got, rep = ctx.camera_covariance_noalloc(d, outs[k])
        fro, scaled = block_errors(got.cpu().numpy(), ref)
        print(f"  fro {fro:.2e} scaled {scaled:.2e}", flush=True)
        assert fro < 1e-6 and scaled < 1e-5, (k, fro, scaled)
        assert fro < 1e-9, (k, fro)  # same kernels: rounding order only
    got, _ = ctx.camera_covariance_noalloc(devs[1], out_paper, gauge=u.GAUGE_PAPER)
    assert block_errors(got.cpu().numpy(), ref_paper)[0] < 1e-9
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    gc.enable()
    assert free1 == free0, (free0, free1)
    # beyond the static scratch: a clean ENOMEM, and the context still works
    big = sg.spiral_slab(0)
    out_big = torch.empty((big.n_cams, 9, 9), dtype=torch.float64, device="cuda:0")
    with pytest.raises(u.UcovError) as e:
        ctx.camera_covariance_noalloc(u.DeviceScene.from_scene(big), out_big)
    assert e.value.kind == "ENOMEM"
    got, _ = ctx.camera_covariance_noalloc(devs[1], outs[1])
    assert block_errors(got.cpu().numpy(), refs[1])[0] < 1e-9
    # the workspace path of the same context is unaffected
    got, _ = ctx.camera_covariance(devs[0])
    assert block_errors(got.cpu().numpy(), refs[0])[0] < 1e-9
    ctx.close()
