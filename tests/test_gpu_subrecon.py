"""GPU parity of sub-reconstruction covariances (Sec. 6) against the oracle,
and their error against the whole reconstruction as the groups grow."""
import numpy as np
import pytest

import scenegen as sg
from oracle import subrecon

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ucov():
    import torch
    import paper_1808_02414_amd as u
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ctx = u.Context(0)
    yield u, ctx
    ctx.close()


def rel_blocks(got, ref):
    return np.linalg.norm(got - ref, axis=(1, 2)) / np.linalg.norm(ref, axis=(1, 2))


@pytest.mark.parametrize("n,m,k,decomp", [(60, 3000, 15, 3), (500, 50000, 100, 2)])
def test_subrecon_matches_oracle(ucov, n, m, k, decomp):
    u, ctx = ucov
    s = sg.spiral_slab(33, n=n, m=m)
    groups = np.stack([sg.view_graph_partition(s, k, seed=d) for d in range(decomp)])
    print(f"subrecon n={n} k={k} decompositions={decomp}", flush=True)
    got, chosen, n_sub, rep = ctx.subrecon_covariance(u.DeviceScene.from_scene(s), groups)
    ref, ref_chosen = subrecon.camera_covariance_min_trace(s, groups)
    err = rel_blocks(got.cpu().numpy(), ref)
    print(f"  {n_sub} sub-reconstructions, max block error {err.max():.2e}", flush=True)
    assert n_sub == sum(int(g.max()) + 1 for g in groups)
    assert err.max() < 1e-6
    # the choice agrees wherever the two candidates' traces are not within rounding
    cand = subrecon.candidates(s, groups)
    tr = np.trace(cand, axis1=2, axis2=3)
    clear = np.abs(np.diff(np.sort(tr, axis=0)[:2], axis=0)[0]) > 1e-9 * tr.min(axis=0)
    assert np.array_equal(chosen[clear], ref_chosen[clear])


def test_subrecon_large_clustered(ucov):
    """1000 cameras in 4 sites (1.16 million observations), three
    decompositions into groups of about 250: the sub-scenes (3.5 million
    candidate observations) are chosen on the device; every block against
    the oracle's sub-reconstructions."""
    import time
    import torch
    u, ctx = ucov
    s = sg.clustered(5, n_clusters=4, per_cluster=250, m=170_000)
    groups = np.stack([sg.view_graph_partition(s, 250, seed=d) for d in range(3)])
    d = u.DeviceScene.from_scene(s)
    print(f"subrecon clustered n={s.n_cams} t={s.n_obs}", flush=True)
    ctx.subrecon_covariance(d, groups)  # workspace
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    got, chosen, n_sub, rep = ctx.subrecon_covariance(d, groups)
    torch.cuda.synchronize()
    print(f"  {n_sub} sub-reconstructions in {1e3 * (time.perf_counter() - t0):.1f} ms", flush=True)
    ref, _ = subrecon.camera_covariance_min_trace(s, groups)
    err = rel_blocks(got.cpu().numpy(), ref)
    print(f"  max block error {err.max():.2e}", flush=True)
    assert err.max() < 1e-6
    again = ctx.subrecon_covariance(d, groups)[0]
    assert torch.equal(again, got)


def test_subrecon_error_falls_with_group_size(ucov):
    """The paper's Fig. 6 on the 500-camera scene: the relative error of the
    minimum-trace covariance against the whole reconstruction, for groups of
    about 25 to 250 cameras (three decompositions each).  The intrinsics
    (f, k1, k2) blocks are gauge-free and bounded from above; the full blocks
    also carry the difference between the sub-reconstructions' gauges."""
    u, ctx = ucov
    s = sg.spiral_slab(0)
    d = u.DeviceScene.from_scene(s)
    full = ctx.camera_covariance(d)[0].cpu().numpy()
    med = {}
    for k in (25, 50, 100, 250):
        groups = np.stack([sg.view_graph_partition(s, k, seed=10 + r) for r in range(3)])
        got = ctx.subrecon_covariance(d, groups)[0].cpu().numpy()
        e_in = rel_blocks(got[:, 6:, 6:], full[:, 6:, 6:])
        e_all = rel_blocks(got, full)
        med[k] = float(np.median(e_in))
        print(f"  k={k}: intrinsics median {np.median(e_in):.3e} p90 {np.percentile(e_in, 90):.3e}; "
              f"whole block median {np.median(e_all):.3e}", flush=True)
        # upper bound: no intrinsics variance below the whole reconstruction's
        dv = np.diagonal(got[:, 6:, 6:], axis1=1, axis2=2) - np.diagonal(full[:, 6:, 6:], axis1=1, axis2=2)
        assert dv.min() >= -1e-9 * np.abs(full[:, 6:, 6:]).max()
    assert med[250] < med[25]
