"""GPU parity of the batched path: every scene of a batch of independent
sub-reconstructions against the FP64 oracle, scene by scene.

The batched entry point gathers the scenes into one concatenation, runs the
scene stage once for all of them and the dense inverses side by side; each
scene's blocks must match the oracle to the same 1e-6 relative Frobenius bar as
a single-scene call, and agree with that call to rounding.
"""
import numpy as np
import pytest

import scenegen as sg
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


def small_batch():
    """Uneven scenes (20-70 cameras, the workload's recipe), plus two tiny
    ones, one of them with information blocks."""
    scenes = sg.batch_scenes(seed=3000, count=8, lo=20, hi=70)
    scenes.insert(3, sg.tiny_circle(22))
    scenes.append(sg.tiny_circle(21, with_info=True))
    return scenes


def test_batched_matches_oracle_per_scene(ucov):
    u, ctx = ucov
    scenes = small_batch()
    print("batched small: sizes", [s.n_cams for s in scenes], flush=True)
    devs = [u.DeviceScene.from_scene(s) for s in scenes]
    views, alphas, rep = ctx.camera_covariance_batched(devs)
    assert rep["bad_scene"] == -1 and len(alphas) == len(scenes)
    for s, v in zip(scenes, views):
        ref = oracle_cov(s)["blocks"]
        fro, scaled = block_errors(v.cpu().numpy(), ref)
        assert fro < 1e-6 and scaled < 1e-5, (s.name, s.n_cams, fro, scaled)
    # the same kernels as a single-scene call: equal up to the order of the
    # camera-pair sums
    for s, v, a in zip(scenes, views, alphas):
        one, rep1 = ctx.camera_covariance(u.DeviceScene.from_scene(s))
        fro, _ = block_errors(v.cpu().numpy(), one.cpu().numpy())
        assert fro < 1e-9, (s.name, fro)
        assert abs(a - rep1["alpha"]) <= 1e-12 * abs(a)


def test_batched_repeat_bitwise_equal(ucov):
    u, ctx = ucov
    devs = [u.DeviceScene.from_scene(s) for s in small_batch()]
    first, _, _ = ctx.camera_covariance_batched(devs)
    first = [v.cpu().numpy() for v in first]
    for _ in range(2):
        again, _, _ = ctx.camera_covariance_batched(devs)
        for a, b in zip(first, again):
            assert np.array_equal(a, b.cpu().numpy())


def test_batched_given_alpha(ucov):
    """A caller-given gauge weight is used for every scene and leaves Z^+ unchanged."""
    u, ctx = ucov
    scenes = small_batch()[:4]
    devs = [u.DeviceScene.from_scene(s) for s in scenes]
    auto, _, _ = ctx.camera_covariance_batched(devs)
    auto = [v.cpu().numpy() for v in auto]
    given, alphas, _ = ctx.camera_covariance_batched(devs, alpha=0.37)
    assert all(a == 0.37 for a in alphas)
    for g, a in zip(given, auto):
        assert block_errors(g.cpu().numpy(), a)[0] < 1e-7


def test_batched_single_scene_and_repeat(ucov):
    """A batch of one equals the single call; a smaller batch in between reuses
    the workspace."""
    u, ctx = ucov
    s = sg.spiral_slab(31, n=45, m=2500)
    d = u.DeviceScene.from_scene(s)
    (v,), _, _ = ctx.camera_covariance_batched([d])
    first = v.cpu().numpy()
    ctx.camera_covariance_batched([u.DeviceScene.from_scene(sg.tiny_circle(2))])
    (v,), _, _ = ctx.camera_covariance_batched([d])
    assert block_errors(v.cpu().numpy(), first)[0] < 1e-9
    ref = oracle_cov(s)["blocks"]
    assert block_errors(first, ref)[0] < 1e-6


@pytest.fixture(scope="module")
def full_workload(ucov):
    """The 256-scene workload (20-400 cameras, 100 points per camera) solved
    by one batched call, as the benchmark runs it."""
    u, ctx = ucov
    scenes = sg.batch_scenes()
    print("batched full: cameras", sum(s.n_cams for s in scenes), flush=True)
    devs = [u.DeviceScene.from_scene(s) for s in scenes]
    views, alphas, rep = ctx.camera_covariance_batched(devs)
    print(f"  report {rep}", flush=True)
    return scenes, [v.cpu().numpy() for v in views], alphas


def test_batched_full_workload_properties(full_workload):
    _, views, alphas = full_workload
    allb = np.concatenate(views)
    assert np.all(np.isfinite(allb))
    assert np.abs(allb - allb.transpose(0, 2, 1)).max() <= 1e-12 * np.abs(allb).max()
    assert np.all(np.diagonal(allb, axis1=1, axis2=2) > 0)
    assert all(a > 0 for a in alphas)


@pytest.mark.parametrize("part", range(4))
def test_batched_full_workload_every_scene(full_workload, part):
    """Every scene of the workload against the oracle (a quarter of the
    scenes per case, the oracle in parallel processes)."""
    from oracle_pool import oracle_blocks
    scenes, views, _ = full_workload
    idx = list(range(part, len(scenes), 4))
    refs = oracle_blocks([scenes[i] for i in idx])
    worst = (0.0, 0.0, -1)
    for i, ref in zip(idx, refs):
        fro, scaled = block_errors(views[i], ref)
        assert fro < 1e-6 and scaled < 1e-5, (i, scenes[i].n_cams, fro, scaled)
        worst = max(worst, (fro, scaled, i))
    print(f"  scenes {idx[0]}::4 worst fro {worst[0]:.2e} scaled {worst[1]:.2e} "
          f"(scene {worst[2]})", flush=True)


def test_batched_errors_name_the_scene(ucov):
    u, ctx = ucov
    good = [sg.tiny_circle(40 + k, n=6, m=80) for k in range(4)]

    def run(scenes):
        return ctx.camera_covariance_batched([u.DeviceScene.from_scene(s) for s in scenes])

    # a local camera index outside its own scene (but inside the concatenation)
    s = good[2]
    bad = sg.Scene(s.cams, s.pts, s.obs_cam.copy(), s.obs_pt.copy())
    bad.obs_cam[5] = s.n_cams
    with pytest.raises(u.UcovError) as e:
        run([good[0], good[1], bad, good[3]])
    assert e.value.kind == "EINVAL" and e.value.scene == 2 and e.value.index == 5

    # a point seen once: EPOINT with the local point index
    s = good[1]
    j = int(s.obs_pt[0])
    sel = (s.obs_pt != j) | (np.arange(s.n_obs) == 0)
    lone = sg.Scene(s.cams, s.pts, s.obs_cam[sel], s.obs_pt[sel])
    with pytest.raises(u.UcovError) as e:
        run([good[0], lone, good[2]])
    assert e.value.kind == "EPOINT" and e.value.scene == 1 and e.value.index == j

    # two disconnected halves in one scene: its gauge is not 7-dimensional
    a, b = sg.tiny_circle(50, n=5, m=60), sg.tiny_circle(51, n=5, m=60)
    two = sg.Scene(np.vstack([a.cams, b.cams]), np.vstack([a.pts, b.pts]),
                   np.concatenate([a.obs_cam, b.obs_cam + 5]).astype(np.int32),
                   np.concatenate([a.obs_pt, b.obs_pt + 60]).astype(np.int32))
    with pytest.raises(u.UcovError) as e:
        run([good[0], good[1], good[2], two])
    assert e.value.kind == "EGAUGE" and e.value.scene == 3

    # the context still works
    views, _, _ = run(good)
    for s, v in zip(good, views):
        assert block_errors(v.cpu().numpy(), oracle_cov(s)["blocks"])[0] < 1e-6


def test_tune_batched_then_solve(ucov):
    """The batched tile-schedule tuning picks one of its candidates; the
    batch solved with it agrees with the untuned schedule to rounding and
    with the oracle."""
    u, ctx = ucov
    scenes = small_batch()
    devs = [u.DeviceScene.from_scene(s) for s in scenes]
    before, _, _ = ctx.camera_covariance_batched(devs)
    before = [v.cpu().numpy() for v in before]
    th, ms = ctx.tune_batched([9 * s.n_cams for s in scenes])
    print(f"  batched threshold {th} ({ms:.3f} ms)", flush=True)
    assert th in (0, 256, 1024, 4096, 1 << 40) and ms > 0.0
    after, _, _ = ctx.camera_covariance_batched(devs)
    for s, a, b in zip(scenes, after, before):
        assert block_errors(a.cpu().numpy(), b)[0] < 1e-9
        assert block_errors(a.cpu().numpy(), oracle_cov(s)["blocks"])[0] < 1e-6


def test_batch_graph_replays_match_eager(ucov):
    """A recorded batch (eager solve, then a captured graph) replays several
    times, with other eager work and synchronisations in between: every
    replay gives the eager call's blocks bit for bit."""
    import torch
    u, ctx = ucov
    scenes = small_batch()
    devs = [u.DeviceScene.from_scene(s) for s in scenes]
    eager, _, _ = ctx.camera_covariance_batched(devs)
    eager = torch.cat(eager).cpu()
    b = ctx.batch(devs)
    assert torch.equal(b.out.cpu(), eager)  # the eager solve inside create
    other = u.DeviceScene.from_scene(sg.spiral_slab(33, n=50, m=3000))
    for k in range(4):
        b.out.zero_()
        rep = b.run()
        assert rep["ms_total"] > 0.0 and rep["bad_scene"] == -1
        assert torch.equal(b.out.cpu(), eager), k
        ctx.camera_covariance(other)  # eager work of the same context between replays
        torch.cuda.synchronize()
    b.close()


def test_batch_graph_follows_new_values(ucov):
    """Between replays the scenes' parameter values may change: a replay
    after moving the cameras of one scene equals a fresh eager solve."""
    import torch
    u, ctx = ucov
    scenes = small_batch()
    devs = [u.DeviceScene.from_scene(s) for s in scenes]
    b = ctx.batch(devs)
    d = devs[2]
    d.cams[:, 6] *= 1.02          # focal lengths
    d.cams[:, 3:6] += 0.01        # centres
    b.run()
    eager, _, _ = ctx.camera_covariance_batched(devs)
    assert torch.equal(b.out, torch.cat(eager))
    b.close()


def test_batch_graph_rejects_grown_structure(ucov):
    """A replay whose scene gained camera pairs (an observation moved to a
    point with more cameras) reports EINVAL without touching memory beyond its
    buffers; restoring the scene makes the next replay good again."""
    import torch
    u, ctx = ucov
    scenes = small_batch()
    devs = [u.DeviceScene.from_scene(s) for s in scenes]
    eager, _, _ = ctx.camera_covariance_batched(devs)
    eager = torch.cat(eager)
    b = ctx.batch(devs)
    # in scene 1, move one observation of a 3-camera point to another
    # 3-camera point that its camera does not see yet: pairs 6 + 6 -> 3 + 10
    s = scenes[1]
    cnt = np.bincount(s.obs_pt, minlength=s.n_pts)
    three = np.flatnonzero(cnt == 3)
    moved = None
    for pa in three:
        for pb in three:
            if pa == pb:
                continue
            cams_b = set(s.obs_cam[s.obs_pt == pb].tolist())
            for o in np.flatnonzero(s.obs_pt == pa):
                if int(s.obs_cam[o]) not in cams_b:
                    moved = (int(o), int(pb))
                    break
            if moved:
                break
        if moved:
            break
    assert moved is not None
    op = s.obs_pt.copy()
    op[moved[0]] = moved[1]
    devs[1].obs_pt.copy_(torch.as_tensor(op, dtype=torch.int32))
    with pytest.raises(u.UcovError) as e:
        b.run()
    assert e.value.kind == "EINVAL"
    devs[1].obs_pt.copy_(torch.as_tensor(s.obs_pt, dtype=torch.int32))
    b.run()
    assert torch.equal(b.out, eager)
    b.close()
