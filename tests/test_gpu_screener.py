"""GPU parity of the learned screener against its FP64 oracle, and what the
trained network gains over screening without it.

Tolerances: features are computed in FP64 and stored in FP32 (1e-5); the
network rounds every product operand to BF16 (8 significant bits, relative
rounding 2^-9) and accumulates in FP32, so its outputs are held to 3e-2 in
relative norm against the FP64 oracle.  Its gradients are compared with the
oracle's BF16 mode (1e-2 per tensor), which takes the ReLU decisions in the
same precision: a pre-activation near zero may switch sign between BF16 and
FP64 operands and then reroutes that unit's gradient entirely.  Adam and the
label transforms run in FP32/FP64 arithmetic (1e-5).
"""
import os
import time

import numpy as np
import pytest

import scenegen as sg
from oracle import screener as osc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ucov():
    import torch
    import paper_1808_02414_amd as u
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ctx = u.Context(0)
    yield u, ctx
    ctx.close()


def cuda(a, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


@pytest.mark.parametrize("maker", [lambda: sg.tiny_circle(3, with_info=True),
                                   lambda: sg.spiral_slab(4, n=20, m=600),
                                   lambda: sg.spiral_slab(8, n=70, m=5000)])
def test_features_match_oracle(ucov, maker):
    u, ctx = ucov
    s = maker()
    print(f"features {s.name} n={s.n_cams}", flush=True)
    got = ctx.screener_features(u.DeviceScene.from_scene(s)).cpu().numpy()
    ref = osc.camera_features(s)
    assert np.allclose(got, ref, rtol=1e-5, atol=1e-6), np.abs(got - ref).max(axis=0)


def mlp_case(seed, batch):
    import torch
    rng = np.random.default_rng(seed)
    p = sg.mlp_init(seed)
    p[np.arange(p.size) % 97 == 0] += 0.05  # some nonzero biases
    mean = rng.normal(0, 1, 55)
    std = rng.uniform(0.5, 2.0, 55)
    x = mean + std * rng.normal(size=(batch, 55))
    t = rng.normal(size=(batch, 45))
    p32 = p.astype(np.float32)
    xs = (x.astype(np.float32).astype(np.float64) - mean.astype(np.float32)) / std.astype(np.float32)
    return (p32, mean.astype(np.float32), std.astype(np.float32), x.astype(np.float32),
            t.astype(np.float32), xs)


@pytest.mark.parametrize("batch", [1, 37, 300, 1024])
def test_mlp_forward_matches_oracle(ucov, batch):
    import torch
    u, ctx = ucov
    p, mean, std, x, t, xs = mlp_case(11, batch)
    y = ctx.mlp_forward(cuda(p, torch.float32), cuda(x, torch.float32),
                        cuda(mean, torch.float32), cuda(std, torch.float32)).cpu().numpy()
    ref, _ = osc.mlp_forward(p.astype(np.float64), xs)
    assert rel(y, ref) < 3e-2, rel(y, ref)


@pytest.mark.parametrize("batch", [5, 300, 2048])
def test_mlp_gradient_matches_oracle(ucov, batch):
    """Against the oracle's BF16 mode, which takes every ReLU decision in the
    kernel's precision (operands rounded to bfloat16); the loss also against
    plain FP64."""
    import torch
    u, ctx = ucov
    p, mean, std, x, t, xs = mlp_case(12, batch)
    g, loss = ctx.mlp_gradient(cuda(p, torch.float32), cuda(x, torch.float32),
                               cuda(t, torch.float32), cuda(mean, torch.float32),
                               cuda(std, torch.float32))
    g = g.cpu().numpy()
    l64, _ = osc.mlp_backward(p.astype(np.float64), xs, t.astype(np.float64))
    assert loss == pytest.approx(l64, rel=3e-2)
    lref, gref = osc.mlp_backward(p.astype(np.float64), xs, t.astype(np.float64), bf16_ops=True)
    assert loss == pytest.approx(lref, rel=1e-3)
    for li, ((Wg, bg), (Wr, br)) in enumerate(zip(osc.split_params(g.astype(np.float64)),
                                                  osc.split_params(gref))):
        print(f"  layer {li}: dW {rel(Wg, Wr):.2e} db {rel(bg, br):.2e}")
        assert rel(Wg, Wr) < 1e-2 and rel(bg, br) < 1e-2, li


def test_train_step_is_gradient_plus_adam(ucov):
    """One training step equals the library's gradient followed by the
    oracle's Adam update (first step, zero moments), to FP32 rounding."""
    import torch
    u, ctx = ucov
    p, mean, std, x, t, xs = mlp_case(13, 256)
    args = (cuda(x, torch.float32), cuda(t, torch.float32), cuda(mean, torch.float32),
            cuda(std, torch.float32))
    g, _ = ctx.mlp_gradient(cuda(p, torch.float32), *args)
    g = g.cpu().numpy().astype(np.float64)
    pt = cuda(p, torch.float32)
    m = torch.zeros_like(pt)
    v = torch.zeros_like(pt)
    ctx.mlp_train(pt, m, v, 1, 1e-3, 256, args[0], args[1], args[2], args[3])
    ref, mref, vref = osc.adam_step(p.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1, 1e-3)
    assert np.abs(pt.cpu().numpy() - ref).max() <= 1e-6
    assert np.allclose(m.cpu().numpy(), mref, rtol=1e-5, atol=1e-12)
    assert np.allclose(v.cpu().numpy(), vref, rtol=1e-5, atol=1e-16)


def test_label_transforms_match_oracle(ucov):
    """Labels and their inverse with the per-camera scale D = s b (b from the
    cameras' Z_ii features) against the oracle's transforms."""
    import torch
    u, ctx = ucov
    from oracle.pipeline import camera_covariance as oracle_cov
    sc = sg.tiny_circle(7)
    S = oracle_cov(sc)["blocks"]
    F = osc.camera_features(sc).astype(np.float32)
    s = osc.label_scale(S, F)
    D = s * osc.block_scale(F)
    raw = osc.log_cholesky(S, D)
    # a spread small enough that some labels reach the clip
    small = (0.05 * raw.std(0) + 0.01).astype(np.float32)
    mean = raw.mean(0).astype(np.float32)
    lab = ctx.screener_labels(cuda(S, torch.float64), cuda(F, torch.float32), cuda(s, torch.float64),
                              cuda(mean, torch.float32), cuda(small, torch.float32)).cpu().numpy()
    ref = osc.standardise(raw, mean, small)
    assert np.abs(ref).max() == osc.LABEL_CLIP
    assert np.abs(lab - ref).max() <= 1e-5 * osc.LABEL_CLIP
    # a spread under which no label is clipped: the inverse map recovers S
    std = (raw.std(0) + 0.1).astype(np.float32)
    lab = ctx.screener_labels(cuda(S, torch.float64), cuda(F, torch.float32), cuda(s, torch.float64),
                              cuda(mean, torch.float32), cuda(std, torch.float32)).cpu().numpy()
    ref = osc.standardise(raw, mean, std)
    assert np.abs(ref).max() < osc.LABEL_CLIP
    assert np.abs(lab - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max())
    cov, spread = ctx.screener_covariance(cuda(lab, torch.float32), cuda(F, torch.float32),
                                          cuda(s, torch.float64), cuda(mean, torch.float32),
                                          cuda(std, torch.float32))
    back = osc.from_log_cholesky(mean + std * lab.astype(np.float64), D)
    assert rel(cov.cpu().numpy(), back) < 1e-10
    assert rel(cov.cpu().numpy(), S) < 1e-4
    Dm = D[:, :, None] * D[:, None, :]
    assert np.allclose(spread.cpu().numpy(), np.trace(S / Dm, axis1=1, axis2=2), rtol=1e-4)


def test_screener_stats_match_numpy(ucov):
    """The library's standardisation statistics against plain numpy on the
    oracle's covariances: feature means and deviations (n - 1), the label
    scale (square root of the lower median of every variance ratio to the
    block-diagonal estimate), and the labels' lower median and scaled median
    absolute deviation (the oracle's transform, in FP32 as the library
    stores the labels)."""
    import torch
    u, ctx = ucov
    from oracle.pipeline import camera_covariance as oracle_cov
    scenes = [sg.tiny_circle(70 + k) for k in range(7)]  # 70 cameras: an even count
    S = np.concatenate([oracle_cov(s)["blocks"] for s in scenes])
    F = np.concatenate([osc.camera_features(s) for s in scenes]).astype(np.float32)
    im, isd, sc, om, osd = ctx.screener_stats(cuda(F, torch.float32), cuda(S, torch.float64))
    F64 = F.astype(np.float64)
    assert np.allclose(im.cpu().numpy(), F64.mean(0), rtol=1e-6, atol=1e-6)
    assert np.allclose(isd.cpu().numpy(), np.maximum(F64.std(0, ddof=1), 1e-6), rtol=1e-5, atol=1e-6)
    sref = osc.label_scale(S, F)
    assert np.allclose(sc.cpu().numpy(), sref, rtol=1e-12)
    raw = osc.log_cholesky(S, sref * osc.block_scale(F)).astype(np.float32).astype(np.float64)
    mref, sdref = osc.label_moments(raw)
    assert np.allclose(om.cpu().numpy(), mref, rtol=1e-5, atol=1e-6)
    assert np.allclose(osd.cpu().numpy(), sdref, rtol=1e-4, atol=1e-6)
    again = ctx.screener_stats(cuda(F, torch.float32), cuda(S, torch.float64))
    for a, b in zip(again, (im, isd, sc, om, osd)):
        assert torch.equal(a, b)


def test_screener_file_round_trip(ucov, tmp_path):
    """ucov_screener_save / ucov_screener_load: every array comes back bit for
    bit, with and without the Adam moments; a corrupted file is rejected."""
    import torch
    u, ctx = ucov
    P = ctx.mlp_param_count()
    g = torch.Generator(device="cpu").manual_seed(5)
    t = {"params": torch.randn(P, generator=g), "in_mean": torch.randn(55, generator=g),
         "in_std": torch.rand(55, generator=g), "scale": torch.rand(9, generator=g).double(),
         "out_mean": torch.randn(45, generator=g), "out_std": torch.rand(45, generator=g),
         "adam_m": torch.randn(P, generator=g), "adam_v": torch.rand(P, generator=g)}
    t = {k: v.cuda().contiguous() for k, v in t.items()}
    path = str(tmp_path / "s.bin")
    ctx.screener_save(path, t, step=1234)
    back, step = ctx.screener_load(path, adam=True)
    assert step == 1234
    for k in t:
        assert torch.equal(back[k], t[k]), k
    plain = {k: v for k, v in t.items() if not k.startswith("adam")}
    ctx.screener_save(path, plain, step=7)
    back, step = ctx.screener_load(path)
    assert step == 7 and set(back) == set(plain)
    with pytest.raises(u.UcovError):
        ctx.screener_load(path, adam=True)  # no moments in this file
    raw = bytearray(open(path, "rb").read())
    raw[100] ^= 1
    open(path, "wb").write(bytes(raw))
    with pytest.raises(u.UcovError):
        ctx.screener_load(path)


def block_rel_errors(got, ref):
    return np.linalg.norm(got - ref, axis=(1, 2)) / np.linalg.norm(ref, axis=(1, 2))


def zii_from_features(F):
    """Rebuild Z_ii from its 45 features (log10 diagonal, correlations)."""
    n = F.shape[0]
    Z = np.zeros((n, 9, 9))
    k = 0
    for a in range(9):
        for b in range(a, 9):
            Z[:, a, b] = F[:, k]
            k += 1
    d = 10.0 ** np.stack([Z[:, a, a] for a in range(9)], 1)
    for a in range(9):
        for b in range(a + 1, 9):
            Z[:, a, b] = Z[:, b, a] = Z[:, a, b] * np.sqrt(d[:, a] * d[:, b])
        Z[:, a, a] = d[:, a]
    return Z


def screener_workload(ctx, jobs, count):
    """Features and exact covariances (device tensors) of the first ``count``
    cameras of the scenes of the given generator jobs (generated in parallel
    processes); a scene the exact path rejects (a degenerate gauge or point)
    is skipped, which the jobs' spare scenes make up for."""
    import torch
    from scene_pool import generate
    import paper_1808_02414_amd as u
    from paper_1808_02414_amd import screener as scr
    F, S, have, skipped = [], [], 0, 0
    for s in generate(jobs):
        if have >= count:
            continue
        try:
            f, c = scr.training_set(ctx, [s])
        except u.UcovError as e:
            assert e.kind in ("EGAUGE", "EPOINT"), e
            skipped += 1
            continue
        F.append(f)
        S.append(c)
        have += f.shape[0]
    assert have >= count, (have, count)
    print(f"  {have} cameras, {skipped} generated scenes rejected by the exact path", flush=True)
    return torch.cat(F)[:count].contiguous(), torch.cat(S)[:count].contiguous()


def c5_set(ctx, seed0, n_tiny, n_spiral, n_clustered, clustered_kw):
    """Cameras of the three scene recipes, exactly n_tiny, n_spiral and
    n_clustered of each (spare scenes of every recipe make up for the rare
    scene the exact path rejects)."""
    import torch
    per = clustered_kw.get("cams", 3000)
    kw = {k: v for k, v in clustered_kw.items() if k != "cams"}
    parts = [screener_workload(ctx, [("clustered", (seed0 + 1000 + k,), kw)
                                     for k in range(-(-n_clustered // per) + 1)], n_clustered),
             screener_workload(ctx, [("spiral_slab", (seed0 + 500 + k,), {})
                                     for k in range(n_spiral // 500 * 11 // 10 + 4)], n_spiral),
             screener_workload(ctx, [("tiny_circle", (seed0 + k,), {}) for k in range(n_tiny // 10 + 100)],
                               n_tiny)]
    return torch.cat([p[0] for p in parts]), torch.cat([p[1] for p in parts])


def test_trained_screener_gains_over_screening_without_it(ucov, tmp_path):
    """The learned screener at its stated size: trained on 200 000 cameras of
    the tiny (60 000 cameras in scenes of 10), spiral (125 000 in scenes of
    500) and clustered (15 000 in scenes of 3 000) recipes, with exact
    covariances from the library as labels, by the library's own kernels;
    evaluated on 10 000 held-out cameras (3 000 tiny, 6 000 spiral and 1 000 of
    a clustered scene of 4 sites of 250 cameras).  Against what screening has
    without it -- the training median of the normalised covariance (scaled
    per camera like the network's output) and the block-diagonal estimate
    (Z_ii)^-1, which needs no inverse of Z but ignores the other cameras'
    uncertainty -- the network must be about three times more accurate
    (median relative Frobenius error per camera block), rank cameras by
    uncertainty like the exact path (Spearman > 0.9), and answer faster than
    the exact path."""
    import torch
    from paper_1808_02414_amd import screener as scr
    u, ctx = ucov
    t0 = time.time()
    F, S = c5_set(ctx, 10000, 60_000, 125_000, 15_000, {})
    print(f"  training cameras {F.shape[0]} ({time.time() - t0:.1f} s)", flush=True)
    assert F.shape[0] == 200_000
    t0 = time.time()
    held_clustered = {"n_clusters": 4, "per_cluster": 250, "m": 170_000, "cams": 1000}
    Fh, Sh = c5_set(ctx, 90000, 3_000, 6_000, 1_000, held_clustered)
    print(f"  held-out cameras {Fh.shape[0]} ({time.time() - t0:.1f} s)", flush=True)
    assert Fh.shape[0] == 10_000
    t0 = time.time()
    model, hist = scr.fit(ctx, F, S, sg.mlp_init(1), epochs=40, batch=512, seed=1)
    torch.cuda.synchronize()
    print(f"  trained in {time.time() - t0:.1f} s: loss first {hist[0]:.4f} last {hist[-1]:.4f}",
          flush=True)
    # the network's last epoch against the constant prediction 0 (the
    # training median of every parameter): at most half its loss
    labels = ctx.screener_labels(S, F, model.scale, model.out_mean, model.out_std)
    base = float((labels.double() ** 2).mean())
    print(f"  loss of the constant prediction {base:.4f}", flush=True)
    loss_ok = hist[-1] < 0.5 * base

    pred, spread = model.predict(ctx, Fh)
    pred_all = pred.clone()
    ref = Sh.cpu().numpy()
    err_net = block_rel_errors(pred.cpu().numpy(), ref)
    # network output 0 is the training median of every parameter
    zero = torch.zeros((Fh.shape[0], 45), dtype=torch.float32, device="cuda")
    mcov, _ = ctx.screener_covariance(zero, Fh, model.scale, model.out_mean, model.out_std)
    err_mean = block_rel_errors(mcov.cpu().numpy(), ref)
    err_zii = block_rel_errors(np.linalg.inv(zii_from_features(Fh.cpu().numpy().astype(np.float64))), ref)
    med = {k: float(np.median(e)) for k, e in (("net", err_net), ("mean", err_mean), ("zii", err_zii))}
    print(f"  held-out median relative error {med}", flush=True)

    D = model.scale.cpu().numpy() * osc.block_scale(Fh.cpu().numpy())
    true_spread = np.trace(ref / (D[:, :, None] * D[:, None, :]), axis1=1, axis2=2)
    from scipy.stats import spearmanr
    rho = spearmanr(spread.cpu().numpy(), true_spread).correlation
    print(f"  spread rank correlation {rho:.3f}", flush=True)
    for name, sel in (("tiny", slice(7000, 10000)), ("spiral", slice(1000, 7000)),
                      ("clustered", slice(0, 1000))):
        print(f"  {name}: median errors net {np.median(err_net[sel]):.3f} "
              f"mean {np.median(err_mean[sel]):.3f} zii {np.median(err_zii[sel]):.3f}", flush=True)
    assert loss_ok, hist
    assert med["net"] < 0.35 * min(med["mean"], med["zii"]), med
    assert rho > 0.9

    # time: screening (features + network) against the exact path, per camera,
    # on held-out spiral scenes
    from scene_pool import generate
    dev_held = [u.DeviceScene.from_scene(s)
                for s in generate([("spiral_slab", (90500 + k,), {}) for k in range(4)])]
    torch.cuda.synchronize()
    t = time.perf_counter()
    for d in dev_held:
        model.predict(ctx, ctx.screener_features(d))
    torch.cuda.synchronize()
    t_screen = time.perf_counter() - t
    t = time.perf_counter()
    for d in dev_held:
        ctx.camera_covariance(d)
    torch.cuda.synchronize()
    t_exact = time.perf_counter() - t
    ncam = sum(d.n_cams for d in dev_held)
    print(f"  screening {ncam / t_screen:.0f} cams/s, exact {ncam / t_exact:.0f} cams/s", flush=True)
    assert t_screen < t_exact

    # screening with fallback: cameras whose predicted spread exceeds the
    # threshold get the exact covariance, the others the network's
    d = dev_held[-1]
    _, sp = model.predict(ctx, ctx.screener_features(d))
    thr = float(torch.quantile(sp, 0.8))
    cov, spread, fallback = model.screen(ctx, d, thr)
    exact = ctx.camera_covariance(d)[0]
    pred, _ = model.predict(ctx, ctx.screener_features(d))
    fb = fallback.cpu().numpy()
    print(f"  screen: {fb.sum()} of {fb.size} cameras fall back", flush=True)
    assert 0 < fb.sum() < fb.size
    # the exact path is bitwise reproducible
    assert torch.equal(cov[fallback], exact[fallback])
    assert bool((spread[~fallback] <= thr).all()) and bool((spread[fallback] > thr).all())
    kept = ~fallback
    assert not bool(torch.isclose(cov[kept], exact[kept], rtol=1e-9, atol=0.0).all())
    err_screen = block_rel_errors(cov.cpu().numpy(), exact.cpu().numpy())
    err_pred = block_rel_errors(pred.cpu().numpy(), exact.cpu().numpy())
    assert np.mean(err_screen) < np.mean(err_pred)

    # the trained screener round-trips through its file, Adam state included
    path = str(tmp_path / "screener.bin")
    model.save(ctx, path)
    loaded = scr.Screener.load(ctx, path, adam=True)
    assert loaded.step == model.step > 0
    again, _ = loaded.predict(ctx, Fh)
    assert torch.equal(again, pred_all)


def test_screener_falls_back_on_non_finite_spread(ucov):
    """A camera whose predicted spread is not a number falls back to the exact
    block (a network whose output is NaN for every input)."""
    import torch
    from paper_1808_02414_amd import screener as scr
    u, ctx = ucov
    s = sg.tiny_circle(8)
    d = u.DeviceScene.from_scene(s)
    P = ctx.mlp_param_count()
    f32 = torch.float32
    params = torch.full((P,), float("nan"), dtype=f32, device="cuda")
    model = scr.Screener(params, torch.zeros(55, dtype=f32, device="cuda"),
                         torch.ones(55, dtype=f32, device="cuda"),
                         torch.ones(9, dtype=torch.float64, device="cuda"),
                         torch.zeros(45, dtype=f32, device="cuda"),
                         torch.ones(45, dtype=f32, device="cuda"))
    cov, spread, fallback = model.screen(ctx, d, threshold=1e30)
    assert bool(torch.isnan(spread).all()) and bool(fallback.all())
    exact, _ = ctx.camera_covariance(d)
    assert torch.equal(cov, exact)
