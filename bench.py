"""Throughput of the exact camera covariance on one MI355X.

Default workload (``--workload clustered3000``): the large scene, 10 sites of
300 cameras (500 000 points, Zipf track lengths, ~3.4 million observations,
Z 27000 x 27000, seed 0).  One step is one call of the whole hot path
(Jacobians, point blocks and Schur scatter, nullspace and gauge, dense
inverse, block extraction) on a scene already resident in HBM, ending with
the n x 81 FP64 covariance blocks in HBM.

``--workload spiral500``: the 500-camera spiral scene (50 000 points, ~300 000
observations, Z 4500 x 4500, seed 0), one call per step.

``--workload batch256``: 256 independent sub-reconstructions (20-400 cameras,
100 points per camera), one batched call per step.

Prints one JSON line with the throughput in cameras/s, the roofline of the
dominant stage (the dense inverse, 2N^3/3 algorithmic flops per scene and
step, timed with HIP events on the library's stream), the CPU oracle timed on
the host cores on a bounded sample of the same workload, and the largest
per-block relative error of the timed call's output against the oracle
(exit status 1 above 1e-6).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6   # MI355X dense FP64 (MFMA and vector)
PEAK_HBM_GBS = 8000.0

METRIC = "cameras/s of exact covariance + MFMA util on Z^-1, at 1e-6 rel err vs FP64"


GOLDEN_C3 = os.path.join(ROOT, "tests", "golden", "clustered3000_blocks.json")
TOLERANCE = 1e-6  # per-block relative Frobenius error against the FP64 oracle


def traffic_profile(workload):
    return os.path.join(ROOT, "profiles", f"dense_inverse_fp64_{workload}_hbm_counters.md")
DEFAULT_TILE_THRESHOLD = 4096  # the library's untuned 32 x 32-tile threshold


BIG_TILES = 512  # FP64 products with this many 128 x 128 tiles run on them


def tile_schedule(n, small):
    """For each product of the dense recursion on an n x n matrix (n a
    multiple of 64), the tile size it runs on under the tile threshold
    `small` (the splits and tile counts of the library's host code): 128 when
    it has at least BIG_TILES tiles of 128 x 128 (a node's paired launch
    twice that), else 64 when it has at least `small` tiles of 64 x 64, else
    32.  Two thresholds with the same schedule
    launch the same kernels."""
    out = []

    def kind(t64, t128, products=1):
        return 128 if t128 >= products * BIG_TILES else (64 if t64 >= small else 32)

    def node(n):
        if n <= 128:
            return
        n1 = (n // 64 // 2) * 64
        n2 = n - n1
        node(n1)
        lower, square = (n2 // 64) * (n1 // 64), (n2 // 64) ** 2
        b1, b2 = -(-n1 // 128), -(-n2 // 128)
        out.extend([kind(lower, b2 * b1), kind(square + lower, b2 * b2 + b2 * b1, 2),
                    kind(lower, b2 * b1)])
        node(n2)

    node(n)
    return tuple(out)


DENSE_SOURCE = os.path.join(ROOT, "paper_1808_02414_amd", "csrc", "dense_kernels.hip")


def recorded_traffic(workload):
    """HBM bytes per step of the dense stage from the committed counter runs
    (FETCH_SIZE and WRITE_SIZE scaled by a plain copy) and the tile threshold
    they were taken with, or None when there are none for this workload or
    the dense kernels have changed since they were taken."""
    try:
        text = open(traffic_profile(workload)).read()
        src = hashlib.sha256(open(DENSE_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None
    t = re.search(r"traffic_bytes_per_step: (\d+)", text)
    h = re.search(r"dense_kernels_sha256: (\w+)", text)
    th = re.search(r"tile_threshold: (\d+)", text)
    if not (t and h) or h.group(1) != src:
        return None
    return int(t.group(1)), int(th.group(1)) if th else DEFAULT_TILE_THRESHOLD


def recorded_traffic_for(args, np_pad):
    """The recorded traffic when the counters were taken with the tile
    schedule this run uses (the single-scene FP64 path only), else None."""
    if args.workload == "batch256" or args.precision != "fp64":
        return None
    rec = recorded_traffic(args.workload)
    if rec is None:
        return None
    used = getattr(args, "tuned_threshold", None) or DEFAULT_TILE_THRESHOLD
    return rec[0] if tile_schedule(np_pad, used) == tile_schedule(np_pad, rec[1]) else None


def _threads():
    try:
        from threadpoolctl import threadpool_info
        return int(max([d.get("num_threads", 1) for d in threadpool_info()] or [1]))
    except Exception:
        return os.cpu_count() or 1


def cpu_baseline(scenes, budget_s=20.0):
    """Time the FP64 oracle (as it stands) on the host: whole scenes of the
    workload in order until about ``budget_s`` seconds have been spent.
    Returns the baseline and the oracle's blocks of the scenes it solved."""
    import numpy as np
    import oracle
    cams, dt, k = 0, 0.0, 0
    ref = []
    for s in scenes:
        t0 = time.perf_counter()
        out = oracle.camera_covariance(s)
        dt += time.perf_counter() - t0
        assert np.all(np.isfinite(out["blocks"]))
        ref.append(out["blocks"])
        cams += s.n_cams
        k += 1
        if dt >= budget_s:
            break
    what = (f"one full oracle solve of the benchmark scene ({cams} cameras)" if len(scenes) == 1
            else f"full oracle solves of the first {k} of {len(scenes)} scenes ({cams} cameras)")
    return {"value": cams / dt, "unit": "cameras/s", "cores": _threads(),
            "kind": "oracle", "seconds": dt, "sample": what}, ref


def cpu_baseline_large(scene, point_stride=10, block=9000):
    """The oracle on the large scene in bounded pieces, each scaled by its
    cost law (one whole solve takes minutes on the host):

    * the scene stage (Jacobians, normal-equation blocks, point-block
      inverses, the Schur complement Z and the nullspace basis) on the
      observations of every ``point_stride``-th point, times point_stride
      (its cost is linear in the observations);
    * the oracle's whole-inverse mode (Jacobi-scaled Cholesky factorisation of
      Z + aQQ^T and its solve against the identity) on the leading
      ``block`` x ``block`` block of that Z, times (N / block)^3.
    """
    import numpy as np
    from oracle import camera, covariance, nullspace, schur
    import scenegen
    sel = scene.obs_pt % point_stride == 0
    keep_pts = np.unique(scene.obs_pt[sel])
    remap = np.full(scene.n_pts, -1, np.int64)
    remap[keep_pts] = np.arange(keep_pts.size)
    sub = scenegen.Scene(scene.cams, scene.pts[keep_pts], scene.obs_cam[sel],
                         remap[scene.obs_pt[sel]].astype(np.int32))
    oc, op = sub.obs_cam.astype(np.int64), sub.obs_pt.astype(np.int64)
    n, m = sub.n_cams, sub.n_pts
    t0 = time.perf_counter()
    JP, JX = camera.jacobians(sub.cams, sub.pts, oc, op)
    Lam = schur.information_blocks(None, oc.size)
    U, V, W = schur.normal_blocks(JP, JX, Lam, oc, op, n, m)
    Vinv, _ = schur.point_block_inverses(V)
    Z = schur.reduced_camera_matrix(U, W, Vinv, oc, op, n, m)
    Hr = nullspace.rotation_blocks(sub.cams, sub.pts, oc, op, JP, JX)
    Q = covariance.orthonormal_basis(nullspace.camera_rows(sub.cams, Hr))
    t_scene = time.perf_counter() - t0
    N = Z.shape[0]
    b = min(block, N)
    Zb = np.ascontiguousarray(Z[:b, :b])
    Qb = np.ascontiguousarray(Q[:b])
    del Z, U, V, W, JP, JX
    t0 = time.perf_counter()
    S = covariance.pseudo_inverse(Zb, Qb, covariance.balanced_alpha(Zb, Qb))
    t_dense = time.perf_counter() - t0
    assert np.all(np.isfinite(S))
    est = point_stride * t_scene + (N / b) ** 3 * t_dense
    return {"value": scene.n_cams / est, "unit": "cameras/s", "cores": _threads(),
            "kind": "oracle", "seconds": t_scene + t_dense, "estimated_solve_s": est,
            "sample": (f"oracle stages on pieces, scaled by their cost law: the scene stage "
                       f"(Jacobians to Z and the nullspace basis) on the observations of every "
                       f"{point_stride}th point ({t_scene:.1f} s, x{point_stride}); the "
                       f"whole-inverse mode (scaled Cholesky factor and solve against the "
                       f"identity) on the leading {b}x{b} block of Z ({t_dense:.1f} s, "
                       f"x(N/{b})^3 = {(N / b) ** 3:.1f}); estimated solve {est:.0f} s for "
                       f"{scene.n_cams} cameras")}


def max_block_error(got, ref):
    """Largest per-block relative Frobenius error of got against ref."""
    import numpy as np
    return float(max(np.linalg.norm(g - r) / np.linalg.norm(r) for g, r in zip(got, ref)))


def golden_c3():
    import numpy as np
    with open(GOLDEN_C3) as f:
        gold = json.load(f)
    ref = np.array([[float(v) for v in b] for b in gold["blocks"]]).reshape(-1, 9, 9)
    return gold["cameras"], ref


def run_single(args, ucov, torch, np, scene):
    ctx = ucov.Context(0)
    dev = ucov.DeviceScene.from_scene(scene, "cuda:0")
    prec = {"fp64": ucov.FP64, "fp32ns": ucov.FP32_NS, "bf16x": ucov.BF16X_NS}[args.precision]
    if args.threshold is not None:
        ctx.set_dense_threshold(9 * scene.n_cams, args.threshold)
        args.tuned_threshold = args.threshold
    elif prec == ucov.FP64 and not args.no_tune:
        # the library's tile-schedule tuning for this size, before the timed steps
        args.tuned_threshold = ctx.tune_dense(9 * scene.n_cams)[0]
    out = torch.empty((scene.n_cams, 9, 9), dtype=torch.float64, device="cuda:0")
    for _ in range(args.warmup):
        ctx.camera_covariance(dev, precision=prec, out=out)
    torch.cuda.synchronize()
    reps = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, rep = ctx.camera_covariance(dev, precision=prec, out=out)
        reps.append(rep)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, reps, [9 * scene.n_cams], out


def run_batch(args, ucov, torch, np, scenes):
    ctx = ucov.Context(0)
    devs = [ucov.DeviceScene.from_scene(s, "cuda:0") for s in scenes]
    if not args.no_tune:
        # the library's batched tile-schedule tuning, before the timed steps
        args.tuned_threshold = ctx.tune_batched([9 * s.n_cams for s in scenes])[0]
    n = sum(s.n_cams for s in scenes)
    out = torch.empty((n, 9, 9), dtype=torch.float64, device="cuda:0")
    for _ in range(args.warmup):
        _, _, rep = ctx.camera_covariance_batched(devs, out=out)
    torch.cuda.synchronize()
    reps = []
    if args.graph:
        # the batch recorded once into a graph and replayed; the stage times
        # come from one eager call
        _, _, eager = ctx.camera_covariance_batched(devs, out=out)
        b = ctx.batch(devs, out=out)
        b.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            rep = b.run()
            reps.append(dict(eager, ms_total=rep["ms_total"]))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        b.close()
        return dt, reps, [9 * s.n_cams for s in scenes], out
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, _, rep = ctx.camera_covariance_batched(devs, out=out)
        reps.append(rep)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, reps, [9 * s.n_cams for s in scenes], out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["spiral500", "batch256", "clustered3000"],
                    default="clustered3000")
    ap.add_argument("--precision", choices=["fp64", "fp32ns", "bf16x"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph", action="store_true",
                    help="batch256: record the batch once into a graph and time its replays")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default dense tile schedule instead of tuning it for the size")
    ap.add_argument("--threshold", type=int, default=None,
                    help="use this tile-schedule threshold instead of tuning (e.g. for a profile)")
    ap.add_argument("--n-cams", type=int, default=500)
    ap.add_argument("--n-pts", type=int, default=50_000)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only copy a buffer of this many MiB 5 times (for scaling HBM counters)")
    args = ap.parse_args()
    if args.calibrate_copy_mib:
        import torch
        n = args.calibrate_copy_mib * (1 << 20) // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read": 8 * n, "bytes_written": 8 * n,
                          "launches": 5}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "sharding across GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import scenegen
    import paper_1808_02414_amd as ucov

    if args.workload == "spiral500":
        scene = scenegen.spiral_slab(0, n=args.n_cams, m=args.n_pts)
        scenes = [scene]
        dt, reps, Ns, out = run_single(args, ucov, torch, np, scene)
        workload = (f"spiral_slab: {scene.n_cams} cameras, {scene.n_pts} points, "
                    f"{scene.n_obs} observations, Z {Ns[0]}x{Ns[0]}, seed 0")
    elif args.workload == "clustered3000":
        print("bench: generating the 3000-camera scene", file=sys.stderr, flush=True)
        scene = scenegen.clustered(0)
        scenes = [scene]
        print("bench: timing", file=sys.stderr, flush=True)
        dt, reps, Ns, out = run_single(args, ucov, torch, np, scene)
        workload = (f"clustered: 10 sites of 300 cameras, {scene.n_pts} points, "
                    f"{scene.n_obs} observations, Z {Ns[0]}x{Ns[0]}, seed 0")
    else:
        if args.precision != "fp64":
            sys.exit("the batched workload runs in FP64")
        scenes = scenegen.batch_scenes()
        dt, reps, Ns, out = run_batch(args, ucov, torch, np, scenes)
        workload = (f"batch_scenes: {len(scenes)} independent spiral scenes, "
                    f"{sum(s.n_cams for s in scenes)} cameras (20-400 per scene), "
                    f"{sum(s.n_pts for s in scenes)} points, {sum(s.n_obs for s in scenes)} "
                    f"observations, seed 1000")
    cams = sum(s.n_cams for s in scenes)
    ms_step = 1e3 * dt / args.steps
    value = cams * args.steps / dt

    inv_ms = float(np.mean([r["ms_inverse"] for r in reps]))
    flops = sum(2.0 * N ** 3 / 3.0 for N in Ns)
    achieved = flops / (inv_ms * 1e-3) / 1e12
    stages = {k: float(np.mean([r[k] for r in reps]))
              for k in ("ms_structure", "ms_schur", "ms_gauge", "ms_inverse", "ms_extract")}
    np_pad = -(-Ns[0] // 64) * 64  # the padded dense size of the (first) scene

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "cameras/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32ns": "f32+f64", "bf16x": "bf16x3+f32+f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": workload, "precision": args.precision,
                   "launch": "graph replay" if args.graph else "eager"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                     # counters taken with the same tile schedule, else null
                     "traffic": recorded_traffic_for(args, np_pad),
                     "kernel": "dense inverse stage (k_leaf_mfma + k_gemm128/64/32s + their _pair launches), "
                               "2N^3/3 flops per scene; traffic in bytes per step"},
        "stages_ms": stages,
        "n_pairs": int(reps[-1]["n_pairs"]),
    }
    if getattr(args, "tuned_threshold", None) is not None:
        line["dense_tile_threshold"] = args.tuned_threshold
    if args.precision != "fp64":
        line["ns_iters"] = int(reps[-1]["ns_iters"])
        line["ns_residual"] = float(reps[-1]["ns_residual"])
    # the timed call's output against the oracle
    got = out.cpu().numpy()
    if args.workload == "clustered3000":
        cams_checked, ref = golden_c3()
        err = max_block_error(got[cams_checked], ref)
        checked = f"{len(cams_checked)} cameras against stored oracle blocks"
    if args.workload == "clustered3000" and not args.no_cpu_baseline:
        print("bench: timing the oracle", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline_large(scenes[0])
    elif args.workload != "clustered3000":
        print("bench: timing the oracle", file=sys.stderr, flush=True)
        base, refs = cpu_baseline(scenes, budget_s=0.0 if args.no_cpu_baseline else 20.0)
        if not args.no_cpu_baseline:
            line["cpu_baseline"] = base
        ncheck = sum(r.shape[0] for r in refs)
        err = max_block_error(got[:ncheck], np.concatenate(refs))
        checked = (f"all {ncheck} cameras" if len(scenes) == 1
                   else f"the {ncheck} cameras of the first {len(refs)} scenes")
    line["check"] = {"max_rel_fro": err, "tolerance": TOLERANCE, "against": "FP64 oracle",
                     "cameras": checked}
    print(json.dumps(line), flush=True)
    if not err <= TOLERANCE:
        print(f"bench: output error {err:.3e} above {TOLERANCE:g}", file=sys.stderr, flush=True)
        sys.exit(1)


if __name__ == "__main__":
    main()
