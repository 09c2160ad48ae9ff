"""Writes ``clustered3000_blocks.json``: the FP64 oracle's covariance blocks of
64 cameras of the large clustered scene (``scenegen.clustered(0)``: 10 sites
of 300 cameras, 500 000 points, Z 27000 x 27000), which the oracle needs
minutes for, so that the GPU test can compare against them.  The cameras
span all ten sites: per site four spread along its ring and the two that
observe the most far (near-zero baseline) points, plus cameras 0, 1, 1499
and 2999.  The file
also holds a hash of the scene's observation structure and checksums of its
parameters, so that the test can tell the scene was generated the same way.

Calls only the oracle and the input generator:

    python tests/golden/make_clustered3000.py
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import scenegen  # noqa: E402
from oracle.pipeline import camera_covariance  # noqa: E402

FIXED = [0, 1, 1499, 2999]
PER_SITE = 300
PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "clustered3000_blocks.json")


def structure_hash(scene):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(scene.obs_cam, np.int32).tobytes())
    h.update(np.ascontiguousarray(scene.obs_pt, np.int32).tobytes())
    return h.hexdigest()


def checksums(scene):
    return {"cams": float(np.abs(scene.cams).sum()), "pts": float(np.abs(scene.pts).sum())}


def choose_cameras(scene):
    """The 64 cameras described above (the far points are those more than
    100 units from every site, the sites lying on a circle of radius 40)."""
    n_sites = scene.n_cams // PER_SITE
    far = np.linalg.norm(scene.pts[:, :2], axis=1) > 140.0
    far_obs = np.bincount(scene.obs_cam[far[scene.obs_pt]], minlength=scene.n_cams)
    out = list(FIXED)
    for c in range(n_sites):
        lo = c * PER_SITE
        for k in np.argsort(-far_obs[lo:lo + PER_SITE], kind="stable")[:2]:
            if lo + int(k) not in out:
                out.append(lo + int(k))
        for off in (37, 112, 187, 262):
            if lo + off not in out:
                out.append(lo + off)
    return sorted(out)


def main():
    t0 = time.time()
    s = scenegen.clustered(0)
    print(f"scene generated in {time.time() - t0:.0f} s", flush=True)
    cameras = choose_cameras(s)
    print(f"{len(cameras)} cameras", flush=True)
    t0 = time.time()
    out = camera_covariance(s, cameras=cameras)
    print(f"oracle in {time.time() - t0:.0f} s", flush=True)
    with open(PATH, "w") as f:
        json.dump({"scene": "scenegen.clustered(0)", "n_cams": s.n_cams, "n_pts": s.n_pts,
                   "n_obs": s.n_obs, "structure_sha256": structure_hash(s),
                   "checksums": checksums(s), "cameras": cameras, "alpha": out["alpha"],
                   "blocks": [[repr(float(v)) for v in b.ravel()] for b in out["blocks"]]},
                  f, indent=1)
    print(f"wrote {PATH}")


if __name__ == "__main__":
    main()
