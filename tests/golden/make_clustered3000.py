"""Writes ``clustered3000_blocks.json``: the FP64 oracle's covariance blocks of
four cameras of the large clustered scene (``scenegen.clustered(0)``: 10
sites of 300 cameras, 500 000 points, Z 27000 x 27000), which the oracle
needs minutes for, so that the GPU test can compare against them.  The file
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

CAMERAS = [0, 1, 1499, 2999]
PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "clustered3000_blocks.json")


def structure_hash(scene):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(scene.obs_cam, np.int32).tobytes())
    h.update(np.ascontiguousarray(scene.obs_pt, np.int32).tobytes())
    return h.hexdigest()


def checksums(scene):
    return {"cams": float(np.abs(scene.cams).sum()), "pts": float(np.abs(scene.pts).sum())}


def main():
    t0 = time.time()
    s = scenegen.clustered(0)
    print(f"scene generated in {time.time() - t0:.0f} s", flush=True)
    t0 = time.time()
    out = camera_covariance(s, cameras=CAMERAS)
    print(f"oracle in {time.time() - t0:.0f} s", flush=True)
    with open(PATH, "w") as f:
        json.dump({"scene": "scenegen.clustered(0)", "n_cams": s.n_cams, "n_pts": s.n_pts,
                   "n_obs": s.n_obs, "structure_sha256": structure_hash(s),
                   "checksums": checksums(s), "cameras": CAMERAS, "alpha": out["alpha"],
                   "blocks": [[repr(float(v)) for v in b.ravel()] for b in out["blocks"]]},
                  f, indent=1)
    print(f"wrote {PATH}")


if __name__ == "__main__":
    main()
