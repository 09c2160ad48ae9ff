"""The FP64 oracle over many scenes in parallel processes (test helper).

Each worker runs the oracle single-threaded on whole scenes; the pool has at
most 16 workers (the host share of one GPU).  Only the tests call this.
"""
from __future__ import annotations

import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor


def _init():
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)


def _blocks(scene):
    from oracle.pipeline import camera_covariance
    return camera_covariance(scene)["blocks"]


def oracle_blocks(scenes, workers: int | None = None):
    """The oracle's (n_s, 9, 9) blocks of every scene, in order."""
    workers = workers or max(1, min(16, os.cpu_count() or 1, len(scenes)))
    with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn"), initializer=_init) as ex:
        return list(ex.map(_blocks, scenes, chunksize=1))
