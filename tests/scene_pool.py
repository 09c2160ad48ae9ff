"""Seeded scenes generated in parallel processes (test helper): at most 16
workers (the host share of one GPU), results in the order asked for."""
from __future__ import annotations

import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor


def _make(job):
    """scenegen.<name>(seed, *rest, **kwargs); a seed whose scene the
    generator rejects as disconnected is replaced by seed + 7919 k (the
    first k that works), so the job list always yields a scene."""
    import scenegen
    name, args, kwargs = job
    seed, rest = args[0], args[1:]
    for k in range(8):
        try:
            return getattr(scenegen, name)(seed + 7919 * k, *rest, **kwargs)
        except RuntimeError as e:
            if "not connected" not in str(e):
                raise
    raise RuntimeError(f"no connected {name} scene near seed {seed}")


def generate(jobs, workers: int | None = None):
    """Yield the scene of every (name, args, kwargs) job (args[0] the seed),
    in order."""
    workers = workers or max(1, min(16, os.cpu_count() or 1, len(jobs)))
    with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        yield from ex.map(_make, jobs, chunksize=1)
