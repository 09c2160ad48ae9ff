"""Seeded scenes generated in parallel processes (test helper): at most 16
workers (the host share of one GPU), results in the order asked for."""
from __future__ import annotations

import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor


def _make(job):
    import scenegen
    name, args, kwargs = job
    return getattr(scenegen, name)(*args, **kwargs)


def generate(jobs, workers: int | None = None):
    """Yield scenegen.<name>(*args, **kwargs) for every (name, args, kwargs)
    job, in order."""
    workers = workers or max(1, min(16, os.cpu_count() or 1, len(jobs)))
    with ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        yield from ex.map(_make, jobs, chunksize=1)
