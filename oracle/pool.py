"""Several reference runs at once in worker processes (test infrastructure:
used by the GPU tests that compare many small models with the reference).

Each worker runs single-threaded (OpenMP off) so that a pool of worker
processes uses the host's cores; the workers never touch a GPU.  The pool is
started with 'spawn', so it is safe from a process that has initialised one.
"""
from __future__ import annotations

import multiprocessing as mp
import os


def _init():
    os.environ["OMP_NUM_THREADS"] = "1"


def _moments_after(args):
    w, dt, steps = args
    from oracle import oracle
    o = oracle.Oracle(w)
    o.step(dt, steps)
    return o.moments()


def moments_after(workloads, dts, steps, processes=None):
    """[(zone_moments, totals)] of every workload after `steps` steps of its dt"""
    n = processes or min(16, len(workloads), os.cpu_count() or 1)
    ctx = mp.get_context("spawn")
    with ctx.Pool(n, initializer=_init) as p:
        return p.map(_moments_after, [(w, dt, steps) for w, dt in zip(workloads, dts)], chunksize=1)
