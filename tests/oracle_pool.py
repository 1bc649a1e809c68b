"""Oracle kernel tables for many planes at once, for the full-size GPU tests: one plane per task
over a pool of fresh interpreters (the test process holds a GPU context, so no fork).  The tables
are the oracle's own (`oracle.kernels.make_tables`, one plane per call)."""
import multiprocessing
import os
import sys

from oracle import kernels

_STATE = {}


def _init_worker(g, phi):
    _STATE["g"], _STATE["phi"] = g, phi


def _one_table(q):
    return kernels.make_tables(_STATE["g"], _STATE["phi"], planes=[q])[q]


def _task_table(task):
    g, phi, q = task
    return kernels.make_tables(g, phi, planes=[q])[q]


def _workers(n):
    return max(1, min(16, n, len(os.sched_getaffinity(0))))


def tables_in_parallel(g, phi, planes, label=""):
    """List over all planes of g: the oracle table of each plane in `planes`, None elsewhere."""
    planes = list(planes)
    workers = _workers(len(planes))
    ctx = multiprocessing.get_context("spawn")
    with ctx.Pool(workers, initializer=_init_worker, initargs=(g, phi)) as pool:
        got = pool.map(_one_table, planes)
    out = [None] * g.nplanes
    for q, t in zip(planes, got):
        out[q] = t
    print(f"[oracle tables] {label} {len(planes)} planes on {workers} processes", file=sys.stderr, flush=True)
    return out


def tables_for_tasks(tasks, label=""):
    """The oracle tables of (geometry, screens, plane) tasks, in order, over one pool."""
    tasks = list(tasks)
    workers = _workers(len(tasks))
    ctx = multiprocessing.get_context("spawn")
    with ctx.Pool(workers) as pool:
        got = pool.map(_task_table, tasks, chunksize=1)
    print(f"[oracle tables] {label} {len(tasks)} tables on {workers} processes", file=sys.stderr, flush=True)
    return got
