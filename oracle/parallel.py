"""Row-parallel evaluation of the oracle -- test and measurement infrastructure only.

TabNet inference treats every row on its own (batch norm uses running statistics), so
the oracle can be run over consecutive row chunks in separate processes and the pieces
put side by side.  This module holds no TabNet arithmetic: it cuts X into chunks, hands
each chunk (and an optional per-chunk payload) to a module-level function in a worker
process, and returns the results in chunk order.

Workers are started with the "spawn" method (safe beside a process that holds a GPU
context) and run their BLAS on one thread each, so `workers` processes use `workers`
cores.  The model parameters are sent once per worker.
"""
from __future__ import annotations

import multiprocessing as mp
import os
from concurrent.futures import ProcessPoolExecutor
from contextlib import contextmanager

_THREAD_VARS = ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS", "MKL_NUM_THREADS")
_PARAMS = None


def default_workers() -> int:
    """Cores this process may run on, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _init(params) -> None:
    global _PARAMS
    _PARAMS = params


def _call(fn, lo, X, payload):
    return lo, fn(_PARAMS, X, payload)


@contextmanager
def _single_threaded_children():
    saved = {k: os.environ.get(k) for k in _THREAD_VARS}
    for k in _THREAD_VARS:
        os.environ[k] = "1"
    try:
        yield
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def map_rows(fn, params, X, chunk: int = 8192, workers: int | None = None, payload=None, inflight: int | None = None):
    """Yield (lo, fn(params, X[lo:hi], payload(lo, hi))) for consecutive chunks of rows, in
    order.  fn must be a module-level function; payload(lo, hi) (optional) builds the
    chunk's extra argument in this process just before the chunk is sent, and at most
    `inflight` chunks (default 2 per worker) are outstanding, so a large batch is never
    held whole by the workers."""
    workers = workers or default_workers()
    inflight = inflight or 2 * workers
    n = X.shape[0]
    bounds = [(lo, min(n, lo + chunk)) for lo in range(0, n, chunk)]
    with _single_threaded_children(), ProcessPoolExecutor(
            max_workers=workers, mp_context=mp.get_context("spawn"), initializer=_init, initargs=(params,)) as ex:
        pending = []
        k = 0
        while k < len(bounds) or pending:
            while k < len(bounds) and len(pending) < inflight:
                lo, hi = bounds[k]
                pending.append(ex.submit(_call, fn, lo, X[lo:hi], None if payload is None else payload(lo, hi)))
                k += 1
            yield pending.pop(0).result()
