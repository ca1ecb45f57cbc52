"""Worker processes for the oracle's point-parallel evaluation.

TEST INFRASTRUCTURE ONLY (see the package docstring).

A process that has initialised the GPU runtime must never fork: the child
would inherit the parent's device files and runtime state. So the pool is
made once, by ``start()``, before the caller touches the GPU (the test
session's configure hook, the top of the benchmark's ``main``), and reused by
every parallel oracle call after that. Large arrays reach the workers through
POSIX shared memory (``share``), never through the fork itself.

If no pool was started, ``get()`` makes one from a fresh 'forkserver' process
(started by fork and exec, so it holds no GPU state) rather than forking the
caller.
"""
from __future__ import annotations

import atexit
import multiprocessing as mp
import os
from multiprocessing import shared_memory

import numpy as np

# The caller plus its workers stay within 16 processes.
MAX_WORKERS = 15

_pool = None
_size = 0


def default_workers() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(MAX_WORKERS, n))


def start(workers: int | None = None, method: str = "fork") -> int:
    """Make the worker pool (idempotent). With method 'fork' this must run
    before the calling process initialises the GPU runtime. Returns the number
    of workers."""
    global _pool, _size
    if _pool is not None:
        return _size
    n = default_workers() if workers is None else max(1, min(MAX_WORKERS, int(workers)))
    # the shared-memory tracker is a child process too: start it now as well
    from multiprocessing import resource_tracker
    resource_tracker.ensure_running()
    ctx = mp.get_context(method)
    _pool = ctx.Pool(n)
    _size = n
    atexit.register(stop)
    return n


def stop() -> None:
    global _pool, _size
    if _pool is not None:
        _pool.terminate()
        _pool.join()
    _pool = None
    _size = 0


def get():
    """The pool and its size (made on first use from a 'forkserver' process
    when ``start()`` was not called)."""
    if _pool is None:
        ctx = mp.get_context("forkserver")
        ctx.set_forkserver_preload(["numpy", "oracle.tdbp"])
        start(method="forkserver")
    return _pool, _size


class Shared:
    """NumPy arrays in named shared memory, released on ``close()``."""

    def __init__(self, **arrays):
        self._blocks = []
        self.specs = {}
        for name, a in arrays.items():
            if a is None:
                self.specs[name] = None
                continue
            a = np.ascontiguousarray(a)
            blk = shared_memory.SharedMemory(create=True, size=max(1, a.nbytes))
            np.ndarray(a.shape, dtype=a.dtype, buffer=blk.buf)[...] = a
            self._blocks.append(blk)
            self.specs[name] = (blk.name, a.shape, a.dtype.str)

    def close(self) -> None:
        for blk in self._blocks:
            blk.close()
            blk.unlink()
        self._blocks = []

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


_attached = {}


def attach(specs: dict) -> dict:
    """Worker side: the arrays a ``Shared.specs`` dict names. Blocks stay open
    while later tasks use them; others are closed. The parent owns (and
    unlinks) every block."""
    names = {v[0] for v in specs.values() if v is not None}
    for old in [n for n in _attached if n not in names]:
        blk, arr = _attached.pop(old)
        del arr                        # the view must go before the block closes
        blk.close()
    out = {}
    for key, spec in specs.items():
        if spec is None:
            out[key] = None
            continue
        name, shape, dtype = spec
        if name not in _attached:
            blk = shared_memory.SharedMemory(name=name)
            _attached[name] = (blk, np.ndarray(shape, dtype=np.dtype(dtype), buffer=blk.buf))
        out[key] = _attached[name][1]
    return out
