import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")
    # The oracle's worker processes are forked here, before anything in this
    # process initialises the GPU runtime (collection below asks torch for a
    # device); a process that holds GPU state never forks.
    from oracle import pool
    pool.start()


def pytest_collection_modifyitems(config, items):
    # GPU tests need a device; skip (not fail) them where there is none so that
    # `-m "not gpu"` and plain runs on a CPU-only host stay green.
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover
        has_gpu = False
    if has_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU on this host")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)
