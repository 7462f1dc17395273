"""Helpers shared by the GPU tests (imported only by tests marked gpu)."""
import contextlib
import sys

import numpy as np


def need_gpu():
    import pytest
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1304_5583_amd import binding
    binding.load_library()   # fails loudly when the HIP library is missing
    return torch


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@contextlib.contextmanager
def one_thread():
    """Run the oracle single-threaded (small problems are faster that way)."""
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        yield
        return
    with threadpool_limits(limits=1):
        yield


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
