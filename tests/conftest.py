import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")

# The oracle runs on small matrices in the CPU tests; many BLAS threads only add
# synchronisation overhead there.
try:
    from threadpoolctl import threadpool_limits as _tpl
    _TPL = _tpl(limits=1)
except Exception:  # pragma: no cover
    _TPL = None
