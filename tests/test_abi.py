"""C-ABI checks that need no GPU: the library loads, exports every function the
headers declare, and validates arguments on the host before any device work."""
import ctypes as C
import glob
import os
import re

import numpy as np
import pytest

from paper_1304_5583_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[a-z_]+\s*\**\s*([a-z_0-9]+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    lib = B.load_library()
    names = _declared_functions()
    assert {"lrr_solve", "dfc_lrr_solve", "dfc_lrr_backward", "lrr_ctx_create"} <= names
    for name in sorted(names):
        assert hasattr(lib, name), f"{name} declared but not exported"


def test_opts_default_values():
    o = B.lrr_opts_default()
    assert o.precision == B.LRR_FP64 and o.mu0 == 1e-6 and o.rho == 1.1
    assert o.mu_max == 1e10 and o.tol == 1e-8 and o.max_iter == 1000
    assert o.fixed_iters == 0 and o.checkpoint_every == 20 and list(o.reserved) == [0] * 3 and o.tune == 0
    assert o.io_type == B.LRR_IO_FP64
    assert o.coords == 0
    assert o.use_graph == 1
    assert "gfx950" in B.lrr_version()


def test_check_partition():
    n = 10
    perm = np.random.default_rng(0).permutation(n)
    assert B.lrr_check_partition(n, perm, [0, 4, 10]) == B.LRR_OK
    assert B.lrr_check_partition(n, perm, [0, 10]) == B.LRR_OK
    assert B.lrr_check_partition(n, perm, [0, 4, 4, 10]) == B.LRR_EINVAL      # empty block
    assert B.lrr_check_partition(n, perm, [1, 4, 10]) == B.LRR_EINVAL        # does not start at 0
    assert B.lrr_check_partition(n, perm, [0, 4, 9]) == B.LRR_EINVAL         # does not end at n
    bad = perm.copy()
    bad[0] = bad[1]
    assert B.lrr_check_partition(n, bad, [0, 4, 10]) == B.LRR_EINVAL         # not a permutation
    bad = perm.copy()
    bad[0] = n
    assert B.lrr_check_partition(n, bad, [0, 4, 10]) == B.LRR_EINVAL         # out of range
    assert "permutation" in B.lrr_last_error()


def test_workspace_bytes_scales_with_problem():
    lib = B.load_library()
    o = B.lrr_opts_default()
    sizes = []
    for n in (200, 2000):
        off = np.array([0, n // 2, n], dtype=np.int32)
        out = C.c_size_t(0)
        assert lib.lrr_workspace_bytes(100, n, 2, B._ip(off), C.byref(o), C.byref(out)) == B.LRR_OK
        sizes.append(out.value)
    assert 0 < sizes[0] < sizes[1]
    # at least the six n x n state matrices
    assert sizes[1] >= 6 * 2000 * 2000 * 8


def test_null_ctx_and_bad_arguments_rejected_on_host():
    lib = B.load_library()
    o = B.lrr_opts_default()
    info = B.lrr_info()
    perm = np.arange(10, dtype=np.int32)
    off = np.array([0, 10], dtype=np.int32)
    st = lib.lrr_solve(None, 5, 10, 10, None, 5, None, 5, 0.1, C.byref(o), None, 10, None, 5,
                       C.byref(info), None)
    assert st == B.LRR_EINVAL
    st = lib.dfc_lrr_solve(None, 5, 10, None, 5, 0.1, 1, B._ip(perm), B._ip(off), C.byref(o), None, 10,
                           None, 5, C.byref(info), None)
    assert st == B.LRR_EINVAL
    dl = C.c_double(0)
    assert lib.dfc_lrr_backward(None, None, 10, C.byref(dl), None, 5, None) == B.LRR_EINVAL
    assert lib.lrr_ctx_create(0, None) == B.LRR_EINVAL
    flags = np.zeros(10, dtype=np.uint8)
    assert lib.lrr_outlier_flags(None, 5, 10, None, 5, None, 5, 0.5, None, None, None) == B.LRR_EINVAL
