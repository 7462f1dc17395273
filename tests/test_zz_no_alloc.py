"""The entry point that allocates no device memory (lrr_diag_spd_inverse_noalloc)
against the allocating one (lrr_diag_spd_inverse), through the C ABI.

Both run the same kernels on the same inputs, so the results must agree to
rounding (bar 1e-13 relative; measured: bitwise equal).  Two calls in a row,
the second with a smaller order: the static work array keeps the first call's
contents, which the second must not read.  Orders above the stated limit are
rejected with LRR_EINVAL."""
import ctypes as C

import numpy as np
import pytest

from gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


def test_spd_inverse_noalloc_matches_allocating_entry():
    torch = need_gpu()
    from paper_1304_5583_amd import binding as B
    lib = B.load_library()
    ctx = B.Context(0)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rng = np.random.default_rng(77)
    for m, n in ((700, 900), (130, 170)):
        say(f"[no-alloc] m={m} n={n}")
        A = rng.standard_normal((m, n))
        At = B.to_device_colmajor(A)
        K1 = torch.full((m, m), float("nan"), dtype=torch.float64, device="cuda")
        K2 = torch.full((m, m), float("nan"), dtype=torch.float64, device="cuda")
        st1 = lib.lrr_diag_spd_inverse(ctx.handle, m, n, C.c_void_p(At.data_ptr()), m,
                                       C.c_void_p(K1.data_ptr()), m, stream)
        st2 = lib.lrr_diag_spd_inverse_noalloc(ctx.handle, m, n, C.c_void_p(At.data_ptr()), m,
                                               C.c_void_p(K2.data_ptr()), m, stream)
        torch.cuda.synchronize()
        assert st1 == B.LRR_OK and st2 == B.LRR_OK
        k1, k2 = K1.cpu().numpy(), K2.cpu().numpy()
        err = float(np.abs(k2 - k1).max() / np.abs(k1).max())
        # and the definition itself: (I + A A^T) K = I
        res = float(np.abs((np.eye(m) + A @ A.T) @ k2 - np.eye(m)).max())
        say(f"  max rel diff vs allocating entry {err:.2e}, residual {res:.2e}")
        assert err <= 1e-13
        assert res <= 1e-9
    m = 1025
    At = torch.zeros((4, m), dtype=torch.float64, device="cuda")
    K = torch.zeros((m, m), dtype=torch.float64, device="cuda")
    st = lib.lrr_diag_spd_inverse_noalloc(ctx.handle, m, 4, C.c_void_p(At.data_ptr()), m,
                                          C.c_void_p(K.data_ptr()), m, stream)
    assert st == B.LRR_EINVAL
    assert "1024" in lib.lrr_last_error(ctx.handle).decode()
