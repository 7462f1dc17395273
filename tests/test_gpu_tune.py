"""The schedule table of the autotuner (lrr_tune_load, opts.tune).

A tuned solve must be bitwise the solve with the entry's options given
explicitly; tune = 0 ignores the table; a malformed table is rejected with the
line named and leaves the previous table in place; NULL clears it."""
import os

import numpy as np
import pytest

from gpu_util import need_gpu

pytestmark = pytest.mark.gpu


def test_tuned_solve_equals_explicit_schedule(tmp_path):
    torch = need_gpu()
    from paper_1304_5583_amd import binding as B
    from paper_1304_5583_amd.datagen import small_problem
    p = small_problem(71, m=48, k=3, r=3, ns=40, n_replace=8, t=3, uneven=(35, 45))
    Mt = B.to_device_colmajor(p.M)
    ctx = B.Context(0)
    maxl = int(np.diff(p.offsets).max())
    path = tmp_path / "table.txt"
    path.write_text("# m n t maxl precision eig_block use_graph check_every coords\n"
                    f"{p.m} {p.n} {p.t} {maxl} 0 32 0 4 1\n")
    B.lrr_tune_load(str(path), ctx=ctx)
    Zt, _, info = B.dfc_lrr_solve(Mt, p.lam, p.perm, p.offsets, opts=B.lrr_opts_default(tune=1), ctx=ctx)
    Ze, _, infe = B.dfc_lrr_solve(Mt, p.lam, p.perm, p.offsets, ctx=ctx,
                                  opts=B.lrr_opts_default(eig_block=32, use_graph=0, check_every=4, coords=1))
    assert torch.equal(Zt, Ze) and info.iters.tolist() == infe.iters.tolist()
    Zd, _, _ = B.dfc_lrr_solve(Mt, p.lam, p.perm, p.offsets, ctx=ctx, opts=B.lrr_opts_default())
    Zu, _, _ = B.dfc_lrr_solve(Mt, p.lam, p.perm, p.offsets, ctx=ctx, opts=B.lrr_opts_default(tune=0))
    assert torch.equal(Zd, Zu)
    # a malformed file is rejected and the loaded table stays
    bad = tmp_path / "bad.txt"
    bad.write_text(f"{p.m} {p.n} {p.t} {maxl} 0 24 0 4 1\n")
    with pytest.raises(B.LRRError) as e:
        B.lrr_tune_load(str(bad), ctx=ctx)
    assert e.value.status == B.LRR_EINVAL and "line 1" in str(e.value)
    Zt2, _, _ = B.dfc_lrr_solve(Mt, p.lam, p.perm, p.offsets, opts=B.lrr_opts_default(tune=1), ctx=ctx)
    assert torch.equal(Zt2, Ze)
    B.lrr_tune_load(None, ctx=ctx)
    Zc, _, _ = B.dfc_lrr_solve(Mt, p.lam, p.perm, p.offsets, opts=B.lrr_opts_default(tune=1), ctx=ctx)
    assert torch.equal(Zc, Zd)


def test_shipped_table_is_well_formed():
    need_gpu()
    from paper_1304_5583_amd import binding as B
    if os.path.exists(B.TUNE_TABLE):
        B.lrr_tune_load(B.TUNE_TABLE, ctx=B.Context(0))
