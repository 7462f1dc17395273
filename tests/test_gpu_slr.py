"""GPU SLR-graph (Section 4.2.2): lrr_slr_graph against the oracle.

Neighbour lists are integer work and must equal the oracle's bit for bit (both
sides form |Z_ij| + |Z_ji| with one FP64 addition and order by it, ties to the
lower index).  The non-negative Lasso has a unique optimal value but, when a
sample's neighbours span fewer dimensions than their number, not unique
weights; so per sample the test compares the optimal objective with the
oracle's (relative 1e-9), checks the GPU weights against the optimality
conditions computed here in FP64 (1e-9 of the sample's scale), recomputes the
objective from the weights, and where D_i^T D_i is positive definite compares
the weights themselves (1e-7).
"""
import numpy as np
import pytest

from gpu_util import need_gpu, one_thread, say

pytestmark = pytest.mark.gpu


def _check_sample(M, i, nbr_i, w_i, obj_i, alpha, ref_obj=None, ref_w=None):
    D = M[:, nbr_i]
    G, b, x = D.T @ D, D.T @ M[:, i], M[:, i]
    scale = max(1.0, np.abs(2 * b - alpha).max(), 2 * np.diag(G).max())
    g = 2 * G @ w_i - 2 * b + alpha
    kkt = np.max(np.where(w_i > 0, np.abs(g), np.maximum(0.0, -g)))
    f = float(np.sum((x - D @ w_i) ** 2) + alpha * w_i.sum())
    assert np.all(w_i >= 0)
    assert kkt <= 1e-9 * scale, kkt / scale
    assert abs(obj_i - f) <= 1e-10 * max(1.0, f)
    if ref_obj is not None:
        assert abs(f - ref_obj) <= 1e-9 * max(1.0, ref_obj), (f, ref_obj)
    if ref_w is not None and np.linalg.eigvalsh(G)[0] > 1e-8 * np.linalg.eigvalsh(G)[-1]:
        assert np.abs(w_i - ref_w).max() <= 1e-7 * max(1.0, np.abs(ref_w).max())


@pytest.mark.parametrize("seed,nk,alpha", [(61, 8, 0.05), (62, 20, 0.05), (63, 5, 0.5), (64, 40, 0.01)])
def test_slr_graph_matches_oracle(seed, nk, alpha):
    """Small union-of-subspaces data, Z from the GPU DFC-LRR solve."""
    need_gpu()
    import oracle
    from oracle import slr
    from paper_1304_5583_amd import binding as B
    from paper_1304_5583_amd.datagen import small_problem
    p = small_problem(seed, m=40, k=4, r=3, ns=30, n_replace=8, t=3)
    Mt = B.to_device_colmajor(p.M)
    Zt, _, _ = B.dfc_lrr_solve(Mt, p.lam, p.perm, p.offsets)
    nbr, w, obj, info = B.lrr_slr_graph(Mt, Zt, nk, alpha)
    Zg = B.from_device_colmajor(Zt)
    nbr, w, obj = nbr.cpu().numpy(), w.cpu().numpy(), obj.cpu().numpy()
    with one_thread():
        rn, rw, robj = slr.slr_graph(p.M, Zg, nk, alpha)
    say(f"[slr s{seed}] n={p.n} nk={nk} alpha={alpha} steps<={info['max_steps']} kkt={info['max_kkt']:.1e} "
        f"nnz={int((w > 0).sum())}")
    assert info["converged"]
    assert np.array_equal(nbr, rn)
    for i in range(p.n):
        _check_sample(p.M, i, nbr[i], w[i], obj[i], alpha, robj[i], rw[i])


def test_slr_graph_workload2_paper_settings():
    """Workload 2 (n = 2000) with the paper's alpha = 0.05 and n_k = 500 on the
    GPU solve's Z: every neighbour list equals the oracle's, every sample's
    weights satisfy the optimality conditions, and on 8 seeded samples the
    optimal objective equals the oracle's."""
    need_gpu()
    from oracle import slr
    from paper_1304_5583_amd import binding as B
    from paper_1304_5583_amd.datagen import make_config
    p = make_config(2)
    Mt = B.to_device_colmajor(p.M)
    Zt, _, _ = B.dfc_lrr_solve(Mt, p.lam, p.perm, p.offsets, want_S=False)
    nk, alpha = 500, 0.05
    nbr, w, obj, info = B.lrr_slr_graph(Mt, Zt, nk, alpha)
    say(f"[slr wl2] steps<={info['max_steps']} kkt={info['max_kkt']:.1e} nnz/sample="
        f"{float((w > 0).sum().item()) / p.n:.1f}")
    assert info["converged"]
    Zg = B.from_device_colmajor(Zt)
    nbr, w, obj = nbr.cpu().numpy(), w.cpu().numpy(), obj.cpu().numpy()
    with one_thread():
        rn = slr.slr_neighbors(Zg, nk)
    assert np.array_equal(nbr, rn)
    rng = np.random.default_rng(77)
    for i in rng.choice(p.n, 8, replace=False):
        D = p.M[:, nbr[i]]
        G, b = D.T @ D, D.T @ p.M[:, i]
        with one_thread():
            rw = slr.nn_lasso(G, b, alpha)
        robj = slr.nn_lasso_objective(G, b, float(p.M[:, i] @ p.M[:, i]), alpha, rw)
        _check_sample(p.M, i, nbr[i], w[i], obj[i], alpha, robj)
    for i in range(0, p.n, 50):
        _check_sample(p.M, i, nbr[i], w[i], obj[i], alpha)


def test_slr_graph_edges_and_errors():
    torch = need_gpu()
    from oracle import slr
    from paper_1304_5583_amd import binding as B
    rng = np.random.default_rng(5)
    m, n = 12, 30
    M = rng.standard_normal((m, n))
    Z = rng.standard_normal((n, n))
    Mt, Zt = B.to_device_colmajor(M), B.to_device_colmajor(Z)
    for nk in (1, n - 1):
        nbr, w, obj, info = B.lrr_slr_graph(Mt, Zt, nk, 0.1)
        assert np.array_equal(nbr.cpu().numpy(), slr.slr_neighbors(Z, nk))
        for i in range(n):
            _check_sample(M, i, nbr.cpu().numpy()[i], w.cpu().numpy()[i], obj.cpu().numpy()[i], 0.1)
    for kw in (dict(nk=0), dict(nk=n), dict(nk=3, alpha=0.0), dict(nk=3, alpha=-1.0)):
        with pytest.raises(B.LRRError) as e:
            B.lrr_slr_graph(Mt, Zt, **kw)
        assert e.value.status == B.LRR_EINVAL
