"""GPU segmentation (Section 4.1.2): lrr_segment against the oracle's segment.

The bar is label equality: the labels from the HIP pipeline (range basis,
left singular vectors, normalised affinity, spectral embedding, k-means) must
equal ``oracle.segment`` on the same Z, element by element, including the -1
of excluded points.  Small cases compare on the oracle's own Z and on the
GPU's Z; the full workloads 2 and 3 compare against the stored oracle labels
(computed by tests/golden/make_golden.py from the oracle's Z); workload 4,
whose SVD the oracle cannot afford, is checked by properties that hold at any
size.
"""
import json
import os

import numpy as np
import pytest

from gpu_util import need_gpu, one_thread, say

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _seg(Z, k, exclude=None, rank_tol=1e-6, rank_bound=0, ctx=None):
    from paper_1304_5583_amd import binding as B
    Zt = B.to_device_colmajor(Z) if isinstance(Z, np.ndarray) else Z
    lab, info = B.lrr_segment(Zt, k, exclude=exclude, rank_tol=rank_tol, rank_bound=rank_bound, ctx=ctx)
    return lab.cpu().numpy(), info


def _small(seed, **kw):
    from paper_1304_5583_amd.datagen import small_problem
    return small_problem(seed, **kw)


CASES = [
    # seed, problem kwargs, rank_tol, rank_bound
    (21, dict(m=40, k=3, r=3, ns=30, n_replace=6, t=1), 1e-6, 0),
    (22, dict(m=48, k=4, r=3, ns=25, n_replace=10, t=2), 1e-6, 0),
    (23, dict(m=64, k=3, r=4, ns=40, n_replace=8, t=3, uneven=(35, 45)), 1e-6, 60),
    (24, dict(m=50, k=5, r=3, ns=24, n_replace=12, t=4, lam=0.25), 1e-3, 0),
    (25, dict(m=80, k=4, r=5, ns=30, n_replace=0, t=2, coeff="uniform", normalize=True), 1e-6, 70),
]


@pytest.mark.parametrize("seed,kw,rank_tol,rank_bound", CASES)
def test_labels_equal_oracle_on_oracle_Z(seed, kw, rank_tol, rank_bound):
    """On the oracle's DFC-LRR Z: GPU labels == oracle labels, with the outlier
    columns excluded, and also without exclusion when the data has no outlier
    columns (with them, each outlier is a component of its own in the affinity
    graph, the eigenvalue 1 of L has multiplicity above k and the embedding,
    hence the labels, are not determined on either side)."""
    need_gpu()
    import oracle
    p = _small(seed, **kw)
    k = p.extra["k"]
    with one_thread():
        ref = oracle.dfc_lrr(p.M, p.lam, p.perm, p.offsets)
    for exclude in (p.outliers,) + (() if p.outliers.any() else (None,)):
        with one_thread():
            want = oracle.segment(ref.Z, k, exclude, rank_tol=rank_tol)
        got, info = _seg(ref.Z, k, exclude, rank_tol=rank_tol, rank_bound=rank_bound)
        say(f"[seg s{seed}] n={p.n} k={k} excl={exclude is not None} rank={info['rank']} "
            f"q={info['range_rank']} p={info['sketch']} it={info['embed_iters']} res={info['embed_resid']:.1e} "
            f"theta_k={info['theta_k']:.4f} theta_k1={info['theta_k1']:.4f} km={info['kmeans_iters']}")
        assert info["converged"]
        assert info["theta_k"] - info["theta_k1"] > 1e-3
        assert np.array_equal(got, want)


def test_labels_equal_oracle_on_gpu_Z():
    """The whole product path: DFC-LRR solve and segmentation on the GPU, labels
    equal to the oracle's segmentation of the oracle's Z."""
    need_gpu()
    import oracle
    from paper_1304_5583_amd import binding as B
    p = _small(31, m=60, k=4, r=4, ns=30, n_replace=12, t=3, uneven=(36, 48))
    Mt = B.to_device_colmajor(p.M)
    Zt, _, info = B.dfc_lrr_solve(Mt, p.lam, p.perm, p.offsets)
    with one_thread():
        ref = oracle.dfc_lrr(p.M, p.lam, p.perm, p.offsets)
        want = oracle.segment(ref.Z, 4, p.outliers)
    got, sinfo = _seg(Zt, 4, p.outliers, rank_bound=int(p.offsets[1] - p.offsets[0]))
    assert np.array_equal(got, want)
    got0, _ = _seg(Zt, 4, p.outliers, rank_bound=0)
    assert np.array_equal(got0, want)


@pytest.mark.parametrize("wl", [2, 3])
def test_full_workload_labels_equal_stored_oracle_labels(wl):
    """Workloads 2 and 3 at full size: GPU solve, GPU segmentation (direct and
    sketched), labels equal to the oracle labels stored for that workload, at
    both rank cuts."""
    need_gpu()
    from paper_1304_5583_amd import binding as B
    from paper_1304_5583_amd.datagen import make_config
    g = json.load(open(os.path.join(GOLD, f"workload{wl}_oracle.json")))
    p = make_config(wl)
    k = p.extra["k"]
    Mt = B.to_device_colmajor(p.M)
    Zt, _, info = B.dfc_lrr_solve(Mt, p.lam, p.perm, p.offsets)
    del Mt
    bound = int(np.diff(p.offsets).max())
    exclude = None if "S_ratio" in g else p.outliers   # every point (Section 4.1.2)
    for rank_tol, key in ((1e-6, "labels"), (1e-3, "labels_rank_tol_1e-3")):
        for rb in (0, bound):
            got, sinfo = _seg(Zt, k, exclude, rank_tol=rank_tol, rank_bound=rb)
            say(f"[seg wl{wl}] tol={rank_tol} bound={rb} rank={sinfo['rank']} q={sinfo['range_rank']} "
                f"it={sinfo['embed_iters']} res={sinfo['embed_resid']:.1e} theta_k={sinfo['theta_k']:.4f} "
                f"theta_k1={sinfo['theta_k1']:.4f} km={sinfo['kmeans_iters']}")
            assert sinfo["converged"]
            assert got.tolist() == g[key]


def test_workload4_properties():
    """Workload 4 (n = 20000) through the sketch, every point clustered (Section
    4.1.2): k clusters, every point labelled, the labels unchanged when the
    sketch grows, and the segmentation accuracy over the generator's clean
    points at least that of the oracle's labels on the smaller workloads of the
    same generator (1.0 there).  The outlier flags of the solve's own S are
    reported (on this workload S = 0: the replaced columns are represented in
    Z, not in S)."""
    need_gpu()
    import oracle
    from paper_1304_5583_amd import binding as B
    from paper_1304_5583_amd.datagen import make_config
    p = make_config(4)
    k = p.extra["k"]
    Mt = B.to_device_colmajor(p.M)
    Zt, St, info = B.dfc_lrr_solve(Mt, p.lam, p.perm, p.offsets)
    flags, nf = B.lrr_outlier_flags(Mt, St, 0.5)
    say(f"[seg wl4] outlier flags from S (delta 0.5): {nf}, of them generator outliers: "
        f"{int((flags.cpu().numpy() & p.outliers).sum())}")
    del Mt, St
    bound = int(np.diff(p.offsets).max())
    got, sinfo = _seg(Zt, k, None, rank_bound=bound)
    say(f"[seg wl4] rank={sinfo['rank']} q={sinfo['range_rank']} it={sinfo['embed_iters']} "
        f"res={sinfo['embed_resid']:.1e} theta_k={sinfo['theta_k']:.4f} theta_k1={sinfo['theta_k1']:.4f} "
        f"km={sinfo['kmeans_iters']}")
    assert sinfo["converged"]
    assert got.min() == 0 and got.max() == k - 1
    kept = got
    # renumbered by first appearance
    _, first = np.unique(kept, return_index=True)
    assert np.all(np.diff(first) > 0)
    acc = oracle.segmentation_accuracy(got, np.where(p.outliers, -1, p.labels))
    say(f"[seg wl4] accuracy={acc:.4f}")
    assert acc >= 0.99
    got2, _ = _seg(Zt, k, None, rank_bound=bound + 64)
    assert np.array_equal(got, got2)


def test_edge_cases():
    """k = 1, k = n_keep, all points but k excluded, and the error paths."""
    torch = need_gpu()
    import oracle
    from paper_1304_5583_amd import binding as B
    p = _small(27, m=30, k=3, r=3, ns=20, n_replace=6, t=1)
    with one_thread():
        ref = oracle.dfc_lrr(p.M, p.lam, p.perm, p.offsets)
    Z = ref.Z
    n = Z.shape[0]
    got, _ = _seg(Z, 1)
    assert np.all(got == 0) and np.array_equal(got, oracle.segment(Z, 1))
    ex = np.ones(n, dtype=bool)
    ex[[3, 17, 40, 41]] = False
    got, _ = _seg(Z, 4, ex)
    with one_thread():
        want = oracle.segment(Z, 4, ex)
    assert np.array_equal(got, want)
    assert sorted(got[~ex].tolist()) == [0, 1, 2, 3]
    got, _ = _seg(Z, n)
    with one_thread():
        assert np.array_equal(got, oracle.segment(Z, n))
    Zt = B.to_device_colmajor(Z)
    for kw in (dict(k=0), dict(k=n + 1), dict(k=3, rank_tol=0.0), dict(k=3, rank_tol=1.0),
               dict(k=3, rank_bound=-1)):
        with pytest.raises(B.LRRError) as e:
            B.lrr_segment(Zt, **kw)
        assert e.value.status == B.LRR_EINVAL
    with pytest.raises(B.LRRError):
        B.lrr_segment(Zt, 3, exclude=np.ones(n, dtype=bool))
    # a rank bound below the rank of Z: the sketch has full rank
    Zr = B.to_device_colmajor(np.random.default_rng(3).standard_normal((n, n)))
    with pytest.raises(B.LRRError) as e:
        B.lrr_segment(Zr, 3, rank_bound=2)
    assert e.value.status == B.LRR_EINVAL


def test_block_diagonal_affinity_recovers_subspaces():
    """Independent subspaces: the shape-interaction matrix V V^T is block
    diagonal up to the point order, so the labels are the subspace memberships
    (renumbered by first appearance) on the GPU as in the oracle."""
    need_gpu()
    import oracle
    rng = np.random.default_rng(5)
    k, r, ns, m = 5, 3, 40, 60
    bases = [np.linalg.qr(rng.standard_normal((m, r)))[0] for _ in range(k)]
    truth = np.repeat(np.arange(k), ns)
    X = np.hstack([b @ rng.standard_normal((r, ns)) for b in bases])
    order = rng.permutation(k * ns)
    X, truth = X[:, order], truth[order]
    _, s, Vt = np.linalg.svd(X, full_matrices=False)
    V = Vt[: k * r].T
    Z = V @ V.T
    got, _ = _seg(Z, k)
    with one_thread():
        want = oracle.segment(Z, k)
    assert np.array_equal(got, want)
    assert oracle.segmentation_accuracy(got, truth) == 1.0


def test_outlier_flags_vs_oracle():
    """lrr_outlier_flags on the S of a GPU solve against oracle.outlier_flags on
    the same S (both FP64; flags compared away from ratios within 1e-12 of the
    threshold), for several thresholds, plus its argument checks."""
    torch = need_gpu()
    import oracle
    from paper_1304_5583_amd import binding as B
    from paper_1304_5583_amd.datagen import make_config, small_problem
    for name, p in (("small", small_problem(51, m=40, k=3, r=3, ns=30, n_replace=6, t=3, lam=0.15)),
                    ("workload 3", make_config(3))):
        Mt = B.to_device_colmajor(p.M)
        _, St, _ = B.dfc_lrr_solve(Mt, p.lam, p.perm, p.offsets)
        S = B.from_device_colmajor(St)
        ratio = np.linalg.norm(S, axis=0) / np.linalg.norm(p.M, axis=0)
        for delta in (0.0, 0.05, 0.1, 0.5):
            flags, cnt = B.lrr_outlier_flags(Mt, St, delta)
            got = flags.cpu().numpy()
            want = oracle.outlier_flags(S, p.M, delta)
            far = np.abs(ratio - delta) > 1e-12
            say(f"[outlier flags {name}] delta={delta} gpu={cnt} oracle={int(want.sum())} "
                f"generator={int(p.outliers.sum())} hits={int((got & p.outliers).sum())}")
            assert cnt == int(got.sum())
            assert np.array_equal(got[far], want[far])
        del Mt, St
    Mt = B.to_device_colmajor(p.M)
    with pytest.raises(B.LRRError):
        B.lrr_outlier_flags(Mt, Mt, -1.0)
    with pytest.raises(B.LRRError):
        B.lrr_outlier_flags(Mt, Mt, float("nan"))
