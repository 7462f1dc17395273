"""Pins of the oracle's footnote variant of Section 2.2 (dfc_lrr_local).

Each block solves Eq. (1) with its own columns as dictionary; the C step is the
best rank-k approximation of diag(Z_1, ..., Z_t).  The checks do not retype the
oracle's formulas: the single-block case is compared with plain LRR on the
unpermuted matrix (equivariance under a permutation of the points), the C step
with a truncated SVD of the assembled n x n block-diagonal matrix (Eckart-Young),
and each block with the duality certificate of Eq. (1) at a slow schedule.
"""
import numpy as np
import pytest

import oracle
from oracle import ALMOptions

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _data(seed, m=24, k=3, r=2, ns=12, n_out=4):
    rng = np.random.default_rng(seed)
    cols = []
    for _ in range(k):
        q, _ = np.linalg.qr(rng.standard_normal((m, r)))
        cols.append(q @ rng.standard_normal((r, ns)))
    M = np.concatenate(cols, axis=1)
    idx = rng.choice(M.shape[1], n_out, replace=False)
    M[:, idx] = rng.standard_normal((m, n_out))
    return M


def _split(n, t, seed):
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n).astype(np.int64)
    cuts = np.sort(rng.choice(np.arange(4, n - 3), t - 1, replace=False)) if t > 1 else np.array([], int)
    return perm, np.concatenate([[0], cuts, [n]]).astype(np.int64)


def test_single_block_is_plain_lrr_of_the_unpermuted_matrix():
    """t = 1, nothing truncated: LRR of M P with dictionary M P is P^T Z P for the
    LRR solution Z of M, so undoing the permutation must give plain LRR of M."""
    M = _data(1)
    n = M.shape[1]
    perm, off = _split(n, 1, 1)
    d = oracle.dfc_lrr_local(M, 0.4, perm, off, rank=-1)
    ref = oracle.lrr_alm(M, M, 0.4)
    assert np.abs(d.Z - ref.J).max() <= 1e-9
    assert np.abs(d.S - ref.E).max() <= 1e-9
    assert d.combine_rank == ref.rank


@pytest.mark.parametrize("rank", [0, 3, 7, -1, 10_000])
def test_combine_is_truncated_svd_of_the_block_diagonal(rank):
    """The C step equals the rank-k truncated SVD of the assembled n x n matrix
    diag(J_1, ..., J_t) (one dense SVD, no per-block factors), and is zero
    outside the diagonal blocks."""
    M = _data(2, ns=14)
    n = M.shape[1]
    perm, off = _split(n, 3, 2)
    d = oracle.dfc_lrr_local(M, 0.35, perm, off, rank=rank)
    B = np.zeros((n, n))
    for i, r in enumerate(d.blocks):
        cols = perm[off[i]:off[i + 1]]
        B[np.ix_(cols, cols)] = r.J
    U, s, Vt = np.linalg.svd(B)
    total = sum(r.rank for r in d.blocks)
    k = {0: max(r.rank for r in d.blocks), -1: total}.get(rank, min(rank, total))
    assert d.combine_rank == k
    ref = (U[:, :k] * s[:k]) @ Vt[:k]
    assert np.linalg.norm(d.Z - ref) <= 1e-9 * max(np.linalg.norm(ref), 1.0)
    inside = np.zeros((n, n), dtype=bool)
    for i in range(len(off) - 1):
        cols = perm[off[i]:off[i + 1]]
        inside[np.ix_(cols, cols)] = True
    assert np.all(d.Z[~inside] == 0.0)
    assert np.linalg.matrix_rank(d.Z, tol=1e-9 * s[0]) == k


def test_each_block_is_a_certified_lrr_solution():
    """Every block estimate solves Eq. (1) for its own columns: at a slow
    penalty schedule the duality gap of Eq. (2) with X = A = C_i vanishes."""
    M = _data(3)
    n = M.shape[1]
    perm, off = _split(n, 2, 3)
    d = oracle.dfc_lrr_local(M, 0.5, perm, off, rank=-1, opts=ALMOptions(rho=1.01, tol=1e-13, max_iter=10000))
    for i, r in enumerate(d.blocks):
        C = M[:, perm[off[i]:off[i + 1]]]
        Z = r.J
        gap, primal = oracle.dual_gap(C, C, Z, C - C @ Z, r.Y1, 0.5)
        assert -1e-12 <= gap <= 1e-8 * primal
    # the block's outlier estimate sits in the original column order
    S_ref = np.concatenate([r.E for r in d.blocks], axis=1)
    assert np.abs(d.S[:, perm] - S_ref).max() == 0.0
