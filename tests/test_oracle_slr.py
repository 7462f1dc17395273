"""Pins of the oracle's SLR-graph (Section 4.2.2): neighbour selection and the
non-negative Lasso of the SPG construction.

The Lasso solver is checked against a closed form (orthonormal basis), against
brute force over all supports on tiny positive-definite problems (the unique
point satisfying the optimality conditions), against a bounded quasi-Newton
library solve on singular problems, and through its optimality conditions.
The neighbour lists are checked by the defining property (every selected
affinity is at least every unselected one, ties to the lower index) on a matrix
with planted ties.
"""
import itertools

import numpy as np
import pytest
import scipy.optimize as so

from oracle import slr


def _kkt(G, b, alpha, w):
    g = 2.0 * G @ w - 2.0 * b + alpha
    return float(np.max(np.where(w > 0, np.abs(g), np.maximum(0.0, -g))))


def test_orthonormal_basis_closed_form():
    """G = I: the minimiser of |w|^2 - 2 b^T w + alpha sum(w), w >= 0, is max(0, b - alpha/2)."""
    rng = np.random.default_rng(1)
    b = rng.standard_normal(12)
    w = slr.nn_lasso(np.eye(12), b, 0.3)
    assert np.abs(w - np.maximum(0.0, b - 0.15)).max() <= 1e-14


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_over_supports(seed):
    """Tiny positive-definite problems: exactly one support S gives a stationary
    point w_S = G_SS^-1 (b_S - alpha/2) > 0 whose outside gradients are >= 0;
    the active-set result must be that point."""
    rng = np.random.default_rng(seed)
    m, k = 9, 6
    D = rng.standard_normal((m, k))
    x = rng.standard_normal(m) + D @ np.abs(rng.standard_normal(k))
    G, b, alpha = D.T @ D, D.T @ x, 0.4 + seed * 0.3
    found = []
    for r in range(k + 1):
        for S in itertools.combinations(range(k), r):
            w = np.zeros(k)
            if S:
                idx = list(S)
                w[idx] = np.linalg.solve(G[np.ix_(idx, idx)], b[idx] - alpha / 2.0)
                if np.any(w[idx] <= 0):
                    continue
            g = 2.0 * G @ w - 2.0 * b + alpha
            if all(g[j] >= -1e-12 for j in range(k) if j not in S):
                found.append(w)
    assert len(found) == 1
    w = slr.nn_lasso(G, b, alpha)
    assert np.abs(w - found[0]).max() <= 1e-10 * max(1.0, np.abs(found[0]).max())


@pytest.mark.parametrize("seed", range(3))
def test_singular_gram_matches_bounded_quasi_newton(seed):
    """More basis columns than dimensions (G singular): the optimal value is
    unique; a bounded L-BFGS solve of the same objective does not beat it, and
    the optimality conditions hold."""
    rng = np.random.default_rng(10 + seed)
    m, k = 8, 14
    D = rng.standard_normal((m, k))
    x = rng.standard_normal(m)
    G, b, alpha = D.T @ D, D.T @ x, 0.2
    w = slr.nn_lasso(G, b, alpha)
    f = slr.nn_lasso_objective(G, b, float(x @ x), alpha, w)
    fun = lambda v: float(np.sum((x - D @ v) ** 2) + alpha * np.sum(v))
    jac = lambda v: -2.0 * D.T @ (x - D @ v) + alpha
    r = so.minimize(fun, np.zeros(k), jac=jac, method="L-BFGS-B", bounds=[(0, None)] * k,
                    options=dict(ftol=1e-15, gtol=1e-12, maxiter=10000))
    assert f <= r.fun + 1e-10
    assert abs(f - fun(w)) <= 1e-12 * max(1.0, f)
    assert np.all(w >= 0) and _kkt(G, b, alpha, w) <= 1e-10


def test_neighbors_are_the_top_affinities_with_index_ties():
    """Every listed neighbour has affinity >= every unlisted one, the list is by
    decreasing affinity with ties to the lower index, and i is never listed."""
    rng = np.random.default_rng(3)
    n, nk = 30, 7
    Z = np.round(rng.standard_normal((n, n)), 1)      # many exact ties in |Z_ij| + |Z_ji|
    nbr = slr.slr_neighbors(Z, nk)
    A = np.abs(Z) + np.abs(Z).T
    for i in range(n):
        lst = nbr[i].tolist()
        assert i not in lst and len(set(lst)) == nk
        rest = [j for j in range(n) if j != i and j not in lst]
        assert min(A[i, lst]) >= max(A[i, rest])
        for a, c in zip(lst, lst[1:]):
            assert A[i, a] > A[i, c] or (A[i, a] == A[i, c] and a < c)
        edge = min(A[i, lst])
        assert all(j > max(q for q in lst if A[i, q] == edge) for j in rest if A[i, j] == edge)


def test_neighbor_rows_match_a_lexicographic_sort():
    """slr_neighbors_rows on a tie-heavy matrix equals numpy's lexicographic
    sort on (-affinity, index) of each row, and slr_neighbors' rows."""
    rng = np.random.default_rng(11)
    n, nk = 300, 40
    Z = np.round(rng.standard_normal((n, n)) * 4) / 4       # many exact ties
    rows = [0, 7, 150, 299]
    got = slr.slr_neighbors_rows(Z, nk, rows)
    for r, i in enumerate(rows):
        a = np.abs(Z[i, :]) + np.abs(Z[:, i])
        j = np.array([q for q in range(n) if q != i])
        order = j[np.lexsort((j, -a[j]))]
        assert np.array_equal(got[r], order[:nk])
    assert np.array_equal(got, slr.slr_neighbors(Z, nk)[rows])


def test_slr_graph_weights_satisfy_optimality():
    """End to end on a small union of subspaces: each sample's weights are
    non-negative and optimal for its neighbour basis."""
    rng = np.random.default_rng(4)
    m, n = 20, 40
    M = np.hstack([np.linalg.qr(rng.standard_normal((m, 2)))[0] @ rng.standard_normal((2, 10)) for _ in range(4)])
    Z = rng.standard_normal((n, n)) * 0.1
    nbr, W, obj = slr.slr_graph(M, Z, 6, 0.05)
    for i in range(n):
        D = M[:, nbr[i]]
        G, b = D.T @ D, D.T @ M[:, i]
        assert np.all(W[i] >= 0)
        assert _kkt(G, b, 0.05, W[i]) <= 1e-9
        assert abs(obj[i] - (np.sum((M[:, i] - D @ W[i]) ** 2) + 0.05 * W[i].sum())) <= 1e-12
