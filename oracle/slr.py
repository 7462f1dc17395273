"""SLR-graph (Section 4.2.2): graph weights from a low-rank coefficient matrix.

TEST INFRASTRUCTURE ONLY (see the oracle package docstring).

The method takes the LRR / DFC-LRR coefficient matrix Z as an affinity, picks
for every sample x_i the n_k samples with the largest affinity to it as the
basis D_i, and solves the non-negative Lasso of the SPG construction (the
optimisation problem of Section 4.2.2's graph-construction list)

    min_w  ||x_i - D_i w||_2^2 + alpha ||w||_1   s.t.  w >= 0;

the non-negative weights define the edges of sample i.

Readings where the paper is silent (listed in the design notes): the affinity of
samples i and j is |Z_ij| + |Z_ji| (Z is not symmetric; both directions of the
representation count), a sample is never its own neighbour, ties in the
affinity go to the lower index, and the neighbours are listed by decreasing
affinity.  The Lasso is written in its Gram form min w^T G w - 2 b^T w +
alpha 1^T w (G = D^T D, b = D^T x) and solved by cyclic exact coordinate
minimisation run until the optimality conditions hold to rounding; G is
singular whenever the neighbours of a sample span fewer dimensions than there
are of them (the normal case here: they come from the sample's own subspace),
so only the optimal value is unique in general, and the weights are unique
when G is positive definite.
"""
from __future__ import annotations

import numpy as np

__all__ = ["slr_neighbors", "nn_lasso", "nn_lasso_objective", "slr_graph"]


def slr_neighbors(Z: np.ndarray, nk: int) -> np.ndarray:
    """(n, nk) int64: row i lists the nk samples j != i with the largest
    |Z_ij| + |Z_ji|, by decreasing affinity, ties to the lower index."""
    Z = np.asarray(Z, dtype=np.float64)
    n = Z.shape[0]
    if not 1 <= nk <= n - 1:
        raise ValueError("need 1 <= nk <= n - 1")
    A = np.abs(Z) + np.abs(Z).T
    out = np.empty((n, nk), dtype=np.int64)
    for i in range(n):
        cand = [j for j in range(n) if j != i]
        cand.sort(key=lambda j: (-A[i, j], j))
        out[i] = cand[:nk]
    return out


def nn_lasso_objective(G: np.ndarray, b: np.ndarray, xx: float, alpha: float, w: np.ndarray) -> float:
    """||x - D w||^2 + alpha sum(w) from the Gram form (G = D^T D, b = D^T x, xx = ||x||^2)."""
    return float(w @ G @ w - 2.0 * b @ w + xx + alpha * np.sum(w))


def nn_lasso(G: np.ndarray, b: np.ndarray, alpha: float, tol: float = 1e-13,
             max_sweeps: int = 200000) -> np.ndarray:
    """Minimiser of w^T G w - 2 b^T w + alpha 1^T w over w >= 0.

    Cyclic coordinate minimisation: coordinate j in turn moves to the exact
    minimiser of the objective along it, max(0, w_j - g_j / (2 G_jj)) with the
    gradient g = 2 G w - 2 b + alpha; the gradient is re-formed from w every
    sweep.  Stops when the optimality conditions hold to tol (relative to the
    problem's scale): |g_j| where w_j > 0, max(0, -g_j) where w_j = 0."""
    G = np.asarray(G, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    k = b.size
    w = np.zeros(k)
    if k == 0:
        return w
    scale = max(1.0, float(np.max(np.abs(2.0 * b - alpha))), float(np.max(np.abs(2.0 * G))))
    for _ in range(max_sweeps):
        g = 2.0 * G @ w - 2.0 * b + alpha
        viol = np.where(w > 0, np.abs(g), np.maximum(0.0, -g))
        if float(np.max(viol)) <= tol * scale:
            break
        for j in range(k):
            if G[j, j] <= 0.0:
                continue                      # a zero column: its weight stays 0 (gradient alpha > 0)
            gj = 2.0 * (G[j] @ w) - 2.0 * b[j] + alpha
            wj = max(0.0, w[j] - gj / (2.0 * G[j, j]))
            w[j] = wj
    return w


def slr_graph(M: np.ndarray, Z: np.ndarray, nk: int, alpha: float):
    """Neighbours (n, nk), weights (n, nk) and the optimal objective per sample."""
    M = np.asarray(M, dtype=np.float64)
    nbr = slr_neighbors(Z, nk)
    n = M.shape[1]
    W = np.zeros((n, nk))
    obj = np.zeros(n)
    for i in range(n):
        D = M[:, nbr[i]]
        G = D.T @ D
        b = D.T @ M[:, i]
        w = nn_lasso(G, b, alpha)
        W[i] = w
        obj[i] = nn_lasso_objective(G, b, float(M[:, i] @ M[:, i]), alpha, w)
    return nbr, W, obj
