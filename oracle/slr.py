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
alpha 1^T w (G = D^T D, b = D^T x) and solved by the active-set method of
Lawson and Hanson with a pivot for entering columns that depend on the free
ones (see nn_lasso), a finite method that ends at the optimality conditions; G is
singular whenever the neighbours of a sample span fewer dimensions than there
are of them (the normal case here: they come from the sample's own subspace),
so only the optimal value is unique in general, and the weights are unique
when G is positive definite.
"""
from __future__ import annotations

import numpy as np

__all__ = ["slr_neighbors", "slr_neighbors_rows", "nn_lasso", "nn_lasso_objective", "slr_graph"]


def slr_neighbors(Z: np.ndarray, nk: int) -> np.ndarray:
    """(n, nk) int64: row i lists the nk samples j != i with the largest
    |Z_ij| + |Z_ji|, by decreasing affinity, ties to the lower index."""
    Z = np.asarray(Z, dtype=np.float64)
    return slr_neighbors_rows(Z, nk, range(Z.shape[0]))


def slr_neighbors_rows(Z: np.ndarray, nk: int, rows) -> np.ndarray:
    """The rows `rows` of slr_neighbors(Z, nk), each formed on its own (for
    sampled checks at sizes where all n rows would take too long)."""
    Z = np.asarray(Z, dtype=np.float64)
    n = Z.shape[0]
    if not 1 <= nk <= n - 1:
        raise ValueError("need 1 <= nk <= n - 1")
    rows = list(rows)
    out = np.empty((len(rows), nk), dtype=np.int64)
    for r, i in enumerate(rows):
        a = np.abs(Z[i, :]) + np.abs(Z[:, i])        # a[j] = |Z_ij| + |Z_ji|
        cand = [j for j in range(n) if j != i]
        cand.sort(key=lambda j: (-a[j], j))
        out[r] = cand[:nk]
    return out


def nn_lasso_objective(G: np.ndarray, b: np.ndarray, xx: float, alpha: float, w: np.ndarray) -> float:
    """||x - D w||^2 + alpha sum(w) from the Gram form (G = D^T D, b = D^T x, xx = ||x||^2)."""
    return float(w @ G @ w - 2.0 * b @ w + xx + alpha * np.sum(w))


def nn_lasso(G: np.ndarray, b: np.ndarray, alpha: float, tol: float = 1e-12, dep_tol: float = 1e-10) -> np.ndarray:
    """Minimiser of w^T G w - 2 b^T w + alpha 1^T w over w >= 0 (alpha > 0).

    The active-set method of Lawson and Hanson (Solving Least Squares Problems,
    1974, ch. 23) in Gram form, with gradient g = 2 G w - 2 b + alpha and the
    free set P kept linearly independent:
      * stop when the optimality conditions hold to tol of the problem's scale
        (|g_j| on P, max(0, -g_j) off P);
      * otherwise the coordinate j off P with the most negative gradient enters;
      * if column j depends on the free columns (its Cholesky pivot falls below
        dep_tol of the largest diagonal entry), D_j = D_P beta and the objective
        falls linearly along w_P -= t beta, w_j += t (its slope is
        alpha (1 - sum(beta)) = g_j < 0): move until the first free weight with
        beta_i > 0 reaches zero and swap it out;
      * then the stationary point s of the face P, G_PP s = b_P - alpha/2, is
        taken if positive; otherwise w moves towards s until the first weight
        reaches zero, that index leaves P, and the face is solved again."""
    G = np.asarray(G, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    k = b.size
    w = np.zeros(k)
    if k == 0:
        return w
    scale = max(1.0, float(np.max(np.abs(2.0 * b - alpha))), float(np.max(np.abs(2.0 * G))))
    dmax = float(np.max(np.diag(G)))
    P: list[int] = []
    for _ in range(10 * k + 20):
        g = 2.0 * G @ w - 2.0 * b + alpha
        free = np.zeros(k, dtype=bool)
        free[P] = True
        viol = np.where(free, np.abs(g), np.maximum(0.0, -g))
        if float(np.max(viol)) <= tol * scale:
            return w
        cand = np.where(free, np.inf, g)
        j = int(np.argmin(cand))
        if not cand[j] < 0:
            # only free coordinates violate: re-solve the face below
            j = -1
        if j >= 0:
            if P:
                L = np.linalg.cholesky(G[np.ix_(P, P)])
                y = np.linalg.solve(L, G[P, j])
                piv = G[j, j] - float(y @ y)
            else:
                piv = G[j, j]
            if piv <= dep_tol * dmax:
                beta = np.linalg.solve(G[np.ix_(P, P)], G[P, j])
                pos = [q for q in range(len(P)) if beta[q] > 0]
                t = min(w[P[q]] / beta[q] for q in pos)
                out = min((q for q in pos if w[P[q]] / beta[q] == t), key=lambda q: P[q])
                for q in range(len(P)):
                    w[P[q]] -= t * beta[q]
                w[j] = t
                w[P[out]] = 0.0
                P = [P[q] for q in range(len(P)) if q != out] + [j]
            else:
                P = P + [j]
        while P:
            s = np.linalg.solve(G[np.ix_(P, P)], b[P] - alpha / 2.0)
            if np.all(s > 0):
                w[:] = 0.0
                w[P] = s
                break
            ratios = [(w[P[q]] / (w[P[q]] - s[q]), P[q]) for q in range(len(P)) if s[q] <= 0]
            t = min(r for r, _ in ratios)
            for q in range(len(P)):
                w[P[q]] += t * (s[q] - w[P[q]])
            gone = {i for r, i in ratios if r == t}
            for i in gone:
                w[i] = 0.0
            P = [i for i in P if i not in gone]
    raise RuntimeError("non-negative Lasso: step limit reached")


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
