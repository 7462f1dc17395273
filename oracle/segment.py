"""Segmentation from an LRR coefficient matrix, and the paper's success criteria.

TEST INFRASTRUCTURE ONLY (see the oracle package docstring).

* ``segment``: Section 4.1.2 builds an affinity U U^T from the top left singular
  vectors of Z, embeds the points spectrally into k dimensions and runs k-means.
  The paper does not fix the number of vectors, the Laplacian, the k-means
  initialisation, tie breaking, or what happens to outlier columns; the readings
  used here are: numerical rank #sigma > 1e-6 sigma_1, affinity |U U^T| over the
  points not marked as outliers (an outlier column is represented by itself, so
  each one is a separate component of the affinity graph and the k leading
  eigenvectors would not be determined), symmetric normalisation D^-1/2 W D^-1/2,
  the k leading eigenvectors with unit rows, Lloyd's k-means started from a
  deterministic farthest-point seeding, labels renumbered by first appearance,
  -1 for the excluded points.  The routine is deterministic and continuous away
  from exact ties, so running it on two Z's tests the Z's, not the clustering.
* ``segmentation_accuracy``: each cluster takes the majority ground-truth label of
  its members; the score is the mean over classes of the fraction of that class
  labelled correctly (Section 4.1.2).  Columns labelled -1 (either side) are
  skipped.
* ``outlier_flags``: the columns the method itself marks as outliers, from the
  column-sparse outlier estimate S of Eq. (1)/(2): column j is flagged when
  ||S[:, j]||_2 > delta ||M[:, j]||_2 (reading: the paper identifies outlier
  columns through the column support of S, Section 4.1.1, with a threshold it
  does not state; delta = 0.1 is used by default).
* ``oracle_constraints``: the success test of Section 4.1.1 -- the oracle
  constraints of the appendix (column space of Z inside the row space of the
  clean data, outlier estimate supported on the outlier columns) within a
  relative tolerance.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

__all__ = ["segment", "segmentation_accuracy", "oracle_constraints", "kmeans", "outlier_flags"]

OUTLIER_DELTA = 0.1


def kmeans(Y: np.ndarray, k: int, max_iter: int = 300):
    """Lloyd's k-means from a farthest-point seeding; returns (labels, inertia).

    Seeding: the point farthest from the centroid, then repeatedly the point
    farthest from the chosen ones (ties to the lowest index).  Assignment ties go
    to the lowest centre index."""
    c0 = int(np.argmax(np.sum((Y - Y.mean(axis=0)) ** 2, axis=1)))
    chosen = [c0]
    d2 = np.sum((Y - Y[c0]) ** 2, axis=1)
    for _ in range(1, k):
        j = int(np.argmax(d2))
        chosen.append(j)
        d2 = np.minimum(d2, np.sum((Y - Y[j]) ** 2, axis=1))
    centers = Y[chosen].copy()
    lab = None
    for _it in range(max_iter):
        dist = np.sum((Y[:, None, :] - centers[None, :, :]) ** 2, axis=2)
        new = np.argmin(dist, axis=1)
        if lab is not None and np.array_equal(new, lab):
            break
        lab = new
        for c in range(k):
            mem = Y[lab == c]
            if len(mem):
                centers[c] = mem.mean(axis=0)
    return lab, float(np.sum((Y - centers[lab]) ** 2))


def _canonical(labels: np.ndarray) -> np.ndarray:
    mapping: dict[int, int] = {}
    out = np.empty_like(labels)
    for i, v in enumerate(labels):
        if v not in mapping:
            mapping[int(v)] = len(mapping)
        out[i] = mapping[int(v)]
    return out


def segment(Z: np.ndarray, k: int, exclude: np.ndarray | None = None,
            rank_tol: float = 1e-6) -> np.ndarray:
    """Labels 0..k-1 for the n points from Z (n x n), Section 4.1.2 pipeline;
    points with exclude[j] True get -1 and stay out of the affinity."""
    n = Z.shape[0]
    U, s, _ = sla.svd(Z, full_matrices=False, lapack_driver="gesdd")
    r = int(np.sum(s > rank_tol * s[0])) if s.size and s[0] > 0 else 0
    r = max(r, 1)
    keep = np.ones(n, dtype=bool) if exclude is None else ~np.asarray(exclude, dtype=bool)
    Ur = U[keep, :r]
    W = np.abs(Ur @ Ur.T)
    d = W.sum(axis=1)
    d[d <= 0] = 1.0
    Dm = 1.0 / np.sqrt(d)
    L = W * Dm[:, None] * Dm[None, :]
    w, vec = sla.eigh(L)
    emb = vec[:, np.argsort(-w, kind="stable")[:k]]
    nrm = np.linalg.norm(emb, axis=1, keepdims=True)
    nrm[nrm == 0] = 1.0
    emb = emb / nrm
    lab, _ = kmeans(emb, k)
    out = -np.ones(n, dtype=np.int64)
    out[keep] = _canonical(lab)
    return out


def segmentation_accuracy(pred: np.ndarray, truth: np.ndarray) -> float:
    """Majority-vote cluster labels, then mean per-class recall (-1 ignored)."""
    keep = (truth >= 0) & (pred >= 0)
    pred, truth = pred[keep], truth[keep]
    assign = {}
    for c in np.unique(pred):
        vals, cnt = np.unique(truth[pred == c], return_counts=True)
        assign[int(c)] = int(vals[np.argmax(cnt)])
    mapped = np.array([assign[int(c)] for c in pred])
    recalls = [float(np.mean(mapped[truth == g] == g)) for g in np.unique(truth)]
    return float(np.mean(recalls))


def outlier_flags(S: np.ndarray, M: np.ndarray, delta: float = OUTLIER_DELTA) -> np.ndarray:
    """Boolean mask of the columns whose outlier estimate carries more than
    delta of the column's norm: ||S[:, j]||_2 > delta ||M[:, j]||_2."""
    s = np.sqrt(np.sum(np.asarray(S, dtype=np.float64) ** 2, axis=0))
    m = np.sqrt(np.sum(np.asarray(M, dtype=np.float64) ** 2, axis=0))
    return s > delta * m


def oracle_constraints(Z: np.ndarray, E: np.ndarray, L0: np.ndarray, outlier_cols: np.ndarray,
                       tol: float = 1e-4) -> tuple[bool, float, float]:
    """Appendix oracle constraints: P_{L0^T} Z = Z and the outlier estimate lives on
    the outlier columns, each within relative Frobenius tolerance ``tol``.

    L0 is the clean data with the outlier columns zeroed (m x n); ``outlier_cols``
    marks the columns of E's block that are outliers.  Returns (ok, ez, ee)."""
    Ul, sl, Vt = sla.svd(L0, full_matrices=False)
    r = int(np.sum(sl > 1e-10 * sl[0]))
    V = Vt[:r].T
    PZ = V @ (V.T @ Z)
    nz = np.linalg.norm(Z)
    ez = float(np.linalg.norm(Z - PZ) / nz) if nz > 0 else 0.0
    ne = np.linalg.norm(E)
    ee = float(np.linalg.norm(E[:, ~outlier_cols]) / ne) if ne > 0 else 0.0
    return (ez <= tol and ee <= tol), ez, ee
