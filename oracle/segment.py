"""Segmentation from an LRR coefficient matrix, and the paper's success criteria.

TEST INFRASTRUCTURE ONLY (see the oracle package docstring).

* ``segment``: Section 4.1.2 builds an affinity U U^T from the top left singular
  vectors of Z, embeds the points spectrally into k dimensions and runs k-means.
  The paper does not fix the number of vectors, the Laplacian, the k-means
  initialisation or tie breaking; the readings used here are: numerical rank
  #sigma > 1e-6 sigma_1, affinity |U U^T|, symmetric normalisation
  D^-1/2 W D^-1/2, the k leading eigenvectors with unit rows, Lloyd's k-means
  with k-means++ seeding from a fixed seed, 10 restarts, lowest inertia, ties to
  the lowest index, labels renumbered by first appearance.  The routine is
  deterministic in Z, so running it on two Z's tests the Z's, not the clustering.
* ``segmentation_accuracy``: each cluster takes the majority ground-truth label of
  its members; the score is the mean over classes of the fraction of that class
  labelled correctly (Section 4.1.2).  Columns with ground truth -1 are skipped.
* ``oracle_constraints``: the success test of Section 4.1.1 -- the oracle
  constraints of the appendix (column space of Z inside the row space of the
  clean data, outlier estimate supported on the outlier columns) within a
  relative tolerance.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

__all__ = ["segment", "segmentation_accuracy", "oracle_constraints", "kmeans"]


def kmeans(Y: np.ndarray, k: int, seed: int = 0, restarts: int = 10, max_iter: int = 300):
    """Lloyd's k-means with k-means++ seeding; returns (labels, inertia)."""
    rng = np.random.default_rng(seed)
    npts = Y.shape[0]
    best_lab, best_in = None, np.inf
    for _ in range(restarts):
        centers = np.empty((k, Y.shape[1]))
        centers[0] = Y[rng.integers(npts)]
        d2 = np.sum((Y - centers[0]) ** 2, axis=1)
        for c in range(1, k):
            tot = d2.sum()
            if tot <= 0:
                idx = int(rng.integers(npts))
            else:
                idx = int(np.searchsorted(np.cumsum(d2), rng.uniform(0, tot)))
                idx = min(idx, npts - 1)
            centers[c] = Y[idx]
            d2 = np.minimum(d2, np.sum((Y - centers[c]) ** 2, axis=1))
        lab = None
        for _it in range(max_iter):
            dist = np.sum((Y[:, None, :] - centers[None, :, :]) ** 2, axis=2)
            new = np.argmin(dist, axis=1)          # ties -> lowest centre index
            if lab is not None and np.array_equal(new, lab):
                break
            lab = new
            for c in range(k):
                mem = Y[lab == c]
                if len(mem):
                    centers[c] = mem.mean(axis=0)
        inertia = float(np.sum((Y - centers[lab]) ** 2))
        if inertia < best_in - 1e-12:
            best_in, best_lab = inertia, lab.copy()
    return best_lab, best_in


def _canonical(labels: np.ndarray) -> np.ndarray:
    mapping: dict[int, int] = {}
    out = np.empty_like(labels)
    for i, v in enumerate(labels):
        if v not in mapping:
            mapping[int(v)] = len(mapping)
        out[i] = mapping[int(v)]
    return out


def segment(Z: np.ndarray, k: int, seed: int = 0, rank_tol: float = 1e-6) -> np.ndarray:
    """Labels 0..k-1 for the n points from Z (n x n), Section 4.1.2 pipeline."""
    U, s, _ = sla.svd(Z, full_matrices=False, lapack_driver="gesdd")
    r = int(np.sum(s > rank_tol * s[0])) if s.size and s[0] > 0 else 0
    r = max(r, 1)
    Ur = U[:, :r]
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
    lab, _ = kmeans(emb, k, seed=seed)
    return _canonical(lab)


def segmentation_accuracy(pred: np.ndarray, truth: np.ndarray) -> float:
    """Majority-vote cluster labels, then mean per-class recall (-1 ignored)."""
    keep = truth >= 0
    pred, truth = pred[keep], truth[keep]
    assign = {}
    for c in np.unique(pred):
        vals, cnt = np.unique(truth[pred == c], return_counts=True)
        assign[int(c)] = int(vals[np.argmax(cnt)])
    mapped = np.array([assign[int(c)] for c in pred])
    recalls = [float(np.mean(mapped[truth == g] == g)) for g in np.unique(truth)]
    return float(np.mean(recalls))


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
