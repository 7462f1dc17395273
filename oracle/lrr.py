"""FP64 CPU oracle for LRR and DFC-LRR.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link
this module: only the test suite, the smoke check of the entry-point module and
the CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
library (it does not import the package that holds the GPU path).

What it computes
----------------
* Eq. (1)/(2) (Sections 1 and 2.2): for observations X (m x l) and dictionary
  A (m x n)

      min  ||Z||_* + lam ||E||_{2,1}   s.t.  X = A Z + E,

  where ||.||_{2,1} is the sum of the column l2 norms (Section 1).
* The solver is the inexact augmented-Lagrange-multiplier method that the paper
  names as its base LRR algorithm (Section 4 preamble).  The paper does not print
  its steps; they are written out here from the augmented Lagrangian of the split
  Z = J:

      L = ||J||_* + lam||E||_{2,1} + <Y1, X - A Z - E> + <Y2, Z - J>
          + mu/2 (||X - A Z - E||_F^2 + ||Z - J||_F^2),

  minimised block by block (J, then Z, then E), followed by dual ascent on Y1, Y2
  and the penalty schedule mu <- min(rho mu, mu_max).  Each minimisation has a
  closed form: singular-value soft-thresholding for J, a linear solve with
  (I + A^T A) for Z, column-wise l2 shrinkage for E.
* Algorithm 1 (DFC-LRR): the columns of M are split into t blocks C_i (the split
  is an input), each block is solved with M as the dictionary (Eq. 2), and the
  C step projects [Z_1 ... Z_t] onto the column space of Z_1 (Section 2.2).
* The alternative of the Section 2.2 footnote (``dfc_lrr_local``): each block
  is solved with C_i in both places of Eq. (1), so Z_i is l x l, and the C step
  is a low-rank approximation of diag(Z_1, ..., Z_t).  The paper does not name
  the approximation or its rank; the reading taken here is the best rank-k
  approximation in the Frobenius norm (truncated SVD), which for a
  block-diagonal matrix keeps the k largest singular triplets pooled over the
  blocks, with k = max_i rank(Z_i) by default (the k' of the run-time remark of
  Section 2.2); k = -1 keeps every triplet.

Readings where the paper is silent (each is listed in the design notes):
update order J -> Z -> E -> (Y1, Y2) -> mu; stop when both residuals are below
``tol`` in the entrywise max-norm, per block, measured before the multiplier
update; the returned estimate of a block is J at termination, which is exactly
low rank and available in factored form (Section 2.2 asks for a factored
estimate); the column space of Z_1 is spanned by the left singular vectors that
survive the last threshold; the same lam is used for every block.

Parity status: every public function here is pinned by the CPU tests
(closed forms, optimality certificates, brute force, invariants).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

__all__ = [
    "ALMOptions", "LRRResult", "DFCResult", "svt", "l21_shrink", "lrr_alm",
    "column_projection", "dfc_lrr", "dfc_lrr_local", "trivial_lambda", "objective", "dual_gap",
]


@dataclass
class ALMOptions:
    """Inexact-ALM constants (not printed in the paper; shared with the GPU path
    as explicit arguments, so parity does not depend on their values)."""

    mu0: float = 1e-6
    rho: float = 1.1
    mu_max: float = 1e10
    tol: float = 1e-8
    max_iter: int = 1000
    fixed_iters: int = 0          # > 0: run exactly this many iterations, no stop test
    solve_form: str = "literal"   # "literal": (I + A^T A); "pushthrough": (I + A A^T)


@dataclass
class LRRResult:
    Z: np.ndarray
    E: np.ndarray
    J: np.ndarray
    U: np.ndarray        # left singular vectors of J (n x r)
    s: np.ndarray        # singular values of J (r), already thresholded
    V: np.ndarray        # right singular vectors of J (l x r)
    Y1: np.ndarray
    Y2: np.ndarray
    mu: float            # penalty after the last update
    tau: float           # threshold 1/mu used by the last singular-value step
    iters: int
    res1: float          # ||X - A Z - E||_max at the last iteration
    res2: float          # ||Z - J||_max at the last iteration
    converged: bool

    @property
    def rank(self) -> int:
        return int(self.s.size)


@dataclass
class DFCResult:
    Z: np.ndarray                  # n x n, original column order
    S: np.ndarray                  # m x n, original column order
    blocks: list = field(default_factory=list)   # LRRResult per block
    U1: np.ndarray | None = None   # basis of the column space of Z_1
    combine_rank: int = 0          # rank of the combined estimate


def svt(Y: np.ndarray, tau: float):
    """Singular-value soft-thresholding: the proximal map of tau*||.||_*.

    Returns (U, s - tau, V) for the singular triplets with s > tau, so that
    SVT(Y) = U diag(s - tau) V^T.  A value exactly equal to tau contributes zero
    either way; it is not counted in the rank."""
    try:
        U, s, Vt = sla.svd(Y, full_matrices=False, lapack_driver="gesdd")
    except np.linalg.LinAlgError:  # pragma: no cover - gesdd convergence failure
        U, s, Vt = sla.svd(Y, full_matrices=False, lapack_driver="gesvd")
    keep = s > tau
    return U[:, keep], s[keep] - tau, Vt[keep, :].T


def l21_shrink(Q: np.ndarray, thr: float) -> np.ndarray:
    """Proximal map of thr*||.||_{2,1}: each column q becomes max(0, 1 - thr/||q||) q."""
    norms = np.sqrt(np.sum(Q * Q, axis=0))
    scale = np.zeros_like(norms)
    big = norms > thr
    scale[big] = 1.0 - thr / norms[big]
    return Q * scale[None, :]


def objective(Z: np.ndarray, E: np.ndarray, lam: float) -> float:
    """||Z||_* + lam ||E||_{2,1} (Eq. 1 / Eq. 2)."""
    return float(np.sum(sla.svdvals(Z)) + lam * np.sum(np.linalg.norm(E, axis=0)))


def dual_gap(X: np.ndarray, A: np.ndarray, Z: np.ndarray, E: np.ndarray, Y1: np.ndarray,
             lam: float) -> tuple[float, float]:
    """Weak-duality gap of Eq. (2) at (Z, E) with the multiplier Y1 as dual point.

    The Lagrange dual of Eq. (2) is  max <Q, X>  s.t. ||A^T Q||_2 <= 1 and every
    column of Q has l2 norm <= lam.  Y1 is scaled into that set, so
    primal - dual >= primal - optimum >= 0.  Returns (gap, primal)."""
    spec = float(sla.svdvals(A.T @ Y1)[0]) if Y1.size else 0.0
    cmax = float(np.max(np.linalg.norm(Y1, axis=0))) / lam if Y1.size else 0.0
    scale = max(1.0, spec, cmax)
    dual = float(np.sum(Y1 * X)) / scale
    primal = objective(Z, E, lam)
    return primal - dual, primal


def trivial_lambda(X: np.ndarray, A: np.ndarray) -> float:
    """Largest lam at which (Z, E) = (0, X) solves Eq. (2).

    At Z = 0, E = X (all columns nonzero) the E-subgradient forces the dual point
    Q = lam * X_bar (X with unit columns); optimality then needs ||A^T Q||_2 <= 1,
    i.e. lam <= 1 / ||A^T X_bar||_2."""
    Xb = X / np.linalg.norm(X, axis=0, keepdims=True)
    return 1.0 / float(sla.svdvals(A.T @ Xb)[0])


def lrr_alm(X: np.ndarray, A: np.ndarray, lam: float, opts: ALMOptions | None = None,
            trace=None) -> LRRResult:
    """Inexact ALM for Eq. (2): X = A Z + E (Eq. 1 when X = A).

    ``trace``, if given, is called after every iteration with a dict of the
    iterates (used by the invariant tests)."""
    opts = opts or ALMOptions()
    X = np.asarray(X, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    m, l = X.shape
    n = A.shape[1]
    if A.shape[0] != m:
        raise ValueError("dictionary and observations must have the same row count")
    Z = np.zeros((n, l))
    J = np.zeros((n, l))
    E = np.zeros((m, l))
    Y1 = np.zeros((m, l))
    Y2 = np.zeros((n, l))
    mu = float(opts.mu0)

    if opts.solve_form == "literal":
        # Z-step normal equations: (I + A^T A) Z = A^T (X - E + Y1/mu) + J - Y2/mu
        chol = sla.cho_factor(np.eye(n) + A.T @ A, lower=True)
    elif opts.solve_form == "pushthrough":
        # same solve through (I + A^T A)^{-1} = I - A^T (I + A A^T)^{-1} A
        chol = sla.cho_factor(np.eye(m) + A @ A.T, lower=True)
    else:
        raise ValueError(opts.solve_form)

    n_iter = opts.fixed_iters if opts.fixed_iters > 0 else opts.max_iter
    U = np.zeros((n, 0))
    s = np.zeros(0)
    V = np.zeros((l, 0))
    res1 = res2 = np.inf
    converged = False
    tau = 1.0 / mu
    it = 0
    for it in range(1, n_iter + 1):
        tau = 1.0 / mu
        # J-step: J = argmin ||J||_*/mu + 1/2 ||J - (Z + Y2/mu)||_F^2
        U, s, V = svt(Z + Y2 / mu, tau)
        J = (U * s) @ V.T
        # Z-step: minimiser of the quadratic part in Z
        if opts.solve_form == "literal":
            rhs = A.T @ (X - E + Y1 / mu) + J - Y2 / mu
            Z = sla.cho_solve(chol, rhs)
        else:
            Q = J - Y2 / mu
            W = sla.cho_solve(chol, (X - E + Y1 / mu) - A @ Q)
            Z = Q + A.T @ W
        AZ = A @ Z
        # E-step: E = argmin lam||E||_{2,1}/mu + 1/2 ||E - (X - A Z + Y1/mu)||_F^2
        E_prev = E
        E = l21_shrink(X - AZ + Y1 / mu, lam / mu)
        # residuals of the two constraints, then dual ascent and penalty update
        R1 = X - AZ - E
        R2 = Z - J
        Y1 = Y1 + mu * R1
        Y2 = Y2 + mu * R2
        mu_used = mu
        mu = min(opts.rho * mu, opts.mu_max)
        res1 = float(np.max(np.abs(R1))) if R1.size else 0.0
        res2 = float(np.max(np.abs(R2))) if R2.size else 0.0
        if trace is not None:
            trace(dict(k=it, Z=Z, J=J, E=E, E_prev=E_prev, Y1=Y1, Y2=Y2, mu=mu_used,
                       U=U, s=s, V=V, res1=res1, res2=res2))
        if opts.fixed_iters <= 0 and res1 < opts.tol and res2 < opts.tol:
            converged = True
            break
    return LRRResult(Z=Z, E=E, J=J, U=U, s=s, V=V, Y1=Y1, Y2=Y2, mu=mu, tau=tau,
                     iters=it, res1=res1, res2=res2, converged=converged)


def column_projection(U1: np.ndarray, blocks: list[np.ndarray]) -> np.ndarray:
    """C step of Algorithm 1: project [Z_1 ... Z_t] onto span(U1) (U1 orthonormal)."""
    Zcat = np.concatenate(blocks, axis=1)
    return U1 @ (U1.T @ Zcat)


def dfc_lrr(M: np.ndarray, lam: float, perm: np.ndarray, offsets: np.ndarray,
            opts: ALMOptions | None = None) -> DFCResult:
    """Algorithm 1 with a given D-step partition.

    Block i holds the original columns perm[offsets[i]:offsets[i+1]].  Every block
    is solved with the full M as dictionary (Eq. 2), so the rows of each block
    estimate index the original points; after the C step the columns are put
    back into the original order."""
    M = np.asarray(M, dtype=np.float64)
    m, n = M.shape
    perm = np.asarray(perm, dtype=np.int64)
    offsets = np.asarray(offsets, dtype=np.int64)
    if sorted(perm.tolist()) != list(range(n)):
        raise ValueError("perm is not a permutation")
    if offsets[0] != 0 or offsets[-1] != n or np.any(np.diff(offsets) <= 0):
        raise ValueError("bad offsets")
    results = []
    for i in range(len(offsets) - 1):
        cols = perm[offsets[i]:offsets[i + 1]]
        results.append(lrr_alm(M[:, cols], M, lam, opts))
    U1 = results[0].U
    Zp = column_projection(U1, [r.J for r in results])
    Z = np.empty((n, n))
    Z[:, perm] = Zp
    S = np.empty((m, n))
    S[:, perm] = np.concatenate([r.E for r in results], axis=1)
    return DFCResult(Z=Z, S=S, blocks=results, U1=U1)


def dfc_lrr_local(M: np.ndarray, lam: float, perm: np.ndarray, offsets: np.ndarray, rank: int = 0,
                  opts: ALMOptions | None = None) -> DFCResult:
    """The footnote alternative of Section 2.2 with a given D-step partition.

    Block i (original columns perm[offsets[i]:offsets[i+1]]) solves Eq. (1) with
    C_i as both dictionary and observations, so its estimate J_i = U_i s_i V_i^T is
    l_i x l_i and indexes the block's own points in rows and columns.  C step:
    the rank-k truncated SVD of diag(J_1, ..., J_t): the k largest singular values
    over all blocks are kept (ties: earlier block, then larger value first within
    a block's descending list), each block keeps its own triplets among them.
    k = 0 means max_i rank(J_i); k = -1 keeps all.  Z (n x n) holds block i's
    result at rows and columns perm[offsets[i]:offsets[i+1]] and zeros elsewhere."""
    M = np.asarray(M, dtype=np.float64)
    m, n = M.shape
    perm = np.asarray(perm, dtype=np.int64)
    offsets = np.asarray(offsets, dtype=np.int64)
    if sorted(perm.tolist()) != list(range(n)):
        raise ValueError("perm is not a permutation")
    if offsets[0] != 0 or offsets[-1] != n or np.any(np.diff(offsets) <= 0):
        raise ValueError("bad offsets")
    results = []
    for i in range(len(offsets) - 1):
        C = M[:, perm[offsets[i]:offsets[i + 1]]]
        results.append(lrr_alm(C, C, lam, opts))
    pool = [(float(r.s[j]), i, j) for i, r in enumerate(results) for j in range(r.s.size)]
    total = len(pool)
    if rank == 0:
        k = max(r.rank for r in results)
    elif rank < 0:
        k = total
    else:
        k = min(rank, total)
    # descending by value; equal values keep the pooled (block, position) order
    order = sorted(range(total), key=lambda q: -pool[q][0])
    kept = [[] for _ in results]
    for q in order[:k]:
        kept[pool[q][1]].append(pool[q][2])
    Z = np.zeros((n, n))
    for i, r in enumerate(results):
        cols = perm[offsets[i]:offsets[i + 1]]
        j = np.array(sorted(kept[i]), dtype=np.int64)
        Zi = (r.U[:, j] * r.s[j]) @ r.V[:, j].T if j.size else np.zeros((cols.size, cols.size))
        Z[np.ix_(cols, cols)] = Zi
    S = np.empty((m, n))
    S[:, perm] = np.concatenate([r.E for r in results], axis=1)
    return DFCResult(Z=Z, S=S, blocks=results, U1=None, combine_rank=k)
