"""Reverse-mode gradient of the unrolled ALM and of the DFC combine (FP64, CPU).

Test infrastructure only (see the package header).  The map differentiated is
the fixed-count iteration of ``lrr.lrr_alm`` (literal Z-step form) with no stop
test, started from zero, followed for DFC by the column projection of
Algorithm 1.  Every step is differentiated by hand from its definition:

  J-step   J = SVT_tau(Z + Y2/mu) = U f(S) V^T with f(s) = (s - tau)_+.  The
           derivative of this spectral function of the singular values is
           self-adjoint; with G' = U^T G V it is
             U [A o sym(G') + B o skew(G')] V^T + (I - U U^T) G V diag(f(s)/s) V^T,
           A_ij = (f_i - f_j)/(s_i - s_j), A_ii = f'(s_i), B_ij = (f_i + f_j)/(s_i + s_j)
           (Candes, Sing-Long and Trzasko, IEEE TSP 2013).
  Z-step   Z = (I + A^T A)^{-1} (A^T (X - E + Y1/mu) + J - Y2/mu).
  E-step   column shrink e = (1 - theta/||q||)_+ q with theta = lambda/mu and
           q = X - A Z + Y1/mu; for ||q|| > theta the column Jacobian is
           (1 - theta/||q||) I + theta q q^T / ||q||^3, and de/dtheta = -q/||q||.
  duals    Y1 += mu (X - A Z - E),  Y2 += mu (Z - J);  mu follows the fixed
           schedule and carries no gradient.
  combine  Z_hat = P1 [J_1 ... J_t] with P1 = U1 U1^T the projector on the range
           of J_1; dP1 = (I - P1) dJ_1 J_1^+ + ((I - P1) dJ_1 J_1^+)^T
           (Golub and Pereyra, SIAM J. Numer. Anal. 1973).
  M        enters each block twice, as the dictionary A and through the block's
           columns X = M[:, C_i]; both contributions are summed.

The reference gradient is pinned to central finite differences of the forward
map in the tests.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from .lrr import ALMOptions, l21_shrink


@dataclass
class Tape:
    """States of the unrolled iteration: states[k] = (Z, E, Y1, Y2) before
    iteration k (k = 0 .. K), mus[k] the penalty used by iteration k."""
    X: np.ndarray
    A: np.ndarray
    lam: float
    states: list
    mus: list
    J: np.ndarray        # J of the last iteration
    Y: np.ndarray        # input of the last J-step


def _svd(Y):
    try:
        return sla.svd(Y, full_matrices=False, lapack_driver="gesdd")
    except np.linalg.LinAlgError:  # pragma: no cover
        return sla.svd(Y, full_matrices=False, lapack_driver="gesvd")


def svt_full(Y: np.ndarray, tau: float):
    """SVT_tau(Y) together with the full thin SVD it came from."""
    U, s, Vt = _svd(Y)
    f = np.maximum(s - tau, 0.0)
    return (U * f) @ Vt, U, s, Vt.T


def svt_backward(G: np.ndarray, Y: np.ndarray, tau: float) -> np.ndarray:
    """Cotangent of Y for J = SVT_tau(Y) given the cotangent G of J."""
    n, l = Y.shape
    if n < l:
        return svt_backward(G.T, Y.T, tau).T
    U, s, Vt = _svd(Y)
    V = Vt.T
    f = np.maximum(s - tau, 0.0)
    above = s > tau
    si, sj = s[:, None], s[None, :]
    fi, fj = f[:, None], f[None, :]
    both_above = above[:, None] & above[None, :]
    one_above = above[:, None] ^ above[None, :]
    A = np.zeros((l, l))
    A[both_above] = 1.0
    diff = si - sj
    with np.errstate(divide="ignore", invalid="ignore"):
        mixed = np.where(one_above, (fi - fj) / np.where(diff == 0, 1.0, diff), 0.0)
    A += mixed
    ssum = si + sj
    with np.errstate(divide="ignore", invalid="ignore"):
        B = np.where(ssum > 0, (fi + fj) / np.where(ssum > 0, ssum, 1.0), 0.0)
    Gp = U.T @ G @ V
    sym = 0.5 * (Gp + Gp.T)
    skew = 0.5 * (Gp - Gp.T)
    out = U @ (A * sym + B * skew) @ Vt
    with np.errstate(divide="ignore", invalid="ignore"):
        fos = np.where(above, f / np.where(s > 0, s, 1.0), 0.0)
    GV = G @ V
    out += (GV - U @ (U.T @ GV)) @ (fos[:, None] * Vt)
    return out


def shrink_backward(q: np.ndarray, ebar: np.ndarray, theta: float):
    """Cotangents (qbar, thetabar) of e = l21_shrink(q, theta) given ebar."""
    nq = np.sqrt(np.sum(q * q, axis=0))
    qbar = np.zeros_like(q)
    thetabar = 0.0
    big = nq > theta
    if np.any(big):
        qb, eb, nb = q[:, big], ebar[:, big], nq[big]
        dot = np.sum(qb * eb, axis=0)
        qbar[:, big] = (1.0 - theta / nb) * eb + theta * qb * (dot / nb ** 3)
        thetabar = float(-np.sum(dot / nb))
    return qbar, thetabar


def unrolled_forward(X: np.ndarray, A: np.ndarray, lam: float, opts: ALMOptions) -> Tape:
    """The fixed-count iteration of lrr_alm (literal form), recording its states."""
    if opts.fixed_iters <= 0:
        raise ValueError("the unrolled map needs fixed_iters > 0")
    X = np.asarray(X, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    m, l = X.shape
    n = A.shape[1]
    Z, E, Y1, Y2 = np.zeros((n, l)), np.zeros((m, l)), np.zeros((m, l)), np.zeros((n, l))
    chol = sla.cho_factor(np.eye(n) + A.T @ A, lower=True)
    mu = float(opts.mu0)
    states, mus = [], []
    J = np.zeros((n, l))
    Y = np.zeros((n, l))
    for _ in range(opts.fixed_iters):
        states.append((Z, E, Y1, Y2))
        mus.append(mu)
        Y = Z + Y2 / mu
        J = svt_full(Y, 1.0 / mu)[0]
        Z = sla.cho_solve(chol, A.T @ (X - E + Y1 / mu) + J - Y2 / mu)
        AZ = A @ Z
        E_new = l21_shrink(X - AZ + Y1 / mu, lam / mu)
        Y1 = Y1 + mu * (X - AZ - E_new)
        Y2 = Y2 + mu * (Z - J)
        E = E_new
        mu = min(opts.rho * mu, opts.mu_max)
    states.append((Z, E, Y1, Y2))
    return Tape(X=X, A=A, lam=float(lam), states=states, mus=mus, J=J, Y=Y)


def unrolled_backward(tape: Tape, Zbar: np.ndarray | None, Jbar: np.ndarray | None):
    """Cotangents (Xbar, Abar, lambar) of the unrolled map given those of its
    final Z and final J."""
    X, A = tape.X, tape.A
    m, l = X.shape
    n = A.shape[1]
    K = np.eye(n) + A.T @ A
    chol = sla.cho_factor(K, lower=True)
    Xbar = np.zeros((m, l))
    Abar = np.zeros((m, n))
    lambar = 0.0
    # cotangents of the state after the iteration being reversed
    cZ = np.zeros((n, l)) if Zbar is None else np.array(Zbar, dtype=np.float64)
    cE = np.zeros((m, l))
    cY1 = np.zeros((m, l))
    cY2 = np.zeros((n, l))
    cJ = np.zeros((n, l)) if Jbar is None else np.array(Jbar, dtype=np.float64)
    for k in range(len(tape.mus) - 1, -1, -1):
        Z0, E0, Y10, Y20 = tape.states[k]
        mu = tape.mus[k]
        tau, theta = 1.0 / mu, tape.lam / mu
        # recompute the iteration's intermediates
        Y = Z0 + Y20 / mu
        J = svt_full(Y, tau)[0]
        Pv = X - E0 + Y10 / mu
        Q = J - Y20 / mu
        Z = sla.cho_solve(chol, A.T @ Pv + Q)
        q = X - A @ Z + Y10 / mu
        # Y1' = Y1 + mu (X - A Z - E'),  Y2' = Y2 + mu (Z - J)
        nY1, nY2 = cY1.copy(), cY2.copy()
        Xbar += mu * cY1
        Zt = cZ - mu * (A.T @ cY1) + mu * cY2
        Abar -= mu * (cY1 @ Z.T)
        Et = cE - mu * cY1
        Jt = cJ - mu * cY2
        # E' = shrink(q, theta)
        qbar, thbar = shrink_backward(q, Et, theta)
        lambar += thbar / mu
        # q = X - A Z + Y1/mu
        Xbar += qbar
        Abar -= qbar @ Z.T
        Zt = Zt - A.T @ qbar
        nY1 += qbar / mu
        # Z = K^{-1} (A^T Pv + Q)
        R = sla.cho_solve(chol, Zt)
        Kbar = -R @ Z.T
        Abar += A @ (Kbar + Kbar.T)
        Abar += Pv @ R.T
        Pbar = A @ R
        Qbar = R
        # Pv = X - E + Y1/mu,  Q = J - Y2/mu
        Xbar += Pbar
        nE = -Pbar
        nY1 += Pbar / mu
        Jt = Jt + Qbar
        nY2 -= Qbar / mu
        # J = SVT(Z + Y2/mu)
        Ybar = svt_backward(Jt, Y, tau)
        cZ = Ybar
        nY2 += Ybar / mu
        cE, cY1, cY2 = nE, nY1, nY2
        cJ = np.zeros((n, l))
    return Xbar, Abar, lambar


def dfc_forward_backward(M: np.ndarray, lam: float, perm, offsets, opts: ALMOptions, dZ: np.ndarray):
    """Unrolled DFC-LRR (Algorithm 1 with fixed-count blocks) and the cotangents
    (Z, Mbar, lambar) of a loss with dL/dZ = dZ."""
    perm = np.asarray(perm, dtype=np.int64)
    tapes = dfc_forward(M, lam, perm, offsets, opts)
    Z, _ = dfc_combine(tapes, perm)
    Mbar, lambar = dfc_backward(tapes, perm, offsets, dZ)
    return Z, Mbar, lambar


def dfc_forward(M: np.ndarray, lam: float, perm, offsets, opts: ALMOptions):
    """The blocks' unrolled forward runs (tapes) of Algorithm 1."""
    M = np.asarray(M, dtype=np.float64)
    perm = np.asarray(perm, dtype=np.int64)
    offsets = np.asarray(offsets, dtype=np.int64)
    return [unrolled_forward(M[:, perm[offsets[i]:offsets[i + 1]]], M, lam, opts)
            for i in range(len(offsets) - 1)]


def dfc_backward(tapes, perm, offsets, dZ):
    """(Mbar, lambar) from the tapes of dfc_forward and dL/dZ of the combined estimate."""
    perm = np.asarray(perm, dtype=np.int64)
    offsets = np.asarray(offsets, dtype=np.int64)
    m, n = tapes[0].A.shape
    Mbar = np.zeros((m, n))
    lambar = 0.0
    Jbars = dfc_combine_backward(tapes, perm, dZ)
    for i, (tp, Jb) in enumerate(zip(tapes, Jbars)):
        Xb, Ab, lb = unrolled_backward(tp, None, Jb)
        cols = perm[offsets[i]:offsets[i + 1]]
        Mbar += Ab
        Mbar[:, cols] += Xb
        lambar += lb
    return Mbar, lambar


def _range_basis(tape: Tape):
    """U1, kept singular values s - tau and right vectors of the final J."""
    tau = 1.0 / tape.mus[-1]
    U, s, Vt = _svd(tape.Y)
    keep = s > tau
    return U[:, keep], s[keep] - tau, Vt[keep].T


def dfc_combine(tapes, perm):
    U1 = _range_basis(tapes[0])[0]
    Jcat = np.concatenate([tp.J for tp in tapes], axis=1)
    Zp = U1 @ (U1.T @ Jcat)
    n = Zp.shape[0]
    Z = np.empty((n, n))
    Z[:, perm] = Zp
    return Z, U1


def dfc_combine_backward(tapes, perm, dZ):
    """Cotangents of the blocks' final J given dL/dZ of the combined estimate."""
    U1, s1, V1 = _range_basis(tapes[0])
    Jcat = np.concatenate([tp.J for tp in tapes], axis=1)
    dZp = np.asarray(dZ, dtype=np.float64)[:, perm]
    dJcat = U1 @ (U1.T @ dZp)
    widths = [tp.J.shape[1] for tp in tapes]
    out = np.split(dJcat, np.cumsum(widths)[:-1], axis=1)
    out = [o.copy() for o in out]
    if U1.shape[1] > 0:
        # dL/dP1 = dZp Jcat^T;  J1bar += (I - P1)(P1bar + P1bar^T)(J1^+)^T
        pinvT = (U1 / s1) @ V1.T                    # (J1^+)^T = U1 diag(1/s) V1^T
        F = dZp @ (Jcat.T @ pinvT) + Jcat @ (dZp.T @ pinvT)
        out[0] += F - U1 @ (U1.T @ F)
    return out
