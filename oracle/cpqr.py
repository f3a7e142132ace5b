"""Interpolative decomposition by column-pivoted Householder QR.

Sec. 2.2, Def. 1: a column ID of C picks skeleton columns S, redundant columns
R and T with ||C_R - C_S T|| <= eps ||C||; the paper computes it by greedy
column-pivoted QR (cost O(m n |S|)).  Sec. 2.3, eq. e:t: one ID of the stacked
matrix serves both A_FR ~ A_FS T and A_RF ~ T^* A_SF.

Rules fixed here where the paper is silent:
* truncation: stop after k steps when the largest trailing column norm is
  <= tol * nu0, nu0 the largest column norm of C (= |R_00|);
* norms: recomputed exactly from the current trailing submatrix at every step
  (no downdating);
* ties: among trailing columns whose norm is >= (1 - TIE) * max, the one with
  the smallest global index is chosen (the uniform grid and the circular proxy
  create exactly equal norms);
* T = R11^{-1} R12, then rows of T are reordered to ascending skeleton ids and
  columns to ascending redundant ids.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

TIE = 1e-8


def householder_cpqr(C: np.ndarray, tol: float, gid: np.ndarray):
    """Column-pivoted Householder QR of C (m x n), truncated by the rule above.

    Returns (k, perm, Rtop) where perm is the column order (perm[:k] are the
    skeleton columns in pivot order) and Rtop is the k x n upper-trapezoidal
    factor in that column order.
    """
    A = np.array(C, dtype=np.complex128, copy=True)
    m, n = A.shape
    gid = np.asarray(gid)
    perm = np.arange(n)
    if n == 0:
        return 0, perm, np.zeros((0, 0), dtype=np.complex128)
    norms0 = np.sqrt(np.sum(np.abs(A) ** 2, axis=0))
    nu0 = norms0.max()
    k = 0
    for j in range(min(m, n)):
        nrm = np.sqrt(np.sum(np.abs(A[j:, j:]) ** 2, axis=0))
        mx = nrm.max()
        if mx <= tol * nu0:
            break
        cand = np.nonzero(nrm >= (1.0 - TIE) * mx)[0] + j
        p = cand[np.argmin(gid[perm[cand]])]
        if p != j:
            A[:, [j, p]] = A[:, [p, j]]
            perm[[j, p]] = perm[[p, j]]
        x = A[j:, j]
        xn = np.linalg.norm(x)
        phase = x[0] / abs(x[0]) if x[0] != 0 else 1.0
        alpha = -phase * xn
        v = x.copy()
        v[0] -= alpha
        vv = np.vdot(v, v).real
        if vv > 0:
            A[j:, j:] -= np.outer(v, (2.0 / vv) * (v.conj() @ A[j:, j:]))
        A[j, j] = alpha
        A[j + 1:, j] = 0.0
        k = j + 1
    return k, perm, np.triu(A[:k, :])


def interpolative_decomposition(C: np.ndarray, tol: float, gid: np.ndarray):
    """ID of C with skeleton/redundant columns in ascending global-index order.

    Returns (S, R, T): local column positions S (k), R (n-k), both sorted by
    gid, and T (k x (n-k)) with C[:, R] ~ C[:, S] @ T.
    """
    gid = np.asarray(gid)
    n = C.shape[1]
    k, perm, Rt = householder_cpqr(C, tol, gid)
    if k == 0:
        S = np.zeros(0, dtype=np.int64)
        R = perm[np.argsort(gid[perm], kind="stable")]
        return S, R, np.zeros((0, n), dtype=np.complex128)
    R11 = Rt[:, :k]
    R12 = Rt[:, k:]
    Tp = scipy.linalg.solve_triangular(R11, R12, lower=False) if n > k else np.zeros((k, 0), complex)
    sk, rd = perm[:k], perm[k:]
    os_ = np.argsort(gid[sk], kind="stable")
    or_ = np.argsort(gid[rd], kind="stable")
    return sk[os_].astype(np.int64), rd[or_].astype(np.int64), Tp[os_][:, or_]
