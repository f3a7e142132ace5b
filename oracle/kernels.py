"""Matrix entries of the dense kernel system A x = b.

Sec. 1, eqs. e:axb / e:aij: A_ij = K(x_i, x_j) for i != j.  The workloads use
A_ij = w K(|x_i - x_j|) off the diagonal and a constant A_ii = d (Sec. 5
discretizes by piecewise-constant collocation with w = h^2, eqs. e:a1, e:b1).

Kernels:
* Laplace    K(r) = -log(r) / (2 pi)               (Sec. 5.1, eq. e:kernel_laplace)
* Helmholtz  K(r) = (i/4) H0^(1)(kappa r),
             H0^(1) = J0 + i Y0                      (Sec. 5.2, eq. e:kernel_helmholtz)
* degenerate K(x, y) = (1 + x.y)^q: exactly low rank, (q+1)(q+2)/2; not from the
  paper, used to make every interpolative decomposition exact so the whole
  algebra reduces to a dense LU solve.

The kernel description is any object with attributes ``kind``, ``kappa``,
``weight``, ``diag`` and ``q``.
"""
from __future__ import annotations

import numpy as np
import scipy.special


def kernel_values(kern, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """K(x_i, y_j) for every row x_i of X (m x 2) and y_j of Y (n x 2), with no
    weight and no diagonal rule.  Returns an m x n complex128 array."""
    X = np.asarray(X, dtype=np.float64).reshape(-1, 2)
    Y = np.asarray(Y, dtype=np.float64).reshape(-1, 2)
    if kern.kind == "degenerate":
        dot = X[:, None, 0] * Y[None, :, 0] + X[:, None, 1] * Y[None, :, 1]
        return ((1.0 + dot) ** int(kern.q)).astype(np.complex128)
    dx = X[:, None, 0] - Y[None, :, 0]
    dy = X[:, None, 1] - Y[None, :, 1]
    r = np.sqrt(dx * dx + dy * dy)
    if kern.kind == "laplace":
        with np.errstate(divide="ignore"):
            return (-np.log(r) / (2.0 * np.pi)).astype(np.complex128)
    if kern.kind == "helmholtz":
        with np.errstate(invalid="ignore"):
            return 0.25j * scipy.special.hankel1(0, kern.kappa * r)
    raise ValueError(f"unknown kernel kind {kern.kind!r}")


def entries(kern, P: np.ndarray, I: np.ndarray, J: np.ndarray) -> np.ndarray:
    """The block A[I, J] of the system matrix for global index arrays I, J into
    the point array P: w K(x_i, x_j) where i != j and d where i == j
    (eq. e:aij with a constant diagonal)."""
    I = np.asarray(I, dtype=np.int64)
    J = np.asarray(J, dtype=np.int64)
    if I.size == 0 or J.size == 0:
        return np.zeros((I.size, J.size), dtype=np.complex128)
    same = I[:, None] == J[None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        A = kern.weight * kernel_values(kern, P[I], P[J])
    A[same] = kern.diag
    return A


def proxy_entries(kern, G: np.ndarray, P: np.ndarray, I: np.ndarray) -> np.ndarray:
    """w K(y_p, x_i) for proxy points y_p (rows) against box points x_i
    (Sec. 2.3, the matrix K_proxy,B of eq. e:proxy); never the diagonal rule."""
    return kern.weight * kernel_values(kern, G, P[np.asarray(I, dtype=np.int64)])


def dense_matrix(kern, P: np.ndarray) -> np.ndarray:
    """The full N x N matrix (tiny N only)."""
    idx = np.arange(P.shape[0])
    return entries(kern, P, idx, idx)
