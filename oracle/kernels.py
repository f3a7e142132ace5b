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
``weight``, ``diag`` and ``q``, and optionally the paper's discretizations
(Sec. 5): ``cell_diag`` with the cell side ``h`` puts the cell integral of K
on the diagonal (eqs. e:a1i, e:b2), and ``bump_a`` > 0 the scattering
potential b(x) = exp(-bump_a |x - bump_c|^2) (Sec. 5.2):

    A_ij = w s_i s_j K(x_i, x_j)  (i != j),   s_i = sqrt(b(x_i)) (1 without a bump),
    A_ii = d + (w / h^2) s_i^2 c(h)  with c(h) the cell integral (0 without cell_diag).

First-kind Laplace (eqs. e:a1, e:a1i): w = h^2, d = 0, cell_diag.
Lippmann-Schwinger Helmholtz (eqs. e:b1, e:b2): w = h^2 kappa^2, d = 1,
cell_diag and the bump.  Both stay symmetric (A_ij = A_ji).
"""
from __future__ import annotations

import numpy as np
import scipy.special

from . import cells


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


def point_scale(kern, X: np.ndarray) -> np.ndarray:
    """s(x) = sqrt(b(x)) of the scattering potential, or ones without one."""
    X = np.asarray(X, dtype=np.float64).reshape(-1, 2)
    a = float(getattr(kern, "bump_a", 0.0))
    if a <= 0.0:
        return np.ones(X.shape[0])
    c = getattr(kern, "bump_c", (0.5, 0.5))
    r2 = (X[:, 0] - c[0]) ** 2 + (X[:, 1] - c[1]) ** 2
    return np.exp(-0.5 * a * r2)


_CELL = {}


def diagonal(kern, X: np.ndarray) -> np.ndarray:
    """A_ii for the points X (rows): d, plus (w / h^2) s_i^2 c(h) with the cell
    integral when ``cell_diag`` is set."""
    X = np.asarray(X, dtype=np.float64).reshape(-1, 2)
    out = np.full(X.shape[0], complex(kern.diag))
    if getattr(kern, "cell_diag", False):
        key = (kern.kind, float(kern.kappa), float(kern.h))
        if key not in _CELL:
            _CELL[key] = cells.cell_integral(kern)
        out = out + (kern.weight / kern.h ** 2) * point_scale(kern, X) ** 2 * _CELL[key]
    return out


def entries(kern, P: np.ndarray, I: np.ndarray, J: np.ndarray) -> np.ndarray:
    """The block A[I, J] of the system matrix for global index arrays I, J into
    the point array P: w s_i s_j K(x_i, x_j) where i != j and the diagonal
    rule where i == j (eq. e:aij)."""
    I = np.asarray(I, dtype=np.int64)
    J = np.asarray(J, dtype=np.int64)
    if I.size == 0 or J.size == 0:
        return np.zeros((I.size, J.size), dtype=np.complex128)
    same = I[:, None] == J[None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        A = kern.weight * kernel_values(kern, P[I], P[J])
    if getattr(kern, "bump_a", 0.0) > 0.0:
        A = A * point_scale(kern, P[I])[:, None] * point_scale(kern, P[J])[None, :]
    if same.any():
        dg = diagonal(kern, P[I])
        ii, jj = np.nonzero(same)
        A[ii, jj] = dg[ii]
    return A


def proxy_entries(kern, G: np.ndarray, P: np.ndarray, I: np.ndarray) -> np.ndarray:
    """w K(y_p, x_i) s_i for proxy points y_p (rows) against box points x_i
    (Sec. 2.3, the matrix K_proxy,B of eq. e:proxy); never the diagonal rule.
    The column scale s_i of the box points is that of A's columns; a row scale
    of the far field does not change the column ID."""
    I = np.asarray(I, dtype=np.int64)
    return kern.weight * kernel_values(kern, G, P[I]) * point_scale(kern, P[I])[None, :]


def proxy_entries_t(kern, G: np.ndarray, P: np.ndarray, I: np.ndarray) -> np.ndarray:
    """(w s_i K(x_i, y_p))^* : the transposed proxy block of eq. e:con's second
    half, rows p, columns i."""
    I = np.asarray(I, dtype=np.int64)
    return (kern.weight * point_scale(kern, P[I])[:, None] * kernel_values(kern, P[I], G)).conj().T


def dense_matrix(kern, P: np.ndarray) -> np.ndarray:
    """The full N x N matrix (tiny N only)."""
    idx = np.arange(P.shape[0])
    return entries(kern, P, idx, idx)
