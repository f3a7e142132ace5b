"""Exact products with A and iterative refinement.

Sec. 5: on a uniform grid A is block-Toeplitz with Toeplitz blocks, so A x is
computed by FFT.  Here the generator g(dx, dy) = w K(h |(dx, dy)|), g(0,0) = d,
for dx, dy in [-(n-1), n-1], is embedded in a 2n x 2n circulant and applied by
2-D FFT.  A blocked direct sum serves point sets that are not grids.

The relative residual is ||A x - b|| / ||b|| per column (Tab. t:notations);
the maximum over columns is reported.
"""
from __future__ import annotations

import numpy as np

from . import kernels
from . import rss


def dense_matvec(kern, P, X):
    return kernels.dense_matrix(kern, P) @ X


def direct_matvec(kern, P, X, block: int = 2048):
    """sum_j A_ij x_j by blocks of rows (any point set, O(N^2))."""
    X = np.asarray(X, dtype=np.complex128)
    sq = X.ndim == 1
    if sq:
        X = X[:, None]
    N = P.shape[0]
    out = np.zeros((N, X.shape[1]), dtype=np.complex128)
    cols = np.arange(N)
    for i0 in range(0, N, block):
        rows = np.arange(i0, min(N, i0 + block))
        out[rows] = kernels.entries(kern, P, rows, cols) @ X
    return out[:, 0] if sq else out


def grid_generator(kern, n: int) -> np.ndarray:
    """g on the (2n-1) x (2n-1) offset lattice, indexed [dy + n - 1, dx + n - 1]:
    w K(h |(dx, dy)|), and 0 at the origin (the diagonal is added apart)."""
    h = 1.0 / n
    d = np.arange(-(n - 1), n)
    DX, DY = np.meshgrid(d, d, indexing="xy")
    pts = np.stack([DX.ravel() * h, DY.ravel() * h], axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        g = kern.weight * kernels.kernel_values(kern, pts, np.zeros((1, 2)))[:, 0]
    g = g.reshape(2 * n - 1, 2 * n - 1)
    g[n - 1, n - 1] = 0.0
    return g


def fft_matvec(kern, n: int, X):
    """A x for the n x n cell-centre grid with user index iy*n + ix, via a
    2n x 2n circulant embedding: A x = s * (G (s * x)) + diag(A) * x with G
    the Toeplitz part (zero diagonal) and s the point scale."""
    X = np.asarray(X, dtype=np.complex128)
    sq = X.ndim == 1
    if sq:
        X = X[:, None]
    P = _grid_points(n)
    s = kernels.point_scale(kern, P)
    dg = kernels.diagonal(kern, P)
    g = grid_generator(kern, n)
    m = 2 * n
    c = np.zeros((m, m), dtype=np.complex128)
    # circulant first column: c[dy mod m, dx mod m] = g(dy, dx)
    idx = np.arange(-(n - 1), n) % m
    c[np.ix_(idx, idx)] = g
    cf = np.fft.fft2(c)
    out = np.empty_like(X)
    for j in range(X.shape[1]):
        xp = np.zeros((m, m), dtype=np.complex128)
        xp[:n, :n] = (s * X[:, j]).reshape(n, n)
        y = np.fft.ifft2(cf * np.fft.fft2(xp))
        out[:, j] = s * y[:n, :n].ravel() + dg * X[:, j]
    return out[:, 0] if sq else out


def _grid_points(n: int) -> np.ndarray:
    """cell centres ((ix + 1/2) h, (iy + 1/2) h) in user order iy * n + ix"""
    h = 1.0 / n
    c = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(c, c, indexing="xy")
    return np.stack([X.ravel(), Y.ravel()], axis=1)


def relres(Ax, B) -> float:
    Ax = np.asarray(Ax).reshape(B.shape[0], -1)
    B = np.asarray(B).reshape(B.shape[0], -1)
    num = np.linalg.norm(Ax - B, axis=0)
    den = np.linalg.norm(B, axis=0)
    return float(np.max(num / np.where(den > 0, den, 1.0)))


def refine(F, matvec, B, tol: float = 1e-12, max_iter: int = 20):
    """x <- F^{-1} b, then x <- x + F^{-1} (b - A x) until the max column relres
    is <= tol.  Returns (x, relres history)."""
    x = rss.solve(F, B)
    hist = []
    for _ in range(max_iter + 1):
        r = np.asarray(B) - matvec(x).reshape(x.shape)
        rr = relres(np.asarray(B) - r, B)
        hist.append(rr)
        if rr <= tol:
            break
        x = x + rss.solve(F, r)
    return x, hist
