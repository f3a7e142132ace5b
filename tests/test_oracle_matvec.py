"""Pins for the oracle's products with A and refinement (oracle/matvec.py).

The BTTB-FFT product and the blocked direct sum are exact linear algebra, so
both must equal the explicit dense product to rounding.  Refinement must
converge to the dense solution (the unique A^{-1} b).
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import kernels, matvec, rss
from paper_2310_15458_amd import workloads as W


@pytest.mark.parametrize("kind,kappa,n", [("laplace", 0, 16), ("helmholtz", 25.0, 24),
                                          ("helmholtz", 50.0, 40), ("laplace", 0, 64)])
def test_fft_and_direct_equal_dense(kind, kappa, n):
    P = W.grid_points(n)
    k = W.grid_kernel(kind, n, kappa)
    X = W.rhs(n * n, 3, 1)
    ref = kernels.dense_matrix(k, P) @ X
    scale = np.abs(ref).max()
    assert np.abs(matvec.fft_matvec(k, n, X) - ref).max() <= 1e-13 * scale
    assert np.abs(matvec.direct_matvec(k, P, X, block=100) - ref).max() <= 1e-13 * scale


def test_refinement_reaches_dense_solution():
    n, leaf = 32, 16
    P = W.grid_points(n)
    k = W.grid_kernel("helmholtz", n, 40.0)
    F = rss.factor(P, k, 1e-3, leaf)      # a loose factorization needs refining
    b = W.rhs(n * n, 2, 8)
    x, hist = matvec.refine(F, lambda v: matvec.fft_matvec(k, n, v), b, tol=1e-13)
    assert hist[-1] <= 1e-13 and len(hist) >= 2
    xd = scipy.linalg.solve(kernels.dense_matrix(k, P), b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-12
