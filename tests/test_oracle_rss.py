"""Pins for the oracle's RS-S factorization and solve (oracle/rss.py).

* Degenerate kernel (1 + x.y)^q: every Schur complement of "diagonal + rank
  (q+1)(q+2)/2" stays in the same spaces (Woodbury), so every ID is exact and
  RS-S must reproduce the dense LU solve to rounding, at any depth.
* Dense-literal RS-S (oracle/dense_literal.py): the full-matrix application of
  the same operators agrees with the block-store version, including the
  skeleton sets, and the far-field entries that the ID drops are measured.
* Accuracy on the workload matrices: relres vs a dense solve below tol.
* Solve identities: linearity, multi-RHS = column-by-column, tol -> 0 gives
  the dense solution, tol >= 1 (k = 0 everywhere) runs.
* Ranks stay bounded across depths.
* Point sets that are not grids: ragged and empty boxes.
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import dense_literal, kernels, matvec, rss
from paper_2310_15458_amd import workloads as W


def _dense_solve(kern, P, b):
    return scipy.linalg.solve(kernels.dense_matrix(kern, P), b)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("n,leaf", [(16, 4), (24, 9), (32, 16)])
@pytest.mark.parametrize("tol", [1e-6, 1e-10])
def test_degenerate_kernel_is_exact(n, leaf, tol):
    P = W.grid_points(n)
    k = W.Kernel("degenerate", weight=1.0 / n ** 2, diag=1.0, q=2)
    F = rss.factor(P, k, tol, leaf)
    assert F.tree.D >= 3
    assert max(r.k for r in F.ledger) <= 6      # exact rank of the kernel
    b = W.rhs(n * n, 2, 5)
    assert _rel(rss.solve(F, b), _dense_solve(k, P, b)) < 1e-12


@pytest.mark.parametrize("kind,kappa,n,leaf", [("laplace", 0, 16, 4), ("helmholtz", 40, 24, 9),
                                               ("laplace", 0, 24, 9)])
def test_dense_literal_agrees(kind, kappa, n, leaf):
    P = W.grid_points(n)
    k = W.grid_kernel(kind, n, kappa)
    F = rss.factor(P, k, 1e-6, leaf)
    LF = dense_literal.factor_literal(P, k, 1e-6, leaf)
    assert F.skeletons.keys() == LF.skeletons.keys()
    for key in F.skeletons:
        assert np.array_equal(F.skeletons[key], LF.skeletons[key])
    b = W.rhs(n * n, 1, 2)[:, 0]
    x = rss.solve(F, b)
    assert _rel(x, dense_literal.solve_literal(LF, b)) < 1e-12
    # the entries the ID drops are of the size the ID promises
    ratios = [r.far_ratio for r in LF.records]
    assert max(ratios) <= 100.0
    # the block store holds exactly the full-matrix entries at each depth start
    for d, (act, Afull) in LF.snapshots.items():
        if d == F.tree.D:
            continue
        # fresh kernel entries between boxes more than 2 apart (Thm. a:bm)
        for b1 in range(4 ** d):
            for b2 in range(4 ** d):
                if F.tree.dist(d, b1, b2) > 2 and act[b1].size and act[b2].size:
                    blk = Afull[np.ix_(act[b1], act[b2])]
                    ref = kernels.entries(k, P, act[b1], act[b2])
                    assert np.allclose(blk, ref, rtol=0, atol=1e-14 * max(1, np.abs(ref).max()))


@pytest.mark.parametrize("kind,kappa", [("laplace", 0.0), ("helmholtz", 25.0), ("helmholtz", 50.0)])
def test_relres_below_tol(kind, kappa):
    n, leaf, tol = 32, 16, 1e-6
    P = W.grid_points(n)
    k = W.grid_kernel(kind, n, kappa)
    F = rss.factor(P, k, tol, leaf)
    b = W.rhs(n * n, 3, 11)
    x = rss.solve(F, b)
    A = kernels.dense_matrix(k, P)
    assert matvec.relres(A @ x, b) < tol
    assert _rel(x, scipy.linalg.solve(A, b)) < tol


def test_solve_identities():
    n, leaf = 24, 9
    P = W.grid_points(n)
    k = W.grid_kernel("helmholtz", n, 30.0)
    F = rss.factor(P, k, 1e-6, leaf)
    B = W.rhs(n * n, 8, 3)
    X = rss.solve(F, B)
    for j in range(8):
        assert np.allclose(rss.solve(F, B[:, j]), X[:, j], rtol=0, atol=1e-14 * np.abs(X).max())
    a, c = 0.3 - 2j, 1.7
    lin = rss.solve(F, a * B[:, 0] + c * B[:, 1])
    assert _rel(lin, a * X[:, 0] + c * X[:, 1]) < 1e-13


def test_tiny_tol_passes_through_to_dense():
    n, leaf = 16, 4
    P = W.grid_points(n)
    k = W.grid_kernel("laplace", n)
    F = rss.factor(P, k, 1e-15, leaf)
    assert all(r.r == 0 for r in F.ledger)           # every box keeps all points
    assert F.root_idx.size == n * n
    b = W.rhs(n * n, 1, 0)
    assert _rel(rss.solve(F, b), _dense_solve(k, P, b)) < 1e-12


def test_tol_one_eliminates_everything():
    n, leaf = 16, 4
    P = W.grid_points(n)
    k = W.grid_kernel("helmholtz", n, 20.0)
    F = rss.factor(P, k, 1.0, leaf)
    assert all(r.k == 0 for r in F.ledger)
    assert F.root_idx.size == 0
    x = rss.solve(F, W.rhs(n * n, 1, 0))
    assert np.all(np.isfinite(x))


def test_ranks_bounded_across_depths():
    # Fig. f:ranks prints no values (parity unpinned); the pin is that ranks
    # stay O(1): no depth's mean rank exceeds a fixed bound at tol 1e-6
    n, leaf = 48, 9
    P = W.grid_points(n)
    for kind, kappa, bound in [("laplace", 0, 40.0), ("helmholtz", 25.0, 48.0)]:
        F = rss.factor(P, W.grid_kernel(kind, n, kappa), 1e-6, leaf)
        means = [np.mean(F.ranks(d)) for d in range(F.tree.D, 1, -1)]
        assert len(means) == 3
        assert max(means) <= bound


def test_scattered_points_with_empty_boxes():
    rng = np.random.default_rng(9)
    # two clusters: many leaf boxes are empty, others ragged
    P = np.vstack([0.05 + 0.3 * rng.random((300, 2)), 0.6 + 0.35 * rng.random((200, 2))])
    k = W.Kernel("helmholtz", kappa=10.0, weight=1.0 / 500, diag=1.0)
    F = rss.factor(P, k, 1e-8, 12)
    assert F.tree.D >= 3
    counts = np.bincount(F.tree.box_of(F.tree.D), minlength=4 ** F.tree.D)
    assert (counts == 0).any()
    b = W.rhs(500, 2, 4)
    x = rss.solve(F, b)
    A = kernels.dense_matrix(k, P)
    assert matvec.relres(A @ x, b) < 1e-7


def test_shallow_tree_is_dense_lu():
    P = W.grid_points(8)
    k = W.grid_kernel("laplace", 8)
    F = rss.factor(P, k, 1e-6, 64)
    assert F.tree.D == 0 and not F.records
    b = W.rhs(64, 1, 0)
    assert _rel(rss.solve(F, b), _dense_solve(k, P, b)) < 1e-13
