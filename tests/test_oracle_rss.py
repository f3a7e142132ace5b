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
* Ranks stay bounded across depths; the ledger matches independent counts.
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


@pytest.mark.parametrize("kind,kappa,growth", [("laplace", 0.0, 2.0), ("helmholtz", 25.0, 3.0),
                                                ("helmholtz", 50.0, 3.0)])
def test_ranks_bounded_across_depths(kind, kappa, growth):
    # Fig. f:ranks shows skeleton ranks that stay O(1) across levels for Laplace
    # and grow only with the box size in wavelengths for Helmholtz (Sec. 5.2:
    # O(kappa D) ranks); it prints no values, so the reading pinned here is:
    # at tol 1e-6 the leaf really compresses (mean rank well below the leaf
    # size), and no upper depth's mean rank exceeds `growth` times the leaf
    # mean (2x Laplace, 3x Helmholtz kappa <= 50).  n = 128 with 64-point
    # leaves gives D = 4 and three compressed depths of 64-point leaves.
    n, leaf = 128, 64
    P = W.grid_points(n)
    F = rss.factor(P, W.grid_kernel(kind, n, kappa), 1e-6, leaf)
    assert F.tree.D == 4
    means = {d: np.mean(F.ranks(d)) for d in range(F.tree.D, 1, -1)}
    assert len(means) == 3
    leaf_mean = means[F.tree.D]
    assert 4.0 <= leaf_mean <= 0.5 * leaf
    for d, mu in means.items():
        assert mu <= growth * leaf_mean, (d, mu, leaf_mean)
    # ranks never exceed the box's own size, and every box of a grid compresses
    for row in F.ledger:
        assert 0 < row.k < row.n


def _exact_householder_flops(m, n, k):
    # step j of a complex Householder QR touches the (m - j) x (n - j) trailing
    # block: one dot product and one update per column, 16 real flops per entry
    return sum(16.0 * (m - j) * (n - j) for j in range(k))


def test_ledger_matches_counts():
    # Every ledger row is checked against counts taken independently of it: the
    # box sizes from the tree and the active sets, the stored arrays of the
    # factor record, the kernel evaluations the oracle really makes, and the
    # operation counts of the textbook algorithms (leading terms).
    n, leaf = 32, 16
    P = W.grid_points(n)
    kern = W.grid_kernel("helmholtz", n, 30.0)
    # every kernel value the oracle computes goes through kernels.kernel_values
    calls = [0]
    real_values = rss.kernels.kernel_values

    def count_values(k, X, Y):
        out = real_values(k, X, Y)
        calls[0] += out.size
        return out

    rss.kernels.kernel_values = count_values
    try:
        F = rss.factor(P, kern, 1e-6, leaf)
    finally:
        rss.kernels.kernel_values = real_values
    npx = 128
    assert calls[0] > 0 and F.kernel_evals == calls[0]
    recs = {(r.depth, r.box): r for r in F.records}
    tree = F.tree
    # the active sets at the start of every depth
    active = {tree.D: tree.members(tree.D)}
    for d in range(tree.D, 2, -1):
        nxt = []
        for p in range(4 ** (d - 1)):
            nxt.append(np.sort(np.concatenate([F.skeletons.get((d, c), active[d][c])
                                               for c in tree.children(d - 1, p)])))
        active[d - 1] = nxt
    order = {d: list(tree.order(d)) for d in active}
    for row in F.ledger:
        d, b = row.depth, row.box
        assert row.n == active[d][b].size
        assert row.k + row.r == row.n
        # sizes of the neighbours when b is eliminated: processed boxes are
        # already reduced to their skeletons
        pos = order[d].index(b)
        done = set(order[d][:pos])

        def size(x):
            return F.skeletons[(d, x)].size if x in done else active[d][x].size
        assert row.m == 2 * sum(size(x) for x in tree.dist2(d, b)) + 2 * npx
        assert row.nN == sum(size(x) for x in tree.nbrs(d, b))
        m_, n_, k_, r_, q_ = row.m, row.n, row.k, row.r, row.k + row.nN
        exact = _exact_householder_flops(m_, n_, k_)
        assert abs(row.flops_id - exact) <= 16.0 * (m_ + n_ + k_) * k_ + 1.0
        if r_ == 0:
            assert row.flops_lu == row.flops_y == row.flops_schur == row.factor_entries == 0
            continue
        rec = recs[(d, b)]
        # complex LU: sum over pivots of 8 (r - j)^2 real flops, leading term
        lu_exact = sum(8.0 * (r_ - j) ** 2 for j in range(r_))
        assert abs(row.flops_lu - lu_exact) <= 8.0 * r_ * r_ + 1.0
        # two triangular solves with q right-hand sides, a q x r x q product
        assert row.flops_y == 2 * 4.0 * r_ * r_ * q_
        assert row.flops_schur == 8.0 * q_ * r_ * q_
        stored = rec.T.size + rec.lu[0].size + rec.X_SR.size + rec.X_NR.size + rec.X_RS.size + rec.X_RN.size
        assert row.factor_entries == stored
    tot = rss.ledger_totals(F)
    assert tot["flops_schur"] == sum(r.flops_schur for r in F.ledger) > 0


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


# --- four-colour schedule (Sec. 3's coloured variant; snapshot reading) ---

@pytest.mark.parametrize("kind,kappa,n,leaf", [("laplace", 0, 16, 4), ("helmholtz", 40, 24, 9),
                                               ("helmholtz", 25, 32, 16)])
def test_four_colour_dense_literal_agrees(kind, kappa, n, leaf):
    # the block-store oracle and the literal full-matrix one, both taking a
    # colour's IDs from the matrix before its first elimination
    P = W.grid_points(n)
    k = W.grid_kernel(kind, n, kappa)
    F = rss.factor(P, k, 1e-6, leaf, rss.Options(colours=4))
    LF = dense_literal.factor_literal(P, k, 1e-6, leaf, colours=4)
    assert F.skeletons.keys() == LF.skeletons.keys()
    for key in F.skeletons:
        assert np.array_equal(F.skeletons[key], LF.skeletons[key])
    b = W.rhs(n * n, 1, 2)[:, 0]
    assert _rel(rss.solve(F, b), dense_literal.solve_literal(LF, b)) < 1e-12
    assert max(r.far_ratio for r in LF.records) <= 100.0


@pytest.mark.parametrize("kind,kappa", [("laplace", 0.0), ("helmholtz", 25.0), ("helmholtz", 50.0)])
def test_four_colour_relres_below_tol(kind, kappa):
    n, leaf, tol = 32, 16, 1e-6
    P = W.grid_points(n)
    k = W.grid_kernel(kind, n, kappa)
    F = rss.factor(P, k, tol, leaf, rss.Options(colours=4))
    b = W.rhs(n * n, 3, 11)
    x = rss.solve(F, b)
    A = kernels.dense_matrix(k, P)
    assert matvec.relres(A @ x, b) < tol
    assert _rel(x, scipy.linalg.solve(A, b)) < tol


def test_four_colour_order_inside_a_colour_is_immaterial():
    # a colour is one concurrent step: eliminating its boxes in the reverse
    # order gives the same skeletons and, to rounding, the same factorization
    n, leaf = 32, 16
    P = W.grid_points(n)
    k = W.grid_kernel("helmholtz", n, 40.0)
    F1 = rss.factor(P, k, 1e-6, leaf, rss.Options(colours=4))
    F2 = rss.factor(P, k, 1e-6, leaf, rss.Options(colours=4, reverse_within_colour=True))
    for key in F1.skeletons:
        assert np.array_equal(F1.skeletons[key], F2.skeletons[key])
    b = W.rhs(n * n, 2, 4)
    assert _rel(rss.solve(F2, b), rss.solve(F1, b)) < 1e-12
    # and the schedule is another elimination order than the nine-colour one
    F9 = rss.factor(P, k, 1e-6, leaf)
    assert any(not np.array_equal(F1.skeletons[key], F9.skeletons[key]) for key in F1.skeletons)
