"""Pins for the oracle's interpolative decomposition (oracle/cpqr.py).

* Def. 1 bound: with the truncation rule, ||C_R - C_S T||_F <= sqrt(r) tol nu0
  (every trailing column norm is <= tol nu0 at truncation, and C_R - C_S T is
  exactly the trailing block in the orthogonal frame);
* T is the least-squares solution of C_S T = C_R;
* on tie-free random matrices the pivots and rank equal LAPACK's column-pivoted
  QR (geqp3) truncated by the same rule;
* ties go to the smallest global index; tol >= 1 gives k = 0; tiny tol on a
  full-rank matrix gives k = n.
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import cpqr


def _lowrank(m, n, rank, seed, decay=1e-1):
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((m, rank)) + 1j * rng.standard_normal((m, rank))
    V = rng.standard_normal((rank, n)) + 1j * rng.standard_normal((rank, n))
    s = decay ** np.arange(rank)
    return (U * s) @ V


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("tol", [1e-3, 1e-6, 1e-9])
def test_id_bound_and_lstsq(seed, tol):
    C = _lowrank(300, 40, 30, seed)
    gid = np.arange(40) * 3 + 5
    S, R, T = cpqr.interpolative_decomposition(C, tol, gid)
    nu0 = np.linalg.norm(C, axis=0).max()
    err = np.linalg.norm(C[:, R] - C[:, S] @ T)
    assert err <= np.sqrt(max(R.size, 1)) * tol * nu0 * (1 + 1e-8)
    if R.size and S.size:
        Tl = np.linalg.lstsq(C[:, S], C[:, R], rcond=None)[0]
        cond = np.linalg.cond(C[:, S])
        assert np.linalg.norm(T - Tl) <= 1e-14 * cond * max(1.0, np.linalg.norm(Tl))
    assert np.all(np.diff(gid[S]) > 0) and np.all(np.diff(gid[R]) > 0)
    assert sorted(np.concatenate([S, R]).tolist()) == list(range(40))


@pytest.mark.parametrize("seed", range(6))
def test_pivots_match_lapack_geqp3(seed):
    rng = np.random.default_rng(100 + seed)
    C = (rng.standard_normal((120, 25)) + 1j * rng.standard_normal((120, 25))) * \
        (0.5 ** np.arange(25))[None, :]
    C = C[:, rng.permutation(25)]
    tol = 1e-4
    k, perm, _ = cpqr.householder_cpqr(C, tol, np.arange(25))
    _, Rl, pl = scipy.linalg.qr(C, mode="economic", pivoting=True)
    d = np.abs(np.diag(Rl))
    kl = int(np.argmax(d <= tol * d[0])) if np.any(d <= tol * d[0]) else 25
    assert k == kl
    assert np.array_equal(perm[:k], pl[:k])


def test_ties_go_to_smallest_global_index():
    rng = np.random.default_rng(3)
    a = rng.standard_normal(50) + 1j * rng.standard_normal(50)
    b = rng.standard_normal(50) + 1j * rng.standard_normal(50)
    b *= np.linalg.norm(a) / np.linalg.norm(b)       # equal norms: an exact tie
    C = np.stack([b, a, 0.1 * a + 0.01 * b], axis=1)
    gid = np.array([9, 4, 1])
    k, perm, _ = cpqr.householder_cpqr(C, 1e-12, gid)
    assert perm[0] == 1                               # gid 4 < gid 9
    gid2 = np.array([2, 4, 1])
    k, perm, _ = cpqr.householder_cpqr(C, 1e-12, gid2)
    assert perm[0] == 0


def test_rank_edges():
    C = _lowrank(80, 20, 20, 1, decay=0.8)
    S, R, T = cpqr.interpolative_decomposition(C, 1.0, np.arange(20))
    assert S.size == 0 and R.size == 20
    S, R, T = cpqr.interpolative_decomposition(C, 1e-15, np.arange(20))
    assert S.size == 20 and R.size == 0 and T.shape == (20, 0)
    S, R, T = cpqr.interpolative_decomposition(np.zeros((10, 5), complex), 1e-6, np.arange(5))
    assert S.size == 0
