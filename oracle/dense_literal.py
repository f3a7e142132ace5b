"""RS-S applied literally to the full N x N matrix (tiny N only).

This is a bookkeeping check of rss.py.  It keeps the whole matrix A~ and
applies, box by box in the same order, the operators of Sec. 2.4 as row and
column operations on all N rows and columns:

  * sparsification (eq. e:s): rows R -= T^* rows S, columns R -= columns S T;
    the entries A~[R, F] and A~[F, R] that the ID makes small are measured and
    then set to exactly zero (F = every active index outside B and N(B));
  * elimination (eq. e:step): with X_RR = A~[R, R], rows S u N -= A~[SuN, R]
    X_RR^{-1} A~[R, :], columns S u N likewise, then A~[R, R] = I.

Nothing here uses the distance-2 block store, Thm. a:bm or the merge rule: the
compression matrix is read straight from A~ (rows of the distance-2 boxes'
active indices, Def. d:m).  So agreement with rss.py checks that the block
store holds exactly the entries the full elimination produces, and the
measured far-field entries check the proxy argument of Sec. 2.3 directly.

The solve builds each V_B = L S^* and W_B = S U of eq. e:sk as explicit N x N
matrices and applies x = W_1 ... W_m Z^{-1} V_m ... V_1 b (eq. e:alg), with
Z^{-1} the identity on eliminated indices and a dense solve on the root.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg

from . import cpqr, kernels
from .tree import Tree


@dataclasses.dataclass
class LiteralRecord:
    S: np.ndarray
    R: np.ndarray
    N: np.ndarray
    T: np.ndarray
    X_RR: np.ndarray
    X_SNR: np.ndarray   # rows S then N, columns R
    X_RSN: np.ndarray   # rows R, columns S then N
    far_ratio: float    # max |A~[F,R]|, |A~[R,F]| (2-norm) / (tol * nu0)


@dataclasses.dataclass
class LiteralFactorization:
    N: int
    records: list
    root_idx: np.ndarray
    root: np.ndarray
    snapshots: dict      # depth -> (list of active sets, A~ copy) at depth start
    skeletons: dict


def factor_literal(P, kern, tol, leaf, n_proxy=0, proxy_radius=1.25, min_depth=2, root=None, colours=9):
    """colours = 4: the four-colour schedule; every ID of a colour is taken
    from the matrix as it stands before the colour's first elimination."""
    P = np.asarray(P, dtype=np.float64)
    tree = Tree(P, leaf, root)
    N = tree.N
    A = kernels.dense_matrix(kern, P)
    npx = n_proxy or (64 if kern.kind == "laplace" else 128)
    records, snaps, skel = [], {}, {}
    if tree.D < min_depth:
        return LiteralFactorization(N, [], np.arange(N), A.copy(), {}, {})
    active = tree.members(tree.D)
    d = tree.D
    while True:
        snaps[d] = ([a.copy() for a in active], A.copy())

        def ident(b):
            I = active[b]
            Mb = tree.dist2(d, b)
            Midx = np.concatenate([active[m] for m in Mb]) if Mb else np.zeros(0, np.int64)
            G = tree.proxy_points(d, b, npx, proxy_radius)
            C = np.vstack([A[np.ix_(Midx, I)], A[np.ix_(I, Midx)].conj().T,
                           kernels.proxy_entries(kern, G, P, I),
                           kernels.proxy_entries_t(kern, G, P, I)])
            Sl, Rl, T = cpqr.interpolative_decomposition(C, tol, I)
            return Sl, Rl, T, np.sqrt(np.sum(np.abs(C) ** 2, axis=0)).max()

        order = tree.order(d, colours)
        snap_ids = {}
        for pos, b in enumerate(order):
            I = active[b]
            n = I.size
            if n == 0:
                continue
            if colours == 4 and (pos == 0 or tree.colour(d, order[pos - 1], 4) != tree.colour(d, b, 4)):
                # first box of a colour: the IDs of the whole colour, from this matrix
                c = tree.colour(d, b, 4)
                snap_ids = {x: ident(x) for x in order if tree.colour(d, x, 4) == c and active[x].size}
            Nb = tree.nbrs(d, b)
            Nidx = np.concatenate([active[x] for x in Nb]) if Nb else np.zeros(0, np.int64)
            Sl, Rl, T, nu0 = snap_ids[b] if colours == 4 else ident(b)
            skel[(d, b)] = I[Sl].copy()
            if Rl.size == 0:
                continue
            S, R = I[Sl], I[Rl]
            # sparsification on the full matrix
            A[R, :] -= T.conj().T @ A[S, :]
            A[:, R] -= A[:, S] @ T
            all_active = np.concatenate(active)
            near = np.concatenate([I, Nidx])
            F = np.setdiff1d(all_active, near)
            far = 0.0
            if F.size:
                far = max(np.linalg.norm(A[np.ix_(F, R)], 2), np.linalg.norm(A[np.ix_(R, F)], 2))
            ratio = far / (tol * nu0) if nu0 > 0 and tol > 0 else 0.0
            # every index outside R, S, N(B) is dropped from R's rows and columns
            rest = np.setdiff1d(np.arange(N), np.concatenate([R, S, Nidx]))
            A[np.ix_(R, rest)] = 0.0
            A[np.ix_(rest, R)] = 0.0
            SN = np.concatenate([S, Nidx])
            X_RR = A[np.ix_(R, R)].copy()
            X_SNR = A[np.ix_(SN, R)].copy()
            X_RSN = A[np.ix_(R, SN)].copy()
            # elimination of R on the full matrix
            A[np.ix_(SN, SN)] -= X_SNR @ np.linalg.solve(X_RR, X_RSN)
            A[np.ix_(SN, R)] = 0.0
            A[np.ix_(R, SN)] = 0.0
            A[np.ix_(R, R)] = np.eye(R.size)
            records.append(LiteralRecord(S, R, Nidx, T, X_RR, X_SNR, X_RSN, ratio))
            active[b] = S.copy()
        if d == min_depth:
            break
        pd = d - 1
        active = [np.sort(np.concatenate([active[c] for c in tree.children(pd, p)]))
                  for p in range(4 ** pd)]
        d = pd
    ridx = np.sort(np.concatenate(active))
    return LiteralFactorization(N, records, ridx, A[np.ix_(ridx, ridx)].copy(), snaps, skel)


def _V(N, rec):
    """V_B = L S^* restricted to the index space (P~ is index selection)."""
    Sst = np.eye(N, dtype=np.complex128)
    Sst[np.ix_(rec.R, rec.S)] = -rec.T.conj().T          # S^*: row R gets -T^* row S
    L = np.eye(N, dtype=np.complex128)
    SN = np.concatenate([rec.S, rec.N])
    Xi = np.linalg.inv(rec.X_RR)
    L[np.ix_(SN, rec.R)] = -rec.X_SNR @ Xi                 # rows S,N -= X_{SN,R} X_RR^{-1} rows R
    Lr = np.eye(N, dtype=np.complex128)
    Lr[np.ix_(rec.R, rec.R)] = Xi                           # scale the R block to identity
    return Lr @ L @ Sst


def _W(N, rec):
    """W_B = S U, so that V_B A W_B has an identity R block decoupled from the rest."""
    Ssp = np.eye(N, dtype=np.complex128)
    Ssp[np.ix_(rec.S, rec.R)] = -rec.T                    # S: column R gets -(column S) T
    U = np.eye(N, dtype=np.complex128)
    SN = np.concatenate([rec.S, rec.N])
    U[np.ix_(rec.R, SN)] = -np.linalg.solve(rec.X_RR, rec.X_RSN)
    return Ssp @ U


def solve_literal(LF: LiteralFactorization, b):
    b = np.asarray(b, dtype=np.complex128)
    z = b.copy()
    for rec in LF.records:
        z = _V(LF.N, rec) @ z
    if LF.root_idx.size:
        z[LF.root_idx] = scipy.linalg.solve(LF.root, z[LF.root_idx])
    for rec in reversed(LF.records):
        z = _W(LF.N, rec) @ z
    return z
