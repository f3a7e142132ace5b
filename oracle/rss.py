"""Strong recursive skeletonization (RS-S): factorization and solve, CPU FP64.

Follows Sec. 2 of the paper step by step.

Factorization (Alg. a:fact):
  for depth d = D (leaves) .. 2, for every box B in the elimination order
  (tree.Tree.order: colour-major), apply the strong skeletonization operator
  Z(A; B) = V A W (eq. e:sk):
    1. ID of the compression matrix (Sec. 2.3, eqs. e:con, e:proxy, Rem. r:t)
         C = [A_{M,B}; A_{B,M}^*; K(proxy, B); K(B, proxy)^*]
       -> skeleton S, redundant R, interpolation T (cpqr.py);
    2. sparsification S^* (P^T A P) S (eq. e:s): with T the redundant rows and
       columns decouple from the far field, leaving
         X_RR = A_RR - T^* A_SR - A_RS T + T^* A_SS T
         X_RS = A_RS - T^* A_SS,   X_SR = A_SR - A_SS T
         X_RN = A_RN - T^* A_SN,   X_NR = A_NR - A_NS T;
    3. X_RR = L_R U_R and block elimination of R (eq. e:step): the Schur
       complement updates [A_SS A_SN; A_NS A_NN] -= [X_SR; X_NR] X_RR^{-1} [X_RS X_RN]
       (Rem. r:nn: only B's neighbours are touched);
    4. B keeps only S.
  Between depths, a parent owns the union of its children's skeletons
  (Sec. 2.5, Fig. f:merge).  Only interactions within box distance 2 are ever
  modified, so blocks of pairs further apart are fresh kernel evaluations
  (Thm. a:bm and the level theorem of Sec. 2.5).  After depth 2 the remaining
  indices are factored densely (the root; Sec. 2.5 footnote: the top level has
  no far field).

Four-colour schedule (Options.colours = 4; Sec. 3's coloured variant, where
only neighbours must differ in colour): the boxes of one colour are at
distance 2, so a box B' of the colour lies in M(B).  Reading: the colour is
one concurrent step taken from a snapshot -- every ID of the colour is
computed from the blocks as they stand before any of its eliminations (B's
compression matrix still holds all of B''s indices, a superset of the rows
a sequential order would give), then every box is sparsified, eliminated and
compacted.  Those steps commute exactly: B's sparsification reads only
blocks with B as an index, which no other box of the colour writes (Rem.
r:nn: B is not a neighbour of B'), and the Schur updates of two boxes meet
only additively on blocks between common neighbours.  The result is a valid
RS-S factorization in another order than the nine-colour one.

Storage: a dense block A[b, b'] for every ordered pair of boxes at distance
<= 2 at the current depth ("explicitly store the modified interactions for
every box", Sec. 3.3).  Each box's active index set is kept sorted by global
index.

Solve (Sec. 2.6): an upward pass in factorization order updating b(B) then
b(N), the root solve, then a downward pass in reverse order reading b(N) and
updating b(B):
  forward : z_R -= T^* z_S;  w = X_RR^{-1} z_R;  z_S -= X_SR w;  z_N -= X_NR w
  backward: z_R  = X_RR^{-1} (z_R - X_RS z_S - X_RN z_N);  z_S -= T z_R
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg

from . import cpqr, kernels
from .tree import Tree


@dataclasses.dataclass
class Options:
    n_proxy: int = 0            # 0 -> 64 for Laplace, 128 otherwise
    proxy_radius: float = 1.25  # proxy circle radius in box-side units
    min_depth: int = 2          # compress depths D .. min_depth
    colours: int = 9            # 9: colour (bx mod 3) + 3 (by mod 3); 4: (bx mod 2) + 2 (by mod 2)
    reverse_within_colour: bool = False  # four colours: eliminate a colour's boxes in descending id
                                         # order (tests of the snapshot reading: no effect but rounding)


@dataclasses.dataclass
class FactorRecord:
    depth: int
    box: int
    S: np.ndarray      # global ids, ascending
    R: np.ndarray      # global ids, ascending
    Nidx: np.ndarray   # global ids of the neighbours' active sets, box order
    T: np.ndarray      # k x r
    lu: tuple          # scipy lu_factor of X_RR
    X_SR: np.ndarray
    X_NR: np.ndarray
    X_RS: np.ndarray
    X_RN: np.ndarray


@dataclasses.dataclass
class LedgerRow:
    depth: int
    box: int
    n: int
    k: int
    r: int
    m: int
    nN: int
    flops_id: float
    flops_lu: float
    flops_y: float
    flops_schur: float
    factor_entries: int


@dataclasses.dataclass
class Factorization:
    tree: Tree
    kern: object
    tol: float
    records: list
    root_idx: np.ndarray
    root_lu: tuple
    ledger: list
    skeletons: dict           # (depth, box) -> sorted global ids kept
    kernel_evals: int = 0

    def ranks(self, d: int) -> list:
        return [r.k for r in self.ledger if r.depth == d]


class _State:
    """Active sets and the block store at one depth."""

    def __init__(self, tree: Tree, d: int, active: list):
        self.tree = tree
        self.d = d
        self.active = active          # list of sorted global id arrays
        self.blocks = {}              # (b, b2) -> ndarray


def _default_npx(kern, n_proxy):
    if n_proxy:
        return int(n_proxy)
    return 64 if kern.kind == "laplace" else 128


def _stencil_pairs(tree: Tree, d: int):
    nb = 1 << d
    for b in range(nb * nb):
        for b2 in [b] + tree.ring(d, b, 1) + tree.ring(d, b, 2):
            yield b, b2


def _leaf_state(tree: Tree, kern, P, counter) -> _State:
    d = tree.D
    st = _State(tree, d, tree.members(d))
    for b, b2 in _stencil_pairs(tree, d):
        st.blocks[(b, b2)] = kernels.entries(kern, P, st.active[b], st.active[b2])
        counter[0] += st.active[b].size * st.active[b2].size
    return st


def _compression_matrix(st: _State, kern, P, b, npx, c_r, counter):
    """C = [A_{M,B}; A_{B,M}^*; K(proxy,B); K(B,proxy)^*] (eqs. e:con, e:proxy)."""
    tree, d = st.tree, st.d
    I = st.active[b]
    rows = []
    Mb = tree.dist2(d, b)
    for m in Mb:
        rows.append(st.blocks[(m, b)])
    for m in Mb:
        rows.append(st.blocks[(b, m)].conj().T)
    G = tree.proxy_points(d, b, npx, c_r)
    rows.append(kernels.proxy_entries(kern, G, P, I))
    # K(B, proxy)^*: entry (p, i) = conj(w K(x_i, y_p))
    rows.append(kernels.proxy_entries_t(kern, G, P, I))
    counter[0] += 2 * npx * I.size
    return np.vstack(rows) if rows else np.zeros((0, I.size), complex)


def _skel_id(st: _State, kern, P, b, tol, opts, counter):
    """The ID of box b from the current blocks (Def. 1, eqs. e:con, e:proxy):
    (Sl, Rl, T, m), or None for an empty box."""
    I = st.active[b]
    if I.size == 0:
        return None
    npx = _default_npx(kern, opts.n_proxy)
    C = _compression_matrix(st, kern, P, b, npx, opts.proxy_radius, counter)
    Sl, Rl, T = cpqr.interpolative_decomposition(C, tol, I)
    return Sl, Rl, T, C.shape[0]


def _skel(st: _State, kern, P, b, tol, opts, records, ledger, skeletons, counter, ident=None):
    """Strong skeletonization of box b; ident: its ID when already taken
    (the four-colour schedule's snapshot), else computed here."""
    tree, d = st.tree, st.d
    I = st.active[b]
    n = I.size
    if n == 0:
        return
    if ident is None:
        ident = _skel_id(st, kern, P, b, tol, opts, counter)
    Sl, Rl, T, m = ident
    k, r = Sl.size, Rl.size
    Nb = tree.nbrs(d, b)
    nN = sum(st.active[x].size for x in Nb)
    idf = 4.0 * (4.0 * m * n * k - 2.0 * (m + n) * k * k + 4.0 * k ** 3 / 3.0)
    skeletons[(d, b)] = I[Sl].copy()
    if r == 0:  # k == n: the box passes through unchanged
        ledger.append(LedgerRow(d, b, n, k, 0, m, nN, idf, 0.0, 0.0, 0.0, 0))
        return
    Abb = st.blocks[(b, b)]
    A_RR = Abb[np.ix_(Rl, Rl)]
    A_RS = Abb[np.ix_(Rl, Sl)]
    A_SR = Abb[np.ix_(Sl, Rl)]
    A_SS = Abb[np.ix_(Sl, Sl)]
    if Nb:
        A_RN = np.hstack([st.blocks[(b, x)][Rl, :] for x in Nb])
        A_SN = np.hstack([st.blocks[(b, x)][Sl, :] for x in Nb])
        A_NR = np.vstack([st.blocks[(x, b)][:, Rl] for x in Nb])
        A_NS = np.vstack([st.blocks[(x, b)][:, Sl] for x in Nb])
    else:
        A_RN = np.zeros((r, 0), complex)
        A_SN = np.zeros((k, 0), complex)
        A_NR = np.zeros((0, r), complex)
        A_NS = np.zeros((0, k), complex)
    Th = T.conj().T
    # sparsification (eq. e:s)
    X_SR = A_SR - A_SS @ T
    X_RS = A_RS - Th @ A_SS
    X_RR = A_RR - Th @ A_SR - A_RS @ T + Th @ A_SS @ T
    X_RN = A_RN - Th @ A_SN
    X_NR = A_NR - A_NS @ T
    # elimination of R (eq. e:step)
    lu = scipy.linalg.lu_factor(X_RR, check_finite=False)
    if np.any(np.diag(lu[0]) == 0):
        raise np.linalg.LinAlgError(f"singular X_RR at depth {d} box {b}")
    Y = scipy.linalg.lu_solve(lu, np.hstack([X_RS, X_RN]), check_finite=False)
    U = np.vstack([X_SR, X_NR]) @ Y
    # scatter the Schur update into the stored blocks (Rem. r:nn)
    targets = [b] + Nb
    rows = [Sl] + [np.arange(st.active[x].size) for x in Nb]
    offs = np.cumsum([0] + [len(x) for x in rows])
    for i1, t1 in enumerate(targets):
        for i2, t2 in enumerate(targets):
            blk = st.blocks[(t1, t2)]
            blk[np.ix_(rows[i1], rows[i2])] -= U[offs[i1]:offs[i1 + 1], offs[i2]:offs[i2 + 1]]
    Nidx = np.concatenate([st.active[x] for x in Nb]) if Nb else np.zeros(0, np.int64)
    records.append(FactorRecord(d, b, I[Sl].copy(), I[Rl].copy(), Nidx, T, lu,
                                X_SR, X_NR, X_RS, X_RN))
    ledger.append(LedgerRow(d, b, n, k, r, m, nN, idf, 8.0 / 3.0 * r ** 3,
                            8.0 * r * r * (k + nN), 8.0 * (k + nN) ** 2 * r,
                            T.size + r * r + 2 * (X_SR.size + X_NR.size)))
    # drop R from every stored block of B
    for b2 in [b] + tree.ring(d, b, 1) + tree.ring(d, b, 2):
        st.blocks[(b, b2)] = st.blocks[(b, b2)][Sl, :]
        st.blocks[(b2, b)] = st.blocks[(b2, b)][:, Sl]
    st.active[b] = I[Sl].copy()


def _assemble(tree, kern, P, d_child, child_state: _State, boxes_i, boxes_j, counter):
    """Block over the union of the child boxes' active sets: a stored block
    where the two child boxes are within distance 2, a fresh kernel block
    otherwise.  Rows/cols returned in ascending global id order."""
    Ii = np.concatenate([child_state.active[c] for c in boxes_i]) if boxes_i else np.zeros(0, np.int64)
    Ij = np.concatenate([child_state.active[c] for c in boxes_j]) if boxes_j else np.zeros(0, np.int64)
    out = np.zeros((Ii.size, Ij.size), dtype=np.complex128)
    oi = np.cumsum([0] + [child_state.active[c].size for c in boxes_i])
    oj = np.cumsum([0] + [child_state.active[c].size for c in boxes_j])
    for a, c in enumerate(boxes_i):
        for bb, c2 in enumerate(boxes_j):
            if tree.dist(d_child, c, c2) <= 2:
                blk = child_state.blocks[(c, c2)]
            else:
                blk = kernels.entries(kern, P, child_state.active[c], child_state.active[c2])
                counter[0] += blk.size
            out[oi[a]:oi[a + 1], oj[bb]:oj[bb + 1]] = blk
    pi = np.argsort(Ii, kind="stable")
    pj = np.argsort(Ij, kind="stable")
    return Ii[pi], Ij[pj], out[np.ix_(pi, pj)]


def _transition(st: _State, kern, P, counter) -> _State:
    """Depth d -> d-1 (Sec. 2.5, Fig. f:merge; Sec. 3.3)."""
    tree, d = st.tree, st.d
    pd = d - 1
    npb = 1 << pd
    kids = [tree.children(pd, p) for p in range(npb * npb)]
    active = []
    for p in range(npb * npb):
        Ip = np.concatenate([st.active[c] for c in kids[p]])
        active.append(np.sort(Ip))
    nst = _State(tree, pd, active)
    for p, p2 in _stencil_pairs(tree, pd):
        _, _, blk = _assemble(tree, kern, P, d, st, kids[p], kids[p2], counter)
        nst.blocks[(p, p2)] = blk
    return nst


def factor(P: np.ndarray, kern, tol: float, leaf: int, opts: Options | None = None,
           root=None) -> Factorization:
    """RS-S factorization (Alg. a:fact with the multilevel recursion of Sec. 2.5)."""
    opts = opts or Options()
    P = np.asarray(P, dtype=np.float64)
    tree = Tree(P, leaf, root)
    counter = [0]
    records, ledger, skeletons = [], [], {}
    if tree.D >= opts.min_depth:
        st = _leaf_state(tree, kern, P, counter)
        d = tree.D
        while True:
            if opts.colours == 4:
                order = tree.order(d, 4)
                for c in range(4):
                    boxes = [b for b in order if tree.colour(d, b, 4) == c]
                    ids = {b: _skel_id(st, kern, P, b, tol, opts, counter) for b in boxes}
                    for b in (boxes[::-1] if opts.reverse_within_colour else boxes):
                        _skel(st, kern, P, b, tol, opts, records, ledger, skeletons, counter, ids[b])
            else:
                for b in tree.order(d):
                    _skel(st, kern, P, b, tol, opts, records, ledger, skeletons, counter)
            if d == opts.min_depth:
                break
            st = _transition(st, kern, P, counter)
            d -= 1
        boxes = list(range(4 ** d))
        ridx, _, Aroot = _assemble(tree, kern, P, d, st, boxes, boxes, counter)
    else:
        ridx = np.arange(tree.N)
        Aroot = kernels.dense_matrix(kern, P)
        counter[0] += Aroot.size
    root_lu = scipy.linalg.lu_factor(Aroot, check_finite=False) if ridx.size else None
    if root_lu is not None and np.any(np.diag(root_lu[0]) == 0):
        raise np.linalg.LinAlgError("singular root matrix")
    return Factorization(tree, kern, tol, records, ridx, root_lu, ledger, skeletons, counter[0])


def solve(F: Factorization, B: np.ndarray) -> np.ndarray:
    """Apply the factored inverse (Sec. 2.6) to B (N x nrhs); returns a new array."""
    z = np.array(B, dtype=np.complex128, copy=True)
    squeeze = z.ndim == 1
    if squeeze:
        z = z[:, None]
    for rec in F.records:
        z[rec.R] -= rec.T.conj().T @ z[rec.S]
        w = scipy.linalg.lu_solve(rec.lu, z[rec.R], check_finite=False)
        z[rec.S] -= rec.X_SR @ w
        if rec.Nidx.size:
            z[rec.Nidx] -= rec.X_NR @ w
    if F.root_idx.size:
        z[F.root_idx] = scipy.linalg.lu_solve(F.root_lu, z[F.root_idx], check_finite=False)
    for rec in reversed(F.records):
        t = z[rec.R] - rec.X_RS @ z[rec.S]
        if rec.Nidx.size:
            t -= rec.X_RN @ z[rec.Nidx]
        z[rec.R] = scipy.linalg.lu_solve(rec.lu, t, check_finite=False)
        z[rec.S] -= rec.T @ z[rec.R]
    return z[:, 0] if squeeze else z


def ledger_totals(F: Factorization) -> dict:
    L = F.ledger
    return {
        "flops_id": sum(r.flops_id for r in L),
        "flops_lu": sum(r.flops_lu for r in L),
        "flops_y": sum(r.flops_y for r in L),
        "flops_schur": sum(r.flops_schur for r in L),
        "factor_entries": sum(r.factor_entries for r in L),
        "kernel_evals": F.kernel_evals,
    }
