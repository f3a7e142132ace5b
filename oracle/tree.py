"""Hierarchical domain decomposition (Sec. 2.1) and box lists.

* The root square [x0, x0+s0] x [y0, y0+s0] is split into four equal children
  recursively; depth d has a 2^d x 2^d grid of boxes (the paper's level
  l = d + 1; its level 1 is the root).
* The leaf depth is the smallest depth at which no box holds more than ``leaf``
  points (Sec. 2.1: subdivide until every box holds O(1) points).
* A point belongs to box (bx, by) = (min(floor((x-x0)/s), 2^d-1), same for y),
  s = s0 / 2^d.  Box id = by * 2^d + bx (row-major).
* N(B): boxes at Chebyshev box distance exactly 1 (Sec. 2.1, at most 8).
* M(B) = N(N(B)) minus (N(B) and B): distance exactly 2 (Def. d:m, at most 16).
* Colour (bx mod 3) + 3 (by mod 3): boxes of one colour are at distance >= 3,
  so by Rem. r:t and Rem. r:nn they read and write disjoint blocks.  Within a
  depth the oracle visits colours 0..8 and, inside a colour, boxes in id
  order -- one admissible instance of "a given ordering" in Alg. a:fact.
* The four-colour schedule (colour (bx mod 2) + 2 (by mod 2)) of Sec. 3's
  coloured variant only keeps neighbours apart: boxes of one colour are at
  distance 2, share neighbours and see each other in their compression
  matrices (rss.factor's snapshot reading).
"""
from __future__ import annotations

import numpy as np

MAX_DEPTH = 15


class Tree:
    def __init__(self, P: np.ndarray, leaf: int, root=None):
        P = np.asarray(P, dtype=np.float64)
        self.P = P
        self.N = P.shape[0]
        if root is None:
            lo = P.min(axis=0) if self.N else np.zeros(2)
            hi = P.max(axis=0) if self.N else np.ones(2)
            if self.N and lo.min() >= 0.0 and hi.max() <= 1.0:
                root = (0.0, 0.0, 1.0)
            else:
                side = float(max(hi - lo)) * (1.0 + 1e-12) or 1.0
                root = (float(lo[0]), float(lo[1]), side)
        self.x0, self.y0, self.s0 = root
        self.leaf = int(leaf)
        d = 0
        while True:
            counts = np.bincount(self.box_of(d), minlength=4 ** d)
            if self.N == 0 or counts.max() <= self.leaf:
                break
            d += 1
            if d > MAX_DEPTH:
                raise ValueError("tree deeper than the supported maximum")
        self.D = d

    # -- geometry ---------------------------------------------------------
    def side(self, d: int) -> float:
        return self.s0 / (1 << d)

    def box_xy(self, d: int):
        nb = 1 << d
        s = self.side(d)
        bx = np.minimum(np.floor((self.P[:, 0] - self.x0) / s), nb - 1).astype(np.int64)
        by = np.minimum(np.floor((self.P[:, 1] - self.y0) / s), nb - 1).astype(np.int64)
        bx = np.maximum(bx, 0)
        by = np.maximum(by, 0)
        return bx, by

    def box_of(self, d: int) -> np.ndarray:
        bx, by = self.box_xy(d)
        return by * (1 << d) + bx

    def members(self, d: int) -> list:
        """Sorted global index array of every box at depth d."""
        b = self.box_of(d)
        order = np.argsort(b, kind="stable")  # stable: ascending global index inside a box
        counts = np.bincount(b, minlength=4 ** d)
        out, pos = [], 0
        for c in counts:
            out.append(order[pos:pos + c].copy())
            pos += c
        return out

    def centre(self, d: int, b: int):
        nb = 1 << d
        s = self.side(d)
        bx, by = b % nb, b // nb
        return (self.x0 + (bx + 0.5) * s, self.y0 + (by + 0.5) * s)

    # -- lists -----------------------------------------------------------
    @staticmethod
    def dist(d: int, a: int, b: int) -> int:
        nb = 1 << d
        return max(abs(a % nb - b % nb), abs(a // nb - b // nb))

    @staticmethod
    def ring(d: int, b: int, r: int) -> list:
        """Boxes at Chebyshev distance exactly r, clipped to the grid, ascending id."""
        nb = 1 << d
        bx, by = b % nb, b // nb
        out = []
        for y in range(by - r, by + r + 1):
            for x in range(bx - r, bx + r + 1):
                if 0 <= x < nb and 0 <= y < nb and max(abs(x - bx), abs(y - by)) == r:
                    out.append(y * nb + x)
        return out

    def nbrs(self, d: int, b: int) -> list:
        return self.ring(d, b, 1)

    def dist2(self, d: int, b: int) -> list:
        return self.ring(d, b, 2)

    @staticmethod
    def colour(d: int, b: int, ncol: int = 9) -> int:
        nb = 1 << d
        if ncol == 4:
            return (b % nb) % 2 + 2 * ((b // nb) % 2)
        return (b % nb) % 3 + 3 * ((b // nb) % 3)

    def order(self, d: int, ncol: int = 9) -> list:
        """Elimination order at depth d: colour-major, id order inside a colour."""
        nb = 1 << d
        boxes = range(nb * nb)
        return [b for c in range(ncol) for b in boxes if self.colour(d, b, ncol) == c]

    @staticmethod
    def children(d: int, p: int) -> list:
        """Children at depth d+1 of box p at depth d, ascending id."""
        nb = 1 << d
        px, py = p % nb, p // nb
        cn = nb * 2
        return [(2 * py + j) * cn + (2 * px + i) for j in range(2) for i in range(2)]

    def proxy_points(self, d: int, b: int, n_px: int, c_r: float) -> np.ndarray:
        """Proxy circle (Sec. 2.3): n_px equispaced points of radius c_r * side
        around the box centre, angles 2 pi p / n_px."""
        cx, cy = self.centre(d, b)
        rad = c_r * self.side(d)
        th = 2.0 * np.pi * np.arange(n_px) / n_px
        return np.stack([cx + rad * np.cos(th), cy + rad * np.sin(th)], axis=1)
