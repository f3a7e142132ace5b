"""Pins for the oracle's quadtree (oracle/tree.py) by brute force."""
import itertools

import numpy as np
import pytest

from oracle.tree import Tree
from paper_2310_15458_amd import workloads as W


def _brute_ring(d, b, r):
    nb = 1 << d
    bx, by = b % nb, b // nb
    out = []
    for c in range(nb * nb):
        cx, cy = c % nb, c // nb
        if max(abs(cx - bx), abs(cy - by)) == r:
            out.append(c)
    return out


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_lists_brute_force(d):
    t = Tree(W.grid_points(8), 1)
    for b in range(4 ** d):
        assert t.nbrs(d, b) == _brute_ring(d, b, 1)
        assert t.dist2(d, b) == _brute_ring(d, b, 2)
        assert len(t.nbrs(d, b)) <= 8 and len(t.dist2(d, b)) <= 16
        # Def. d:m: M(B) = N(N(B)) \ (N(B) u B)
        nn = set()
        for x in t.nbrs(d, b):
            nn.update(t.nbrs(d, x))
        assert sorted(nn - set(t.nbrs(d, b)) - {b}) == t.dist2(d, b)


@pytest.mark.parametrize("d", [2, 3, 4, 5])
def test_colour_classes_are_far_apart(d):
    nb = 1 << d
    for c in range(9):
        boxes = [b for b in range(nb * nb) if Tree.colour(d, b) == c]
        for a, b in itertools.combinations(boxes, 2):
            assert Tree.dist(d, a, b) >= 3


@pytest.mark.parametrize("n,leaf,D", [(64, 64, 3), (256, 64, 5), (512, 64, 6), (48, 36, 3),
                                      (32, 64, 2), (96, 64, 4), (128, 64, 4), (8, 64, 0)])
def test_depth_rule(n, leaf, D):
    t = Tree(W.grid_points(n), leaf)
    assert t.D == D
    counts = np.bincount(t.box_of(t.D), minlength=4 ** t.D)
    assert counts.max() <= leaf
    if t.D > 0:
        assert np.bincount(t.box_of(t.D - 1)).max() > leaf


def test_members_partition_sorted():
    P = np.random.default_rng(1).random((500, 2))
    t = Tree(P, 20)
    for d in range(t.D + 1):
        m = t.members(d)
        allm = np.concatenate(m)
        assert np.array_equal(np.sort(allm), np.arange(500))
        for b, idx in enumerate(m):
            assert np.all(np.diff(idx) > 0)
            bx, by = t.box_xy(d)
            assert np.all(by[idx] * (1 << d) + bx[idx] == b)


def test_children_and_parent_geometry():
    t = Tree(W.grid_points(16), 4)
    for d in range(3):
        for p in range(4 ** d):
            cx, cy = t.centre(d, p)
            for c in t.children(d, p):
                x, y = t.centre(d + 1, c)
                assert abs(abs(x - cx) - t.side(d) / 4) < 1e-15
                assert abs(abs(y - cy) - t.side(d) / 4) < 1e-15


@pytest.mark.parametrize("c_r", [1.25, 2.5])
def test_proxy_circle_separates_box_from_far_field(c_r):
    t = Tree(W.grid_points(32), 16)
    d = 3
    b = 27
    G = t.proxy_points(d, b, 64, c_r)
    cx, cy = t.centre(d, b)
    rad = np.hypot(G[:, 0] - cx, G[:, 1] - cy)
    assert np.allclose(rad, c_r * t.side(d), rtol=1e-14)
    # the circle encloses the box (corner at sqrt(2)/2 side) and excludes F \ M
    # (Chebyshev distance >= 2.5 sides from the centre)
    assert c_r * t.side(d) > np.sqrt(2) / 2 * t.side(d)
    assert np.max(np.maximum(np.abs(G[:, 0] - cx), np.abs(G[:, 1] - cy))) <= 2.5 * t.side(d) + 1e-15
