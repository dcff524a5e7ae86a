"""Pins for the oracle's tree and lists (CPU only).

Pinned to what the paper prints and to what the definitions force:
* fig:tree -- the index-halving tree of [1..400];
* fig:matrix_strong_1d_lvl3 -- the admissible (blue) and inadmissible (red)
  block sets of the depth-3 tree on a grid over [0, 1];
* the list-size bounds of the section on rank-structured matrices
  (at most 3^d neighbors, at most 6^d - 3^d interaction-list boxes);
* list symmetry and the exact cover of the matrix by admissible blocks of
  all levels plus the leaf neighbor blocks.
"""
import json
import os

import numpy as np
import pytest

import workloads
from oracle import OTree

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_example_1d.json")))


def heap_pairs(T, l, which):
    p, i = (T.intl if which == "int" else T.nei)[l]
    out = set()
    for a in range(T.nbox(l)):
        for b in i[p[a]:p[a + 1]]:
            out.add((a + 2 ** l, int(b) + 2 ** l))
    return out


def test_index_tree_matches_fig_tree():
    T = OTree(workloads.grid_1d(400), 100, "index_binary", "weak")
    got = {}
    heap = 1
    for l in range(3):
        for b in range(T.nbox(l)):
            s0, s1 = T.box_range(l, b)
            got["I%d" % (2 ** l + b)] = [s0 + 1, s1]
    for k, v in GOLD["index_tree"].items():
        assert got[k] == v, (k, got[k], v)
    assert T.L == 2
    assert np.array_equal(T.perm, np.arange(400))


def test_worked_example_block_sets():
    # 64 grid points on [0,1] with leaf size 8 give the paper's depth-3 tree
    T = OTree(workloads.grid_1d(64), 8, "geometric", "strong")
    assert T.L == 3 and [T.nbox(l) for l in range(4)] == [1, 2, 4, 8]
    assert heap_pairs(T, 2, "int") == set(map(tuple, GOLD["admissible_level2"]))
    assert heap_pairs(T, 3, "int") == set(map(tuple, GOLD["admissible_level3"]))
    assert heap_pairs(T, 3, "nei") == set(map(tuple, GOLD["inadmissible_leaf"]))
    assert heap_pairs(T, 1, "int") == set()


def _check_lists(T):
    d = T.dim
    for l in range(T.nlev):
        nb = T.nbox(l)
        nei = [set(map(int, T.neighbors(l, b))) for b in range(nb)]
        itl = [set(map(int, T.interaction(l, b))) for b in range(nb)]
        for a in range(nb):
            assert a in nei[a]
            assert not (nei[a] & itl[a])
            for b in nei[a]:
                assert a in nei[b]
            for b in itl[a]:
                assert a in itl[b]
    return True


def _exact_cover(T):
    n = T.n
    cover = np.zeros((n, n), np.int32)
    for l in range(T.nlev):
        for a in range(T.nbox(l)):
            a0, a1 = T.box_range(l, a)
            for b in T.interaction(l, a):
                b0, b1 = T.box_range(l, int(b))
                cover[a0:a1, b0:b1] += 1
    for a in range(T.nbox(T.L)):
        a0, a1 = T.box_range(T.L, a)
        for b in T.neighbors(T.L, a):
            b0, b1 = T.box_range(T.L, int(b))
            cover[a0:a1, b0:b1] += 1
    return cover


@pytest.mark.parametrize("dim,n,leaf,seed", [(1, 300, 7, 1), (2, 700, 12, 2), (3, 900, 20, 3), (2, 500, 5, 4)])
def test_random_trees_lists_and_cover(dim, n, leaf, seed):
    T = OTree(workloads.random_points(n, dim, seed), leaf, "geometric", "strong")
    _check_lists(T)
    assert np.all(_exact_cover(T) == 1)
    # every level partitions all points, boxes hold at most `leaf` at the leaf level
    for l in range(T.nlev):
        assert T.start[l][0] == 0 and T.start[l][-1] == n
        assert np.all(np.diff(T.start[l]) > 0)
    assert np.max(np.diff(T.start[T.L])) <= leaf
    assert sorted(T.perm.tolist()) == list(range(n))


def test_curve_and_sphere_cover():
    T = OTree(workloads.star_curve(1500), 20, "geometric", "strong")
    assert np.all(_exact_cover(T) == 1)
    T = OTree(workloads.sphere(1200, 9), 30, "geometric", "strong")
    assert np.all(_exact_cover(T) == 1)
    T = OTree(workloads.uniform_line(1000, 1), 64, "index_binary", "weak")
    assert np.all(_exact_cover(T) == 1)


@pytest.mark.parametrize("dim,side", [(1, 64), (2, 16), (3, 8)])
def test_list_bounds_on_uniform_grids(dim, side):
    g = (np.arange(side) + 0.5) / side
    pts = np.stack(np.meshgrid(*([g] * dim), indexing="ij"), -1).reshape(-1, dim)
    T = OTree(pts, 1, "geometric", "strong")
    for l in range(T.nlev):
        for b in range(T.nbox(l)):
            assert len(T.neighbors(l, b)) <= 3 ** dim
            assert len(T.interaction(l, b)) <= 6 ** dim - 3 ** dim
    # an interior box of a full grid reaches both bounds
    l = T.L
    assert max(len(T.neighbors(l, b)) for b in range(T.nbox(l))) == 3 ** dim
    assert max(len(T.interaction(l, b)) for b in range(T.nbox(l))) == 6 ** dim - 3 ** dim


def test_morton_order_and_carried_leaves():
    # three clusters of very different density: leaves stop at different depths
    rng = np.random.default_rng(5)
    pts = np.concatenate([rng.uniform(0, 0.01, (200, 2)), rng.uniform(0.5, 1.0, (60, 2)),
                          np.array([[0.9, 0.02]])])
    T = OTree(pts, 16, "geometric", "strong")
    assert np.all(_exact_cover(T) == 1)
    for l in range(1, T.nlev):
        for b in range(T.nbox(l)):
            P = T.parent[l][b]
            s0, s1 = T.box_range(l, b)
            p0, p1 = T.box_range(l - 1, P)
            assert p0 <= s0 and s1 <= p1
            if p1 - p0 <= 16:   # a leaf is carried unchanged
                assert (s0, s1) == (p0, p1) and T.blev[l][b] == T.blev[l - 1][P]
    # every point's integer cell lies inside its box's cube at every level
    lo = pts.min(0)
    s = (pts.max(0) - lo).max()
    c = np.minimum(2 ** 21 - 1, np.floor(((pts - lo) / s) * 2 ** 21)).astype(np.int64)
    for l in range(T.nlev):
        for b in range(T.nbox(l)):
            s0, s1 = T.box_range(l, b)
            size = 2 ** (21 - T.blev[l][b])
            cc = c[T.perm[s0:s1]]
            assert np.all(cc >= T.org[l][b, :2]) and np.all(cc < T.org[l][b, :2] + size)
