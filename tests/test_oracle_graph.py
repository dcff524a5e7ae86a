"""Pins for the oracle's constraint graphs and DSatur coloring (CPU only).

* fig:graph_strong_1d_lvl3: 12 vertices, 54 edges, the paper's vertex
  grouping (e.g. A_{8,11} and A_{9,11} share one constraint set) and its
  6-coloring (color classes compared up to relabeling);
* fig:graph_strong_1d_leaf: 22 vertices, 80 edges and 3 colors;
* level 2 of the example: 4 mutually incompatible test matrices;
* DSatur (alg:dsatur) never uses more than deg(G)+1 colors, always yields a
  valid coloring and is exact on bipartite graphs;
* the general patterns of fig:h1activations are valid colorings of our
  graphs on uniform grids (the chi <= 6^d and chi_leaf <= 3^d argument);
  DSatur stays within those bounds in 1D and 2D.
"""
import json
import os

import numpy as np
import pytest

import workloads
from oracle import OTree, dsatur

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_example_1d.json")))


def _name(pair):
    return "%dx%d" % tuple(pair)


def _vertex_of_pair(T, l, G):
    out = {}
    off = 2 ** l if l < T.nlev else 2 ** T.L
    for a, b, v in zip(G.pair_a, G.pair_b, G.pair_v):
        out[(int(a) + off, int(b) + off)] = int(v)
    return out


def _check_graph(T, G, gold, level):
    vp = _vertex_of_pair(T, level, G)
    # every figure node is one vertex; all its labelled pairs map to it
    node_vertex = {}
    for name, node in gold["vertices"].items():
        pairs = [tuple(p) for p in node["pairs"]]
        vs = {vp[p] for p in pairs}
        assert len(vs) == 1, (name, vs)
        node_vertex[name] = vs.pop()
    assert len(set(node_vertex.values())) == G.nv == len(gold["vertices"])
    # edges
    got = set()
    for u in range(G.nv):
        for w in G.adj[G.xadj[u]:G.xadj[u + 1]]:
            got.add(frozenset((u, int(w))))
    want = {frozenset((node_vertex[a], node_vertex[b])) for a, b in gold["edges"]}
    assert got == want
    # coloring equals the figure's up to relabeling
    classes = {}
    for name, node in gold["vertices"].items():
        classes.setdefault(node["fill"], set()).add(node_vertex[name])
    ours = {}
    for v in range(G.nv):
        ours.setdefault(int(G.color[v]), set()).add(v)
    assert sorted(map(sorted, classes.values())) == sorted(map(sorted, ours.values()))
    return node_vertex


def test_level3_graph_matches_paper():
    T = OTree(workloads.grid_1d(64), 8, "geometric", "strong")
    G = T.graphs[3]
    assert G.nv == 12 and G.nedges == 54 and G.ncolors == 6
    _check_graph(T, G, GOLD["graph_level3"], 3)


def test_leaf_graph_matches_paper():
    T = OTree(workloads.grid_1d(64), 8, "geometric", "strong")
    G = T.leaf_graph
    assert G.nv == 22 and G.nedges == 80 and G.ncolors == 3
    _check_graph(T, G, GOLD["graph_leaf"], T.nlev)


def test_level2_four_test_matrices():
    T = OTree(workloads.grid_1d(64), 8, "geometric", "strong")
    G = T.graphs[2]
    assert G.nv == 4 and G.nedges == 6 and G.ncolors == 4


def test_hodlr_two_colors_per_level():
    T = OTree(workloads.uniform_line(1024, 1), 64, "index_binary", "weak")
    assert T.sampled_levels() == [1, 2, 3, 4]
    assert [T.graphs[l].ncolors for l in T.sampled_levels()] == [2, 2, 2, 2]
    assert T.leaf_graph.ncolors == 1


def _valid(G):
    for u in range(G.nv):
        for w in G.adj[G.xadj[u]:G.xadj[u + 1]]:
            if G.color[u] == G.color[int(w)]:
                return False
    return True


def _incompatible(G, u, w):
    su = set(map(int, G.vset[G.vset_ptr[u]:G.vset_ptr[u + 1]]))
    sw = set(map(int, G.vset[G.vset_ptr[w]:G.vset_ptr[w + 1]]))
    bu, bw = int(G.vbox[u]), int(G.vbox[w])
    return bu != bw and (bu in sw or bw in su)


@pytest.mark.parametrize("dim,n,leaf,seed", [(1, 200, 6, 1), (2, 400, 10, 2), (3, 500, 16, 3)])
def test_random_graphs_valid_and_bounded(dim, n, leaf, seed):
    T = OTree(workloads.random_points(n, dim, seed), leaf, "geometric", "strong")
    for g in list(range(T.nlev)) + [T.nlev]:
        G = T.graphs[g]
        if G.nv == 0:
            continue
        assert _valid(G)
        maxdeg = int(np.max(np.diff(G.xadj)))
        assert G.ncolors <= maxdeg + 1
        # brute force: the edge set is exactly the incompatible vertex pairs
        for u in range(G.nv):
            nb = set(map(int, G.adj[G.xadj[u]:G.xadj[u + 1]]))
            for w in range(G.nv):
                if w != u:
                    assert (w in nb) == _incompatible(G, u, w)
        # each pair's vertex is its constraint set (active box, boxes to zero)
        lev = g if g < T.nlev else T.L
        for a, b, v in zip(G.pair_a, G.pair_b, G.pair_v):
            assert G.vbox[v] == b
            if g < T.nlev:
                want = set(map(int, T.neighbors(lev, int(a)))) | set(map(int, T.interaction(lev, int(a))))
            else:
                want = set(map(int, T.neighbors(lev, int(a))))
            assert set(map(int, G.vset[G.vset_ptr[v]:G.vset_ptr[v + 1]])) == want


@pytest.mark.parametrize("dim,side", [(1, 64), (2, 16), (3, 8)])
def test_general_pattern_colors_are_valid(dim, side):
    """The general test-matrix patterns (fig:h1activations): activating the
    boxes that share a position modulo 6 (levels) or modulo 3 (leaf) in every
    dimension satisfies every constraint set, so that assignment must be a
    valid coloring of our graphs -- which bounds chi by 6^d and 3^d."""
    g = (np.arange(side) + 0.5) / side
    pts = np.stack(np.meshgrid(*([g] * dim), indexing="ij"), -1).reshape(-1, dim)
    T = OTree(pts, 1, "geometric", "strong")

    def pattern(G, l, mod):
        size = 2 ** (21 - l)
        pos = T.org[l][G.vbox, :dim] // size
        col = np.zeros(G.nv, np.int64)
        for d in range(dim):
            col = col * mod + pos[:, d] % mod
        return col

    for l in T.sampled_levels():
        G = T.graphs[l]
        col = pattern(G, l, 6)
        for u in range(G.nv):
            nb = G.adj[G.xadj[u]:G.xadj[u + 1]]
            assert not np.any(col[nb] == col[u])
        if dim <= 2:
            assert G.ncolors <= 6 ** dim
    G = T.leaf_graph
    col = pattern(G, T.L, 3)
    for u in range(G.nv):
        nb = G.adj[G.xadj[u]:G.xadj[u + 1]]
        assert not np.any(col[nb] == col[u])
    if dim <= 2:
        assert G.ncolors <= 3 ** dim


def test_dsatur_exact_on_bipartite_and_cycles():
    rng = np.random.default_rng(0)
    for trial in range(20):
        n1, n2 = rng.integers(2, 30, size=2)
        edges = set()
        for _ in range(rng.integers(1, 120)):
            edges.add((int(rng.integers(0, n1)), int(n1 + rng.integers(0, n2))))
        nv = n1 + n2
        nb = [[] for _ in range(nv)]
        for a, b in edges:
            nb[a].append(b); nb[b].append(a)
        xadj = np.zeros(nv + 1, np.int64)
        adj = []
        for v in range(nv):
            s = sorted(set(nb[v]))
            adj += s
            xadj[v + 1] = len(adj)
        col, nc = dsatur(xadj, np.array(adj, np.int32))
        assert nc == 2
    # odd cycle needs 3, even cycle 2, clique K_n needs n
    for n, want in [(5, 3), (8, 2), (9, 3)]:
        xadj = np.arange(0, 2 * n + 1, 2, dtype=np.int64)
        adj = np.array([[(v - 1) % n, (v + 1) % n] for v in range(n)]).reshape(-1)
        adj = np.sort(adj.reshape(n, 2), axis=1).reshape(-1).astype(np.int32)
        assert dsatur(xadj, adj)[1] == want
    n = 7
    xadj = np.arange(0, n * (n - 1) + 1, n - 1, dtype=np.int64)
    adj = np.array([w for v in range(n) for w in range(n) if w != v], np.int32)
    col, nc = dsatur(xadj, adj)
    assert nc == n and sorted(col.tolist()) == list(range(n))
