"""The library's host combinatorics against the oracle, bit for bit (CPU).

Tree order, box ranges, parents, cube origins, neighbor and interaction
lists, constraint graphs (vertex order, active boxes, adjacency, pair ->
vertex maps) and DSatur colorings must be identical: the two sides are
written independently (the library draws neighbor candidates from the parent
level and dedups parent neighbor sets; the oracle scans every box pair).
Also checks that libhm.so exports every entry point include/hm.h declares.
"""
import os
import re

import numpy as np
import pytest

import workloads
from oracle import OTree

hm = pytest.importorskip("paper_2205_03406_amd")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "hm.h")).read()
    declared = set(re.findall(r"\b(hm_[a-z0-9_]+)\s*\(", hdr))
    declared.discard("hm_apply_fn")
    assert declared, "no declarations found"
    lib = hm.lib()
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert declared == set(hm.EXPORTED)


def compare(points, leaf, kind="geometric", adm="strong"):
    O = OTree(points, leaf, kind, adm)
    T = hm.Tree(points, leaf, kind, adm).color()
    assert T.nlev == O.nlev
    assert np.array_equal(T.perm(), O.perm)
    for l in range(O.nlev):
        start, parent, org, blev = T.level(l)
        assert np.array_equal(start, O.start[l])
        assert np.array_equal(parent, O.parent[l])
        if kind == "geometric":
            assert np.array_equal(org, O.org[l])
            assert np.array_equal(blev, O.blev[l])
        for which, mine in ((hm.HM_LIST_NEIGHBOR, O.nei[l]), (hm.HM_LIST_INTERACTION, O.intl[l])):
            ptr, idx = T.list(l, which)
            assert np.array_equal(ptr, mine[0]), (l, which)
            assert np.array_equal(idx, mine[1]), (l, which)
    for g in list(range(O.nlev)) + [-1]:
        G = T.graph(g)
        OG = O.graphs[g if g >= 0 else O.nlev]
        assert G.nv == OG.nv
        assert np.array_equal(G.vbox, OG.vbox)
        assert np.array_equal(G.xadj, OG.xadj)
        assert np.array_equal(G.adj, OG.adj)
        assert np.array_equal(G.pair_a, OG.pair_a)
        assert np.array_equal(G.pair_b, OG.pair_b)
        assert np.array_equal(G.pair_v, OG.pair_v)
        assert G.ncolors == OG.ncolors
        assert np.array_equal(G.color, OG.color)
    return O, T


def test_worked_example():
    O, T = compare(workloads.grid_1d(64), 8)
    assert T.graph(3).ncolors == 6 and T.graph(-1).ncolors == 3


def test_fig_tree_index_halving():
    compare(workloads.grid_1d(400), 100, "index_binary", "weak")


def test_hodlr_config():
    inst = workloads.config(0)
    compare(inst.points, inst.leaf, inst.tree, inst.adm)


def test_star_curve_full_size():
    inst = workloads.config(1)
    compare(inst.points, inst.leaf, inst.tree, inst.adm)


def test_sphere_reduced():
    inst = workloads.config(2, n=8192)
    compare(inst.points, inst.leaf, inst.tree, inst.adm)


@pytest.mark.parametrize("dim,n,leaf,seed", [(1, 777, 9, 1), (2, 1500, 13, 2), (3, 2000, 20, 3),
                                             (2, 300, 1, 4), (3, 64, 100, 5), (1, 1, 4, 6)])
def test_random_sets(dim, n, leaf, seed):
    compare(workloads.random_points(n, dim, seed), leaf)


def test_clusters_and_duplicates():
    rng = np.random.default_rng(9)
    pts = np.concatenate([rng.uniform(0, 1e-3, (300, 2)), rng.uniform(0.4, 1.0, (200, 2)),
                          np.repeat(np.array([[0.7, 0.1]]), 5, axis=0)])
    compare(pts, 12)
    compare(workloads.ellipse(3000, 1.7, 0.6), 64)


def test_weak_on_geometric_tree():
    compare(workloads.random_points(900, 2, 8), 30, "geometric", "weak")


def test_color_entry_point_matches_oracle_dsatur():
    from oracle import dsatur
    rng = np.random.default_rng(1)
    for trial in range(10):
        nv = int(rng.integers(1, 200))
        E = set()
        for _ in range(int(rng.integers(0, 4 * nv))):
            a, b = rng.integers(0, nv, 2)
            if a != b:
                E.add((int(a), int(b)))
                E.add((int(b), int(a)))
        nb = [[] for _ in range(nv)]
        for a, b in E:
            nb[a].append(b)
        xadj = np.zeros(nv + 1, np.int64)
        adj = []
        for v in range(nv):
            adj += sorted(nb[v])
            xadj[v + 1] = len(adj)
        adj = np.array(adj, np.int32)
        c1, n1 = hm.color(xadj, adj)
        c2, n2 = dsatur(xadj, adj)
        assert n1 == n2 and np.array_equal(c1, c2)


def test_errors_are_reported():
    with pytest.raises(hm.HMError):
        hm.Tree(np.zeros((0, 2)), 8)
    with pytest.raises(hm.HMError):
        hm.Tree(np.array([[np.nan, 0.0]]), 8)
    with pytest.raises(hm.HMError):
        hm.Tree(workloads.random_points(10, 2, 1), 4, "index_binary", "strong")
    T = hm.Tree(workloads.grid_1d(64), 8).color()
    G = T.graph(3)
    bad = np.zeros(G.nv, np.int32)
    with pytest.raises(hm.HMError):
        T.set_colors(3, bad)
    # a valid caller coloring (all distinct) is accepted
    T.set_colors(3, np.arange(G.nv, dtype=np.int32))
    assert T.graph(3).ncolors == G.nv


def test_single_hip_runtime_per_process():
    """Importing the binding, then torch, must leave one HIP runtime (and one
    HSA runtime) mapped: two copies would manage the same device apart."""
    import subprocess
    import sys
    code = ("import paper_2205_03406_amd, torch\n"
            "m = open('/proc/self/maps').read().splitlines()\n"
            "print(len({l.split()[-1] for l in m if 'libamdhip64' in l}),"
            " len({l.split()[-1] for l in m if 'libhsa-runtime64' in l}))\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split() == ["1", "1"], out.stdout


@pytest.mark.parametrize("case", ["worked", "curve", "sphere", "hodlr"])
def test_uniform_graphs_match_oracle(case):
    """Stage-1 graphs of uniform H^1 (vertices, adjacency, DSatur colors)
    equal the oracle's, level by level."""
    from oracle import UniformGraph
    if case == "worked":
        args = (workloads.grid_1d(64), 8, "geometric", "strong")
    elif case == "curve":
        args = (workloads.star_curve(3000), 32, "geometric", "strong")
    elif case == "sphere":
        args = (workloads.sphere(3000, 4), 64, "geometric", "strong")
    else:
        args = (workloads.uniform_line(1024, 1), 64, "index_binary", "weak")
    O = OTree(*args)
    T = hm.Tree(*args)
    for l in range(O.nlev):
        UG = UniformGraph(O, l)
        vbox, xadj, adj, col, nc = T.uniform_graph(l)
        assert np.array_equal(vbox, UG.vbox), l
        assert np.array_equal(xadj, UG.xadj), l
        assert np.array_equal(adj, UG.adj), l
        assert np.array_equal(col, UG.color) and nc == UG.ncolors, l


@pytest.mark.parametrize("dim,noise", [(4, 0.0), (4, 0.05), (6, 0.01), (8, 0.0), (8, 0.005)])
def test_noisy_lines_in_more_dimensions(dim, noise):
    """Trees of d > 3 (2^d children, floor(63 / d) key bits): tree order,
    boxes, lists, graphs and colors equal to the oracle's."""
    compare(workloads.noisy_line(3000, dim, noise), 32)
