"""Colors of the incompatibility graphs for points with low-dimensional
structure (section on exploiting low-dimensional structure,
fig:line_with_noise): a uniform grid on a randomly oriented line through
[0, 1]^d, perturbed by Gaussian noise, d = 1..8.  The paper prints no values;
what it states, and what is checked here on the library's host trees
(bit-identical to the oracle's, test_host_parity):

* on the exact line the number of colors grows modestly with d;
* with noise it grows rapidly with d (the effective dimension rises to d);
* more noise never needs fewer colors here, and every coloring is proper.
"""
import numpy as np
import pytest

import workloads

hm = pytest.importorskip("paper_2205_03406_amd")

DIMS = (1, 2, 3, 4, 6, 8)


def max_colors(dim, noise, n=3000, leaf=32):
    T = hm.Tree(workloads.noisy_line(n, dim, noise), leaf).color()
    best = 0
    for l in range(1, T.nlev):
        G = T.graph(l)
        if G.nv:
            for v in range(G.nv):   # proper coloring
                nb = G.adj[G.xadj[v]:G.xadj[v + 1]]
                assert not np.any(G.color[nb] == G.color[v])
        best = max(best, G.ncolors)
    return best


def test_colors_against_dimension_and_noise():
    table = {(d, s): max_colors(d, s) for d in DIMS for s in (0.0, 0.002, 0.01)}
    print("\nmax colors per level (rows d, columns noise 0 / 0.002 / 0.01):")
    for d in DIMS:
        print(d, [table[(d, s)] for s in (0.0, 0.002, 0.01)])
    line = [table[(d, 0.0)] for d in DIMS]
    noisy = [table[(d, 0.01)] for d in DIMS]
    # the 1D grid needs the 6 colors of the worked example's level graphs
    assert line[0] == 6
    # exact line: modest growth (a few colors per added dimension)
    assert line[-1] <= 5 * line[0]
    assert all(b >= a for a, b in zip(line, line[1:]))
    # noise: the count grows much faster with d than on the line
    assert noisy[-1] >= 5 * line[-1]
    assert noisy[-1] >= 8 * noisy[1]
    for d in DIMS[2:]:
        assert table[(d, 0.0)] <= table[(d, 0.002)] <= table[(d, 0.01)], d
