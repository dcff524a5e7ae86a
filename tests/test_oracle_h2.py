"""Pins of the oracle's H^2 compression (section on H^2 compression,
alg:h2_pseudocode, alg:apply_h2_level_truncated).

* Exact recovery of synthetic H^2 matrices (nested bases) at fixed rank and
  in tolerance mode, 1D/2D/3D and HODLR trees, to 1e-12.
* The parent augmentation is load-bearing: with it removed (planted here, in
  the oracle) the nested bases cannot represent the coarse blocks and the
  same matrices are far from recovered.
* The upward / downward apply equals the dense matrix assembled from the
  bases implied by the nesting (a second, bottom-up construction), and its
  adjoint equals the transpose.
* On the star-curve log kernel: error within 20 tol, storage below the
  uniform H^1 form and that below the H^1 form, and the matvec counts
  sum(chi_unif) r + chi_leaf m through A and sum(chi) kmax through A*.
"""
import numpy as np
import pytest

import oracle
import oracle.h2 as h2mod
import workloads
from synth import exact_h2

TREES = {
    "curve": lambda: (workloads.star_curve(900), 20, "geometric", "strong"),
    "strong2d": lambda: (workloads.random_points(700, 2, 11), 16, "geometric", "strong"),
    "strong3d": lambda: (workloads.random_points(900, 3, 12), 24, "geometric", "strong"),
    "hodlr": lambda: (workloads.uniform_line(512, 3), 32, "index_binary", "weak"),
}


def _assembled(H):
    """Dense original-order matrix from the implied long bases, block by block."""
    T = H.T
    U, V = H.effective_bases()
    M = np.zeros((T.n, T.n))
    for l in H.levels:
        for a, b, B in H.B[l]:
            a0, a1 = T.box_range(l, a)
            b0, b1 = T.box_range(l, b)
            M[a0:a1, b0:b1] += U[l][a] @ B @ V[l][b].T
    for a, b, D in H.near:
        a0, a1 = T.box_range(T.L, a)
        b0, b1 = T.box_range(T.L, b)
        M[a0:a1, b0:b1] += D
    out = np.empty_like(M)
    out[np.ix_(T.perm, T.perm)] = M
    return out


@pytest.mark.parametrize("name", list(TREES))
def test_exact_recovery(name):
    T = oracle.OTree(*TREES[name]())
    A = exact_h2(T, 4, seed=5)
    H = oracle.compress_h2(T, oracle.DenseBlackBox(A), 10, k=4, seed=77)
    assert np.linalg.norm(H.dense() - A) <= 1e-12 * np.linalg.norm(A)
    Ht = oracle.compress_h2(T, oracle.DenseBlackBox(A), 14, tol=1e-9, seed=78)
    assert np.linalg.norm(Ht.dense() - A) <= 1e-12 * np.linalg.norm(A)
    assert Ht.saturated == 0


def test_augmentation_is_needed(monkeypatch):
    T = oracle.OTree(*TREES["curve"]())
    A = exact_h2(T, 4, seed=5)
    monkeypatch.setattr(h2mod, "augment_gaussian",
                        lambda seed, level, pas, row0, krows, ncols: np.zeros((krows, ncols)))
    H = oracle.compress_h2(T, oracle.DenseBlackBox(A), 10, k=4, seed=77)
    assert np.linalg.norm(H.dense() - A) > 1e-6 * np.linalg.norm(A)


@pytest.mark.parametrize("name", ["curve", "strong2d", "hodlr"])
def test_apply_matches_nested_assembly(name):
    T = oracle.OTree(*TREES[name]())
    pts = T.points
    K = oracle.kernel_matrix(pts, pts, "log")
    H = oracle.compress_h2(T, oracle.DenseBlackBox(K), 16, tol=1e-6, seed=9)
    D = H.dense()
    M = _assembled(H)
    assert np.linalg.norm(D - M) <= 1e-13 * np.linalg.norm(M)
    X = np.random.default_rng(2).standard_normal((T.n, 3))
    Yt = H.apply(X[T.perm], transpose=True)
    want = (M.T @ X)[T.perm]
    assert np.linalg.norm(Yt - want) <= 1e-13 * np.linalg.norm(want)


def test_kernel_accuracy_storage_counts():
    pts = workloads.star_curve(1500)
    T = oracle.OTree(pts, 64, "geometric", "strong")
    K = oracle.kernel_matrix(pts, pts, "log")
    tol, r = 1e-8, 24
    bb = oracle.CountingBlackBox(oracle.DenseBlackBox(K))
    H = oracle.compress_h2(T, bb, r, tol=tol, seed=3)
    err = np.linalg.norm(H.dense() - K) / np.linalg.norm(K)
    assert err <= 20 * tol, err
    Hu = oracle.compress_uniform(T, oracle.DenseBlackBox(K), r, tol=tol, seed=3)
    Hn = oracle.compress(T, oracle.DenseBlackBox(K), r, tol=tol, seed=3)
    assert H.floats() < oracle.uniform_floats(Hu) < Hn.floats()
    chi_u = [oracle.UniformGraph(T, l).ncolors for l in T.sampled_levels()]
    chi = [T.graphs[l].ncolors for l in T.sampled_levels()]
    assert bb.cols_A == r * sum(chi_u) + T.leaf_graph.ncolors * T.leaf_max() == H.cols_A
    assert bb.cols_At == (r - 10) * sum(chi) == H.cols_At
    assert H.saturated == 0


def test_augment_gaussian_draws():
    G = oracle.augment_gaussian(42, 3, 2, 117, 5, 7)
    assert G.shape == (5, 7)
    for i in range(5):
        want = oracle.gaussian_block(42, 3, 2, (1 << 31) + i, [117], 7)[0]
        assert np.array_equal(G[i], want)
    # the draws are not those of the stage-1 test matrix of the same row
    assert not np.allclose(G[0], oracle.gaussian_block(42, 3, 2, 0, [117], 7)[0])
