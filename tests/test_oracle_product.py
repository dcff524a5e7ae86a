"""Pins of the oracle's operator black boxes (compressed operators and their
products) and of compressing a product of compressed operators.

* The applies of a compressed operator equal its block-by-block assembly
  (and the adjoint its transpose), on 1D, 2D and HODLR trees.
* A product black box equals the product of the dense matrices.
* Compressing an H^1 matrix given only through its own applies recovers it
  (it is exactly H^1 on the same tree: fixed rank at its own rank).
* Compressing the product of two compressed kernel operators at tol 1e-8
  reaches the dense product within a few tol, and the black box is called
  exactly sum(chi_l) r + chi_leaf m times through A and sum(chi_l) r
  through A*.
"""
import numpy as np
import pytest

import oracle
import workloads
from synth import exact_h1


def _tree(case):
    if case == "curve":
        return oracle.OTree(workloads.star_curve(700), 20, "geometric", "strong")
    if case == "strong2d":
        return oracle.OTree(workloads.random_points(500, 2, 4), 16, "geometric", "strong")
    return oracle.OTree(workloads.uniform_line(256, 2), 16, "index_binary", "weak")


@pytest.mark.parametrize("case", ["curve", "strong2d", "hodlr"])
def test_hmatrix_blackbox_matches_assembly(case):
    T = _tree(case)
    A = exact_h1(T, 3, seed=2)
    H = oracle.compress(T, oracle.DenseBlackBox(A), 8, k=3, seed=5)
    M = oracle.assemble(H)
    assert np.linalg.norm(M - A) <= 1e-11 * np.linalg.norm(A)
    bb = oracle.HMatrixBlackBox(H)
    X = np.random.default_rng(1).standard_normal((T.n, 5))
    assert np.allclose(bb.apply(X), M @ X, rtol=0, atol=1e-12 * np.abs(M).sum())
    assert np.allclose(bb.applyT(X), M.T @ X, rtol=0, atol=1e-12 * np.abs(M).sum())


def test_product_blackbox_is_the_product():
    rng = np.random.default_rng(3)
    A, B = rng.standard_normal((40, 40)), rng.standard_normal((40, 40))
    P = oracle.ProductBlackBox(oracle.DenseBlackBox(A), oracle.DenseBlackBox(B))
    X = rng.standard_normal((40, 3))
    assert np.allclose(P.apply(X), (A @ B) @ X, atol=1e-12)
    assert np.allclose(P.applyT(X), (A @ B).T @ X, atol=1e-12)


@pytest.mark.parametrize("case", ["curve", "hodlr"])
def test_recompressing_a_compressed_operator(case):
    T = _tree(case)
    A = exact_h1(T, 3, seed=7)
    H = oracle.compress(T, oracle.DenseBlackBox(A), 8, k=3, seed=5)
    H2 = oracle.compress(T, oracle.HMatrixBlackBox(H), 8, k=3, seed=11)
    assert np.linalg.norm(oracle.assemble(H2) - A) <= 1e-10 * np.linalg.norm(A)


def test_product_of_compressed_kernels():
    pts = workloads.star_curve(1500)
    T = oracle.OTree(pts, 64, "geometric", "strong")
    K = oracle.kernel_matrix(pts, pts, "log")
    H = oracle.compress(T, oracle.DenseBlackBox(K), 24, tol=1e-10, seed=1)
    bb = oracle.CountingBlackBox(oracle.ProductBlackBox(oracle.HMatrixBlackBox(H),
                                                        oracle.HMatrixBlackBox(H)))
    tol = 1e-8
    HP = oracle.compress(T, bb, 24, tol=tol, seed=2)
    KK = K @ K
    err = np.linalg.norm(HP.dense() - KK) / np.linalg.norm(KK)
    assert err <= 5 * tol, err
    chis = [T.graphs[l].ncolors for l in T.sampled_levels()]
    assert bb.cols_At == 24 * sum(chis)
    assert bb.cols_A == 24 * sum(chis) + T.leaf_graph.ncolors * T.leaf_max()
    assert HP.saturated == 0
