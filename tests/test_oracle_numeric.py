"""Pins for the oracle's numerical half (CPU only).

* Philox4x32-10 against its published known-answer vectors;
* Box-Muller output against the moments of the standard normal;
* test matrices against eq:h1constraints for every pair, and against the
  printed block patterns of eq:neartestmatrices and of the leaf example;
* exact recovery: alg:compress_double_random is exact on blocks of rank k,
  so a synthetic non-symmetric H^1 matrix with rank-k admissible blocks must
  come back to rounding error (catches a dropped or mis-signed peel, a
  transposed Z pass, a wrong Psi color or a wrong coupling solve);
* per block: the error never exceeds a small multiple of the optimal
  truncation error given by the exact block's singular values (Eckart-Young);
* matvec counts: sum over levels of chi_l r columns through A* and that plus
  chi_leaf m through A (config 1 gives exactly 304 and 240).
"""
import os

import numpy as np
import pytest

import workloads
from oracle import (CountingBlackBox, DenseBlackBox, KernelBlackBox, OTree, compress,
                    gaussian_block, kernel_matrix, leaf_test_matrix, philox4x32_10,
                    rel_fro_error_dense)
from oracle import test_matrix as make_test_matrix
from synth import exact_h1

HERE = os.path.dirname(__file__)


def test_philox_known_answers():
    n = 0
    for line in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        out = philox4x32_10(w[0], w[1], w[2], w[3], w[4], w[5])
        assert [int(x) for x in out] == w[6:10]
        n += 1
    assert n == 3


def test_gaussian_moments():
    z = gaussian_block(1234, 3, 0, 2, np.arange(40000), 10)
    assert np.all(np.isfinite(z))
    x = z.reshape(-1)
    assert abs(x.mean()) < 0.01
    assert abs(x.var() - 1) < 0.01
    assert abs(np.mean(x ** 4) - 3) < 0.06
    assert abs(np.mean(np.abs(x) <= 1.0) - 0.682689492) < 0.005
    # the two Box-Muller outputs of one draw are uncorrelated, as are columns
    assert abs(np.corrcoef(z[:, 0], z[:, 1])[0, 1]) < 0.02
    assert abs(np.corrcoef(z[:, 0], z[:, 2])[0, 1]) < 0.02
    # different counters give different streams
    z2 = gaussian_block(1234, 3, 1, 2, np.arange(100), 10)
    assert not np.allclose(z[:100], z2)
    # rows are independent of which other rows were drawn
    assert np.array_equal(gaussian_block(1234, 3, 0, 2, [17, 5], 10), z[[17, 5]])


def _constraints_hold(T, l, Om, r, transpose=False):
    G = T.graphs[l]
    idx = {(int(a), int(b)): q for q, (a, b) in enumerate(zip(G.pair_a, G.pair_b))}
    for (a, b), q in idx.items():
        if transpose:
            c = int(G.color[G.pair_v[idx[(b, a)]]])
            row_box, col_box = b, a
        else:
            c = int(G.color[G.pair_v[q]])
            row_box, col_box = a, b
        blk = Om[:, c * r:(c + 1) * r]
        s0, s1 = T.box_range(l, col_box)
        assert np.all(blk[s0:s1] != 0)
        zero = set(map(int, T.neighbors(l, row_box))) | set(map(int, T.interaction(l, row_box)))
        zero.discard(col_box)
        for g in zero:
            g0, g1 = T.box_range(l, g)
            assert np.all(blk[g0:g1] == 0)


@pytest.mark.parametrize("pts,leaf", [(workloads.random_points(600, 2, 3), 12),
                                      (workloads.star_curve(1000), 16),
                                      (workloads.sphere(900, 2), 24)])
def test_test_matrices_satisfy_constraints(pts, leaf):
    T = OTree(pts, leaf, "geometric", "strong")
    for l in T.sampled_levels():
        Om = make_test_matrix(T, l, 0, 99, 6)
        _constraints_hold(T, l, Om, 6)
        Ps = make_test_matrix(T, l, 1, 99, 6)
        _constraints_hold(T, l, Ps, 6, transpose=True)


def test_worked_example_test_matrix_patterns():
    T = OTree(workloads.grid_1d(64), 8, "geometric", "strong")
    r = 4
    Om = make_test_matrix(T, 3, 0, 5, r)
    act = []
    for c in range(T.graphs[3].ncolors):
        boxes = set()
        for b in range(8):
            s0, s1 = T.box_range(3, b)
            if np.any(Om[s0:s1, c * r:(c + 1) * r] != 0):
                boxes.add(b + 8)
        act.append(frozenset(boxes))
    # eq:neartestmatrices: {G8,G14}, {G9,G15}, {G10}, {G11}, {G12}, {G13}
    assert set(act) == {frozenset(s) for s in ({8, 14}, {9, 15}, {10}, {11}, {12}, {13})}
    Ol = leaf_test_matrix(T)
    m = T.leaf_max()
    act = []
    for c in range(T.leaf_graph.ncolors):
        boxes = set()
        for b in range(8):
            s0, s1 = T.box_range(3, b)
            blk = Ol[s0:s1, c * m:(c + 1) * m]
            if np.any(blk != 0):
                assert np.array_equal(blk[:, :s1 - s0], np.eye(s1 - s0))
                boxes.add(b + 8)
        act.append(frozenset(boxes))
    assert set(act) == {frozenset(s) for s in ({8, 11, 14}, {9, 12, 15}, {10, 13})}


@pytest.mark.parametrize("case", ["strong2d", "strong3d", "curve", "hodlr"])
def test_exact_recovery(case):
    if case == "strong2d":
        T = OTree(workloads.random_points(700, 2, 11), 16, "geometric", "strong")
    elif case == "strong3d":
        T = OTree(workloads.random_points(800, 3, 12), 24, "geometric", "strong")
    elif case == "curve":
        T = OTree(workloads.star_curve(900), 20, "geometric", "strong")
    else:
        T = OTree(workloads.uniform_line(512, 3), 32, "index_binary", "weak")
    k = 4
    A = exact_h1(T, k, seed=5)
    assert not np.allclose(A, A.T)
    bb = DenseBlackBox(A)
    H = compress(T, bb, r=k + 6, k=k, seed=77)
    assert rel_fro_error_dense(H, A) < 1e-12
    Ht = compress(T, bb, r=k + 10, tol=1e-9, seed=78)
    assert rel_fro_error_dense(Ht, A) < 1e-11
    for blocks in Ht.ranks().values():
        for ku, kv in blocks:
            assert ku <= k and kv <= k


def test_exact_recovery_catches_planted_mistakes():
    """The exact-recovery pin fails when a mistake is planted in the oracle."""
    import oracle.numeric as on
    T = OTree(workloads.random_points(500, 2, 21), 16, "geometric", "strong")
    A = exact_h1(T, 3, seed=6)
    bb = DenseBlackBox(A)
    good = rel_fro_error_dense(compress(T, bb, r=9, k=3, seed=1), A)
    assert good < 1e-12
    # transposed Z pass: sample A instead of A*
    bad_bb = DenseBlackBox(A)
    bad_bb.applyT = bad_bb.apply
    assert rel_fro_error_dense(compress(T, bad_bb, r=9, k=3, seed=1), A) > 1e-3
    # dropped peeling: subtract nothing from the samples
    orig = on.HMatrix.apply

    def no_peel(self, X, levels=None, near=True, transpose=False):
        if levels is not None:
            return np.zeros((self.T.n, X.shape[1]))
        return orig(self, X, levels, near, transpose)

    on.HMatrix.apply = no_peel
    try:
        assert rel_fro_error_dense(compress(T, bb, r=9, k=3, seed=1), A) > 1e-3
    finally:
        on.HMatrix.apply = orig


def test_hodlr_config_accuracy_and_counts():
    inst = workloads.config(0)
    T = OTree(inst.points, inst.leaf, inst.tree, inst.adm)
    kb = KernelBlackBox(inst.points, inst.kernel)
    bb = CountingBlackBox(kb)
    H = compress(T, bb, inst.r, k=inst.rank, seed=inst.seed)
    assert (bb.cols_A, bb.cols_At) == (304, 240)
    A = kb.dense()
    assert rel_fro_error_dense(H, A) < 1e-8
    # per block: at most 10x the optimal rank-k truncation error, above a
    # rounding floor set by the whole matrix (the peel subtracts coarser levels)
    floor = 1e-13 * np.linalg.norm(A)
    for l, blocks in H.lowrank.items():
        for a, b, U, B, V in blocks:
            a0, a1 = T.box_range(l, a)
            b0, b1 = T.box_range(l, b)
            Ab = A[np.ix_(T.perm[a0:a1], T.perm[b0:b1])]
            s = np.linalg.svd(Ab, compute_uv=False)
            opt = np.sqrt(np.sum(s[inst.rank:] ** 2))
            err = np.linalg.norm(Ab - U @ B @ V.T)
            assert err <= 10 * opt + floor, (l, a, b, err, opt)
    # leaf blocks are the dense blocks up to the peeling residue
    for a, b, D in H.near:
        a0, a1 = T.box_range(T.L, a)
        b0, b1 = T.box_range(T.L, b)
        Ab = A[np.ix_(T.perm[a0:a1], T.perm[b0:b1])]
        assert np.linalg.norm(D - Ab) <= 1e-9 * np.linalg.norm(Ab) + floor


def test_curve_tolerance_mode():
    inst = workloads.config(1, n=2048)
    T = OTree(inst.points, inst.leaf, inst.tree, inst.adm)
    kb = KernelBlackBox(inst.points, inst.kernel)
    bb = CountingBlackBox(kb)
    r = 24
    H = compress(T, bb, r, tol=inst.tol, seed=inst.seed)
    chis = [T.graphs[l].ncolors for l in T.sampled_levels()]
    assert bb.cols_At == sum(chis) * r
    assert bb.cols_A == sum(chis) * r + T.leaf_graph.ncolors * T.leaf_max()
    A = kb.dense()
    assert rel_fro_error_dense(H, A) < 1e-8
    assert H.saturated == 0
    for l, blocks in H.lowrank.items():
        for a, b, U, B, V in blocks:
            a0, a1 = T.box_range(l, a)
            b0, b1 = T.box_range(l, b)
            Ab = A[np.ix_(T.perm[a0:a1], T.perm[b0:b1])]
            err = np.linalg.norm(Ab - U @ B @ V.T)
            assert err <= 10 * inst.tol * np.linalg.norm(Ab), (l, a, b, err)
    X = np.random.default_rng(0).standard_normal((T.n, 3))
    assert np.linalg.norm(H.matvec(X) - A @ X) <= 1e-7 * np.linalg.norm(A @ X)


def test_error_estimators():
    from oracle.numeric import power_error, probe_error
    rng = np.random.default_rng(3)
    Q1, _ = np.linalg.qr(rng.standard_normal((60, 60)))
    Q2, _ = np.linalg.qr(rng.standard_normal((60, 60)))
    s = np.r_[10.0, np.linspace(4, 1, 59)]
    A = Q1 @ np.diag(s) @ Q2.T
    E = Q1 @ np.diag(np.r_[0.5, np.zeros(59)]) @ Q2.T   # ||E|| = 0.5, ||A|| = 10
    S = np.diag(s)
    Es = np.diag(np.r_[0.5, np.zeros(59)])
    assert abs(power_error(lambda X: Es @ X, lambda X: Es @ X, lambda X: S @ X, 60) - 0.05) < 1e-6
    assert probe_error(lambda X: A @ X, lambda X: A @ X, 60) == 0.0
    pe = probe_error(lambda X: A @ X, lambda X: (A - E) @ X, 60, nprobe=4000)
    assert abs(pe - np.linalg.norm(E) / np.linalg.norm(A)) < 0.01


def test_kernel_matrix_hand_values():
    """The kernels of the experiments at hand-computed points: log|x - y| is
    log 5 and 1/|x - y| is 1/5 at (0, 0)-(3, 4) (a 3-4-5 triangle), 0 on the
    diagonal and between coincident points; 1D and 3D distances likewise
    (a slip such as log r^2 for log r, or a squared distance, fails)."""
    P = np.array([[0.0, 0.0], [3.0, 4.0], [3.0, 4.0], [-1.0, 0.0]])
    L = kernel_matrix(P, P, "log")
    R = kernel_matrix(P, P, "inv_r")
    assert L[0, 1] == pytest.approx(np.log(5.0), rel=1e-15)
    assert L[1, 0] == pytest.approx(np.log(5.0), rel=1e-15)
    assert R[0, 1] == pytest.approx(0.2, rel=1e-15)
    assert L[0, 3] == 0.0 and R[0, 3] == 1.0          # |x - y| = 1
    assert L[1, 2] == 0.0 and R[1, 2] == 0.0          # coincident points
    assert np.all(np.diag(L) == 0.0) and np.all(np.diag(R) == 0.0)
    assert L[3, 1] == pytest.approx(0.5 * np.log(32.0), rel=1e-15)   # (4, 4): sqrt 32
    x = np.array([[0.25], [2.25]])
    assert kernel_matrix(x, x, "log")[0, 1] == pytest.approx(np.log(2.0), rel=1e-15)
    assert kernel_matrix(x, x, "inv_r")[1, 0] == pytest.approx(0.5, rel=1e-15)
    q = np.array([[1.0, 2.0, 2.0], [0.0, 0.0, 0.0]])   # |q| = 3
    assert kernel_matrix(q, q, "inv_r")[0, 1] == pytest.approx(1.0 / 3.0, rel=1e-15)
    assert kernel_matrix(q, q, "log")[0, 1] == pytest.approx(np.log(3.0), rel=1e-15)
    # the black box applies the same matrix, rows included
    bb = KernelBlackBox(P, "log", dense_cache=False)
    X = np.eye(4)
    assert np.allclose(bb.apply(X), L, rtol=0, atol=1e-15)
    assert np.allclose(bb.rows([1, 3], X), L[[1, 3]], rtol=0, atol=1e-15)
