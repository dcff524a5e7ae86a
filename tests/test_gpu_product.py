"""Compressing products of compressed operators (hm_hmatrix_blackbox,
hm_product_blackbox) and the adjoint apply (hm_matvec_op) on the GPU.

Bars: the adjoint apply equals the exported factors applied by the oracle's
adjoint loop within 1e-13 relative (FP32: 1e-5); an H^1 matrix given only
through its own applies is recovered within 1e-10; the product of two
compressed kernel operators compresses to the same blocks as the oracle's
compression of the oracle's product (within 10 tol of the block norm), to
within 5 tol of the dense product, with the oracle's matvec counts; the mixed
form within 1e-5 of FP64.
"""
import numpy as np
import pytest

import oracle
import workloads
from synth import exact_h1
from devutil import to_dev, to_host, dense_of

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_03406_amd as m
    return m


def _exported(hm, H, O):
    Hc = oracle.HMatrix(O)
    for l in O.sampled_levels():
        Hc.lowrank[l] = H.export_level(l)
    Hc.near = H.export_near()
    return Hc


@pytest.mark.parametrize("case", ["curve", "sphere"])
def test_adjoint_apply(hm, case):
    if case == "curve":
        inst = workloads.config(1, n=3000)
        args = (inst.points, inst.leaf, inst.tree, inst.adm)
        kernel = "log"
    else:
        args = (workloads.sphere(3000, 3), 128, "geometric", "strong")
        kernel = "inv_r"
    O = oracle.OTree(*args)
    T = hm.Tree(*args).color()
    H = hm.compress(T, T.kernel_blackbox(kernel), tol=1e-8, r=24, seed=3)
    ref = oracle.HMatrixBlackBox(_exported(hm, H, O))
    for nrhs in (1, 9):
        X = np.random.default_rng(nrhs).standard_normal((O.n, nrhs))
        want = ref.applyT(X)
        Y = hm.colmajor(O.n, nrhs)
        H.matvec(to_dev(X), Y, trans=True)
        assert np.linalg.norm(to_host(Y) - want) <= 1e-13 * np.linalg.norm(want)
        # tree order
        Yt = hm.colmajor(O.n, nrhs)
        H.matvec(to_dev(X[O.perm]), Yt, order=hm.HM_ORDER_TREE, trans=True)
        assert np.linalg.norm(to_host(Yt) - want[O.perm]) <= 1e-13 * np.linalg.norm(want)
        Y32 = hm.colmajor(O.n, nrhs, dtype=torch.float32)
        H.matvec(to_dev(X, torch.float32), Y32, trans=True)
        assert np.linalg.norm(to_host(Y32) - want) <= 1e-5 * np.linalg.norm(want)
        # and the forward apply against the same reference
        Yf = hm.colmajor(O.n, nrhs)
        H.matvec(to_dev(X), Yf)
        wf = ref.apply(X)
        assert np.linalg.norm(to_host(Yf) - wf) <= 1e-13 * np.linalg.norm(wf)


@pytest.mark.parametrize("order", ["original", "tree"])
def test_recompress_through_own_applies(hm, order):
    args = (workloads.random_points(700, 2, 11), 16, "geometric", "strong")
    O = oracle.OTree(*args)
    T = hm.Tree(*args).color()
    A = exact_h1(O, 4, seed=5)
    H = hm.compress(T, hm.dense_blackbox(to_dev(A)), rank=4, r=10, seed=77)
    bb = H.blackbox(hm.HM_ORDER_TREE if order == "tree" else hm.HM_ORDER_ORIGINAL)
    H2 = hm.compress(T, bb, rank=4, r=10, seed=78)
    assert np.linalg.norm(dense_of(hm, H2, O.n) - A) <= 1e-10 * np.linalg.norm(A)


def test_product_of_compressed_kernels(hm):
    pts = workloads.star_curve(1500)
    args = (pts, 64, "geometric", "strong")
    O = oracle.OTree(*args)
    T = hm.Tree(*args).color()
    K = oracle.kernel_matrix(pts, pts, "log")
    H = hm.compress(T, T.kernel_blackbox("log"), tol=1e-10, r=24, seed=1)
    Ho = oracle.compress(O, oracle.DenseBlackBox(K), 24, tol=1e-10, seed=1)
    tol = 1e-8
    bh = H.blackbox(hm.HM_ORDER_TREE)
    P = hm.product_blackbox(bh, bh)
    HP = hm.compress(T, P, tol=tol, r=24, seed=2)
    ob = oracle.CountingBlackBox(oracle.ProductBlackBox(oracle.HMatrixBlackBox(Ho),
                                                        oracle.HMatrixBlackBox(Ho)))
    HPo = oracle.compress(O, ob, 24, tol=tol, seed=2)
    KK = K @ K
    floor = 1e-12 * np.linalg.norm(KK)
    worst = 0.0
    for l in O.sampled_levels():
        for (a, b, U, B, V), (a2, b2, U2, B2, V2) in zip(HP.export_level(l), HPo.lowrank[l]):
            assert (a, b) == (a2, b2)
            a0, a1 = O.box_range(l, a)
            b0, b1 = O.box_range(l, b)
            nb = np.linalg.norm(KK[np.ix_(O.perm[a0:a1], O.perm[b0:b1])])
            d = np.linalg.norm(U @ B @ V.T - U2 @ B2 @ V2.T)
            worst = max(worst, d / nb)
            assert d <= 10 * tol * nb + floor, (l, a, b, d, nb)
    D = dense_of(hm, HP, O.n)
    err = np.linalg.norm(D - KK) / np.linalg.norm(KK)
    st = HP.stats()
    print("product: err %.2e, worst block diff %.1e, cols %d/%d" % (err, worst, st["cols_A"],
                                                                   st["cols_At"]))
    assert err <= 5 * tol
    assert (st["cols_A"], st["cols_At"]) == (ob.cols_A, ob.cols_At)
    assert st["saturated"] == 0


def test_product_mixed_and_symmetric(hm):
    inst = workloads.config(1, n=4096)
    T = hm.Tree(inst.points, inst.leaf, inst.tree, inst.adm).color()
    kb = T.kernel_blackbox("log")
    H = hm.compress(T, kb, tol=1e-10, r=24, seed=4)
    bh = H.blackbox(hm.HM_ORDER_TREE)
    P = hm.product_blackbox(bh, bh)
    assert P.symmetric == 0
    # the product of the same symmetric box is symmetric: one call per level
    assert hm.product_blackbox(kb, kb).symmetric == 1
    H64 = hm.compress(T, P, tol=1e-6, r=24, seed=9)
    H32 = hm.compress(T, P, tol=1e-6, r=24, seed=9, prec=hm.HM_PREC_MIXED)
    X = np.random.default_rng(0).standard_normal((T.n, 3))
    a, b = hm.colmajor(T.n, 3), hm.colmajor(T.n, 3)
    H64.matvec(to_dev(X), a)
    H32.matvec(to_dev(X), b)
    a, b = to_host(a), to_host(b)
    d = np.linalg.norm(a - b) / np.linalg.norm(a)
    print("mixed vs FP64 product: %.2e" % d)
    assert d <= 1e-5
    # the product applied through its factors
    Y = hm.colmajor(T.n, 3)
    Z = hm.colmajor(T.n, 3)
    H.matvec(to_dev(X), Z)
    H.matvec(Z, Y)
    want = to_host(Y)
    assert np.linalg.norm(a - want) <= 5e-6 * np.linalg.norm(want)
