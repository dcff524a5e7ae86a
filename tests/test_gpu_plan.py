"""Compression plans: the device pipeline captured once into a HIP graph and
replayed.  Every replay must give exactly what an eager compression of the
same tree, black box and options gives (same launches on the same data), with
the program's own eager work and synchronizations between the replays; a
black box whose device data change between replays gives the compression of
the new operator."""
import numpy as np
import pytest

import oracle
import workloads
from devutil import to_dev, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_03406_amd as m
    return m


def _apply(hm, H, X, dt=None):
    Y = hm.colmajor(X.shape[0], X.shape[1], dtype=dt or torch.float64)
    H.matvec(to_dev(X, dt), Y)
    return to_host(Y)


@pytest.mark.parametrize("prec", [0, 1])
def test_plan_replays_equal_eager(hm, prec):
    inst = workloads.config(1, n=3000)
    T = hm.Tree(inst.points, inst.leaf, inst.tree, inst.adm).color()
    bb = T.kernel_blackbox("log")
    tol = 1e-8 if prec == 0 else 1e-6
    He = hm.compress(T, bb, tol=tol, r=24, seed=7, prec=prec)
    X = np.random.default_rng(1).standard_normal((T.n, 3))
    want = _apply(hm, He, X)
    P = hm.Plan(T, bb, tol=tol, r=24, seed=7, prec=prec)
    print("graph nodes:", P.graph_nodes)
    assert P.graph_nodes > 10
    for k in range(3):
        # eager work of the program between replays
        Z = hm.colmajor(T.n, 5)
        Z.normal_()
        W = hm.colmajor(T.n, 5)
        T.kernel_apply("log", Z, W)
        torch.cuda.synchronize()
        P.execute()
        got = _apply(hm, P.hmatrix(), X)
        assert np.array_equal(got, want), k
        assert P.hmatrix().stats()["nfloats"] == He.stats()["nfloats"]


def test_plan_on_a_forest(hm):
    parts = [workloads.ellipse(n, a, b) for n, a, b in [(2500, 1.4, 0.6), (900, 1.0, 1.0),
                                                        (1700, 0.7, 1.9)]]
    F = hm.Tree(parts, 64).color()
    bb = F.kernel_blackbox("log")
    He = hm.compress(F, bb, tol=1e-6, r=24, seed=104, prec=hm.HM_PREC_MIXED)
    X = np.random.default_rng(2).standard_normal((F.n, 2))
    want = _apply(hm, He, X)
    P = hm.Plan(F, bb, tol=1e-6, r=24, seed=104, prec=hm.HM_PREC_MIXED)
    for _ in range(2):
        P.execute()
        torch.cuda.synchronize()
        assert np.array_equal(_apply(hm, P.hmatrix(), X), want)


def test_plan_follows_black_box_data(hm):
    """Dense black box: scaling A in place between replays scales the
    compressed operator (pivoting and ranks do not change under a power of
    two, so the factors scale exactly)."""
    pts = workloads.star_curve(900)
    T = hm.Tree(pts, 32).color()
    A = oracle.kernel_matrix(pts, pts, "log")
    Ad = to_dev(A)
    bb = hm.dense_blackbox(Ad)
    P = hm.Plan(T, bb, tol=1e-8, r=24, seed=3)
    X = np.random.default_rng(3).standard_normal((T.n, 2))
    y1 = _apply(hm, P.hmatrix(), X)
    Ad.mul_(2.0)
    torch.cuda.synchronize()
    P.execute()
    y2 = _apply(hm, P.hmatrix(), X)
    assert np.array_equal(y2, 2.0 * y1)
    Ad.mul_(0.5)
    torch.cuda.synchronize()
    P.execute()
    assert np.array_equal(_apply(hm, P.hmatrix(), X), y1)
    # and the plan's result is a compression of A
    assert np.linalg.norm(y1 - A @ X) <= 1e-7 * np.linalg.norm(A @ X)
