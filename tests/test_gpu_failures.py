"""Failure paths of hm_compress through the C ABI: a caller's black box that
returns nonzero (HM_E_CALLBACK), on its first call or after some samples
were taken, and one whose samples hold a NaN (HM_E_NUMERIC).  The
compression fails with that code and makes no H-matrix, every device block
it took is back with the caller's allocator afterwards (only the tree's
device copy, made by an earlier compression, stays), and the same tree
compresses normally right after, to the same operator as before."""
import gc

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


def _settle():
    gc.collect()
    torch.cuda.synchronize()


def _apply(hm, H, X):
    Y = hm.colmajor(X.shape[0], X.shape[1])
    H.matvec(X, Y)
    return to_host(Y)


@pytest.fixture(scope="module")
def setup(hm):
    inst = workloads.config(1, n=2048)
    pts = inst.points
    T = hm.Tree(pts, inst.leaf, inst.tree, inst.adm).color()
    A = oracle.kernel_matrix(pts, pts, inst.kernel)
    Ad = to_dev(A)
    dense = hm.dense_blackbox(Ad)
    X = to_dev(np.random.default_rng(8).standard_normal((pts.shape[0], 3)))
    return inst, T, A, dense, X


def test_callback_failure(hm, setup):
    inst, T, A, dense, X = setup
    al = hm.TorchAllocator()
    kw = dict(tol=1e-8, r=24, seed=inst.seed, allocator=al)
    H = hm.compress(T, dense, **kw)
    want = _apply(hm, H, X)
    del H
    _settle()
    held = al.live_bytes()  # the tree's device copy (made by that compression)
    assert held > 0
    calls = []

    for fail_at in (0, 3):
        def apply(ctx, trans, n, ncols, dtype, Xp, ldx, Yp, ldy, stream, fail_at=fail_at):
            calls.append(ncols)
            if len(calls) > fail_at:
                return 7
            return dense.apply(dense.ctx, trans, n, ncols, dtype, Xp, ldx, Yp, ldy, stream)

        fn = hm.APPLY_FN(apply)
        bb = hm.BlackBox(fn, None, dense.order, dense.symmetric, dense.dtypes)
        calls.clear()
        with pytest.raises(hm.HMError) as e:
            hm.compress(T, bb, **kw)
        assert e.value.code == hm.HM_E_CALLBACK, e.value
        assert len(calls) == fail_at + 1  # nothing called after the failure
        _settle()
        assert al.live_bytes() == held, (fail_at, al.live_bytes(), held)
    H = hm.compress(T, dense, **kw)
    assert np.array_equal(_apply(hm, H, X), want)
    del H
    _settle()
    assert al.live_bytes() == held


def test_nan_in_samples(hm, setup):
    inst, T, A, dense, X = setup
    al = hm.TorchAllocator()
    kw = dict(tol=1e-8, r=24, seed=inst.seed, allocator=al)
    H = hm.compress(T, dense, **kw)
    want = _apply(hm, H, X)
    del H
    _settle()
    held = al.live_bytes()
    for bad in (np.nan, np.inf):
        B = A.copy()
        B[5, 1000] = bad  # one entry: its row's samples carry it
        bd = hm.dense_blackbox(to_dev(B))
        with pytest.raises(hm.HMError) as e:
            hm.compress(T, bd, **kw)
        assert e.value.code == hm.HM_E_NUMERIC, e.value
        del bd
        _settle()
        assert al.live_bytes() == held, (bad, al.live_bytes(), held)
    H = hm.compress(T, dense, **kw)
    assert np.array_equal(_apply(hm, H, X), want)
