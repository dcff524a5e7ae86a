"""hm_matvec_static (the apply that allocates nothing: its scratch is the
library's static device array) against hm_matvec_op on the same H-matrices:
two calls in a row, the second with fewer right-hand sides, both orders,
FP64 and FP32, forward and adjoint, for the H^1, uniform H^1 and H^2
formats, and a call with enough right-hand sides to go through the static
scratch in several column blocks.  Every column is computed by the same
kernels, so the results must agree to rounding (1e-14 relative in FP64,
1e-6 in FP32)."""
import ctypes as C

import numpy as np
import pytest

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


def _both(hm, H, n, nrhs, dtype, order, trans, seed):
    X = np.random.default_rng(seed).standard_normal((n, nrhs))
    Xd = to_dev(X, dtype)
    Ya = hm.colmajor(n, nrhs, dtype=dtype)
    Yb = hm.colmajor(n, nrhs, dtype=dtype)
    Yb.fill_(12345.0)  # stale contents the static call must overwrite
    H.matvec(Xd, Ya, order=order, trans=trans)
    # through the C ABI directly: no Python-side allocation between the calls
    lib = hm.lib()
    rc = lib.hm_matvec_static(H.h, 1 if trans else 0, nrhs,
                              hm.HM_F32 if dtype == torch.float32 else hm.HM_F64,
                              C.c_void_p(Xd.data_ptr()), n, C.c_void_p(Yb.data_ptr()), n, order,
                              None)
    assert rc == 0, hm.lib().hm_last_error()
    a, b = to_host(Ya), to_host(Yb)
    return np.linalg.norm(a - b) / np.linalg.norm(a)


@pytest.mark.parametrize("fmt", ["h1", "uniform", "h2"])
def test_static_matvec_matches_matvec(hm, fmt):
    inst = workloads.config(1, n=4096)
    T = hm.Tree(inst.points, inst.leaf, inst.tree, inst.adm).color()
    kw = dict(h1={}, uniform=dict(uniform=True), h2=dict(h2=True))[fmt]
    H = hm.compress(T, T.kernel_blackbox(inst.kernel), tol=1e-8, r=24, seed=inst.seed, **kw)
    n = T.n
    for dtype, bar in ((torch.float64, 1e-14), (torch.float32, 1e-6)):
        for order in (hm.HM_ORDER_ORIGINAL, hm.HM_ORDER_TREE):
            for trans in (False, True):
                for nrhs, seed in ((37, 1), (5, 2)):   # second call smaller
                    d = _both(hm, H, n, nrhs, dtype, order, trans, seed)
                    assert d <= bar, (fmt, dtype, order, trans, nrhs, d)


def test_static_matvec_in_column_blocks(hm):
    """Enough right-hand sides that the 64 MiB scratch holds only part of
    them at once (order conversion copies of 2 n columns each), then a
    small call after it."""
    inst = workloads.config(1)
    T = hm.Tree(inst.points, inst.leaf, inst.tree, inst.adm).color()
    H = hm.compress(T, T.kernel_blackbox(inst.kernel), tol=1e-8, r=24, seed=inst.seed)
    n = T.n
    assert 2 * n * 8 * 700 > 64 << 20
    for nrhs, seed in ((700, 3), (3, 4)):
        d = _both(hm, H, n, nrhs, torch.float64, hm.HM_ORDER_ORIGINAL, False, seed)
        assert d <= 1e-14, (nrhs, d)
