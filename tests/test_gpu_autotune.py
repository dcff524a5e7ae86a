"""Kernel-apply autotuner: the first launch of a shape times every column
tile width on the real operands, later launches reuse the decision.  Every
width computes the same values bit for bit, so tuned and cached launches must
agree exactly, and both must match the oracle's kernel rows."""
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


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("ncols", [40, 333])
def test_tuned_and_cached_launches_agree(hm, dtype, ncols):
    pts = workloads.ellipse(3001, 1.3, 0.7)
    T = hm.Tree(pts, 64)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    X = np.random.default_rng(ncols).standard_normal((T.n, ncols))
    Xd = to_dev(X, tdt)
    Y1 = hm.colmajor(T.n, ncols, dtype=tdt)
    Y2 = hm.colmajor(T.n, ncols, dtype=tdt)
    T.kernel_apply("log", Xd, Y1, order=hm.HM_ORDER_ORIGINAL)   # tunes this shape
    T.kernel_apply("log", Xd, Y2, order=hm.HM_ORDER_ORIGINAL)   # reuses the decision
    a, b = to_host(Y1), to_host(Y2)
    assert np.array_equal(a, b)
    table = hm.autotune_table()
    print(table)
    assert ("ncols=%d " % ncols) in table
    kb = oracle.KernelBlackBox(pts, "log", dense_cache=False)
    rows = np.arange(0, T.n, 13)
    want = kb.rows(rows, X)
    tol = 1e-13 if dtype == "f64" else 1e-6
    assert np.linalg.norm(a[rows] - want) <= tol * np.linalg.norm(want)
