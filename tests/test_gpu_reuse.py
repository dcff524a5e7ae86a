"""Device blocks are reused across compressions (H-matrices, trees and a
compression's scratch return to a per-device cache): a compression must not
depend on what an earlier one left in its buffers.

Bar: compressing A, then a different problem B (another size, every format),
then A again gives bit-identical applies of A."""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_03406_amd as m
    return m


def _apply(hm, H, n, seed):
    X = hm.colmajor(n, 3)
    X.copy_(torch.from_numpy(np.random.default_rng(seed).standard_normal((n, 3))))
    Y = hm.colmajor(n, 3)
    H.matvec(X, Y)
    torch.cuda.synchronize()
    return Y.cpu().numpy()


@pytest.mark.parametrize("fmt", ["h1", "uniform", "h2"])
def test_compression_independent_of_reused_blocks(hm, fmt):
    kw = {"h1": {}, "uniform": {"uniform": True}, "h2": {"h2": True, "rank": 12}}[fmt]
    tol = 0.0 if "rank" in kw else 1e-8
    inst = workloads.config(1, n=3000)
    TA = hm.Tree(inst.points, inst.leaf, inst.tree, inst.adm).color()
    HA = hm.compress(TA, TA.kernel_blackbox("log"), tol=tol, r=24, seed=3, **kw)
    first = _apply(hm, HA, TA.n, 1)
    del HA
    pts = workloads.random_points(5000, 2, 21)
    TB = hm.Tree(pts, 48, "geometric", "strong").color()
    for f in ({}, {"uniform": True}, {"h2": True, "rank": 10}):
        HB = hm.compress(TB, TB.kernel_blackbox("log"), tol=0.0 if "rank" in f else 1e-6, r=20,
                         seed=5, **f)
        _apply(hm, HB, TB.n, 2)
        del HB
    del TB
    HA2 = hm.compress(TA, TA.kernel_blackbox("log"), tol=tol, r=24, seed=3, **kw)
    again = _apply(hm, HA2, TA.n, 1)
    assert np.array_equal(first, again)
