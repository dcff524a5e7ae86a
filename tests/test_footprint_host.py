"""hm_compress_footprint on the host (no device work): the device bytes a
compression will hold at once, as the server reserves them.  Checked here
for the properties the sizes must have; the GPU test of the server
(test_request_footprints_cover_their_allocations) checks the same estimate
against the peak a counting allocator sees."""
import pytest

import workloads

pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hm():
    import paper_2205_03406_amd as m
    return m


@pytest.fixture(scope="module")
def tree(hm):
    inst = workloads.config(1, n=4096)
    return hm.Tree(inst.points, inst.leaf, inst.tree, inst.adm).color()


def test_footprint_orders(hm, tree):
    fp = lambda **kw: hm.compress_footprint(tree, **kw)
    h1 = fp(tol=1e-8, r=24)
    assert h1 > 0
    # more columns per test matrix: wider samples and scratch
    assert fp(tol=1e-8, r=32) > h1
    # FP32 samples and scratch in the mixed form
    assert fp(tol=1e-8, r=24, prec=hm.HM_PREC_MIXED) < h1
    # H^2 keeps no per-pair bases and no per-pair partial projections
    assert fp(tol=1e-8, r=24, h2=True) < fp(tol=1e-8, r=24, uniform=True)
    # fixed rank 14 and tolerance mode with r = 24 size everything for the
    # same largest rank (kmax = r - p = 14): the same estimate
    assert fp(rank=14, r=24) == fp(tol=1e-8, r=24)
    # the default r = rank + p
    assert fp(rank=14) == fp(rank=14, r=24)


def test_footprint_errors(hm, tree):
    with pytest.raises(hm.HMError) as e:
        hm.compress_footprint(tree, tol=1e-8, r=80)
    assert e.value.code == hm.HM_E_ARG
    with pytest.raises(hm.HMError) as e:
        hm.compress_footprint(tree, tol=1e-8)  # tolerance mode without r
    assert e.value.code == hm.HM_E_ARG
    inst = workloads.config(1, n=1024)
    bare = hm.Tree(inst.points, inst.leaf, inst.tree, inst.adm)  # not colored
    with pytest.raises(hm.HMError) as e:
        hm.compress_footprint(bare, tol=1e-8, r=24)
    assert e.value.code == hm.HM_E_STATE
