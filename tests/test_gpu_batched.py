"""Batched compression (hm_build_forest): many independent instances in one
pass of the level pipeline, against the same instances compressed one at a
time and against the oracle's kernel rows.

Bars: test matrices bit-exact per instance (same Philox stream: key seed + i,
rows counted from the instance's first row); kernel apply equal to the
per-instance apply up to 1e-14 relative (same summation order, so normally
bit-exact); compressed operators equal to the per-instance compressions
within 1e-10 relative (the pipeline is the same per instance; only the
grouping of independent work differs); the mixed form within 1e-5 of the
FP64 form; each instance within its tolerance of the kernel matrix.
"""
import numpy as np
import pytest

import oracle
import workloads
from devutil import to_dev, to_host

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SMALL = [(3000, 1.7, 0.6), (700, 1.0, 1.0), (1800, 0.5, 2.0), (64, 1.2, 0.9), (2500, 2.0, 1.9),
         (130, 0.8, 1.3)]


@pytest.fixture(scope="module")
def hm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_03406_amd as m
    return m


def _parts():
    return [workloads.ellipse(n, a, b) for n, a, b in SMALL]


def test_forest_test_matrices_match_instances(hm):
    parts = _parts()
    F = hm.Tree(parts, 64).color()
    singles = [hm.Tree(p, 64).color() for p in parts]
    off = F.instances()
    r, seed = 24, 77
    for l in range(1, F.nlev):
        nc = F.graph(l).ncolors
        if nc == 0:
            continue
        for pas in (0, 1):
            out = hm.colmajor(F.n, nc * r)
            F.test_matrix(l, pas, r, seed, out)
            got = to_host(out)
            for i, T in enumerate(singles):
                rows = got[off[i]:off[i + 1]]
                if l > T.L or T.graph(l).ncolors == 0:
                    assert not rows.any()
                    continue
                nci = T.graph(l).ncolors
                o = hm.colmajor(T.n, nci * r)
                T.test_matrix(l, pas, r, seed + i, o)
                want = to_host(o)
                assert np.array_equal(rows[:, :nci * r], want), (l, pas, i)
                assert not rows[:, nci * r:].any()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_forest_kernel_apply_is_block_diagonal(hm, dtype):
    parts = _parts()
    F = hm.Tree(parts, 64)
    off = F.instances()
    tdt = torch.float64 if dtype == "f64" else torch.float32
    X = np.random.default_rng(3).standard_normal((F.n, 40))
    Y = hm.colmajor(F.n, 40, dtype=tdt)
    F.kernel_apply("log", to_dev(X, tdt), Y)          # tree order
    got = to_host(Y)
    for i, p in enumerate(parts):
        T = hm.Tree(p, 64)
        Yi = hm.colmajor(T.n, 40, dtype=tdt)
        T.kernel_apply("log", to_dev(X[off[i]:off[i + 1]], tdt), Yi)
        want = to_host(Yi)
        err = np.linalg.norm(got[off[i]:off[i + 1]] - want) / np.linalg.norm(want)
        assert err <= 1e-14, (i, err)
    # original order against the oracle's rows of the block-diagonal kernel
    if dtype == "f64":
        Yo = hm.colmajor(F.n, 40)
        F.kernel_apply("log", to_dev(X), Yo, order=hm.HM_ORDER_ORIGINAL)
        go = to_host(Yo)
        for i, p in enumerate(parts):
            kb = oracle.KernelBlackBox(p, "log", dense_cache=False)
            rows = np.arange(0, p.shape[0], 7)
            want = kb.rows(rows, X[off[i]:off[i + 1]])
            assert np.linalg.norm(go[off[i] + rows] - want) <= 1e-13 * np.linalg.norm(want)


def _compress_pair(hm, parts, prec, tol, r, seed):
    F = hm.Tree(parts, 64).color()
    HF = hm.compress(F, F.kernel_blackbox("log"), tol=tol, r=r, seed=seed, prec=prec)
    singles = []
    for i, p in enumerate(parts):
        T = hm.Tree(p, 64).color()
        singles.append((T, hm.compress(T, T.kernel_blackbox("log"), tol=tol, r=r, seed=seed + i,
                                       prec=prec)))
    return F, HF, singles


def test_forest_compression_equals_instances(hm):
    parts = _parts()
    tol, r, seed = 1e-8, 24, 500
    F, HF, singles = _compress_pair(hm, parts, hm.HM_PREC_F64, tol, r, seed)
    off = F.instances()
    X = np.random.default_rng(9).standard_normal((F.n, 3))
    Y = hm.colmajor(F.n, 3)
    HF.matvec(to_dev(X), Y)
    got = to_host(Y)
    st = HF.stats()
    sts = [H.stats() for _, H in singles]
    assert st["npairs"] == sum(s["npairs"] for s in sts)
    assert st["nnear"] == sum(s["nnear"] for s in sts)
    assert st["max_rank"] == max(s["max_rank"] for s in sts)
    assert st["saturated"] == 0
    assert abs(st["nfloats"] - sum(s["nfloats"] for s in sts)) <= 5e-3 * st["nfloats"]
    assert abs(st["flops_blackbox"] - sum(s["flops_blackbox"] for s in sts)) <= \
        1e-12 * st["flops_blackbox"]
    for i, (T, H) in enumerate(singles):
        Yi = hm.colmajor(T.n, 3)
        H.matvec(to_dev(X[off[i]:off[i + 1]]), Yi)
        want = to_host(Yi)
        d = np.linalg.norm(got[off[i]:off[i + 1]] - want) / np.linalg.norm(want)
        print("instance", i, "n", T.n, "forest vs alone", d)
        assert d <= 1e-10, (i, d)
        # and the instance against its kernel matrix
        A = oracle.kernel_matrix(parts[i], parts[i], "log")
        e = np.linalg.norm(got[off[i]:off[i + 1]] - A @ X[off[i]:off[i + 1]]) / \
            np.linalg.norm(A @ X[off[i]:off[i + 1]])
        assert e <= 10 * tol, (i, e)


def test_forest_mixed_against_fp64(hm):
    parts = _parts()
    F = hm.Tree(parts, 64).color()
    bb = F.kernel_blackbox("log")
    H64 = hm.compress(F, bb, tol=1e-6, r=24, seed=9)
    H32 = hm.compress(F, bb, tol=1e-6, r=24, seed=9, prec=hm.HM_PREC_MIXED)
    X = np.random.default_rng(4).standard_normal((F.n, 4))
    Y64, Y32 = hm.colmajor(F.n, 4), hm.colmajor(F.n, 4)
    H64.matvec(to_dev(X), Y64)
    H32.matvec(to_dev(X), Y32)
    a, b = to_host(Y64), to_host(Y32)
    err = np.linalg.norm(a - b) / np.linalg.norm(a)
    print("mixed vs fp64 (forest):", err)
    assert err <= 1e-5


def test_full_size_batched_ellipses(hm):
    """The batched workload at full size: 64 ellipses, N log-uniform in
    [2048, 32768], tol 1e-6, mixed precision.  No rank saturation; rows of
    H X against kernel rows computed one by one, for every instance."""
    insts = workloads.batched_ellipses()
    r = insts[0].r
    parts = [inst.points for inst in insts]
    F = hm.Tree(parts, 64).color()
    H = hm.compress(F, F.kernel_blackbox("log"), tol=insts[0].tol, r=r, seed=insts[0].seed,
                    prec=hm.HM_PREC_MIXED)
    st = H.stats()
    print("batched:", F.n, "points;", {k: st[k] for k in ("cols_A", "cols_At", "max_rank",
                                                          "saturated", "leaf_colors")},
          [c for c in st["colors"] if c])
    assert st["saturated"] == 0
    off = F.instances()
    X = np.random.default_rng(12).standard_normal((F.n, 2))
    Y = hm.colmajor(F.n, 2)
    H.matvec(to_dev(X), Y)
    got = to_host(Y)
    worst = 0.0
    for i, inst in enumerate(insts):
        kb = oracle.KernelBlackBox(inst.points, "log", dense_cache=False)
        rows = np.random.default_rng(100 + i).choice(inst.points.shape[0], 8, replace=False)
        want = kb.rows(rows, X[off[i]:off[i + 1]])
        e = np.linalg.norm(got[off[i] + rows] - want) / np.linalg.norm(want)
        worst = max(worst, e)
    print("worst sampled-row error over instances:", worst)
    assert worst <= 1e-5
