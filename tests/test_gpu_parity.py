"""GPU parity: every step of the path through the C ABI against the oracle.

Tolerances (FP64 path): Philox words bit-exact; Gaussians within 8 ulps
(libm vs device log/sin/cos); kernel apply within 1e-13 relative Frobenius
and, element by element, within 1e-13 of sum_j |A_ij X_j| (the scale of a
sum's rounding); reconstructed blocks within 1e-10 of the block norm plus a
floor of 1e-12 ||A|| wherever the GPU and the oracle chose the same ranks (a
pivot chosen differently between near-equal column norms moves the basis
but not the block); a rank decided differently at the tolerance is counted
(at most 1 % of the blocks) and held to 10 tol; the whole operator within
1e-8 of the oracle's.  Mixed path (FP32 kernel apply and peel): 1e-5
relative Frobenius against the FP64 oracle.
"""
import numpy as np
import pytest

import workloads
import oracle
from synth import exact_h1
from devutil import PerturbedDense, level_worst, to_dev, to_host, dense_of, pair_parity, block_norms

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_03406_amd as m
    return m


def test_device_properties(hm):
    p = torch.cuda.get_device_properties(0)
    print("device:", p.name, "gcnArch:", getattr(p, "gcnArchName", "?"),
          "CUs:", p.multi_processor_count, "mem GB:", p.total_memory / 2 ** 30,
          "smem/block:", getattr(p, "shared_memory_per_block", "?"))


def test_philox_known_answers(hm):
    rows = []
    for line in open("tests/golden/philox4x32_10_kat.txt"):
        if not line.startswith("#") and line.strip():
            rows.append([int(x, 16) for x in line.split()])
    for w in rows:
        ctr = np.array(w[:4], np.uint32)
        c = torch.from_numpy(ctr.view(np.int32)).cuda()
        out = torch.zeros(4, dtype=torch.int32, device="cuda")
        hm.philox(c, w[4], w[5], out)
        got = out.cpu().numpy().view(np.uint32)
        assert [int(x) for x in got] == w[6:10]
    # many counters against the oracle
    rng = np.random.default_rng(1)
    ctr = rng.integers(0, 2 ** 32, size=(5000, 4), dtype=np.uint64).astype(np.uint32)
    c = torch.from_numpy(ctr.reshape(-1).view(np.int32)).cuda()
    out = torch.zeros(5000 * 4, dtype=torch.int32, device="cuda")
    hm.philox(c, 0x12345678, 0x9abcdef0, out)
    got = out.cpu().numpy().view(np.uint32).reshape(5000, 4)
    want = np.stack(oracle.philox4x32_10(ctr[:, 0], ctr[:, 1], ctr[:, 2], ctr[:, 3],
                                         0x12345678, 0x9abcdef0), axis=1)
    assert np.array_equal(got, want)


TREES = [
    ("grid", lambda: (workloads.grid_1d(64), 8, "geometric", "strong")),
    ("hodlr", lambda: (workloads.uniform_line(1024, 1), 64, "index_binary", "weak")),
    ("curve", lambda: (workloads.star_curve(2048), 64, "geometric", "strong")),
    ("sphere", lambda: (workloads.sphere(2500, 3), 128, "geometric", "strong")),
]


@pytest.mark.parametrize("name,make", TREES)
def test_test_matrices(hm, name, make):
    pts, leaf, kind, adm = make()
    T = hm.Tree(pts, leaf, kind, adm).color()
    O = oracle.OTree(pts, leaf, kind, adm)
    for r in (6, 7):
        for l in O.sampled_levels():
            for pas in (0, 1):
                want = oracle.test_matrix(O, l, pas, 2024, r)
                out = hm.colmajor(T.n, want.shape[1])
                T.test_matrix(l, pas, r, 2024, out)
                got = to_host(out)
                assert np.array_equal(got == 0, want == 0)
                nz = want != 0
                assert np.max(np.abs(got[nz] - want[nz]) / np.abs(want[nz])) < 8 * 2.2e-16 * 4
                out32 = hm.colmajor(T.n, want.shape[1], dtype=torch.float32)
                T.test_matrix(l, pas, r, 2024, out32)
                assert np.allclose(to_host(out32), want.astype(np.float32), rtol=3e-7, atol=0)


KAPPLY = [(1, "log", 1000, 37), (2, "log", 1500, 300), (3, "inv_r", 1333, 70), (2, "log", 65, 1),
          (3, "inv_r", 17, 16), (2, "inv_r", 700, 129), (1, "log", 3000, 257)]


@pytest.mark.parametrize("dim,kernel,n,ncols", KAPPLY)
def test_kernel_apply(hm, dim, kernel, n, ncols):
    pts = workloads.random_points(n, dim, 100 + n)
    T = hm.Tree(pts, 32, "geometric", "strong")
    perm = T.perm()
    X = np.random.default_rng(n).standard_normal((n, ncols))
    A = oracle.kernel_matrix(pts, pts, kernel)
    want = A @ X                               # original order
    # element-wise scale of a sum's rounding: sum_j |A_ij X_jc|
    scale = np.abs(A) @ np.abs(X)
    Xd, Yd = to_dev(X), hm.colmajor(n, ncols)
    T.kernel_apply(kernel, Xd, Yd, order=hm.HM_ORDER_ORIGINAL)
    got = to_host(Yd)
    assert np.linalg.norm(got - want) <= 1e-13 * np.linalg.norm(want)
    assert np.max(np.abs(got - want) / scale) <= 1e-13
    Xt = to_dev(X[perm])                       # tree order
    T.kernel_apply(kernel, Xt, Yd, order=hm.HM_ORDER_TREE)
    assert np.linalg.norm(to_host(Yd) - want[perm]) <= 1e-13 * np.linalg.norm(want)
    X32, Y32 = to_dev(X, torch.float32), hm.colmajor(n, ncols, dtype=torch.float32)
    T.kernel_apply(kernel, X32, Y32, order=hm.HM_ORDER_ORIGINAL)
    got32 = to_host(Y32)
    assert np.linalg.norm(got32 - want) <= 2e-5 * np.linalg.norm(want)
    # FP32 inputs: X rounded to FP32 (u32 per term) plus the FP32 kernel values
    assert np.max(np.abs(got32 - want) / scale) <= 1e-5


def _block_parity(T, O, Hg, Ho, A, rel=1e-10, mismatch_rel=None):
    """Every admissible block U B V* and every leaf block against the
    oracle's: within rel of the block norm where the ranks agree; a rank
    decided differently (a singular value at the tolerance) is counted and
    held to mismatch_rel.  Returns (worst, mismatches, blocks)."""
    floor = 1e-12 * np.linalg.norm(A)

    def pairs():
        for l in O.sampled_levels():
            g = Hg.export_level(l)
            o = Ho.lowrank[l]
            assert len(g) == len(o)
            for (a, b, U, B, V), (a2, b2, U2, B2, V2) in zip(g, o):
                assert (a, b) == (a2, b2)
                # orthonormal bases
                if U.shape[1]:
                    assert np.allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-12)
                if V.shape[1]:
                    assert np.allclose(V.T @ V, np.eye(V.shape[1]), atol=1e-12)
                yield (l, a, b, U @ B @ V.T, U2 @ B2 @ V2.T, (U.shape[1], V.shape[1]),
                       (U2.shape[1], V2.shape[1]))
    res = pair_parity(O, pairs(), block_norms(O, A), rel,
                      rel if mismatch_rel is None else mismatch_rel, floor)
    gn = Hg.export_near()
    assert len(gn) == len(Ho.near)
    lim = rel if res[1] == 0 else (rel if mismatch_rel is None else mismatch_rel)
    for (a, b, D), (a2, b2, D2) in zip(gn, Ho.near):
        assert (a, b) == (a2, b2)
        assert np.linalg.norm(D - D2) <= lim * np.linalg.norm(D2) + floor
    return res


@pytest.mark.parametrize("case", ["strong2d", "curve", "hodlr", "strong3d"])
def test_exact_recovery_dense_blackbox(hm, case):
    if case == "strong2d":
        args = (workloads.random_points(700, 2, 11), 16, "geometric", "strong")
    elif case == "strong3d":
        args = (workloads.random_points(900, 3, 12), 24, "geometric", "strong")
    elif case == "curve":
        args = (workloads.star_curve(900), 20, "geometric", "strong")
    else:
        args = (workloads.uniform_line(512, 3), 32, "index_binary", "weak")
    O = oracle.OTree(*args)
    T = hm.Tree(*args).color()
    A = exact_h1(O, 4, seed=5)
    Ad = to_dev(A)
    bb = hm.dense_blackbox(Ad)
    H = hm.compress(T, bb, rank=4, r=10, seed=77)
    n = O.n
    D = dense_of(hm, H, n)
    assert np.linalg.norm(D - A) <= 1e-11 * np.linalg.norm(A)
    Ho = oracle.compress(O, oracle.DenseBlackBox(A), 10, k=4, seed=77)
    assert _block_parity(T, O, H, Ho, A, rel=1e-10)[1] == 0
    st = H.stats()
    chis = [T.graph(l).ncolors for l in O.sampled_levels()]
    assert st["cols_At"] == 10 * sum(chis)
    assert st["cols_A"] == 10 * sum(chis) + T.graph(-1).ncolors * O.leaf_max()
    # tolerance mode finds the exact ranks
    Ht = hm.compress(T, bb, tol=1e-9, r=14, seed=78)
    assert np.linalg.norm(dense_of(hm, Ht, n) - A) <= 1e-10 * np.linalg.norm(A)
    assert Ht.stats()["max_rank"] <= 4


def test_hodlr_config_parity(hm):
    inst = workloads.config(0)
    O = oracle.OTree(inst.points, inst.leaf, inst.tree, inst.adm)
    T = hm.Tree(inst.points, inst.leaf, inst.tree, inst.adm).color()
    bb = T.kernel_blackbox(inst.kernel)
    H = hm.compress(T, bb, rank=inst.rank, r=inst.r, seed=inst.seed)
    st = H.stats()
    assert (st["cols_A"], st["cols_At"]) == (304, 240)
    A = oracle.kernel_matrix(inst.points, inst.points, inst.kernel)
    Ho = oracle.compress(O, oracle.DenseBlackBox(A), inst.r, k=inst.rank, seed=inst.seed)
    assert _block_parity(T, O, H, Ho, A)[1] == 0
    D = dense_of(hm, H, O.n)
    assert np.linalg.norm(D - A) <= 1e-8 * np.linalg.norm(A)


@pytest.mark.parametrize("n,r", [(2048, 24), (4096, 24), (3000, 48)])
def test_curve_tolerance_parity(hm, n, r):
    inst = workloads.config(1, n=n)
    O = oracle.OTree(inst.points, inst.leaf, inst.tree, inst.adm)
    T = hm.Tree(inst.points, inst.leaf, inst.tree, inst.adm).color()
    bb = T.kernel_blackbox(inst.kernel)
    H = hm.compress(T, bb, tol=inst.tol, r=r, seed=inst.seed)
    A = oracle.kernel_matrix(inst.points, inst.points, inst.kernel)
    Ho = oracle.compress(O, oracle.DenseBlackBox(A), r, tol=inst.tol, seed=inst.seed)
    worst, mism, nblk = _block_parity(T, O, H, Ho, A, rel=1e-10, mismatch_rel=10 * inst.tol)
    D = dense_of(hm, H, O.n)
    whole = np.linalg.norm(D - Ho.dense()) / np.linalg.norm(A)
    print("curve N=%d: worst block diff %.1e, rank mismatches %d of %d, whole %.1e"
          % (n, worst, mism, nblk, whole))
    assert mism <= 0.01 * nblk
    assert whole <= 1e-8
    assert np.linalg.norm(D - A) <= inst.tol * np.linalg.norm(A)
    assert H.stats()["saturated"] == 0


def test_sphere_tolerance_parity(hm):
    inst = workloads.config(2, n=3000)
    O = oracle.OTree(inst.points, inst.leaf, inst.tree, inst.adm)
    T = hm.Tree(inst.points, inst.leaf, inst.tree, inst.adm).color()
    bb = T.kernel_blackbox(inst.kernel)
    H = hm.compress(T, bb, tol=inst.tol, r=inst.r, seed=inst.seed)
    A = oracle.kernel_matrix(inst.points, inst.points, inst.kernel)
    Ho = oracle.compress(O, oracle.DenseBlackBox(A), inst.r, tol=inst.tol, seed=inst.seed)
    worst, mism, nblk = _block_parity(T, O, H, Ho, A, rel=1e-10, mismatch_rel=10 * inst.tol)
    D = dense_of(hm, H, O.n)
    whole = np.linalg.norm(D - Ho.dense()) / np.linalg.norm(A)
    print("sphere N=3000: worst block diff %.1e, rank mismatches %d of %d, whole %.1e"
          % (worst, mism, nblk, whole))
    assert mism <= 0.01 * nblk
    assert whole <= 1e-8
    assert np.linalg.norm(D - A) <= 5 * inst.tol * np.linalg.norm(A)


def test_matvec_against_exported_factors(hm):
    inst = workloads.config(1, n=3000)
    O = oracle.OTree(inst.points, inst.leaf, inst.tree, inst.adm)
    T = hm.Tree(inst.points, inst.leaf, inst.tree, inst.adm).color()
    H = hm.compress(T, T.kernel_blackbox("log"), tol=1e-8, r=24, seed=3)
    Hc = oracle.HMatrix(O)          # the GPU factors, applied by the oracle's loop
    for l in O.sampled_levels():
        Hc.lowrank[l] = H.export_level(l)
    Hc.near = H.export_near()
    for nrhs in (1, 7, 64):
        X = np.random.default_rng(nrhs).standard_normal((O.n, nrhs))
        want = Hc.matvec(X)
        Y = hm.colmajor(O.n, nrhs)
        H.matvec(to_dev(X), Y)
        assert np.linalg.norm(to_host(Y) - want) <= 1e-13 * np.linalg.norm(want)
        Yt = hm.colmajor(O.n, nrhs)
        H.matvec(to_dev(X[O.perm]), Yt, order=hm.HM_ORDER_TREE)
        assert np.linalg.norm(to_host(Yt) - want[O.perm]) <= 1e-13 * np.linalg.norm(want)
        Y32 = hm.colmajor(O.n, nrhs, dtype=torch.float32)
        H.matvec(to_dev(X, torch.float32), Y32)
        assert np.linalg.norm(to_host(Y32) - want) <= 1e-5 * np.linalg.norm(want)


@pytest.mark.parametrize("cfg,n,tol,r", [(1, 4096, 1e-6, 24), (1, 4096, 1e-8, 24),
                                         (2, 4000, 1e-6, 32)])
def test_mixed_precision_against_oracle(hm, cfg, n, tol, r):
    """Mixed form (FP32 kernel apply and peel, FP64 QR and couplings)
    against the FP64 oracle's compression of the same inputs, tolerance and
    r: the operators within 1e-5 of each other (relative Frobenius)."""
    inst = workloads.config(cfg, n=n)
    O = oracle.OTree(inst.points, inst.leaf, inst.tree, inst.adm)
    T = hm.Tree(inst.points, inst.leaf, inst.tree, inst.adm).color()
    bb = T.kernel_blackbox(inst.kernel)
    A = oracle.kernel_matrix(inst.points, inst.points, inst.kernel)
    Ho = oracle.compress(O, oracle.DenseBlackBox(A), r, tol=tol, seed=inst.seed)
    H32 = hm.compress(T, bb, tol=tol, r=r, seed=inst.seed, prec=hm.HM_PREC_MIXED)
    D32, Do = dense_of(hm, H32, T.n), Ho.dense()
    e = np.linalg.norm(D32 - Do) / np.linalg.norm(Do)
    print("mixed vs FP64 oracle (%s, tol %g): %.2e; mixed vs dense %.2e, oracle vs dense %.2e"
          % (inst.name, tol, e, np.linalg.norm(D32 - A) / np.linalg.norm(A),
             np.linalg.norm(Do - A) / np.linalg.norm(A)))
    assert e <= 1e-5
    assert H32.stats()["saturated"] == 0


def test_full_size_star_curve_sampled_rows(hm):
    """The benchmark workload (N = 16384, tol 1e-8) in the launch shape the
    benchmark times; rows of H X checked against the kernel rows one by one."""
    inst = workloads.config(1)
    T = hm.Tree(inst.points, inst.leaf, inst.tree, inst.adm).color()
    bb = T.kernel_blackbox(inst.kernel)
    H = hm.compress(T, bb, tol=inst.tol, r=24, seed=inst.seed)
    st = H.stats()
    assert st["saturated"] == 0 and st["max_rank"] <= 14
    X = np.random.default_rng(5).standard_normal((T.n, 8))
    Y = hm.colmajor(T.n, 8)
    H.matvec(to_dev(X), Y)
    got = to_host(Y)
    rows = np.random.default_rng(6).choice(T.n, 96, replace=False)
    kb = oracle.KernelBlackBox(inst.points, inst.kernel, dense_cache=False)
    want = kb.rows(rows, X)
    assert np.linalg.norm(got[rows] - want) <= 1e-7 * np.linalg.norm(want)


def test_full_size_sphere_sampled_rows(hm):
    """The 3D workload at full size (N = 65536 on the unit sphere, 1/r kernel,
    leaves <= 128, tol 1e-6, r = 32: at r = 24 a few blocks reach the rank
    cap r - p): no rank saturation, and rows of H X against kernel rows
    computed one by one."""
    inst = workloads.config(2)
    T = hm.Tree(inst.points, inst.leaf, inst.tree, inst.adm).color()
    bb = T.kernel_blackbox(inst.kernel)
    assert inst.r == 32
    H = hm.compress(T, bb, tol=inst.tol, r=inst.r, seed=inst.seed)
    st = H.stats()
    print("sphere N=65536:", {k: st[k] for k in ("cols_A", "cols_At", "max_rank", "saturated",
                                               "leaf_colors", "nfloats")},
          [c for c in st["colors"] if c])
    assert st["saturated"] == 0
    X = np.random.default_rng(7).standard_normal((T.n, 4))
    Y = hm.colmajor(T.n, 4)
    H.matvec(to_dev(X), Y)
    got = to_host(Y)
    rows = np.random.default_rng(8).choice(T.n, 64, replace=False)
    kb = oracle.KernelBlackBox(inst.points, inst.kernel, dense_cache=False)
    want = kb.rows(rows, X)
    err = np.linalg.norm(got[rows] - want) / np.linalg.norm(want)
    print("sampled-row error", err)
    assert err <= 10 * inst.tol


def test_saturation_retry_and_strict(hm):
    """Tolerance mode with too few columns: blocks reach the cap r - p.
    max_retries recompresses with r + 8 until no block does; HM_FLAG_STRICT
    turns a remaining saturation into HM_E_SATURATED."""
    inst = workloads.config(2, n=3000)
    T = hm.Tree(inst.points, inst.leaf, inst.tree, inst.adm).color()
    bb = T.kernel_blackbox(inst.kernel)
    H0 = hm.compress(T, bb, tol=inst.tol, r=16, seed=inst.seed)
    assert H0.stats()["saturated"] > 0 and H0.stats()["retries"] == 0
    H = hm.compress(T, bb, tol=inst.tol, r=16, seed=inst.seed, max_retries=4)
    st = H.stats()
    print("retries", st["retries"], "r", st["r"], "max rank", st["max_rank"])
    assert st["saturated"] == 0 and st["retries"] >= 1 and st["r"] == 16 + 8 * st["retries"]
    # the retried result is the compression at the final r
    H2 = hm.compress(T, bb, tol=inst.tol, r=st["r"], seed=inst.seed)
    X = np.random.default_rng(3).standard_normal((T.n, 2))
    a, b = hm.colmajor(T.n, 2), hm.colmajor(T.n, 2)
    H.matvec(to_dev(X), a)
    H2.matvec(to_dev(X), b)
    assert np.array_equal(to_host(a), to_host(b))
    with pytest.raises(hm.HMError) as e:
        hm.compress(T, bb, tol=inst.tol, r=16, seed=inst.seed, strict=True)
    assert e.value.code == hm.HM_E_SATURATED


@pytest.mark.parametrize("fmt", ["h1", "uniform", "h2"])
def test_tree_without_sampled_levels(hm, fmt):
    """A point set small enough that no level has an admissible pair: the
    compression is the leaf pass alone, exactly the dense matrix (the
    neighbor blocks cover it)."""
    pts = workloads.random_points(100, 2, 21)
    T = hm.Tree(pts, 64).color()
    A = oracle.kernel_matrix(pts, pts, "log")
    kw = dict(h1={}, uniform=dict(uniform=True), h2=dict(h2=True))[fmt]
    H = hm.compress(T, T.kernel_blackbox("log"), tol=1e-8, r=24, seed=3, **kw)
    st = H.stats()
    assert st["npairs"] == 0
    X = np.random.default_rng(2).standard_normal((100, 3))
    Y = hm.colmajor(100, 3)
    H.matvec(to_dev(X), Y)
    assert np.linalg.norm(to_host(Y) - A @ X) <= 1e-13 * np.linalg.norm(A @ X)


def test_pattern_peel_with_many_boxes_per_item(hm):
    """The projection's segment list holds at most 256 boxes of the sampled
    level per item.  HODLR trees on N = 4096 points: with leaves of 8 (512
    leaves) the level-1 column boxes hold exactly 256 boxes of the finest
    level, the most a list takes; with leaves of 4 they hold 512, and the
    projection sweeps such items densely instead.  Fixed rank 12 lies well
    below the blocks' numerical rank (error 1.2e-6), so the truncated factors
    move with rounding: each block is held to 10 times the oracle's own
    response to a one-ulp perturbation of its products (as for the uniform
    format at fixed rank), the whole operator likewise, and the error against
    the kernel matrix to 1.5 times the oracle's."""
    for n, leaf in ((4096, 8), (4096, 4)):
        pts = workloads.uniform_line(n, 7)
        T = hm.Tree(pts, leaf, "index_binary", "weak").color()
        O = oracle.OTree(pts, leaf, "index_binary", "weak")
        A = oracle.kernel_matrix(pts, pts, "log")
        H = hm.compress(T, T.kernel_blackbox("log"), rank=12, r=22, seed=17)
        Ho = oracle.compress(O, oracle.DenseBlackBox(A), 22, k=12, seed=17)
        Hp = oracle.compress(O, PerturbedDense(A, seed=1), 22, k=12, seed=17)
        blocks = {l: H.export_level(l) for l in O.sampled_levels()}
        bn = block_norms(O, A)
        sens = level_worst(O, Ho.lowrank, Hp.lowrank, bn)
        gpu = level_worst(O, Ho.lowrank, blocks, bn)
        D, Do, Dp = dense_of(hm, H, n), Ho.dense(), Hp.dense()
        nA = np.linalg.norm(A)
        whole, whole_p = np.linalg.norm(D - Do) / nA, np.linalg.norm(Dp - Do) / nA
        err, err_o = np.linalg.norm(D - A) / nA, np.linalg.norm(Do - A) / nA
        print("leaf %d: err %.2e (oracle %.2e), GPU vs oracle %.1e (rounding response %.1e), "
              "per level %s against %s" % (leaf, err, err_o, whole, whole_p,
                                           ["%.1e" % gpu[l] for l in sorted(gpu)],
                                           ["%.1e" % sens[l] for l in sorted(sens)]))
        for l in gpu:
            assert gpu[l] <= 10 * sens[l] + 1e-10, (leaf, l, gpu[l], sens[l])
        assert whole <= 10 * whole_p + 1e-10
        assert err <= 1.5 * err_o + 1e-12
