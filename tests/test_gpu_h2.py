"""H^2 compression on the GPU (hm_compress with HM_FORMAT_H2) against the
oracle's compress_h2.

The row bases follow the paper's rule (plain sum of the stage-2 samples,
augmented); the Gaussian-weighted extension is checked against the
oracle's extension.

Bars (FP64): exact H^2 matrices recovered to 1e-11 relative, every block
(through the nested bases) equal to the oracle's within 1e-10 of the block
norm, the finest level's bases equal to the oracle's singular vectors
within 1e-9 (same signs: the largest entry positive), float and matvec
counts equal to the oracle's; kernel matrices: blocks within 1e-10 of the
block norm of the oracle's (plus 1e-12 ||A||) where the ranks agree (rank
mismatches counted, at most 1 %, held to 10 tol), error equal to the
oracle's, storage below the uniform H^1 form.  Mixed within 1e-5 of the
FP64 oracle at fixed rank; a forest equal to its instances alone within
1e-10; plan replays equal to eager.
"""
import numpy as np
import pytest

import oracle
import workloads
from synth import exact_h2
from devutil import PerturbedDense, level_worst, to_dev, to_host, dense_of, pair_parity, block_norms

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_03406_amd as m
    return m


TREES = {
    "strong2d": lambda: (workloads.random_points(700, 2, 11), 16, "geometric", "strong"),
    "strong3d": lambda: (workloads.random_points(900, 3, 12), 24, "geometric", "strong"),
    "curve": lambda: (workloads.star_curve(900), 20, "geometric", "strong"),
    "hodlr": lambda: (workloads.uniform_line(512, 3), 32, "index_binary", "weak"),
}


def _parity(O, H, Ho, A, rel, mismatch_rel=None):
    """Every block through the nested bases against the oracle's
    (pair_parity).  Returns (worst difference where the ranks agree, rank
    mismatches, blocks)."""
    Ue, Ve = Ho.effective_bases()

    def pairs():
        for l in Ho.levels:
            g = H.export_level(l)
            o = Ho.B[l]
            assert len(g) == len(o)
            for (a, b, U, B, V), (a2, b2, B2) in zip(g, o):
                assert (a, b) == (a2, b2)
                yield (l, a, b, U @ B @ V.T, Ue[l][a] @ B2 @ Ve[l][b].T, B.shape, B2.shape)
    return pair_parity(O, pairs(), block_norms(O, A), rel,
                       rel if mismatch_rel is None else mismatch_rel,
                       1e-12 * np.linalg.norm(A))


@pytest.mark.parametrize("name", ["strong2d", "strong3d", "curve", "hodlr"])
def test_h2_exact_recovery(hm, name):
    args = TREES[name]()
    O = oracle.OTree(*args)
    T = hm.Tree(*args).color()
    A = exact_h2(O, 4, seed=5)
    bb = hm.dense_blackbox(to_dev(A))
    H = hm.compress(T, bb, rank=4, r=10, seed=77, h2=True)
    D = dense_of(hm, H, O.n)
    assert np.linalg.norm(D - A) <= 1e-11 * np.linalg.norm(A)
    Ho = oracle.compress_h2(O, oracle.DenseBlackBox(A), 10, k=4, seed=77)
    assert _parity(O, H, Ho, A, rel=1e-10)[1] == 0
    # the finest level's bases are the oracle's singular vectors, signs included
    f = Ho.levels[-1]
    seen = set()
    for a, b, U, B, V in H.export_level(f):
        if a in seen:
            continue
        seen.add(a)
        assert U.shape == Ho.Ulong[a].shape
        assert np.max(np.abs(U - Ho.Ulong[a])) <= 1e-9, (a, np.max(np.abs(U - Ho.Ulong[a])))
    st = H.stats()
    assert st["format"] == hm.HM_FORMAT_H2
    assert st["nfloats"] == Ho.floats()
    assert (st["cols_A"], st["cols_At"]) == (Ho.cols_A, Ho.cols_At)
    Ht = hm.compress(T, bb, tol=1e-9, r=14, seed=78, h2=True)
    assert np.linalg.norm(dense_of(hm, Ht, O.n) - A) <= 1e-10 * np.linalg.norm(A)


@pytest.mark.parametrize("n,tol", [(1500, 1e-8), (3000, 1e-6)])
def test_h2_kernel_parity(hm, n, tol):
    """Tolerance mode: every block within 1e-10 of the oracle's where the
    ranks agree (mismatches counted, held to 10 tol), error equal to the
    oracle's, storage and device memory below the uniform form."""
    inst = workloads.config(1, n=n)
    O = oracle.OTree(inst.points, inst.leaf, inst.tree, inst.adm)
    T = hm.Tree(inst.points, inst.leaf, inst.tree, inst.adm).color()
    A = oracle.kernel_matrix(inst.points, inst.points, inst.kernel)
    H = hm.compress(T, T.kernel_blackbox(inst.kernel), tol=tol, r=24, seed=inst.seed, h2=True)
    Ho = oracle.compress_h2(O, oracle.DenseBlackBox(A), 24, tol=tol, seed=inst.seed)
    worst, mism, nblk = _parity(O, H, Ho, A, rel=1e-10, mismatch_rel=10 * tol)
    D = dense_of(hm, H, O.n)
    err = np.linalg.norm(D - A) / np.linalg.norm(A)
    err_o = np.linalg.norm(Ho.dense() - A) / np.linalg.norm(A)
    st = H.stats()
    Hu = hm.compress(T, T.kernel_blackbox(inst.kernel), tol=tol, r=24, seed=inst.seed,
                     uniform=True)
    print("h2: err %.2e (oracle %.2e), worst block diff %.1e, rank mismatches %d of %d, "
          "floats %d (oracle %d, uniform %d)"
          % (err, err_o, worst, mism, nblk, st["nfloats"], Ho.floats(), Hu.stats()["nfloats"]))
    assert mism <= 0.01 * nblk
    assert abs(err - err_o) <= 0.05 * err_o + 1e-12
    assert abs(st["nfloats"] - Ho.floats()) <= 0.01 * Ho.floats()
    assert st["nfloats"] < Hu.stats()["nfloats"]
    assert st["saturated"] == 0
    # device memory: no per-pair copies, products or plans beside the nested form
    print("device MB: h2 %.1f, uniform %.1f" % (st["device_bytes"] / 2**20,
                                                Hu.stats()["device_bytes"] / 2**20))
    assert 0 < st["device_bytes"] < Hu.stats()["device_bytes"]


def test_h2_gamma_extension_parity(hm):
    """The Gaussian-weighted row-basis combination (HM_FLAG_MIX_GAMMA, an
    extension) against the oracle's combine="gaussian" at fixed rank."""
    inst = workloads.config(1, n=1500)
    O = oracle.OTree(inst.points, inst.leaf, inst.tree, inst.adm)
    T = hm.Tree(inst.points, inst.leaf, inst.tree, inst.adm).color()
    A = oracle.kernel_matrix(inst.points, inst.points, inst.kernel)
    H = hm.compress(T, T.kernel_blackbox(inst.kernel), rank=14, r=24, seed=inst.seed, h2=True,
                    combine="gaussian")
    Ho = oracle.compress_h2(O, oracle.DenseBlackBox(A), 24, k=14, seed=inst.seed,
                            combine="gaussian")
    worst, mism, nblk = _parity(O, H, Ho, A, rel=1e-10)
    assert mism == 0
    err = np.linalg.norm(dense_of(hm, H, O.n) - A) / np.linalg.norm(A)
    err_o = np.linalg.norm(Ho.dense() - A) / np.linalg.norm(A)
    print("h2 gamma extension: err %.2e (oracle %.2e), worst block diff %.1e" % (err, err_o, worst))
    assert abs(err - err_o) <= 0.05 * err_o + 1e-12


def test_h2_mixed_against_oracle(hm):
    """Mixed form at the paper's fixed rank against the FP64 oracle's H^2
    compression of the same inputs: within 1e-5 of it."""
    inst = workloads.config(1, n=4096)
    O = oracle.OTree(inst.points, inst.leaf, inst.tree, inst.adm)
    T = hm.Tree(inst.points, inst.leaf, inst.tree, inst.adm).color()
    bb = T.kernel_blackbox(inst.kernel)
    A = oracle.kernel_matrix(inst.points, inst.points, inst.kernel)
    Ho = oracle.compress_h2(O, oracle.DenseBlackBox(A), 24, k=14, seed=5)
    H32 = hm.compress(T, bb, rank=14, r=24, seed=5, h2=True, prec=hm.HM_PREC_MIXED)
    D32, Do = dense_of(hm, H32, T.n), Ho.dense()
    d = np.linalg.norm(D32 - Do) / np.linalg.norm(Do)
    e32 = np.linalg.norm(D32 - A) / np.linalg.norm(A)
    eo = np.linalg.norm(Do - A) / np.linalg.norm(A)
    print("mixed H2 vs FP64 oracle: %.2e; errors %.2e (oracle %.2e)" % (d, e32, eo))
    assert d <= 1e-5
    assert e32 <= eo + 1e-5


def test_h2_forest_matches_instances(hm):
    parts = [workloads.ellipse(n, a, b) for n, a, b in [(2500, 1.4, 0.6), (900, 1.0, 1.0),
                                                        (1700, 0.7, 1.9)]]
    F = hm.Tree(parts, 64).color()
    off = F.instances()
    seed = 31
    Hf = hm.compress(F, F.kernel_blackbox("log"), tol=1e-6, r=24, seed=seed, h2=True)
    X = np.random.default_rng(1).standard_normal((F.n, 3))
    Yf = hm.colmajor(F.n, 3)
    Hf.matvec(to_dev(X), Yf, order=hm.HM_ORDER_TREE)
    got = to_host(Yf)
    for i, p in enumerate(parts):
        T = hm.Tree(p, 64).color()
        Hi = hm.compress(T, T.kernel_blackbox("log"), tol=1e-6, r=24, seed=seed + i, h2=True)
        Yi = hm.colmajor(T.n, 3)
        Hi.matvec(to_dev(X[off[i]:off[i + 1]]), Yi, order=hm.HM_ORDER_TREE)
        want = to_host(Yi)
        d = np.linalg.norm(got[off[i]:off[i + 1]] - want) / np.linalg.norm(want)
        assert d <= 1e-10, (i, d)


def test_h2_plan_replays(hm):
    inst = workloads.config(1, n=3000)
    T = hm.Tree(inst.points, inst.leaf, inst.tree, inst.adm).color()
    bb = T.kernel_blackbox("log")
    He = hm.compress(T, bb, tol=1e-8, r=24, seed=7, h2=True)
    X = np.random.default_rng(1).standard_normal((T.n, 3))
    Y = hm.colmajor(T.n, 3)
    He.matvec(to_dev(X), Y)
    want = to_host(Y)
    P = hm.Plan(T, bb, tol=1e-8, r=24, seed=7, h2=True)
    for k in range(3):
        Z = hm.colmajor(T.n, 5)
        Z.normal_()
        W = hm.colmajor(T.n, 5)
        T.kernel_apply("log", Z, W)
        torch.cuda.synchronize()
        P.execute()
        Y2 = hm.colmajor(T.n, 3)
        P.hmatrix().matvec(to_dev(X), Y2)
        assert np.array_equal(to_host(Y2), want), k


def _oracle_blocks(Ho):
    Ue, Ve = Ho.effective_bases()
    return {l: [(a, b, Ue[l][a], B, Ve[l][b]) for (a, b, B) in Ho.B[l]] for l in Ho.levels}


def test_h2_kernel_fixed_rank_parity(hm):
    """Fixed rank (the setting of the paper's experiments).  The row bases
    come from the plain sum of the stage-2 samples, which is numerically
    rank-deficient for many boxes at rank 14 (its trailing singular values
    sit at the rounding level), so the directions it leaves undetermined are
    set by rounding and a correct implementation is unique only up to that:
    the oracle compressing through a black box perturbed by one rounding
    unit per entry moves blocks by up to about 1e-6 of their norm.  The GPU
    must stay within 10 times that response on every level and on the whole
    operator, with the error within 1.5 times the oracle's and equal
    stored-value counts.  (The column bases are not unique either: at rank 14
    the samples of well-separated blocks have trailing singular values at the
    rounding level.)"""
    inst = workloads.config(1, n=3000)
    O = oracle.OTree(inst.points, inst.leaf, inst.tree, inst.adm)
    T = hm.Tree(inst.points, inst.leaf, inst.tree, inst.adm).color()
    A = oracle.kernel_matrix(inst.points, inst.points, inst.kernel)
    H = hm.compress(T, T.kernel_blackbox(inst.kernel), rank=14, r=24, seed=inst.seed, h2=True)
    Ho = oracle.compress_h2(O, oracle.DenseBlackBox(A), 24, k=14, seed=inst.seed)
    Hp = oracle.compress_h2(O, PerturbedDense(A, seed=1), 24, k=14, seed=inst.seed)
    bo = _oracle_blocks(Ho)
    bg = {l: H.export_level(l) for l in Ho.levels}
    bn = block_norms(O, A)
    sens = level_worst(O, bo, _oracle_blocks(Hp), bn)
    gpu = level_worst(O, bo, bg, bn)
    Do, Dp, D = Ho.dense(), Hp.dense(), dense_of(hm, H, O.n)
    nA = np.linalg.norm(A)
    whole, whole_p = np.linalg.norm(D - Do) / nA, np.linalg.norm(Dp - Do) / nA
    err, err_o = np.linalg.norm(D - A) / nA, np.linalg.norm(Do - A) / nA
    print("h2 fixed rank: err %.2e (oracle %.2e), GPU vs oracle %.1e (rounding response %.1e), "
          "per level %s against %s" % (err, err_o, whole, whole_p,
                                       ["%.1e" % gpu[l] for l in sorted(gpu)],
                                       ["%.1e" % sens[l] for l in sorted(sens)]))
    for l in gpu:
        assert gpu[l] <= 10 * sens[l] + 1e-10, (l, gpu[l], sens[l])
    assert whole <= 10 * whole_p + 1e-10
    assert err <= 1.5 * err_o + 1e-12
    assert H.stats()["nfloats"] == Ho.floats()


def test_h2_apply_matches_oracle_passes(hm):
    """The device apply through the nested representation (upward pass,
    couplings, downward pass) against the oracle's, forward and adjoint,
    FP64 and FP32 right-hand sides."""
    inst = workloads.config(1, n=3000)
    O = oracle.OTree(inst.points, inst.leaf, inst.tree, inst.adm)
    T = hm.Tree(inst.points, inst.leaf, inst.tree, inst.adm).color()
    A = oracle.kernel_matrix(inst.points, inst.points, inst.kernel)
    # tolerance mode: the compression is unique (blocks agree to 1e-10), so
    # the two applies can be compared at a tight bar
    H = hm.compress(T, T.kernel_blackbox(inst.kernel), tol=1e-8, r=24, seed=inst.seed, h2=True)
    Ho = oracle.compress_h2(O, oracle.DenseBlackBox(A), 24, tol=1e-8, seed=inst.seed)
    perm = O.perm
    for nrhs in (1, 5, 300):
        X = np.random.default_rng(nrhs).standard_normal((O.n, nrhs))
        want = Ho.matvec(X)
        Y = hm.colmajor(O.n, nrhs)
        H.matvec(to_dev(X), Y)
        assert np.linalg.norm(to_host(Y) - want) <= 1e-9 * np.linalg.norm(want), nrhs
        wt = np.empty_like(X)
        wt[perm] = Ho.apply(X[perm], transpose=True)
        Yt = hm.colmajor(O.n, nrhs)
        H.matvec(to_dev(X), Yt, trans=True)
        assert np.linalg.norm(to_host(Yt) - wt) <= 1e-9 * np.linalg.norm(wt), nrhs
        Y32 = hm.colmajor(O.n, nrhs, dtype=torch.float32)
        H.matvec(to_dev(X, torch.float32), Y32)
        assert np.linalg.norm(to_host(Y32) - want) <= 1e-5 * np.linalg.norm(want), nrhs
