"""Device-array helpers shared by the GPU tests (plain torch marshalling)."""
import numpy as np


def to_dev(X, dtype=None):
    """A host array as an (n, ncols) column-major CUDA tensor."""
    import torch
    X = np.asarray(X)
    if X.ndim == 1:
        X = X.reshape(-1, 1)
    t = torch.from_numpy(np.ascontiguousarray(X.T)).to("cuda")
    if dtype is not None:
        t = t.to(dtype)
    return t.t()


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def dense_of(hm, H, n):
    """The dense matrix an H-matrix applies (original order), column by column."""
    I = hm.colmajor(n, n)
    I.zero_()
    I.diagonal().fill_(1.0)
    Y = hm.colmajor(n, n)
    H.matvec(I, Y, order=hm.HM_ORDER_ORIGINAL)
    return to_host(Y)


def pair_parity(O, pairs, A_norm_of, rel, mismatch_rel, floor):
    """Per-block parity of admissible pairs.

    pairs: iterable of (level, a, b, gpu_block, oracle_block, gpu_ranks,
    oracle_ranks) with the blocks as dense |a| x |b| arrays (U B V*).  Where
    the GPU and the oracle chose the same ranks the difference must be within
    rel * ||A(I_a, I_b)||_F + floor; a rank chosen differently (a singular
    value at the tolerance, decided differently by rounding) is counted and
    held to mismatch_rel instead.  Returns (worst relative difference where
    the ranks agree, number of rank mismatches, number of blocks)."""
    worst = 0.0
    mism = 0
    nblk = 0
    for l, a, b, G, W, rg, ro in pairs:
        nblk += 1
        nb = A_norm_of(l, a, b)
        d = np.linalg.norm(G - W)
        if tuple(rg) == tuple(ro):
            worst = max(worst, d / max(nb, 1e-300))
            assert d <= rel * nb + floor, (l, a, b, d, nb, rg)
        else:
            mism += 1
            assert d <= mismatch_rel * nb + floor, (l, a, b, d, nb, rg, ro)
    return worst, mism, nblk


def block_norms(O, A):
    """||A(I_a, I_b)||_F for boxes of level l (tree order), from the dense
    original-order matrix A."""
    perm = O.perm

    def f(l, a, b):
        a0, a1 = O.box_range(l, a)
        b0, b1 = O.box_range(l, b)
        return np.linalg.norm(A[np.ix_(perm[a0:a1], perm[b0:b1])])
    return f


class PerturbedDense:
    """Dense black box (as oracle.DenseBlackBox) whose products carry a
    relative perturbation of one rounding unit per entry (2^-53 times a
    standard normal): the size of the difference two correct FP64
    implementations of the same product may show.  Compressing through it
    measures how far rounding alone moves the oracle's result."""

    def __init__(self, A, seed=0):
        self.A = A
        self.rng = np.random.default_rng(seed)

    def _p(self, Y):
        return Y * (1.0 + 2.0 ** -53 * self.rng.standard_normal(Y.shape))

    def apply(self, X):
        return self._p(self.A @ X)

    def applyT(self, X):
        return self._p(self.A.T @ X)


def level_worst(O, blocks_a, blocks_b, A_norm_of):
    """Per level, the largest ||X_ab - Y_ab||_F / ||A(I_a, I_b)||_F over the
    admissible pairs, X and Y the blocks U B V* of two compressions given as
    {level: [(a, b, U, B, V), ...]} in the same pair order."""
    out = {}
    for l in blocks_a:
        w = 0.0
        for (a, b, U, B, V), (a2, b2, U2, B2, V2) in zip(blocks_a[l], blocks_b[l]):
            assert (a, b) == (a2, b2)
            d = np.linalg.norm(U @ B @ V.T - U2 @ B2 @ V2.T)
            w = max(w, d / max(A_norm_of(l, a, b), 1e-300))
        out[l] = w
    return out
