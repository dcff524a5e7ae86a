"""Test-only synthetic operators built on the oracle's tree.

``exact_h1(T, k, seed)`` returns a dense, non-symmetric matrix whose
admissible blocks have rank exactly k (random factors) and whose leaf
neighbor blocks are dense random: colored peeling must recover it to
rounding error (alg:compress_double_random is exact on rank-k blocks).
"""
import numpy as np


def exact_h1(T, k, seed=0, scale_by_level=True):
    rng = np.random.default_rng(seed)
    A = np.zeros((T.n, T.n))
    for l in range(T.nlev):
        s = 2.0 ** (-l) if scale_by_level else 1.0
        for a in range(T.nbox(l)):
            a0, a1 = T.box_range(l, a)
            for b in T.interaction(l, a):
                b0, b1 = T.box_range(l, int(b))
                X = rng.standard_normal((a1 - a0, k))
                Y = rng.standard_normal((b1 - b0, k))
                A[a0:a1, b0:b1] = s * (X @ Y.T) / np.sqrt((a1 - a0) * (b1 - b0))
    for a in range(T.nbox(T.L)):
        a0, a1 = T.box_range(T.L, a)
        for b in T.neighbors(T.L, a):
            b0, b1 = T.box_range(T.L, int(b))
            A[a0:a1, b0:b1] = rng.standard_normal((a1 - a0, b1 - b0))
    # A above is in tree order; return it in original point order
    out = np.empty_like(A)
    out[np.ix_(T.perm, T.perm)] = A
    return out
