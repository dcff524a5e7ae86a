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


def exact_uniform_h1(T, k, seed=0):
    """Dense non-symmetric matrix with uniform H^1 structure of rank k: one
    column basis per row box and one row basis per column box at every level
    (orthonormal, k columns, or all rows of a smaller box), a random coupling
    per admissible pair, dense random leaf neighbor blocks.  Uniform
    compression with r >= k + p must recover it to rounding error."""
    rng = np.random.default_rng(seed)
    A = np.zeros((T.n, T.n))
    for l in range(T.nlev):
        U, V = {}, {}
        for a in range(T.nbox(l)):
            if len(T.interaction(l, a)) == 0:
                continue
            a0, a1 = T.box_range(l, a)
            ka = min(k, a1 - a0)
            U[a] = np.linalg.qr(rng.standard_normal((a1 - a0, ka)))[0]
            V[a] = np.linalg.qr(rng.standard_normal((a1 - a0, ka)))[0]
        for a in U:
            a0, a1 = T.box_range(l, a)
            for b in T.interaction(l, a):
                b = int(b)
                b0, b1 = T.box_range(l, b)
                B = rng.standard_normal((U[a].shape[1], V[b].shape[1])) * 2.0 ** (-l)
                A[a0:a1, b0:b1] = U[a] @ B @ V[b].T
    for a in range(T.nbox(T.L)):
        a0, a1 = T.box_range(T.L, a)
        for b in T.neighbors(T.L, a):
            b0, b1 = T.box_range(T.L, int(b))
            A[a0:a1, b0:b1] = rng.standard_normal((a1 - a0, b1 - b0))
    out = np.empty_like(A)
    out[np.ix_(T.perm, T.perm)] = A
    return out
