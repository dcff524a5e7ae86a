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


def exact_h2(T, k, seed=0):
    """Dense non-symmetric matrix with H^2 structure: every box with a
    non-empty far field (an interaction list on its level or above) has
    nested column and row bases; orthonormal long bases (k columns, or all
    rows of a smaller box) on the finest sampled level, random transfer
    matrices above it (k_tau = min(k, sum of the children's ranks), the
    implied bases orthonormalized, which keeps them nested), a
    random coupling per admissible pair, dense random leaf neighbor blocks.
    H^2 compression with r >= k + p must recover it to rounding error."""
    rng = np.random.default_rng(seed)
    sampled = T.sampled_levels()
    A = np.zeros((T.n, T.n))
    if sampled:
        levels = list(range(sampled[0], sampled[-1] + 1))
        has = {}
        for l in levels:
            par = T.parent[l]
            has[l] = [a for a in range(T.nbox(l))
                      if len(T.interaction(l, a)) or (l - 1 in has and int(par[a]) in has[l - 1])]
        f = levels[-1]
        U, V = {f: {}}, {f: {}}
        for a in has[f]:
            a0, a1 = T.box_range(f, a)
            ka = min(k, a1 - a0)
            U[f][a] = np.linalg.qr(rng.standard_normal((a1 - a0, ka)))[0]
            V[f][a] = np.linalg.qr(rng.standard_normal((a1 - a0, ka)))[0]
        for i in range(len(levels) - 2, -1, -1):
            l, lc = levels[i], levels[i + 1]
            U[l], V[l] = {}, {}
            parc = T.parent[lc]
            for tau in has[l]:
                t0, t1 = T.box_range(l, tau)
                ch = [int(c) for c in np.nonzero(parc == tau)[0]]
                for Out, Fine in ((U, U), (V, V)):
                    kt = min(k, sum(Fine[lc][c].shape[1] for c in ch))
                    M = np.zeros((t1 - t0, kt))
                    for c in ch:
                        c0, c1 = T.box_range(lc, c)
                        M[c0 - t0:c1 - t0] = Fine[lc][c] @ rng.standard_normal((Fine[lc][c].shape[1], kt))
                    # orthonormal and still nested: M R^-1 = blockdiag(children) (G R^-1)
                    Out[l][tau] = np.linalg.qr(M)[0]
        for l in levels:
            for a in has[l]:
                a0, a1 = T.box_range(l, a)
                for b in T.interaction(l, a):
                    b = int(b)
                    b0, b1 = T.box_range(l, b)
                    B = rng.standard_normal((U[l][a].shape[1], V[l][b].shape[1])) * 2.0 ** (-l)
                    A[a0:a1, b0:b1] = U[l][a] @ B @ V[l][b].T
    for a in range(T.nbox(T.L)):
        a0, a1 = T.box_range(T.L, a)
        for b in T.neighbors(T.L, a):
            b0, b1 = T.box_range(T.L, int(b))
            A[a0:a1, b0:b1] = rng.standard_normal((a1 - a0, b1 - b0))
    out = np.empty_like(A)
    out[np.ix_(T.perm, T.perm)] = A
    return out
