"""FP64 numerical half of the oracle (test infrastructure only).

Written from Levitt & Martinsson, arXiv 2205.03406:

* randomized sampling with oversampling p (section "Randomized compression");
* per-pair recovery U = qr(Y,k), V = qr(Z,k),
  B = (G2* U)^+ G2* A G1 (V* G1)^+  (alg:compress_double_random);
* the level loop of alg:h1_pseudocode: colored test matrices satisfying
  eq:h1constraints (one per color of the level's incompatibility graph),
  samples of A - A^(l) and A* - A^(l)*, where A^(l) is the level-truncated
  matrix applied with the factors already computed;
* leaf extraction with identity test matrices (section on extracting
  inadmissible blocks).

Readings where the paper is silent (listed in the design notes):

* A^(l) subtracted while sampling level l holds exactly the levels already
  compressed (coarser than l); at the leaf pass it holds every level.
* qr(Y, k) is column-pivoted Householder QR (eq:QR), truncated to the first
  k columns of Q.  Fixed-rank mode: k = min(k, rows, r).  Tolerance mode:
  k = first j with |R_jj| <= tol |R_00|, capped at r - p (a cap hit is
  reported as saturation).
* the Psi pass uses the same coloring as the Omega pass: the A*-constraint
  set of pair (a, b) is the Omega constraint set of pair (b, a);
* test-matrix entries are standard normals from Philox4x32-10 (Salmon et al.,
  SC'11) and the Box-Muller transform, keyed by (seed) with counter
  (row in tree order, column pair, color, 4*level + pass); rows of boxes
  that a color does not activate are zero.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

MASK = np.uint64(0xFFFFFFFF)
_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = np.uint64(0x9E3779B9), np.uint64(0xBB67AE85)
PASS_OMEGA, PASS_PSI = 0, 1


# ----------------------------------------------------------------- Philox
def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11).

    Each round multiplies words 0 and 2 by the two round multipliers, and the
    new state is (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); the key is bumped
    by the two Weyl constants between rounds.  Inputs broadcast; returns four
    uint32 arrays.
    """
    c = [np.asarray(x).astype(np.uint64) & MASK for x in (c0, c1, c2, c3)]
    c = np.broadcast_arrays(*c)
    c = [x.copy() for x in c]
    k0 = np.uint64(int(k0) & 0xFFFFFFFF)
    k1 = np.uint64(int(k1) & 0xFFFFFFFF)
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + _W0) & MASK
            k1 = (k1 + _W1) & MASK
        p0 = _M0 * c[0]
        p1 = _M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return [x.astype(np.uint32) for x in c]


def _unit(a, b):
    """53-bit uniform in (0, 1) from two 32-bit words."""
    m = (a.astype(np.uint64) << np.uint64(21)) | (b.astype(np.uint64) >> np.uint64(11))
    return m.astype(np.float64) * 2.0 ** -53 + 2.0 ** -54


def gaussian_block(seed: int, level: int, pas: int, color: int, rows, r: int) -> np.ndarray:
    """Standard normals G[i, j] for the given tree-order rows, j < r."""
    rows = np.asarray(rows, np.uint64).reshape(-1, 1)
    npair = (r + 1) // 2
    jp = np.arange(npair, dtype=np.uint64).reshape(1, -1)
    a0, a1, a2, a3 = philox4x32_10(rows, jp, color, 4 * level + pas,
                                   seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    u1, u2 = _unit(a0, a1), _unit(a2, a3)
    rad = np.sqrt(-2.0 * np.log(u1))
    th = 6.283185307179586 * u2
    out = np.empty((rows.shape[0], 2 * npair))
    out[:, 0::2] = rad * np.cos(th)
    out[:, 1::2] = rad * np.sin(th)
    return out[:, :r]


def test_matrix(T, level: int, pas: int, seed: int, r: int) -> np.ndarray:
    """Colored test matrix of one level (eq:neartestmatrices), tree order,
    N x (ncolors * r): color c activates the boxes that are the active box of
    a vertex of color c; all other rows of that column block are zero."""
    G = T.graphs[level]
    out = np.zeros((T.n, G.ncolors * r))
    for c in range(G.ncolors):
        for b in sorted(set(int(x) for x in G.vbox[G.color == c])):
            s0, s1 = T.box_range(level, b)
            out[s0:s1, c * r:(c + 1) * r] = gaussian_block(seed, level, pas, c, np.arange(s0, s1), r)
    return out


def leaf_test_matrix(T) -> np.ndarray:
    """Identity test matrices of the leaf pass, N x (ncolors_leaf * m) with
    m the largest leaf box: color c puts an identity on every active box."""
    G = T.leaf_graph
    m = T.leaf_max()
    out = np.zeros((T.n, G.ncolors * m))
    for c in range(G.ncolors):
        for b in sorted(set(int(x) for x in G.vbox[G.color == c])):
            s0, s1 = T.box_range(T.L, b)
            out[s0 + np.arange(s1 - s0), c * m + np.arange(s1 - s0)] = 1.0
    return out


# ----------------------------------------------------------------- black boxes
def kernel_matrix(P: np.ndarray, Q: np.ndarray, kernel: str) -> np.ndarray:
    """K(p_i, q_j): log|p-q| or 1/|p-q|, and 0 where the points coincide."""
    d = P[:, None, :] - Q[None, :, :]
    r2 = np.einsum("ijk,ijk->ij", d, d)
    out = np.zeros_like(r2)
    nz = r2 > 0
    if kernel == "log":
        out[nz] = 0.5 * np.log(r2[nz])
    elif kernel == "inv_r":
        out[nz] = 1.0 / np.sqrt(r2[nz])
    else:
        raise ValueError(kernel)
    return out


class KernelBlackBox:
    """Y = A X with A(i,j) = K(x_i, x_j) formed block by block (original
    point order).  The kernels are symmetric, so A* = A."""

    def __init__(self, points: np.ndarray, kernel: str, block: int = 2048, dense_cache: bool = True):
        self.P = np.ascontiguousarray(points, np.float64)
        if self.P.ndim == 1:
            self.P = self.P.reshape(-1, 1)
        self.kernel = kernel
        self.block = block
        self._dense = None
        if dense_cache and self.P.shape[0] <= 20000:
            self._dense = kernel_matrix(self.P, self.P, kernel)

    def dense(self):
        return self._dense if self._dense is not None else kernel_matrix(self.P, self.P, self.kernel)

    def apply(self, X):
        if self._dense is not None:
            return self._dense @ X
        n = self.P.shape[0]
        Y = np.empty((n, X.shape[1]))
        for i0 in range(0, n, self.block):
            i1 = min(n, i0 + self.block)
            Y[i0:i1] = kernel_matrix(self.P[i0:i1], self.P, self.kernel) @ X
        return Y

    applyT = apply

    def rows(self, idx, X):
        """Selected rows of A X, each computed from its own kernel row."""
        return kernel_matrix(self.P[np.asarray(idx)], self.P, self.kernel) @ X


class DenseBlackBox:
    def __init__(self, A):
        self.A = np.asarray(A, np.float64)

    def apply(self, X):
        return self.A @ X

    def applyT(self, X):
        return self.A.T @ X


class CountingBlackBox:
    """Counts the columns passed through A and through A*."""

    def __init__(self, inner):
        self.inner = inner
        self.cols_A = 0
        self.cols_At = 0

    def apply(self, X):
        self.cols_A += X.shape[1]
        return self.inner.apply(X)

    def applyT(self, X):
        self.cols_At += X.shape[1]
        return self.inner.applyT(X)


# ----------------------------------------------------------------- H-matrix
class HMatrix:
    """H^1 representation: A(I_a, I_b) ~ U B V* for admissible pairs of every
    level, plus dense leaf blocks for neighbor pairs of the leaf level."""

    def __init__(self, T):
        self.T = T
        self.lowrank = {}     # level -> list of (a, b, U, B, V)
        self.near = []        # list of (a, b, D)
        self.saturated = 0

    def apply(self, X, levels=None, near=True, transpose=False):
        """Tree-order product with the levels listed (all if None)."""
        T = self.T
        Y = np.zeros((T.n, X.shape[1]))
        for l, blocks in self.lowrank.items():
            if levels is not None and l not in levels:
                continue
            for a, b, U, B, V in blocks:
                a0, a1 = T.box_range(l, a)
                b0, b1 = T.box_range(l, b)
                if transpose:
                    Y[b0:b1] += V @ (B.T @ (U.T @ X[a0:a1]))
                else:
                    Y[a0:a1] += U @ (B @ (V.T @ X[b0:b1]))
        if near:
            for a, b, D in self.near:
                a0, a1 = T.box_range(T.L, a)
                b0, b1 = T.box_range(T.L, b)
                if transpose:
                    Y[b0:b1] += D.T @ X[a0:a1]
                else:
                    Y[a0:a1] += D @ X[b0:b1]
        return Y

    def matvec(self, X):
        """Original-order product H X."""
        T = self.T
        X = np.asarray(X, np.float64).reshape(T.n, -1)
        Yt = self.apply(X[T.perm])
        Y = np.empty_like(Yt)
        Y[T.perm] = Yt
        return Y

    def dense_tree(self):
        return self.apply(np.eye(self.T.n))

    def dense(self):
        """Original-order dense matrix (small N only)."""
        T = self.T
        Dt = self.dense_tree()
        D = np.empty_like(Dt)
        D[np.ix_(T.perm, T.perm)] = Dt
        return D

    def ranks(self):
        return {l: [(U.shape[1], V.shape[1]) for (_, _, U, _, V) in b] for l, b in self.lowrank.items()}

    def floats(self):
        n = 0
        for blocks in self.lowrank.values():
            for _, _, U, B, V in blocks:
                n += U.size + B.size + V.size
        for _, _, D in self.near:
            n += D.size
        return n


def _basis(S: np.ndarray, k: int, tol: float, r: int, p: int):
    """qr(S, k): the first k columns of Q of a column-pivoted QR of S."""
    m = S.shape[0]
    kmax = min(m, S.shape[1])
    if kmax == 0:
        return np.zeros((m, 0)), False
    Q, R, _ = scipy.linalg.qr(S, mode="economic", pivoting=True)
    sat = False
    if k > 0:
        kk = min(k, kmax)
    else:
        d = np.abs(np.diag(R))
        kk = kmax
        for j in range(kmax):
            if not (d[j] > tol * d[0]):
                kk = j
                break
        if kk > r - p:
            kk, sat = r - p, True
    return Q[:, :kk], sat


def compress(T, bb, r: int, k: int = 0, tol: float = 0.0, p: int = 10, seed: int = 0,
             return_samples: bool = False):
    """alg:h1_pseudocode on tree T with black box ``bb`` (apply / applyT act in
    original point order).  Fixed rank when k > 0, else tolerance ``tol``."""
    if r <= 0:
        r = k + p
    H = HMatrix(T)
    perm = T.perm
    n = T.n

    def to_orig(Xt):
        X = np.empty_like(Xt)
        X[perm] = Xt
        return X

    samples = {}
    for l in T.sampled_levels():
        G = T.graphs[l]
        pair_index = {(int(a), int(b)): q for q, (a, b) in enumerate(zip(G.pair_a, G.pair_b))}
        done = list(H.lowrank.keys())
        Om = test_matrix(T, l, PASS_OMEGA, seed, r)
        Ps = test_matrix(T, l, PASS_PSI, seed, r)
        Y = bb.apply(to_orig(Om))[perm] - H.apply(Om, levels=done, near=False)
        Z = bb.applyT(to_orig(Ps))[perm] - H.apply(Ps, levels=done, near=False, transpose=True)
        if return_samples:
            samples[l] = (Om, Ps, Y, Z)
        blocks = []
        for q in range(len(G.pair_a)):
            a, b = int(G.pair_a[q]), int(G.pair_b[q])
            cu = int(G.color[G.pair_v[q]])
            cv = int(G.color[G.pair_v[pair_index[(b, a)]]])
            a0, a1 = T.box_range(l, a)
            b0, b1 = T.box_range(l, b)
            SU = Y[a0:a1, cu * r:(cu + 1) * r]
            SV = Z[b0:b1, cv * r:(cv + 1) * r]
            U, s1 = _basis(SU, k, tol, r, p)
            V, s2 = _basis(SV, k, tol, r, p)
            H.saturated += int(s1) + int(s2)
            G1 = Om[b0:b1, cu * r:(cu + 1) * r]
            G2 = Ps[a0:a1, cv * r:(cv + 1) * r]
            if U.shape[1] == 0 or V.shape[1] == 0:
                B = np.zeros((U.shape[1], V.shape[1]))
            else:
                B = np.linalg.pinv(G2.T @ U) @ (G2.T @ SU) @ np.linalg.pinv(V.T @ G1)
            blocks.append((a, b, U, B, V))
        H.lowrank[l] = blocks

    # leaf pass: identity test matrices, subtract every compressed level
    G = T.leaf_graph
    m = T.leaf_max()
    Om = leaf_test_matrix(T)
    Y = bb.apply(to_orig(Om))[perm] - H.apply(Om, near=False)
    if return_samples:
        samples["leaf"] = (Om, Y)
    for q in range(len(G.pair_a)):
        a, b = int(G.pair_a[q]), int(G.pair_b[q])
        c = int(G.color[G.pair_v[q]])
        a0, a1 = T.box_range(T.L, a)
        b0, b1 = T.box_range(T.L, b)
        H.near.append((a, b, Y[a0:a1, c * m:c * m + (b1 - b0)].copy()))
    if return_samples:
        return H, samples
    return H


# ----------------------------------------------------------------- errors
def rel_fro_error_dense(H: HMatrix, A: np.ndarray) -> float:
    D = H.dense()
    return float(np.linalg.norm(D - A) / np.linalg.norm(A))


def probe_error(apply_exact, apply_approx, n: int, nprobe: int = 128, seed: int = 7) -> float:
    """||(A - H) G||_F / ||A G||_F with Gaussian probes G (n x nprobe)."""
    G = np.random.default_rng(seed).standard_normal((n, nprobe))
    E = apply_exact(G)
    return float(np.linalg.norm(E - apply_approx(G)) / np.linalg.norm(E))


def power_error(apply_diff, apply_diffT, apply_A, n: int, iters: int = 20, seed: int = 11) -> float:
    """Relative operator-norm error by power iteration (20 steps, as in the
    paper's experiments section): ||A - H|| / ||A||."""
    rng = np.random.default_rng(seed)

    def norm_est(f, fT):
        x = rng.standard_normal((n, 1))
        x /= np.linalg.norm(x)
        s = 0.0
        for _ in range(iters):
            y = f(x)
            z = fT(y)
            s = np.linalg.norm(y)
            nz = np.linalg.norm(z)
            if nz == 0:
                return 0.0
            x = z / nz
        return float(s)

    return norm_est(apply_diff, apply_diffT) / norm_est(apply_A, apply_A)
