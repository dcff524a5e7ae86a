"""H^2 compression (section "H^2 matrix compression", alg:h2_pseudocode,
alg:apply_h2_level_truncated): oracle, test infrastructure only.

An H^2 matrix keeps long bases only at the finest level; a coarser box tau
stores short (transfer) matrices, one per child a, with
U_tau(I_tau(a), :) = U_a Ushort_tau[a] (eq:nested_basis), so the bases are
nested.  The compression follows the uniform H^1 one (two stages per level,
same test matrices and Psi) with three changes:

* bases come from the SVD of the sample, and the singular values are kept;
* the sample of a box a with parent tau is augmented with a sample of the
  parent's far field restricted to a's rows: U_tau(I_tau(a), :) S_tau G,
  G Gaussian, so the basis of a spans what its parent's basis needs;
* after the children of tau have their long bases, tau's short bases are
  the least-squares transfers Ushort_tau[a] = U_a* U_tau(I_tau(a), :) and
  the long basis of tau is dropped.

The row bases come from the plain sum of the stage-2 blocks, augmented:
V_b = svd(sum over a in int(b) of Z(I_b, block of (b, a)) + V_tau(I_tau(b), :)
S_tau G, k), as alg:h2_pseudocode writes it (combine="gaussian" selects the
Gamma-weighted combination of the uniform module's extension instead).

The level-truncated matrix A^(l) subtracted while sampling level l is the
H^2 matrix built so far (every coarser level), applied by the upward pass,
couplings and downward pass of alg:apply_h2_level_truncated with the long
bases of the finest level built so far.

Readings (listed in the design notes):
* the augmented sample is the sum Y(I_a, :) + U_tau(I_tau(a), :) S_tau G
  as the formula of the section writes it, which makes G a k_tau x r (for
  V: k_tau x kmax) Gaussian matrix where the text calls it k x k;
  G row i, column j is the Gaussian of counter (first tree row of a, j/2,
  2^31 + i, 4 level + 2) for U and (..., 4 level + 3) for V (the high
  color slot keeps these draws apart from the test matrices and the
  mixing matrices);
* every box whose far field is not empty gets a basis: a box without an
  interaction list (so no stage-1 sample) whose parent has a basis takes
  the SVD of the augmentation alone; bases exist on every level from the
  first sampled level to the last one;
* rank rules as in the uniform compression: U by qr(., k)'s rule (cap
  r - p, saturation) on the singular values, V up to kmax with no cap;
  singular vectors are signed so that their largest entry is positive;
* B_ab = Z(I_b, block of (b, a))[:, :k_a]* V_b as in the uniform form;
  A^(l)'s near blocks are not part of the level-truncated product (the
  near field is only known after the leaf pass), so the final line of
  alg:apply_h2_level_truncated adds them only in the full apply;
* the leaf pass is that of the other forms, subtracting the whole H^2 part.
"""
from __future__ import annotations

import numpy as np

from .numeric import gaussian_block, leaf_test_matrix
from .uniform import COMBINE, UniformGraph, mixing_matrix, uniform_test_matrix

AUG_SLOT = 1 << 31


def augment_gaussian(seed, level, pas, row0, krows, ncols):
    """G (krows x ncols): row i from counter (row0, column pair, 2^31 + i,
    4 level + pas)."""
    if krows == 0:
        return np.zeros((0, ncols))
    return np.vstack([gaussian_block(seed, level, pas, AUG_SLOT + i, [row0], ncols)[0]
                      for i in range(krows)])


def svd_basis(S, k, tol, cap):
    """Left singular vectors and values of S, truncated to k (fixed rank)
    or to the singular values above tol * s_0, at most cap (tolerance);
    returns (U, s, saturated)."""
    m, c = S.shape
    kmax = min(m, c)
    if kmax == 0:
        return np.zeros((m, 0)), np.zeros(0), False
    U, s, _ = np.linalg.svd(S, full_matrices=False)
    # sign convention: the entry of largest magnitude of every singular
    # vector is positive (the first one on ties)
    idx = np.argmax(np.abs(U), axis=0)
    U = U * np.where(U[idx, np.arange(U.shape[1])] < 0, -1.0, 1.0)
    if k > 0:
        kk = min(k, kmax)
        return U[:, :kk], s[:kk], False
    if not s[0] > 0:
        return np.zeros((m, 0)), np.zeros(0), False
    kk = int(np.sum(s > tol * s[0]))
    sat = kk > cap
    kk = min(kk, cap)
    return U[:, :kk], s[:kk], sat


class H2Matrix:
    """levels: the levels with bases, coarsest first.  At the finest level,
    Ulong / Vlong[b]; at every coarser level l, Ushort / Vshort[l][tau] =
    {child: transfer}.  B[l]: list of (a, b, B) in the pair order of the
    level graph.  near: leaf blocks (a, b, D)."""

    def __init__(self, T):
        self.T = T
        self.levels = []
        self.Ushort, self.Vshort = {}, {}
        self.Ulong, self.Vlong = {}, {}
        self.B = {}
        self.near = []
        self.saturated = 0
        self.cols_A = self.cols_At = 0

    def _children(self, l, tau):
        par = self.T.parent[l + 1]
        return [int(c) for c in np.nonzero(par == tau)[0]]

    def apply(self, X, finest=None, Ulong=None, Vlong=None, transpose=False, near=True):
        """Tree-order product (alg:apply_h2_level_truncated).  finest: the
        finest level included (default: all), with its long bases."""
        T = self.T
        Y = np.zeros((T.n, X.shape[1]))
        lv = [l for l in self.levels if finest is None or l <= finest]
        if lv:
            f = lv[-1]
            UL = self.Ulong if Ulong is None else Ulong
            VL = self.Vlong if Vlong is None else Vlong
            Uin, Uout = (VL, UL) if transpose else (UL, VL)   # out: applied to q
            Sin, Sout = (self.Vshort, self.Ushort) if transpose else (self.Ushort, self.Vshort)
            # outgoing expansions at the finest level, then upward
            qh = {f: {}}
            for b, Vb in Uout.items():
                b0, b1 = T.box_range(f, b)
                qh[f][b] = Vb.T @ X[b0:b1]
            for i in range(len(lv) - 2, -1, -1):
                l = lv[i]
                qh[l] = {}
                for tau, ch in Sout[l].items():
                    acc = 0.0
                    for a, Vs in ch.items():
                        acc = acc + Vs.T @ qh[lv[i + 1]][a]
                    qh[l][tau] = acc
            # couplings and downward pass
            uh = {}
            for i, l in enumerate(lv):
                uh[l] = {}
                for a, b, B in self.B[l]:
                    if transpose:
                        a, b, B = b, a, B.T
                    if b not in qh[l]:
                        continue
                    uh[l][a] = uh[l].get(a, 0.0) + B @ qh[l][b]
                if i > 0:
                    lp = lv[i - 1]
                    for tau, ch in Sin[lp].items():
                        if tau not in uh[lp]:
                            continue
                        for a, Us in ch.items():
                            uh[l][a] = uh[l].get(a, 0.0) + Us @ uh[lp][tau]
            for a, ua in uh[f].items():
                a0, a1 = T.box_range(f, a)
                Y[a0:a1] += Uin[a] @ ua
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
        T = self.T
        X = np.asarray(X, np.float64).reshape(T.n, -1)
        Yt = self.apply(X[T.perm])
        Y = np.empty_like(Yt)
        Y[T.perm] = Yt
        return Y

    def dense(self):
        T = self.T
        Dt = self.apply(np.eye(T.n))
        D = np.empty_like(Dt)
        D[np.ix_(T.perm, T.perm)] = Dt
        return D

    def effective_bases(self):
        """Long bases of every level implied by the nesting:
        U_tau(I_tau(a), :) = U_a Ushort_tau[a], from the finest level up."""
        T = self.T
        if not self.levels:
            return {}, {}
        f = self.levels[-1]
        U = {f: dict(self.Ulong)}
        V = {f: dict(self.Vlong)}
        for i in range(len(self.levels) - 2, -1, -1):
            l, lc = self.levels[i], self.levels[i + 1]
            U[l], V[l] = {}, {}
            for which, Sh, Out, Fine in ((0, self.Ushort, U, U), (1, self.Vshort, V, V)):
                for tau, ch in Sh[l].items():
                    t0, t1 = T.box_range(l, tau)
                    k = next(iter(ch.values())).shape[1] if ch else 0
                    M = np.zeros((t1 - t0, k))
                    for a, Ss in ch.items():
                        a0, a1 = T.box_range(lc, a)
                        M[a0 - t0:a1 - t0] = Fine[lc][a] @ Ss
                    Out[l][tau] = M
        return U, V

    def floats(self):
        n = sum(U.size for U in self.Ulong.values()) + sum(V.size for V in self.Vlong.values())
        for Sh in (self.Ushort, self.Vshort):
            for l in Sh:
                for ch in Sh[l].values():
                    n += sum(M.size for M in ch.values())
        n += sum(B.size for l in self.B for (_, _, B) in self.B[l])
        n += sum(D.size for (_, _, D) in self.near)
        return n


def compress_h2(T, bb, r, k=0, tol=0.0, p=10, seed=0, combine="sum"):
    """H^2 compression of the black box bb (apply / applyT in the original
    point order), alg:h2_pseudocode in its H^2 branch.  combine as in
    compress_uniform ("sum" is the paper's rule)."""
    if combine not in COMBINE:
        raise ValueError("combine must be one of %s" % (COMBINE,))
    if r <= 0:
        r = k + p
    kmax = k if k > 0 else r - p
    H = H2Matrix(T)
    perm = T.perm
    sampled = T.sampled_levels()
    if sampled:
        H.levels = list(range(sampled[0], sampled[-1] + 1))

    def to_orig(Xt):
        X = np.empty_like(Xt)
        X[perm] = Xt
        return X

    Up, Vp, Sup, Svp = {}, {}, {}, {}   # long bases and values of the previous level
    for l in H.levels:
        fin = H.levels.index(l) - 1
        fl = H.levels[fin] if fin >= 0 else None

        def peel(Xt, transpose):
            if fl is None:
                return 0.0
            return H.apply(Xt, finest=fl, Ulong=Up, Vlong=Vp, transpose=transpose, near=False)

        nb = T.nbox(l)
        par = T.parent[l]
        has_parent = lambda a: fl is not None and int(par[a]) in Up
        boxes = [a for a in range(nb) if len(T.interaction(l, a)) or has_parent(a)]
        UG = UniformGraph(T, l)
        vcol = {int(a): int(c) for a, c in zip(UG.vbox, UG.color)}
        # stage 1
        Y = None
        if UG.nv:
            Om = uniform_test_matrix(T, l, UG, seed, r)
            Y = bb.apply(to_orig(Om))[perm] - peel(Om, False)
            H.cols_A += Om.shape[1]
        U, Su = {}, {}
        for a in boxes:
            a0, a1 = T.box_range(l, a)
            S = np.zeros((a1 - a0, r))
            if a in vcol:
                c = vcol[a]
                S += Y[a0:a1, c * r:(c + 1) * r]
            if has_parent(a):
                tau = int(par[a])
                t0 = T.box_range(l - 1, tau)[0]
                Ut = Up[tau][a0 - t0:a1 - t0]
                S += (Ut * Sup[tau]) @ augment_gaussian(seed, l, 2, a0, Ut.shape[1], r)
            U[a], Su[a], sat = svd_basis(S, k, tol, r - p)
            H.saturated += int(sat)
        # stage 2
        G = T.graphs[l]
        pidx = {(int(a), int(b)): q for q, (a, b) in enumerate(zip(G.pair_a, G.pair_b))}
        Z = None
        if G.nv:
            Ps = np.zeros((T.n, G.ncolors * kmax))
            for v, a in enumerate(G.vbox):
                a = int(a)
                c = int(G.color[v])
                a0, a1 = T.box_range(l, a)
                Ps[a0:a1, c * kmax:c * kmax + U[a].shape[1]] = U[a]
            Z = bb.applyT(to_orig(Ps))[perm] - peel(Ps, True)
            H.cols_At += Ps.shape[1]
        V, Sv = {}, {}
        for b in boxes:
            b0, b1 = T.box_range(l, b)
            S = np.zeros((b1 - b0, kmax))
            for a in T.interaction(l, b):
                cq = int(G.color[G.pair_v[pidx[(b, int(a))]]])
                blk = Z[b0:b1, cq * kmax:(cq + 1) * kmax]
                if combine == "sum":
                    S += blk
                else:
                    S += blk @ mixing_matrix(seed, l, T.box_range(l, int(a))[0], kmax)
            if has_parent(b):
                tau = int(par[b])
                t0 = T.box_range(l - 1, tau)[0]
                Vt = Vp[tau][b0 - t0:b1 - t0]
                S += (Vt * Svp[tau]) @ augment_gaussian(seed, l, 3, b0, Vt.shape[1], kmax)
            V[b], Sv[b], _ = svd_basis(S, k, tol, kmax)
        H.B[l] = []
        for q in range(len(G.pair_a)):
            a, b = int(G.pair_a[q]), int(G.pair_b[q])
            cq = int(G.color[G.pair_v[pidx[(b, a)]]])
            b0, b1 = T.box_range(l, b)
            Zb = Z[b0:b1, cq * kmax:cq * kmax + U[a].shape[1]]
            H.B[l].append((a, b, Zb.T @ V[b]))
        # nest the previous level into this one
        if fl is not None:
            H.Ushort[fl], H.Vshort[fl] = {}, {}
            for tau in Up:
                t0 = T.box_range(fl, tau)[0]
                cu, cv = {}, {}
                for a in np.nonzero(par == tau)[0]:
                    a = int(a)
                    a0, a1 = T.box_range(l, a)
                    cu[a] = U[a].T @ Up[tau][a0 - t0:a1 - t0]
                    cv[a] = V[a].T @ Vp[tau][a0 - t0:a1 - t0]
                H.Ushort[fl][tau], H.Vshort[fl][tau] = cu, cv
        Up, Vp, Sup, Svp = U, V, Su, Sv
    H.Ulong, H.Vlong = Up, Vp

    # leaf pass
    GL = T.leaf_graph
    m = T.leaf_max()
    Om = leaf_test_matrix(T)
    Y = bb.apply(to_orig(Om))[perm] - H.apply(Om, near=False)
    H.cols_A += Om.shape[1]
    for q in range(len(GL.pair_a)):
        a, b = int(GL.pair_a[q]), int(GL.pair_b[q])
        c = int(GL.color[GL.pair_v[q]])
        a0, a1 = T.box_range(T.L, a)
        b0, b1 = T.box_range(T.L, b)
        H.near.append((a, b, Y[a0:a1, c * m:c * m + (b1 - b0)].copy()))
    return H
