"""Uniform H^1 compression (section "Uniform H^1 matrix compression"):
oracle, test infrastructure only.

A uniform H^1 matrix keeps one column basis U_a per box a and one row basis
V_b per box b, shared by every admissible pair: A(I_a, I_b) ~ U_a B_ab V_b*.
Per sampled level, coarsest first:

* stage 1: one constraint set per box a with a non-empty interaction list
  (eq:unifh1constraints): the test matrix is a Gaussian block on every box of
  the interaction list of a and zero on every neighbor of a.  Two boxes
  conflict when a box active for one lies in the zero set of the other.  The
  coloring gives one test matrix per color; Y = (A - A^(l)) Omega and
  U_a = qr(Y(I_a, block of a's color)).
* stage 2: the Psi pass of the non-uniform method with the Gaussian blocks
  replaced by the bases just computed: for the pair (a, b), Psi holds U_a on
  box a and zeros on the other boxes of b's parent's neighborhood, so
  Z = (A - A^(l))* Psi gives Z(I_b, block) = A(I_a, I_b)* U_a.  Then
  V_b = qr(sum over a in the interaction list of b of Z(I_b, block of (b, a)), k)
  (alg:h2_pseudocode, "sum samples and orthonormalize") and
  B_ab = Z(I_b, block)* V_b.

Readings (listed in the design notes): the Psi constraint of pair (a, b) is
written in the paper with the roles of a and b exchanged; it is the Omega
constraint set of the non-uniform pair (b, a), so the non-uniform level graph
and its coloring serve stage 2 unchanged.  Stage-1 draws use pass number 2 of
the counter-based generator.  Psi blocks are kmax = k (or r - p) columns wide,
U_a in the first k_a of them (zero beyond), so each summed block is
A(I_a, I_b)* U_a padded with zero columns.  The rank of V_b follows the rule
of qr(., k) on the kmax-column sum (at most the largest k_a; saturation is
counted in stage 1 only).

Extension (not the paper's rule, opt-in with combine="gaussian", no parity
claim against the paper): each term is first multiplied by a Gaussian
kmax x kmax matrix Gamma_a (pass 3 of the generator, counter (first row of
box a, column pair, row of Gamma, 4 level + 3)), a randomized sample of the
side-by-side blocks instead of their sum.
The leaf pass is the non-uniform one.
"""
from __future__ import annotations

import numpy as np

from .comb import dsatur
from .numeric import (HMatrix, _basis, gaussian_block, leaf_test_matrix)

PASS_UNIFORM, PASS_MIX = 2, 3


COMBINE = ("sum", "gaussian")


def mixing_matrix(seed, level, row0, kmax):
    """Gamma_a (kmax x kmax) of the combine="gaussian" extension: row i from
    the counter (row0, column pair, i, 4 level + 3), row0 = the first tree
    row of box a."""
    return np.vstack([gaussian_block(seed, level, PASS_MIX, i, [row0], kmax)[0]
                      for i in range(kmax)])


class UniformGraph:
    """Constraint incompatibility graph of the stage-1 sets of one level."""

    def __init__(self, T, l):
        verts = [b for b in range(T.nbox(l)) if len(T.interaction(l, b))]
        act = {a: set(int(x) for x in T.interaction(l, a)) for a in verts}
        zero = {a: set(int(x) for x in T.neighbors(l, a)) for a in verts}
        adj = [[] for _ in verts]
        for i, a in enumerate(verts):
            for j, b in enumerate(verts):
                if i != j and (act[a] & zero[b] or act[b] & zero[a]):
                    adj[i].append(j)
        self.vbox = np.array(verts, np.int32)
        self.xadj = np.zeros(len(verts) + 1, np.int64)
        self.xadj[1:] = np.cumsum([len(x) for x in adj])
        self.adj = np.array([j for x in adj for j in x], np.int32)
        self.active = act
        self.color, self.ncolors = dsatur(self.xadj, self.adj)

    @property
    def nv(self):
        return len(self.vbox)

    @property
    def nedges(self):
        return int(self.xadj[-1]) // 2


def uniform_test_matrix(T, l, UG, seed, r, colors=None):
    """Stage-1 test matrix of level l, tree order, N x (ncolors * r): color c
    holds the Gaussian block of every box active for a vertex of color c."""
    col = UG.color if colors is None else np.asarray(colors)
    nc = int(col.max()) + 1 if len(col) else 0
    out = np.zeros((T.n, nc * r))
    for c in range(nc):
        boxes = sorted(set(b for v, a in enumerate(UG.vbox) if col[v] == c for b in UG.active[int(a)]))
        for b in boxes:
            s0, s1 = T.box_range(l, b)
            out[s0:s1, c * r:(c + 1) * r] = gaussian_block(seed, l, PASS_UNIFORM, c,
                                                           np.arange(s0, s1), r)
    return out


def _qr_rank(S, k, tol):
    """qr(S, k) of a stage-2 sum block: its columns are the kmax columns of
    the Psi blocks, so the rank is at most the largest k_a and no cap
    applies (a saturated stage 1 already counted the shortfall)."""
    Q, _ = _basis(S, k, tol, S.shape[1] + 1, 1)   # cap = all columns
    return Q


def compress_uniform(T, bb, r, k=0, tol=0.0, p=10, seed=0, return_graphs=False, combine="sum"):
    """Uniform H^1 compression of the black box bb (apply / applyT in the
    original point order), alg:h2_pseudocode in its uniform H^1 branch.
    Returns an HMatrix whose blocks are (a, b, U_a, B_ab, V_b) in the pair
    order of the level graph, with the per-box bases in H.ubasis[l] /
    H.vbasis[l].  combine="sum" (default) forms V_b from the plain sum of
    the sample blocks as the paper does; "gaussian" is the extension of the
    module docstring."""
    if combine not in COMBINE:
        raise ValueError("combine must be one of %s" % (COMBINE,))
    if r <= 0:
        r = k + p
    kmax = k if k > 0 else r - p
    H = HMatrix(T)
    H.ubasis, H.vbasis = {}, {}
    H.cols_A = H.cols_At = 0
    perm = T.perm
    graphs = {}

    def to_orig(Xt):
        X = np.empty_like(Xt)
        X[perm] = Xt
        return X

    for l in T.sampled_levels():
        done = list(H.lowrank.keys())
        UG = UniformGraph(T, l)
        graphs[l] = UG
        # stage 1: column bases
        Om = uniform_test_matrix(T, l, UG, seed, r)
        Y = bb.apply(to_orig(Om))[perm] - H.apply(Om, levels=done, near=False)
        H.cols_A += Om.shape[1]
        U = {}
        for v, a in enumerate(UG.vbox):
            a = int(a)
            c = int(UG.color[v])
            a0, a1 = T.box_range(l, a)
            U[a], s = _basis(Y[a0:a1, c * r:(c + 1) * r], k, tol, r, p)
            H.saturated += int(s)
        # stage 2: Psi from the bases, row bases and couplings
        G = T.graphs[l]
        pair_index = {(int(a), int(b)): q for q, (a, b) in enumerate(zip(G.pair_a, G.pair_b))}
        Ps = np.zeros((T.n, G.ncolors * kmax))
        for v, a in enumerate(G.vbox):
            a = int(a)
            c = int(G.color[v])
            a0, a1 = T.box_range(l, a)
            Ps[a0:a1, c * kmax:c * kmax + U[a].shape[1]] = U[a]
        Z = bb.applyT(to_orig(Ps))[perm] - H.apply(Ps, levels=done, near=False, transpose=True)
        H.cols_At += Ps.shape[1]
        V = {}
        for b in sorted(set(int(x) for x in G.pair_b)):
            b0, b1 = T.box_range(l, b)
            S = np.zeros((b1 - b0, kmax))
            for a in T.interaction(l, b):
                cq = int(G.color[G.pair_v[pair_index[(b, int(a))]]])
                blk = Z[b0:b1, cq * kmax:(cq + 1) * kmax]
                if combine == "sum":
                    S += blk
                else:
                    S += blk @ mixing_matrix(seed, l, T.box_range(l, int(a))[0], kmax)
            V[b] = _qr_rank(S, k, tol)
        blocks = []
        for q in range(len(G.pair_a)):
            a, b = int(G.pair_a[q]), int(G.pair_b[q])
            cq = int(G.color[G.pair_v[pair_index[(b, a)]]])
            b0, b1 = T.box_range(l, b)
            Zb = Z[b0:b1, cq * kmax:cq * kmax + U[a].shape[1]]
            blocks.append((a, b, U[a], Zb.T @ V[b], V[b]))
        H.lowrank[l] = blocks
        H.ubasis[l], H.vbasis[l] = U, V

    # leaf pass: identity test matrices, subtract every compressed level
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
    if return_graphs:
        return H, graphs
    return H


def uniform_floats(H):
    """Stored values of a uniform H^1 matrix: each basis once, B per pair,
    the leaf blocks."""
    n = 0
    for l in H.lowrank:
        n += sum(U.size for U in H.ubasis[l].values())
        n += sum(V.size for V in H.vbasis[l].values())
        n += sum(B.size for (_, _, _, B, _) in H.lowrank[l])
    n += sum(D.size for (_, _, D) in H.near)
    return n
