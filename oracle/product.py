"""Black boxes built from compressed operators (test infrastructure only).

The problem statement (introduction) only asks for fast routines applying A
and A*; the operator-multiplication experiment of the experiments section
compresses a product whose factors are themselves fast operators.  Here the
factors are H^1 matrices of this oracle:

* HMatrixBlackBox(H): A X = H X and A* X = H* X in the original point order
  (every admissible block U B V*, the leaf blocks D; the adjoint applies
  V B* U* and D*);
* ProductBlackBox(A, B): (A B) X = A (B X), (A B)* X = B* (A* X);
* assemble(H): the dense matrix of H put together block by block (a second
  construction, independent of the applies, to check them against).
"""
from __future__ import annotations

import numpy as np


class HMatrixBlackBox:
    def __init__(self, H):
        self.H = H

    def _apply(self, X, transpose):
        T = self.H.T
        X = np.asarray(X, np.float64).reshape(T.n, -1)
        Yt = self.H.apply(X[T.perm], transpose=transpose)
        Y = np.empty_like(Yt)
        Y[T.perm] = Yt
        return Y

    def apply(self, X):
        return self._apply(X, False)

    def applyT(self, X):
        return self._apply(X, True)


class ProductBlackBox:
    def __init__(self, A, B):
        self.A, self.B = A, B

    def apply(self, X):
        return self.A.apply(self.B.apply(X))

    def applyT(self, X):
        return self.B.applyT(self.A.applyT(X))


def assemble(H):
    """Dense original-order matrix of H from its blocks."""
    T = H.T
    M = np.zeros((T.n, T.n))
    for l, blocks in H.lowrank.items():
        for a, b, U, B, V in blocks:
            a0, a1 = T.box_range(l, a)
            b0, b1 = T.box_range(l, b)
            M[a0:a1, b0:b1] += U @ B @ V.T
    for a, b, D in H.near:
        a0, a1 = T.box_range(T.L, a)
        b0, b1 = T.box_range(T.L, b)
        M[a0:a1, b0:b1] += D
    out = np.empty_like(M)
    out[np.ix_(T.perm, T.perm)] = M
    return out
