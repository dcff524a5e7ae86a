"""ctypes wrapper of the oracle's plain-C combinatorics (``comb.c``).

Test infrastructure only.  ``build()`` compiles ``comb.c`` with gcc into
``liborc_comb.so`` beside this file.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liborc_comb.so")
_lib = None


def build(force: bool = True) -> str:
    src = os.path.join(_HERE, "comb.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared",
                               "-ffp-contract=off", "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build(force=True)
    lib = C.CDLL(_SO)
    P = C.c_void_p
    i64p = np.ctypeslib.ndpointer(np.int64, flags="C")
    i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
    f64p = np.ctypeslib.ndpointer(np.float64, flags="C")
    lib.orc_build.restype = P
    lib.orc_build.argtypes = [f64p, C.c_int64, C.c_int, C.c_int, C.c_int, C.c_int]
    lib.orc_nlev.argtypes = [P]
    lib.orc_nbox.argtypes = [P, C.c_int]
    lib.orc_perm.argtypes = [P, i64p]
    lib.orc_boxes.argtypes = [P, C.c_int, i64p, i32p, i64p, i32p]
    lib.orc_list_len.argtypes = [P, C.c_int, C.c_int]
    lib.orc_list.argtypes = [P, C.c_int, C.c_int, i32p, i32p]
    lib.orc_graph_sizes.argtypes = [P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int64),
                                    C.POINTER(C.c_int), C.POINTER(C.c_int)]
    lib.orc_graph.argtypes = [P, C.c_int, i32p, i32p, i32p, i64p, i32p, i32p, i32p, i32p]
    lib.orc_dsatur.restype = C.c_int
    lib.orc_dsatur.argtypes = [C.c_int, i64p, i32p, i32p]
    lib.orc_free.argtypes = [P]
    _lib = lib
    return lib


def dsatur(xadj: np.ndarray, adj: np.ndarray) -> tuple[np.ndarray, int]:
    """DSatur (alg:dsatur) with ties broken by degree, then lower id."""
    lib = _load()
    nv = len(xadj) - 1
    col = np.zeros(max(nv, 1), np.int32)
    nc = lib.orc_dsatur(nv, np.ascontiguousarray(xadj, np.int64),
                        np.ascontiguousarray(adj if len(adj) else np.zeros(1, np.int32), np.int32), col)
    return col[:nv], int(nc)


class Graph:
    """One constraint incompatibility graph (def:incompatibility_graph)."""

    def __init__(self, vbox, vset_ptr, vset, xadj, adj, pa, pb, pv):
        self.vbox, self.vset_ptr, self.vset = vbox, vset_ptr, vset
        self.xadj, self.adj = xadj, adj
        self.pair_a, self.pair_b, self.pair_v = pa, pb, pv
        self.color, self.ncolors = dsatur(xadj, adj)

    @property
    def nv(self):
        return len(self.vbox)

    @property
    def nedges(self):
        return int(self.xadj[-1]) // 2


class OTree:
    """Box tree, lists and graphs for one point set.

    ``kind``: "geometric" (2^d-tree, section on rank-structured matrices) or
    "index_binary" (index halving, fig:tree).  ``adm``: "strong" or "weak".
    """

    def __init__(self, points: np.ndarray, leaf: int, kind: str = "geometric", adm: str = "strong"):
        """points: N x d, 1 <= d <= 8 (2^d-trees; integer cells of 21 bits per
        coordinate for d <= 3, floor(63 / d) bits above)."""
        lib = _load()
        pts = np.ascontiguousarray(points, np.float64)
        if pts.ndim == 1:
            pts = pts.reshape(-1, 1)
        n, dim = pts.shape
        if not 1 <= dim <= 8:
            raise ValueError("points must have 1 to 8 coordinates")
        if kind == "index_binary" and adm != "weak":
            raise ValueError("the index-halving tree is only used with weak admissibility")
        self.n, self.dim, self.leaf, self.kind, self.adm = n, dim, leaf, kind, adm
        self.points = pts
        h = lib.orc_build(pts, n, dim, leaf, 1 if kind == "index_binary" else 0, 1 if adm == "weak" else 0)
        try:
            self.nlev = lib.orc_nlev(h)
            self.perm = np.zeros(max(n, 1), np.int64)
            lib.orc_perm(h, self.perm)
            self.perm = self.perm[:n]
            self.start, self.parent, self.org, self.blev = [], [], [], []
            self.nei, self.intl = [], []
            for l in range(self.nlev):
                nb = lib.orc_nbox(h, l)
                s = np.zeros(nb + 1, np.int64); p = np.zeros(nb, np.int32)
                os_ = max(3, dim)
                o = np.zeros(nb * os_, np.int64); b = np.zeros(nb, np.int32)
                lib.orc_boxes(h, l, s, p, o, b)
                self.start.append(s); self.parent.append(p)
                self.org.append(o.reshape(nb, os_)); self.blev.append(b)
                lists = []
                for which in (0, 1):
                    ln = lib.orc_list_len(h, l, which)
                    ptr = np.zeros(nb + 1, np.int32); idx = np.zeros(max(ln, 1), np.int32)
                    lib.orc_list(h, l, which, ptr, idx)
                    lists.append((ptr, idx[:ln]))
                self.nei.append(lists[0]); self.intl.append(lists[1])
            self.graphs = []
            for g in range(self.nlev + 1):
                nv, nadj, nset, npairs = C.c_int(), C.c_int64(), C.c_int(), C.c_int()
                lib.orc_graph_sizes(h, g, C.byref(nv), C.byref(nadj), C.byref(nset), C.byref(npairs))
                nv, nadj, nset, npairs = nv.value, nadj.value, nset.value, npairs.value
                vbox = np.zeros(max(nv, 1), np.int32); vptr = np.zeros(nv + 1, np.int32)
                vset = np.zeros(max(nset, 1), np.int32); xadj = np.zeros(nv + 1, np.int64)
                adj = np.zeros(max(nadj, 1), np.int32)
                pa = np.zeros(max(npairs, 1), np.int32); pb = np.zeros(max(npairs, 1), np.int32)
                pv = np.zeros(max(npairs, 1), np.int32)
                lib.orc_graph(h, g, vbox, vptr, vset, xadj, adj, pa, pb, pv)
                self.graphs.append(Graph(vbox[:nv], vptr, vset[:nset], xadj, adj[:nadj],
                                         pa[:npairs], pb[:npairs], pv[:npairs]))
        finally:
            lib.orc_free(h)
        self.L = self.nlev - 1
        self.leaf_graph = self.graphs[self.nlev]

    # --- convenience -------------------------------------------------------
    def nbox(self, l):
        return len(self.start[l]) - 1

    def box_range(self, l, b):
        return int(self.start[l][b]), int(self.start[l][b + 1])

    def neighbors(self, l, b):
        p, i = self.nei[l]
        return i[p[b]:p[b + 1]]

    def interaction(self, l, b):
        p, i = self.intl[l]
        return i[p[b]:p[b + 1]]

    def sampled_levels(self):
        """Levels that hold at least one admissible pair, coarsest first."""
        return [l for l in range(1, self.nlev) if len(self.graphs[l].pair_a) > 0]

    def leaf_max(self):
        s = self.start[self.L]
        return int(np.max(np.diff(s))) if len(s) > 1 else 0
