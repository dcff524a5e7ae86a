"""Host structure of the batched form (hm_build_forest), CPU only.

A forest of independent instances must hold, for each instance, exactly the
tree, lists, graphs and colors that the instance gets on its own (box, vertex
and row ids shifted by the instance's offsets; a shallower tree carried down
unchanged), and nothing may join two instances.  The single-instance
structures themselves are pinned bit-exactly to the oracle elsewhere.
"""
import numpy as np
import pytest

import paper_2205_03406_amd as hm
import workloads

NEI, INT = hm.HM_LIST_NEIGHBOR, hm.HM_LIST_INTERACTION


def _instances():
    return [
        ("ellipses", [workloads.ellipse(n, a, b) for n, a, b in
                      [(2900, 1.7, 0.6), (300, 1.0, 1.0), (1500, 0.5, 2.0), (64, 1.2, 0.9),
                       (65, 1.0, 0.7), (900, 2.0, 1.9)]], 64, "geometric", "strong"),
        ("spheres", [workloads.sphere(n, seed) for n, seed in [(2000, 11), (700, 12), (130, 13)]],
         128, "geometric", "strong"),
        ("lines", [workloads.uniform_line(n, seed) for n, seed in [(1024, 1), (300, 2), (513, 3)]],
         64, "index_binary", "weak"),
    ]


def _ids(case):
    return case[0]


@pytest.mark.parametrize("case", _instances(), ids=_ids)
def test_forest_is_the_union_of_its_instances(case):
    _, parts, leaf, kind, adm = case
    F = hm.Tree(parts, leaf, kind, adm).color()
    singles = [hm.Tree(p, leaf, kind, adm).color() for p in parts]
    off = F.instances()
    assert np.array_equal(off, np.concatenate([[0], np.cumsum([p.shape[0] for p in parts])]))
    assert F.nlev == max(T.nlev for T in singles)
    fperm = F.perm()
    for i, T in enumerate(singles):
        assert np.array_equal(fperm[off[i]:off[i + 1]], T.perm() + off[i])

    # box offsets of every instance at every level
    boff = []
    for l in range(F.nlev):
        start, parent, org, blev = F.level(l)
        b = np.searchsorted(start[:-1], off[:-1], side="left")
        boff.append(np.append(b, len(parent)))
    for l in range(F.nlev):
        start, parent, org, blev = F.level(l)
        nptr, nidx = F.list(l, NEI)
        iptr, iidx = F.list(l, INT)
        for i, T in enumerate(singles):
            sl = min(l, T.L)
            s_start, s_parent, s_org, s_blev = T.level(sl)
            b0, b1 = boff[l][i], boff[l][i + 1]
            assert np.array_equal(start[b0:b1] - off[i], s_start[:-1])
            assert np.array_equal(org[b0:b1], s_org) and np.array_equal(blev[b0:b1], s_blev)
            if l == 0:
                assert np.all(parent[b0:b1] == -1)
            elif l > T.L:  # carried: each box is its own parent's copy
                assert np.array_equal(parent[b0:b1] - boff[l - 1][i], np.arange(b1 - b0))
            else:
                assert np.array_equal(parent[b0:b1] - boff[l - 1][i], s_parent)
            sp, si = T.list(sl, NEI)
            got = [nidx[nptr[b]:nptr[b + 1]] - b0 for b in range(b0, b1)]
            want = [si[sp[b]:sp[b + 1]] for b in range(b1 - b0)]
            assert all(np.array_equal(g, w) for g, w in zip(got, want))
            sp, si = T.list(sl, INT)
            for b in range(b0, b1):
                g = iidx[iptr[b]:iptr[b + 1]]
                if l > T.L:
                    assert len(g) == 0
                else:
                    assert np.array_equal(g - b0, si[sp[b - b0]:sp[b - b0 + 1]])

    # graphs: disjoint unions with instance-major vertex ids, same colors
    for g in list(range(F.nlev)) + [-1]:
        FG = F.graph(g)
        bl = F.nlev - 1 if g == -1 else g
        v0 = 0
        ncol = 0
        for i, T in enumerate(singles):
            if g != -1 and g > T.L:
                continue
            SG = T.graph(g)
            nv = SG.nv
            b0 = boff[bl][i]
            assert np.array_equal(FG.vbox[v0:v0 + nv] - b0, SG.vbox)
            xa = FG.xadj[v0:v0 + nv + 1]
            assert np.array_equal(xa - xa[0], SG.xadj)
            assert np.array_equal(FG.adj[xa[0]:xa[-1]] - v0, SG.adj)
            assert np.array_equal(FG.color[v0:v0 + nv], SG.color)
            sel = (FG.pair_a >= b0) & (FG.pair_a < b0 + (boff[bl][i + 1] - b0))
            assert np.array_equal(FG.pair_a[sel] - b0, SG.pair_a)
            assert np.array_equal(FG.pair_b[sel] - b0, SG.pair_b)
            assert np.array_equal(FG.pair_v[sel] - v0, SG.pair_v)
            ncol = max(ncol, SG.ncolors)
            v0 += nv
        assert v0 == FG.nv
        assert FG.ncolors == ncol
        # DSatur on the whole disjoint union gives the same colors
        if FG.nv:
            col, nc = hm.color(FG.xadj, FG.adj)
            assert np.array_equal(col, FG.color) and nc == ncol
        # no edge and no pair between instances
        if FG.nv:
            inst_of_box = np.searchsorted(boff[bl], np.arange(boff[bl][-1]), side="right") - 1
            vinst = inst_of_box[FG.vbox]
            src = np.repeat(np.arange(FG.nv), np.diff(FG.xadj))
            assert np.array_equal(vinst[src], vinst[FG.adj])
            assert np.array_equal(inst_of_box[FG.pair_a], inst_of_box[FG.pair_b])


def test_forest_arguments():
    with pytest.raises(hm.HMError):
        hm.Tree([np.zeros((0, 2)), workloads.ellipse(100, 1.0, 1.0)], 64)
    with pytest.raises(hm.HMError):
        hm.Tree([workloads.uniform_line(100, 1)], 64, "index_binary", "strong")
    T = hm.Tree(workloads.ellipse(500, 1.0, 1.0), 64)
    assert np.array_equal(T.instances(), [0, 500])
