"""Pins of the oracle's tree, lists and colours against brute-force definitions.

Paper: Sec. 2.2 (N_i includes the box itself; I_i = children of the parent's
neighbours that are not neighbours), Sec. 2.3 (|N| <= 27, |I| <= 189 in 3D).
"""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle.tree import Tree, morton_key


def brute_lists(tree, l):
    lev = tree.levels[l]
    C = lev.coords
    nbrs, inter = [], []
    for i in range(lev.nb):
        nb = [j for j in range(lev.nb) if np.max(np.abs(C[i] - C[j])) <= 1]
        pi = C[i] // 2
        it = [j for j in range(lev.nb)
              if np.max(np.abs(C[j] // 2 - pi)) <= 1 and np.max(np.abs(C[i] - C[j])) > 1]
        nbrs.append(nb)
        inter.append(it)
    return nbrs, inter


@pytest.mark.parametrize("n,dim,depth,seed", [(400, 2, 4, 3), (900, 3, 3, 5), (200, 1, 5, 8)])
def test_lists_match_brute_force(n, dim, depth, seed):
    pts = W.uniform_cube(n, dim, seed)
    tr = Tree(pts, depth)
    for l in range(2, depth + 1):
        nb, it = brute_lists(tr, l)
        assert [sorted(x) for x in tr.levels[l].nbrs] == nb
        assert [sorted(x) for x in tr.levels[l].inter] == it


def test_list_sizes_bounded_3d():
    pts = W.uniform_cube(20000, 3, 11)
    tr = Tree(pts, 4)
    for l in range(2, 5):
        lev = tr.levels[l]
        assert max(len(x) for x in lev.nbrs) <= 27
        assert max(len(x) for x in lev.inter) <= 189
    # a fully occupied interior box reaches both bounds at level 4
    lev = tr.levels[4]
    assert max(len(x) for x in lev.nbrs) == 27
    assert max(len(x) for x in lev.inter) == 189


def test_points_partitioned_and_inside_boxes():
    pts = W.clustered(8, 500, 0.05, 31, 32)
    tr = Tree(pts, 5)
    L = tr.L
    lev = tr.levels[L]
    assert tr.leaf_start[0] == 0 and tr.leaf_start[-1] == pts.shape[0]
    assert sorted(tr.perm.tolist()) == list(range(pts.shape[0]))
    h = tr.box_size(L)
    for i in range(lev.nb):
        P = tr.points[tr.leaf_points(i)]
        lo = tr.origin + lev.coords[i] * h
        assert np.all(P >= lo - 1e-12) and np.all(P <= lo + h + 1e-12)
    # boxes in strictly increasing Morton order at every level
    for l in range(2, L + 1):
        k = morton_key(tr.levels[l].coords, l)
        assert np.all(np.diff(k.astype(np.int64)) > 0)


def test_colour_classes_have_disjoint_neighbourhoods():
    pts = W.uniform_cube(3000, 3, 13)
    tr = Tree(pts, 3)
    lev = tr.levels[3]
    for c in set(lev.colour.tolist()):
        members = [i for i in range(lev.nb) if lev.colour[i] == c]
        for a, b in itertools.combinations(members, 2):
            assert not (set(lev.nbrs[a]) & set(lev.nbrs[b]))
    assert len(set(lev.colour.tolist())) == 27


def test_children_and_parent_consistent():
    pts = W.uniform_cube(5000, 2, 17)
    tr = Tree(pts, 5)
    for l in range(2, 5):
        lev, ch = tr.levels[l], tr.levels[l + 1]
        for p in range(lev.nb):
            for c in lev.children[p]:
                assert ch.parent[c] == p
                assert np.all(ch.coords[c] // 2 == lev.coords[p])
        assert sum(len(x) for x in lev.children) == ch.nb
