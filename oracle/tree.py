"""Uniform 2^d-tree, lists and elimination colours (oracle; test infrastructure).

Paper passages followed:
  * Sec. 2.1: the domain is subdivided recursively into clusters Omega_i^(l),
    level 0 is the root and the leaves sit at level L.
  * Sec. 2.2 (after the redirection equations): N_i is the neighbour list of
    a cluster, itself included; I_i is its interaction list, the clusters
    that are children of its parent's neighbours without being neighbours.
  * Sec. 2.2 (merge equations): C_p is the children list of a parent.
  * Sec. 2.3: in 3D, |N_i| <= 3^3 and |I_i| <= 6^3 - 3^3.
  * Sec. 3 opening: a uniform tree.

Readings (where the paper is silent): the root is the tight bounding cube of the points,
slightly enlarged so the largest coordinate falls inside; the leaf level L is
the requested depth; empty boxes are dropped; points are ordered by the
Morton key of their leaf box and then by original index; boxes at one level
are kept in Morton order. Colour (independent-set class) of a box is
sum_k (c_k mod 3) 3^k over its integer coordinates c.
"""
from __future__ import annotations

import itertools

import numpy as np


def morton_key(coords: np.ndarray, bits: int) -> np.ndarray:
    """Interleave the bits of integer box coordinates (dimension 0 least significant)."""
    coords = np.asarray(coords, dtype=np.uint64)
    d = coords.shape[1]
    key = np.zeros(coords.shape[0], dtype=np.uint64)
    for b in range(bits):
        for k in range(d):
            bit = (coords[:, k] >> np.uint64(b)) & np.uint64(1)
            key |= bit << np.uint64(b * d + k)
    return key


def colour_of(coords: np.ndarray) -> np.ndarray:
    """Independent-set class: boxes of one colour are >= 3 apart in some coordinate."""
    coords = np.asarray(coords, dtype=np.int64)
    d = coords.shape[1]
    return sum((coords[:, k] % 3) * (3 ** k) for k in range(d))


class Level:
    """Occupied boxes of one level, in Morton order."""

    def __init__(self, l: int, coords: np.ndarray, d: int):
        self.l = l
        self.coords = coords                      # (nb, d) int64
        self.nb = coords.shape[0]
        self.index = {tuple(c): i for i, c in enumerate(coords.tolist())}
        self.colour = colour_of(coords) if self.nb else np.zeros(0, np.int64)
        self.parent = None                        # (nb,) index into level l-1
        self.children: list[list[int]] = [[] for _ in range(self.nb)]
        self.nbrs: list[list[int]] = []           # N(i), Morton order, includes i
        self.inter: list[list[int]] = []          # I(i), Morton order


def leaf_boxes(points: np.ndarray, depth: int):
    """Root cube (origin, side) and the integer leaf-box coordinates (n, d) of every point."""
    lo = points.min(axis=0)
    hi = points.max(axis=0)
    centre = 0.5 * (lo + hi)
    side = float(np.max(hi - lo)) * (1.0 + 1e-12)
    if side == 0.0:
        side = 1.0
    origin = centre - 0.5 * side
    inv = 1.0 / side
    t = (points - origin) * inv
    nl = 1 << depth
    c = np.floor(t * float(nl)).astype(np.int64)
    c = np.clip(c, 0, nl - 1)
    return origin, side, c


class Tree:
    """Cluster tree of a point cloud (Sec. 2.1, 2.3, 3)."""

    def __init__(self, points: np.ndarray, depth: int):
        points = np.ascontiguousarray(points, dtype=np.float64)
        n, d = points.shape
        if depth < 2:
            raise ValueError("the method needs a leaf level L >= 2 (no well-separated pairs above)")
        self.n, self.d, self.L = n, d, depth
        self.origin, self.side, c = leaf_boxes(points, depth)
        keys = morton_key(c, depth)
        # stable order: leaf key, then original index
        self.perm = np.lexsort((np.arange(n), keys))
        self.points = points[self.perm]
        leaf_c = c[self.perm]
        leaf_keys = keys[self.perm]

        # leaf boxes and point ranges
        uk, start = np.unique(leaf_keys, return_index=True)
        self.leaf_start = np.append(start, n).astype(np.int64)
        self.levels: dict[int, Level] = {}
        self.levels[depth] = Level(depth, leaf_c[start], d)
        for l in range(depth - 1, 1, -1):
            child = self.levels[l + 1]
            pc = child.coords >> 1
            pk = morton_key(pc, l)
            uk, first, inv_idx = np.unique(pk, return_index=True, return_inverse=True)
            lev = Level(l, pc[first], d)
            child.parent = inv_idx.astype(np.int64)
            for ci, p in enumerate(child.parent):
                lev.children[p].append(ci)
            self.levels[l] = lev
        for l in range(2, depth + 1):
            self._lists(l)

    def box_size(self, l: int) -> float:
        return self.side / (1 << l)

    def box_centre(self, l: int, i: int) -> np.ndarray:
        h = self.box_size(l)
        return self.origin + (self.levels[l].coords[i] + 0.5) * h

    def leaf_points(self, i: int) -> slice:
        return slice(int(self.leaf_start[i]), int(self.leaf_start[i + 1]))

    def _lists(self, l: int) -> None:
        """N(i) (adjacent incl. self) and I(i) (children of parent's neighbours, not adjacent)."""
        lev = self.levels[l]
        d = self.d
        offs1 = list(itertools.product((-1, 0, 1), repeat=d))
        lev.nbrs = []
        lev.inter = []
        for i in range(lev.nb):
            ci = lev.coords[i]
            nb = []
            for o in offs1:
                j = lev.index.get(tuple((ci + np.array(o)).tolist()))
                if j is not None:
                    nb.append(j)
            lev.nbrs.append(sorted(nb))
            if l == 2:
                # every level-1 box neighbours every other level-1 box
                lev.inter.append([j for j in range(lev.nb) if j not in set(nb)])
                continue
            pc = ci >> 1
            cand = []
            for o in offs1:
                q = pc + np.array(o)
                for cb in itertools.product((0, 1), repeat=d):
                    cc = tuple((2 * q + np.array(cb)).tolist())
                    j = lev.index.get(cc)
                    if j is not None and int(np.max(np.abs(np.array(cc) - ci))) > 1:
                        cand.append(j)
            lev.inter.append(sorted(cand))

    def elimination_order(self, l: int) -> list[int]:
        """Boxes of level l by (colour, Morton position): one batch per colour class."""
        lev = self.levels[l]
        return sorted(range(lev.nb), key=lambda i: (int(lev.colour[i]), i))

    def adjacent(self, l: int, i: int, j: int) -> bool:
        lev = self.levels[l]
        return int(np.max(np.abs(lev.coords[i] - lev.coords[j]))) <= 1
