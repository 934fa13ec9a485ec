"""Block elimination on the graph of a block system (oracle; test infrastructure).

Sec. 2.1 (graph representation, the 3x3 example and its figure): a vertex is
a block of unknowns, an edge (i, j) is the block A_ij; eliminating a vertex
p replaces every edge (a, b) between its neighbours by A_ab - A_ap A_pp^-1 A_pb
and updates the right-hand side b_a - A_ap A_pp^-1 b_p.
App. C: on the 2-block H-matrix in extended form, eliminating the two x
blocks first (level-by-level order) leaves the system
[[-V0^T A00^-1 U0, -I], [-I, -V1^T A11^-1 U1]] in the auxiliary variables.
"""
from __future__ import annotations

import numpy as np


class BlockGraph:
    def __init__(self, sizes: dict):
        self.sizes = dict(sizes)
        self.E: dict = {}
        self.b: dict = {k: np.zeros(v) for k, v in sizes.items()}

    def set(self, a, c, B):
        self.E[(a, c)] = np.asarray(B, dtype=np.float64)

    def edge(self, a, c):
        return self.E.get((a, c), np.zeros((self.sizes[a], self.sizes[c])))

    def eliminate(self, p):
        """Remove vertex p; every pair of its neighbours gets the Schur fill."""
        App = self.edge(p, p)
        rows = [a for (a, c) in self.E if c == p and a != p]
        cols = [c for (a, c) in self.E if a == p and c != p]
        rows = list(dict.fromkeys(rows))
        cols = list(dict.fromkeys(cols))
        for a in rows:
            Aap = self.E[(a, p)]
            for c in cols:
                fill = -Aap @ np.linalg.solve(App, self.E[(p, c)])
                self.E[(a, c)] = self.edge(a, c) + fill
            self.b[a] = self.b[a] - Aap @ np.linalg.solve(App, self.b[p])
        for key in [k for k in self.E if p in k]:
            del self.E[key]
        del self.sizes[p]
        del self.b[p]

    def dense(self, order):
        offs = np.concatenate([[0], np.cumsum([self.sizes[v] for v in order])]).astype(int)
        M = np.zeros((offs[-1], offs[-1]))
        for ia, a in enumerate(order):
            for ic, c in enumerate(order):
                if (a, c) in self.E:
                    M[offs[ia]:offs[ia + 1], offs[ic]:offs[ic + 1]] = self.E[(a, c)]
        return M
