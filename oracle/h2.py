"""The H2 representation R1 of A and its fast product (oracle; test infrastructure).

Sec. 2.1: well-separated blocks are replaced by U_i K_ij V_j^T with nested
bases; eq. (A_decomp_l3) splits A into a sparse near field S^(L) plus
U^(L) K^(L) V^(L)T, and eq. (A_decomp_l2) splits K^(L) again one level up,
down to level 2 (no well-separated pairs exist at level 1). In FMM terms U is
L2P/L2L, K is M2L and V^T is P2M/M2M; the near-field blocks are P2P.

The operators come from Chebyshev interpolation (Sec. 3 opening):
  leaf U_i = V_i: Lagrange basis of box i at its points   (m_i x n^d)
  transfer child c -> parent: T_c[m, m'] = l^parent_{m'}(xi^c_m)  (n^d x n^d)
  M2L K_ij[m, m'] = K(|xi^i_m - xi^j_{m'}|) for j in I(i)         (n^d x n^d)
  P2P S_ij = A[points_i, points_j] for j in N(i)

R1 is this plain interpolation form. The matrix it represents, A~, is the
system the factorization inverts and GMRES solves.
"""
from __future__ import annotations

import numpy as np

from . import chebyshev as cheb
from . import kernels as kern
from .tree import Tree, leaf_boxes


class H2:
    def __init__(self, tree: Tree, kind: str, param: float, shift: float, n: int):
        self.tree, self.kind, self.param, self.shift, self.n = tree, kind, param, shift, n
        d = tree.d
        self.q = n ** d
        L = tree.L
        lev = tree.levels[L]
        h = tree.box_size(L)
        # leaf interpolation matrices
        self.Ubar = []
        for i in range(lev.nb):
            P = tree.points[tree.leaf_points(i)]
            Xref = (P - tree.box_centre(L, i)) * (2.0 / h)
            self.Ubar.append(cheb.lagrange_nd(n, Xref))
        # child-to-parent transfer, one per child position (bit k set = upper half in dim k)
        g = cheb.node_grid(n, d)
        self.T = {}
        for bits in range(1 << d):
            sgn = np.array([1.0 if (bits >> k) & 1 else -1.0 for k in range(d)])
            self.T[bits] = cheb.lagrange_nd(n, 0.5 * g + 0.5 * sgn)
        self._m2l_cache: dict = {}

    def child_bits(self, l: int, c: int) -> int:
        cc = self.tree.levels[l].coords[c]
        return int(sum(((int(cc[k]) & 1) << k) for k in range(self.tree.d)))

    def m2l(self, l: int, i: int, j: int) -> np.ndarray:
        """K_ij between the Chebyshev nodes of boxes i and j at level l."""
        tr = self.tree
        lev = tr.levels[l]
        delta = tuple((lev.coords[j] - lev.coords[i]).tolist())
        key = (l, delta)
        if key not in self._m2l_cache:
            h = tr.box_size(l)
            g = cheb.node_grid(self.n, tr.d) * (0.5 * h)
            Xi = g
            Xj = g + np.array(delta, dtype=np.float64) * h
            self._m2l_cache[key] = kern.block(self.kind, self.param, Xi, Xj)
        return self._m2l_cache[key]

    def p2p(self, i: int, j: int) -> np.ndarray:
        tr = self.tree
        Pi = tr.points[tr.leaf_points(i)]
        Pj = tr.points[tr.leaf_points(j)]
        B = kern.block(self.kind, self.param, Pi, Pj)
        if i == j:
            B[np.diag_indices_from(B)] += self.shift
        return B

    def matvec_tree(self, X: np.ndarray) -> np.ndarray:
        """A~ X with X in tree (permuted) point order, X of shape (N, k)."""
        tr = self.tree
        L = tr.L
        X = np.asarray(X, dtype=np.float64)
        if X.ndim == 1:
            X = X[:, None]
        k = X.shape[1]
        # upward pass: multipoles w (y in the paper's notation)
        w = {L: [self.Ubar[i].T @ X[tr.leaf_points(i)] for i in range(tr.levels[L].nb)]}
        for l in range(L - 1, 1, -1):
            lev = tr.levels[l]
            w[l] = []
            for p in range(lev.nb):
                acc = np.zeros((self.q, k))
                for c in lev.children[p]:
                    acc += self.T[self.child_bits(l + 1, c)].T @ w[l + 1][c]
                w[l].append(acc)
        # interaction lists: locals g (z in the paper's notation)
        g = {}
        for l in range(2, L + 1):
            lev = tr.levels[l]
            g[l] = []
            for i in range(lev.nb):
                acc = np.zeros((self.q, k))
                for j in lev.inter[i]:
                    acc += self.m2l(l, i, j) @ w[l][j]
                g[l].append(acc)
        # downward pass
        for l in range(3, L + 1):
            lev = tr.levels[l]
            for c in range(lev.nb):
                g[l][c] = g[l][c] + self.T[self.child_bits(l, c)] @ g[l - 1][lev.parent[c]]
        out = np.zeros((tr.n, k))
        lev = tr.levels[L]
        for i in range(lev.nb):
            s = tr.leaf_points(i)
            out[s] = self.Ubar[i] @ g[L][i]
            for j in lev.nbrs[i]:
                out[s] += self.p2p(i, j) @ X[tr.leaf_points(j)]
        return out

    def matvec(self, X: np.ndarray) -> np.ndarray:
        """A~ X in the caller's point order."""
        tr = self.tree
        X = np.asarray(X, dtype=np.float64)
        vec = X.ndim == 1
        Xt = (X[:, None] if vec else X)[tr.perm]
        Yt = self.matvec_tree(Xt)
        Y = np.empty_like(Yt)
        Y[tr.perm] = Yt
        return Y[:, 0] if vec else Y

    def dense(self) -> np.ndarray:
        """A~ as a dense matrix in the caller's order (small N only)."""
        return self.matvec(np.eye(self.tree.n))


def h2_rows(points, kind: str, param: float, shift: float, depth: int, n: int, X, rows) -> np.ndarray:
    """Rows `rows` (caller order) of A~ X, one target at a time, straight from the black-box FMM definition.

    For a target point r_i in leaf box b_L with ancestors b_l:
      (A~ X)_i = sum_{j in N(b_L)} K(|r_i - r_j|) X_j + s X_i
               + sum_{l=2..L} sum_{C in I(b_l)} L_{b_l}(r_i) K(xi^{b_l}, xi^C) W^C,
      W^C = sum_{j in C} L_C(r_j)^T X_j,
    with L_B the tensor Lagrange basis on the Chebyshev nodes xi^B of box B (Sec. 2.1 lists; Sec. 3
    opening). Moments and local evaluations are taken directly at every level rather than through the
    child transfers: interpolating a degree n-1 Lagrange polynomial on a child's n nodes is exact, so the
    two forms represent the same A~ and differ by rounding only. Cost O(N n^d) per level plus O(n^2d |I|)
    per target, so it serves at sizes where the full oracle H2 is too slow to build.
    """
    P = np.ascontiguousarray(points, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    vec = X.ndim == 1
    X2 = X[:, None] if vec else X
    N, d = P.shape
    L = depth
    origin, side, cL = leaf_boxes(P, L)
    g = cheb.node_grid(n, d)
    out = np.zeros((len(rows), X2.shape[1]))
    # direct moments of every occupied box at every level
    mom = {}
    for l in range(2, L + 1):
        h = side / (1 << l)
        cl = cL >> (L - l)
        boxes, inv = np.unique(cl, axis=0, return_inverse=True)
        inv = inv.reshape(-1)
        centres = origin + (cl + 0.5) * h
        Lp = cheb.lagrange_nd(n, (P - centres) * (2.0 / h))            # (N, n^d)
        W = np.zeros((boxes.shape[0], n ** d, X2.shape[1]))
        np.add.at(W, inv, Lp[:, :, None] * X2[:, None, :])
        mom[l] = (boxes, W, h)
    for t, i in enumerate(rows):
        i = int(i)
        bL = cL[i]
        near = np.max(np.abs(cL - bL), axis=1) <= 1
        r = np.sqrt(np.sum((P[near] - P[i]) ** 2, axis=1))
        acc = kern.kernel_of_r(kind, param, r) @ X2[near] + shift * X2[i]
        for l in range(2, L + 1):
            boxes, W, h = mom[l]
            b = bL >> (L - l)
            far = np.max(np.abs(boxes - b), axis=1) > 1
            if l > 2:
                far &= np.max(np.abs((boxes >> 1) - (b >> 1)), axis=1) <= 1
            if not np.any(far):
                continue
            Xi = g * (0.5 * h)
            Xj = (g[None, :, :] * (0.5 * h) + ((boxes[far] - b) * h)[:, None, :]).reshape(-1, d)
            K = kern.block(kind, param, Xi, Xj)                          # (n^d, |I| n^d)
            loc = K @ W[far].reshape(-1, X2.shape[1])
            ci = origin + (b + 0.5) * h
            acc = acc + cheb.lagrange_nd(n, ((P[i] - ci) * (2.0 / h))[None, :])[0] @ loc
        out[t] = acc
    return out[:, 0] if vec else out
