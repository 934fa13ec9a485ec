"""Extended sparse system E, orthonormal bases, weights and sigma_0 (oracle; test infrastructure).

Paper passages followed:
  * Sec. 2.1, eqs. (y3), (y2), (z2), (z3), (decomposition_compact) and
    (Ax=b_extended): auxiliary multipole variables y^(l) = V^(l)T x^(l) and
    local variables z^(l) turn A x = b into the sparse system E. Row order
    x, (V^T x - y), (-z + K y + U z_parent) per level, variable order
    x, z^(l), y^(l) per level, which keeps E symmetric when A is symmetric.
  * Sec. 3 opening: after Chebyshev interpolation an additional SVD reduces
    the rank. Reading: an exact QR of the interpolation bases, bottom-up, so
    every basis is orthonormal (its R factor folds into K and the transfers);
    rank = min(rows, n^d), no numerical truncation at this step.
  * Sec. 2.2, footnote on initial weights: Sigma_U of a box is obtained by an
    SVD of the block row U K V^T of its far field. Reading: the far field of a
    box is its interaction list at its own level together with the far field
    of its parent reached through the transfer, so a direction that only an
    ancestor's far field uses does not get a zero weight.
  * Sec. 2.4, eq. (methods_SVD_rank_spectralnorm): ranks are decided against
    eps * sigma_0(E), sigma_0 the largest singular value of E. Reading: E is
    symmetric for the radial kernels, so sigma_0 is the largest eigenvalue
    magnitude of E, taken from a deterministic Lanczos process on E (start
    vector all ones; three-term recurrence; stopped when the largest Ritz
    value magnitude changes by <= 1e-12 relatively, at most 300 steps); the
    kept directions are those with sigma strictly above
    tau = max(eps, 64 u) sigma_0 (u the unit roundoff of the factor
    precision); where U and V of a box keep different counts, both keep the
    larger count so that the z/y identity blocks stay square.
"""
from __future__ import annotations

import numpy as np

from .h2 import H2
from .tree import Tree


def left_svd(M: np.ndarray):
    """Full left singular vectors W (r x r) and singular values padded with zeros to r."""
    r = M.shape[0]
    if r == 0:
        return np.zeros((0, 0)), np.zeros(0)
    if M.shape[1] == 0:
        return np.eye(r), np.zeros(r)
    W, s, _ = np.linalg.svd(M, full_matrices=True)
    sp = np.zeros(r)
    sp[: s.shape[0]] = s
    return W, sp


class R2:
    """Orthonormal-basis H2 operators of E, weighted and truncated at tau."""

    def __init__(self, h2: H2, eps: float, unit_roundoff: float = 2.0 ** -53,
                 sigma0: float | None = None, rank_max: int = 0, weights: bool = True):
        self.h2 = h2
        tr = h2.tree
        self.tree = tr
        L = tr.L
        self.L = L
        q = h2.q
        # --- exact QR of the interpolation bases, bottom-up -------------------
        self.Q = {}                       # leaf orthonormal bases (m_i x r_i)
        R = {L: []}
        for i in range(tr.levels[L].nb):
            Ub = h2.Ubar[i]
            Qi, Ri = np.linalg.qr(Ub, mode="reduced")
            self.Q[i] = Qi
            R[L].append(Ri)
        self.r = {L: [R[L][i].shape[0] for i in range(tr.levels[L].nb)]}
        self.PU = {}                      # per level l > 2: list of (r_c x r_parent)
        self.PV = {}
        for l in range(L - 1, 1, -1):
            lev = tr.levels[l]
            R[l] = []
            self.r[l] = []
            PU_child = [None] * tr.levels[l + 1].nb
            for p in range(lev.nb):
                cs = lev.children[p]
                M = np.vstack([R[l + 1][c] @ h2.T[h2.child_bits(l + 1, c)] for c in cs])
                Qp, Rp = np.linalg.qr(M, mode="reduced")
                R[l].append(Rp)
                self.r[l].append(Rp.shape[0])
                off = 0
                for c in cs:
                    rc = R[l + 1][c].shape[0]
                    PU_child[c] = Qp[off:off + rc]
                    off += rc
            self.PU[l + 1] = PU_child
            self.PV[l + 1] = [b.copy() for b in PU_child]
        # M2L blocks in the orthonormal bases
        self.K = {}
        for l in range(2, L + 1):
            lev = tr.levels[l]
            Kl = {}
            for i in range(lev.nb):
                for j in lev.inter[i]:
                    Kl[(i, j)] = R[l][i] @ h2.m2l(l, i, j) @ R[l][j].T
            self.K[l] = Kl
        # leaf near field (P2P)
        levL = tr.levels[L]
        self.S = {}
        for i in range(levL.nb):
            for j in levL.nbrs[i]:
                self.S[(i, j)] = h2.p2p(i, j)
        self.U = {i: self.Q[i] for i in self.Q}
        self.V = {i: self.Q[i].copy() for i in self.Q}

        # --- sigma_0 and tau ----------------------------------------------------
        self.sigma0_estimated = None
        if sigma0 is None:
            sigma0 = self.lanczos_sigma0()
            self.sigma0_estimated = sigma0
        self.sigma0 = float(sigma0)
        self.tau = max(eps, 64.0 * unit_roundoff) * self.sigma0
        self.rank_max = rank_max

        # --- weights, rotation, truncation --------------------------------------
        if weights:
            self._weights_and_truncate()

    # ------------------------------------------------------------------ E x
    def vec_layout(self):
        """Sizes of the blocks of a vector of E: x, then z^(l), y^(l) for l = L..2."""
        tr = self.tree
        out = [("x", None, tr.n)]
        for l in range(self.L, 1, -1):
            out.append(("z", l, sum(self.r[l])))
            out.append(("y", l, sum(self.r[l])))
        return out

    def _split(self, v):
        tr = self.tree
        parts = {}
        o = 0
        parts["x"] = v[o:o + tr.n]
        o += tr.n
        for l in range(self.L, 1, -1):
            rs = self.r[l]
            for t in ("z", "y"):
                blocks = []
                for ri in rs:
                    blocks.append(v[o:o + ri])
                    o += ri
                parts[(t, l)] = blocks
        return parts

    def _join(self, parts):
        seq = [parts["x"]]
        for l in range(self.L, 1, -1):
            for t in ("z", "y"):
                seq.extend(parts[(t, l)])
        return np.concatenate(seq) if seq else np.zeros(0)

    def size(self):
        return sum(s for _, _, s in self.vec_layout())

    def apply_E(self, v, transpose=False):
        """E v (or E^T v) for the orthonormal, unweighted operators (eq. Ax=b_extended)."""
        tr = self.tree
        L = self.L
        P = self._split(v)
        levL = tr.levels[L]
        out = {"x": np.zeros(tr.n)}
        for l in range(L, 1, -1):
            out[("z", l)] = [np.zeros(ri) for ri in self.r[l]]
            out[("y", l)] = [np.zeros(ri) for ri in self.r[l]]
        x = P["x"]
        if not transpose:
            # x rows: S x + U z^(L)
            for i in range(levL.nb):
                s = tr.leaf_points(i)
                acc = self.U[i] @ P[("z", L)][i]
                for j in levL.nbrs[i]:
                    acc = acc + self.S[(i, j)] @ x[tr.leaf_points(j)]
                out["x"][s] = acc
            for l in range(L, 1, -1):
                lev = tr.levels[l]
                for i in range(lev.nb):
                    # row (V^T x^(l) - y^(l)), x^(l) = x at the leaves, y^(l+1) above
                    if l == L:
                        vt = self.V[i].T @ x[tr.leaf_points(i)]
                    else:
                        vt = np.zeros(self.r[l][i])
                        for c in lev.children[i]:
                            vt = vt + self.PV[l + 1][c].T @ P[("y", l + 1)][c]
                    out[("z", l)][i] = vt - P[("y", l)][i]
                    # row (-z^(l) + K y^(l) + U z^(l-1))
                    acc = -P[("z", l)][i]
                    for j in lev.inter[i]:
                        acc = acc + self.K[l][(i, j)] @ P[("y", l)][j]
                    if l > 2:
                        acc = acc + self.PU[l][i] @ P[("z", l - 1)][lev.parent[i]]
                    out[("y", l)][i] = acc
            return self._join(out)
        # transpose: the row blocks of v are (x rows, z-type rows, y-type rows)
        for i in range(levL.nb):
            s = tr.leaf_points(i)
            acc = self.V[i] @ P[("z", L)][i]
            for j in levL.nbrs[i]:
                acc = acc + self.S[(j, i)].T @ x[tr.leaf_points(j)]
            out["x"][s] = acc
        for l in range(L, 1, -1):
            lev = tr.levels[l]
            for i in range(lev.nb):
                # column z_i^(l): from x^(l) rows (U) and from y-type row (-I)
                if l == L:
                    uz = self.U[i].T @ x[tr.leaf_points(i)]
                else:
                    uz = np.zeros(self.r[l][i])
                    for c in lev.children[i]:
                        uz = uz + self.PU[l + 1][c].T @ P[("y", l + 1)][c]
                out[("z", l)][i] = uz - P[("y", l)][i]
                # column y_i^(l): from z-type row (-I), y-type rows (K^T), z-type row of parent (PV)
                acc = -P[("z", l)][i]
                for j in lev.inter[i]:
                    acc = acc + self.K[l][(j, i)].T @ P[("y", l)][j]
                if l > 2:
                    acc = acc + self.PV[l][i] @ P[("z", l - 1)][lev.parent[i]]
                out[("y", l)][i] = acc
        return self._join(out)

    def dense_E(self):
        n = self.size()
        I = np.eye(n)
        return np.column_stack([self.apply_E(I[:, k]) for k in range(n)])

    def lanczos_sigma0(self, maxit: int = 300, rtol: float = 1e-12) -> float:
        """Largest |eigenvalue| of the symmetric E by the Lanczos process (Ritz values of the tridiagonal)."""
        n = self.size()
        q = np.ones(n) / np.sqrt(n)
        q_prev = np.zeros(n)
        alphas, betas = [], []
        beta = 0.0
        theta_old = None
        theta = 0.0
        self.sigma0_steps = 0
        for k in range(maxit):
            w = self.apply_E(q) - beta * q_prev
            alpha = float(q @ w)
            w = w - alpha * q
            alphas.append(alpha)
            T = np.diag(alphas) + np.diag(betas, 1) + np.diag(betas, -1)
            ev = np.linalg.eigvalsh(T)
            theta = float(max(abs(ev[0]), abs(ev[-1])))
            self.sigma0_steps = k + 1
            if theta_old is not None and abs(theta - theta_old) <= rtol * theta:
                break
            theta_old = theta
            beta = float(np.linalg.norm(w))
            if beta == 0.0:
                break
            betas.append(beta)
            q_prev, q = q, w / beta
        return theta

    def power_sigma0(self, maxit: int = 200, rtol: float = 1e-10) -> float:
        n = self.size()
        v = np.ones(n) / np.sqrt(n)
        s_old = -1.0
        s = 0.0
        for k in range(maxit):
            w = self.apply_E(v)
            s = float(np.linalg.norm(w))
            if k > 0 and abs(s - s_old) <= rtol * s:
                break
            s_old = s
            u = self.apply_E(w, transpose=True)
            nu = float(np.linalg.norm(u))
            if nu == 0.0:
                break
            v = u / nu
        return s

    # ---------------------------------------------------------- weights
    def _weights_and_truncate(self):
        tr = self.tree
        L = self.L
        WU, WV, sU, sV = {}, {}, {}, {}
        GU, GV = {}, {}
        for l in range(2, L + 1):
            lev = tr.levels[l]
            WU[l], WV[l], sU[l], sV[l], GU[l], GV[l] = [], [], [], [], [], []
            for i in range(lev.nb):
                ri = self.r[l][i]
                colsU = [self.K[l][(i, j)] for j in lev.inter[i]]
                colsV = [self.K[l][(j, i)].T for j in lev.inter[i]]
                if l > 2:
                    p = lev.parent[i]
                    colsU.append(self.PU[l][i] @ GU[l - 1][p])
                    colsV.append(self.PV[l][i] @ GV[l - 1][p])
                MU = np.hstack(colsU) if colsU else np.zeros((ri, 0))
                MV = np.hstack(colsV) if colsV else np.zeros((ri, 0))
                W, s = left_svd(MU)
                WU[l].append(W)
                sU[l].append(s)
                GU[l].append(W * s[None, :])
                W, s = left_svd(MV)
                WV[l].append(W)
                sV[l].append(s)
                GV[l].append(W * s[None, :])
        # ranks kept
        self.k_init = {}
        for l in range(2, L + 1):
            ks = []
            for i in range(tr.levels[l].nb):
                kU = int(np.sum(sU[l][i] > self.tau))
                kV = int(np.sum(sV[l][i] > self.tau))
                k = max(kU, kV)
                if self.rank_max > 0:
                    k = min(k, self.rank_max)
                ks.append(k)
            self.k_init[l] = ks
        # rotate and truncate every operator
        k = self.k_init
        for i in range(tr.levels[L].nb):
            self.U[i] = self.Q[i] @ WU[L][i][:, :k[L][i]]
            self.V[i] = self.Q[i] @ WV[L][i][:, :k[L][i]]
        for l in range(2, L + 1):
            newK = {}
            for (i, j), B in self.K[l].items():
                newK[(i, j)] = WU[l][i][:, :k[l][i]].T @ B @ WV[l][j][:, :k[l][j]]
            self.K[l] = newK
            if l > 2:
                lev = tr.levels[l]
                for i in range(lev.nb):
                    p = lev.parent[i]
                    self.PU[l][i] = WU[l][i][:, :k[l][i]].T @ self.PU[l][i] @ WU[l - 1][p][:, :k[l - 1][p]]
                    self.PV[l][i] = WV[l][i][:, :k[l][i]].T @ self.PV[l][i] @ WV[l - 1][p][:, :k[l - 1][p]]
        self.SU = {l: [sU[l][i][:k[l][i]].copy() for i in range(tr.levels[l].nb)] for l in range(2, L + 1)}
        self.SV = {l: [sV[l][i][:k[l][i]].copy() for i in range(tr.levels[l].nb)] for l in range(2, L + 1)}
        self.r_pre = self.r
        self.r = {l: list(k[l]) for l in k}
