"""Level-by-level IFMM elimination, compression, merge and solve (oracle; test infrastructure).

Paper passages followed:
  * Alg. 1 (overall algorithm): eliminate level L, L-1, ..., 2 updating the
    right-hand side, form the parent-level operators after each level, solve
    the dense system of y^(2), then substitute back down the tree.
  * Alg. 2 (elimination of level l): for each box i eliminate x~_i and z_i
    together; the fill-in between every pair of nodes of its neighbourhood is
    either added to an existing edge or, when the two boxes are
    well-separated and at least one side is a not-yet-eliminated x~,
    compressed and redirected.
  * Sec. 2.2, eqs. (P2P_kj), (P2P_jk): a well-separated fill-in is low rank.
  * Sec. 2.2, eqs. (U_j_recomp) to (V_prime): the new basis of box j comes from
    a recompression of the weighted old basis concatenated with the fill-in;
    r_j and t_j express the old basis in the new one.
  * Sec. 2.2, eqs. (K_kj_update), (K_qj_update), (K_jq_update),
    (U_parent_j_update), (V_parent_j_update) and Alg. 3: every edge of y_j and
    the transfers to the parent are rewritten in the new basis, and the fill
    is redirected through the M2L edge K.
  * Sec. 2.2, eqs. (y_merge), (y_merge_2), (U_merge), (V_merge), (K_merge):
    after a level the y of the children form x~ of the parent and the edges
    between them form the parent's near-field blocks.
  * Sec. 2.4, eq. (methods_SVD_rank_spectralnorm): rank rule against tau.

Readings (where the paper is silent or ambiguous):
  * Boxes of a level are taken in colour order (independent sets), Morton
    order inside a colour; F of box i lists x~_j of not-yet-eliminated
    neighbours, then y_h of eliminated neighbours (Morton order each), then y_i.
  * Pivoting: partial pivoting inside each pivot block [[S_ii, U_i], [V_i^T, 0]].
  * Aggregated compression: after eliminating box i, every not-yet-eliminated
    neighbour j with well-separated fill is recompressed once, from
    [U_j Sigma_U | all its well-separated fill blocks of this elimination]
    (and the same for V); this equals the paper's two-step route (truncated
    SVD of each fill, then recompression with U' Sigma') up to the order in
    which pairs are folded in. r_j = Uhat_j^T U_j and t_j = Vhat_j^T V_j, which
    equal Sigma_hat phi_j Sigma_U^-1 and Sigma_hat psi_j Sigma_V^-1 exactly.
  * mode="literal" follows the paper's pairwise route instead: unordered
    well-separated pairs of F one at a time (F order), a truncated SVD of
    each directed fill block, recompression of the bases with the compressed
    fill, the edge rewrite of Alg. 3 and the redirect, before the next pair.
    Both modes are exact as eps -> 0 and agree with each other to O(eps).
  * After each merge the parent bases [U_p Sigma_U] and [V_p Sigma_V] are
    recompressed at tau, so every pivot block starts with orthonormal bases
    and at most as many basis columns as x~ rows.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .extended import R2
from .h2 import H2
from .tree import Tree


def _svd_left(M: np.ndarray):
    """Left singular vectors and values of M (LAPACK); empty-safe."""
    m = M.shape[0]
    if m == 0 or M.shape[1] == 0:
        return np.zeros((m, 0)), np.zeros(0)
    W, s, _ = np.linalg.svd(M, full_matrices=False)
    return W, s


class LevelState:
    """The part of the graph of E that lives at level l while it is eliminated."""

    def __init__(self, l: int):
        self.l = l
        self.m: list[int] = []          # size of x~_i
        self.r: list[int] = []          # size of z_i and y_i
        self.S: dict = {}               # (i, j) -> x~_i row, x~_j column   (m_i x m_j)
        self.U: list = []               # x~_i row, z_i column              (m_i x r_i)
        self.V: list = []               # V_i, so that z_i row holds V_i^T  (m_i x r_i)
        self.SU: list = []
        self.SV: list = []
        self.K: dict = {}               # (i, j) -> y_i row, y_j column     (r_i x r_j)
        self.Kcols: dict = {}           # i -> set of j with an edge (i, j)
        self.Krows: dict = {}           # j -> set of i with an edge (i, j)
        self.XY: dict = {}              # (j, h) -> x~_j row, y_h column    (m_j x r_h)
        self.YX: dict = {}              # (h, j) -> y_h row, x~_j column    (r_h x m_j)
        self.PU: list | None = None     # y_i row, z_parent column          (r_i x r_p)
        self.PV: list | None = None     # z_parent row holds PV_i^T         (r_i x r_p)

    def k(self, i: int, j: int) -> np.ndarray:
        B = self.K.get((i, j))
        if B is None:
            B = np.zeros((self.r[i], self.r[j]))
            self.setk(i, j, B)
        return B

    def setk(self, i: int, j: int, B: np.ndarray) -> None:
        self.K[(i, j)] = B
        self.Kcols.setdefault(i, set()).add(j)
        self.Krows.setdefault(j, set()).add(i)

    def setK_all(self, K: dict) -> None:
        self.K, self.Kcols, self.Krows = {}, {}, {}
        for (i, j), B in K.items():
            self.setk(i, j, B.copy())


class Elim:
    """Stored factors of one elimination (Alg. 1 decouples elimination and substitution)."""
    __slots__ = ("i", "m", "r", "F", "lu", "piv", "W", "EFP")

    def __init__(self, i, m, r, F, lu, piv, W, EFP):
        self.i, self.m, self.r, self.F, self.lu, self.piv, self.W, self.EFP = i, m, r, F, lu, piv, W, EFP


class IFMM:
    """FP64 IFMM on a point cloud: build, factorize, solve, matvec (oracle)."""

    def __init__(self, points, kind, param, shift, depth, order, eps, sigma0=None,
                 rank_max=0, unit_roundoff=2.0 ** -53, class_shuffle_seed=None, mode="aggregated"):
        if mode not in ("aggregated", "literal"):
            raise ValueError("mode must be 'aggregated' or 'literal'")
        self.mode = mode
        self.tree = Tree(points, depth)
        self.h2 = H2(self.tree, kind, param, shift, order)
        self.r2 = R2(self.h2, eps, unit_roundoff=unit_roundoff, sigma0=sigma0, rank_max=rank_max)
        self.tau = self.r2.tau
        self.rank_max = rank_max
        self.class_shuffle_seed = class_shuffle_seed
        self.factored = False
        self.stats = {"rank_history": []}

    # ------------------------------------------------------------ public
    def matvec(self, x):
        return self.h2.matvec(x)

    def factorize(self):
        tr, r2 = self.tree, self.r2
        L = tr.L
        self.elims: dict[int, list[Elim]] = {}
        self.final_r: dict[int, list[int]] = {}
        st = self._leaf_state()
        for l in range(L, 1, -1):
            self._eliminate_level(st)
            self.final_r[l] = list(st.r)
            if l > 2:
                st = self._merge(st)
            else:
                self._top(st)
        self.factored = True

    def solve(self, b):
        if not self.factored:
            raise RuntimeError("factorize first")
        tr = self.tree
        b = np.asarray(b, dtype=np.float64)
        vec = b.ndim == 1
        B = (b[:, None] if vec else b)[tr.perm]
        X = self._solve_tree(B)
        out = np.empty_like(X)
        out[tr.perm] = X
        return out[:, 0] if vec else out

    # ------------------------------------------------------------ set-up
    def _leaf_state(self) -> LevelState:
        tr, r2 = self.tree, self.r2
        L = tr.L
        lev = tr.levels[L]
        st = LevelState(L)
        for i in range(lev.nb):
            s = tr.leaf_points(i)
            st.m.append(s.stop - s.start)
            st.r.append(r2.r[L][i])
            st.U.append(r2.U[i].copy())
            st.V.append(r2.V[i].copy())
            st.SU.append(r2.SU[L][i].copy())
            st.SV.append(r2.SV[L][i].copy())
        st.S = {key: B.copy() for key, B in r2.S.items()}
        st.setK_all(r2.K[L])
        if L > 2:
            st.PU = [B.copy() for B in r2.PU[L]]
            st.PV = [B.copy() for B in r2.PV[L]]
        return st

    # ------------------------------------------------------- elimination
    def _eliminate_level(self, st: LevelState) -> None:
        tr = self.tree
        l = st.l
        lev = tr.levels[l]
        eliminated = np.zeros(lev.nb, dtype=bool)
        recs = []
        order = tr.elimination_order(l)
        if self.class_shuffle_seed is not None:
            # any order inside a colour class gives the same result (independent sets)
            g = np.random.Generator(np.random.PCG64(self.class_shuffle_seed + l))
            col = lev.colour
            out = []
            for c in sorted(set(int(col[i]) for i in order)):
                members = [i for i in order if int(col[i]) == c]
                out.extend(g.permutation(members).tolist())
            order = out
        for i in order:
            recs.append(self._eliminate_box(st, i, eliminated))
            eliminated[i] = True
        self.elims[l] = recs

    def _eliminate_box(self, st: LevelState, i: int, eliminated) -> Elim:
        tr = self.tree
        l = st.l
        lev = tr.levels[l]
        m_i, r_i = st.m[i], st.r[i]
        p = m_i + r_i
        nb = [j for j in lev.nbrs[i] if j != i]
        F = [("x", j) for j in nb if not eliminated[j]] + \
            [("y", h) for h in nb if eliminated[h]] + [("y", i)]
        dims = [st.m[b] if t == "x" else st.r[b] for t, b in F]
        offs = np.concatenate([[0], np.cumsum(dims)]).astype(int)
        f = int(offs[-1])

        # pivot block E_PP = [[S_ii, U_i], [V_i^T, 0]]
        EPP = np.zeros((p, p))
        EPP[:m_i, :m_i] = st.S[(i, i)]
        EPP[:m_i, m_i:] = st.U[i]
        EPP[m_i:, :m_i] = st.V[i].T
        # couplings E_PF (rows x~_i, z_i) and E_FP (columns x~_i, z_i)
        EPF = np.zeros((p, f))
        EFP = np.zeros((f, p))
        for a, (t, b) in enumerate(F):
            sl = slice(offs[a], offs[a + 1])
            if t == "x":
                EPF[:m_i, sl] = st.S[(i, b)]
                EFP[sl, :m_i] = st.S[(b, i)]
            elif b != i:
                EPF[:m_i, sl] = st.XY.get((i, b), np.zeros((m_i, st.r[b])))
                EFP[sl, :m_i] = st.YX.get((b, i), np.zeros((st.r[b], m_i)))
            else:
                # z_i row has -I at y_i; y_i row has -I at z_i
                EPF[m_i:, sl] = -np.eye(r_i)
                EFP[sl, m_i:] = -np.eye(r_i)
        if p > 0:
            lu, piv = sla.lu_factor(EPP, check_finite=True)
            W = sla.lu_solve((lu, piv), EPF)
        else:
            lu, piv, W = EPP, np.zeros(0, dtype=np.int32), np.zeros((0, f))
        D = -EFP @ W                                    # Schur complement fill, F x F
        rec = Elim(i, m_i, r_i, list(zip(F, dims)), lu, piv, W, EFP)

        def blk(a, c):
            return D[offs[a]:offs[a + 1], offs[c]:offs[c + 1]]

        def box(node):
            return node[1]

        # classify every ordered pair of F
        ws_pairs = []
        for a, na in enumerate(F):
            for c, nc in enumerate(F):
                ta, ba = na
                tc, bc = nc
                near = tr.adjacent(l, ba, bc)
                if ta == "y" and tc == "y":
                    st.setk(ba, bc, st.k(ba, bc) + blk(a, c))
                elif near:
                    if ta == "x" and tc == "x":
                        st.S[(ba, bc)] = st.S[(ba, bc)] + blk(a, c)
                    elif ta == "x":
                        st.XY[(ba, bc)] = st.XY.get((ba, bc), np.zeros((st.m[ba], st.r[bc]))) + blk(a, c)
                    else:
                        st.YX[(ba, bc)] = st.YX.get((ba, bc), np.zeros((st.r[ba], st.m[bc]))) + blk(a, c)
                else:
                    ws_pairs.append((a, c))

        if self.mode == "literal":
            self._compress_pairwise(st, F, ws_pairs, blk)
            return rec
        # aggregated recompression of every not-yet-eliminated neighbour with ws fill
        new_basis = {}
        for a, (ta, j) in enumerate(F):
            if ta != "x":
                continue
            cols = [blk(a, c) for (a2, c) in ws_pairs if a2 == a]
            rows = [blk(c, a).T for (c, a2) in ws_pairs if a2 == a]
            if not cols and not rows:
                continue
            MU = np.hstack([st.U[j] * st.SU[j][None, :]] + cols)
            MV = np.hstack([st.V[j] * st.SV[j][None, :]] + rows)
            new_basis[j] = self._recompress(MU, MV, st.m[j])
        self._apply_basis_change(st, new_basis)
        # redirect the well-separated fill through K (eq. K_kj_update)
        for (a, c) in ws_pairs:
            ta, ba = F[a]
            tc, bc = F[c]
            B = blk(a, c)
            if ta == "x":
                B = new_basis[ba][0].T @ B
            if tc == "x":
                B = B @ new_basis[bc][2]
            self._redirect_add(st, ba, bc, B)
        return rec

    def _compress_pairwise(self, st: LevelState, F, ws_pairs, blk) -> None:
        """The paper's own route for the well-separated fill of one elimination (Alg. 2 and 3).

        Unordered pairs {a, c} of F (a before c in F's order) are taken one at a time. Each of the two
        directed fill blocks D(a, c), D(c, a) is approximated by its truncated SVD U' S' V'^T at tau (eqs.
        P2P_kj and P2P_jk; only the x~ side of an x~-y fill is compressed). Then the bases of the x~ boxes
        involved are recompressed from [U_j Sigma_U | U' S'] and [V_j Sigma_V | V' S'] (eqs. U_j_recomp
        and V_j_recomp), every edge of y_j is rewritten in the new bases (Alg. 3), and the compressed fill
        is added to K (eq. K_kj_update) in those new bases. The next pair sees the updated bases.
        """
        wset = set(ws_pairs)
        done = set()
        for (a, c) in ws_pairs:
            key = (min(a, c), max(a, c))
            if key in done:
                continue
            done.add(key)
            lo, hi = key
            addU, addV, pending = {}, {}, []
            for (p, q) in ((lo, hi), (hi, lo)):
                if (p, q) not in wset:
                    continue
                tp, bp = F[p]
                tq, bq = F[q]
                Uq, sq, Vq = self._truncated_svd(blk(p, q))
                if sq.shape[0] == 0:
                    continue
                if tp == "x":
                    addU.setdefault(bp, []).append(Uq * sq[None, :])
                if tq == "x":
                    addV.setdefault(bq, []).append(Vq * sq[None, :])
                pending.append((tp, bp, tq, bq, Uq, sq, Vq))
            if not pending:
                continue
            new_basis = {}
            for j in sorted(set(addU) | set(addV)):
                MU = np.hstack([st.U[j] * st.SU[j][None, :]] + addU.get(j, []))
                MV = np.hstack([st.V[j] * st.SV[j][None, :]] + addV.get(j, []))
                new_basis[j] = self._recompress_full(MU, MV, st.m[j])
            self._apply_basis_change(st, new_basis)
            for (tp, bp, tq, bq, Uq, sq, Vq) in pending:
                left = st.U[bp].T @ Uq if tp == "x" else Uq
                right = Vq.T @ st.V[bq] if tq == "x" else Vq.T
                self._redirect_add(st, bp, bq, (left * sq[None, :]) @ right)

    def _truncated_svd(self, B: np.ndarray):
        """U', S', V' of B keeping the singular values strictly above tau (eq. methods_SVD_rank_spectralnorm)."""
        if B.size == 0:
            return np.zeros((B.shape[0], 0)), np.zeros(0), np.zeros((B.shape[1], 0))
        U, s, Vt = np.linalg.svd(B, full_matrices=False)
        k = int(np.sum(s > self.tau))
        return U[:, :k], s[:k], Vt[:k].T

    def _recompress_full(self, MU, MV, m_j):
        """As _recompress, with complete left singular bases so that a side that resolves fewer directions
        than the common rank is completed by orthonormal vectors of weight zero."""
        def full(M):
            if M.shape[0] == 0:
                return np.zeros((0, 0)), np.zeros(0)
            W, s, _ = np.linalg.svd(M, full_matrices=True)
            sp = np.zeros(M.shape[0])
            sp[:s.shape[0]] = s[:M.shape[0]]
            return W, sp
        Uh, sU = full(MU)
        Vh, sV = full(MV)
        k = min(max(int(np.sum(sU > self.tau)), int(np.sum(sV > self.tau))), m_j)
        if self.rank_max > 0:
            k = min(k, self.rank_max)
        return Uh[:, :k], sU[:k].copy(), Vh[:, :k], sV[:k].copy()

    def _redirect_add(self, st: LevelState, a: int, c: int, B: np.ndarray) -> None:
        """K(a, c) += compressed fill, eqs. (K_kj_update) and Alg. 3."""
        st.setk(a, c, st.k(a, c) + B)

    def _recompress(self, MU, MV, m_j):
        """Truncated SVD of the weighted bases: (Uhat, sU, Vhat, sV), common rank k."""
        Uh, sU = _svd_left(MU)
        Vh, sV = _svd_left(MV)
        kU = int(np.sum(sU > self.tau))
        kV = int(np.sum(sV > self.tau))
        k = min(max(kU, kV), m_j)
        if self.rank_max > 0:
            k = min(k, self.rank_max)
        sUp = np.zeros(k)
        sVp = np.zeros(k)
        sUp[:min(k, sU.shape[0])] = sU[:k]
        sVp[:min(k, sV.shape[0])] = sV[:k]
        return Uh[:, :k], sUp, Vh[:, :k], sVp

    def _apply_basis_change(self, st: LevelState, new_basis: dict) -> None:
        """Rewrite every edge of y_j, z_j in the new basis (eqs. K_qj_update ... V_parent_j_update)."""
        if not new_basis:
            return
        rt = {}
        for j, (Uh, sU, Vh, sV) in new_basis.items():
            rt[j] = (Uh.T @ st.U[j], Vh.T @ st.V[j])     # r_j, t_j
        touched = set()
        for j in rt:
            for c in st.Kcols.get(j, ()):
                touched.add((j, c))
            for a in st.Krows.get(j, ()):
                touched.add((a, j))
        for (a, c) in touched:
            B = st.K[(a, c)]
            if a in rt:
                B = rt[a][0] @ B
            if c in rt:
                B = B @ rt[c][1].T
            st.K[(a, c)] = B
        for j, (Uh, sU, Vh, sV) in new_basis.items():
            if st.PU is not None:
                st.PU[j] = rt[j][0] @ st.PU[j]
                st.PV[j] = rt[j][1] @ st.PV[j]
            st.U[j], st.SU[j], st.V[j], st.SV[j] = Uh, sU, Vh, sV
            st.r[j] = Uh.shape[1]

    # ------------------------------------------------------------- merge
    def _merge(self, st: LevelState) -> LevelState:
        """Children's y become the parent's x~ (eqs. y_merge ... K_merge), then recompress bases."""
        tr, r2 = self.tree, self.r2
        l = st.l
        lp = l - 1
        levp = tr.levels[lp]
        nt = LevelState(lp)
        offs = {}
        for p in range(levp.nb):
            cs = levp.children[p]
            o = 0
            for c in cs:
                offs[c] = (o, o + st.r[c])
                o += st.r[c]
            nt.m.append(o)
            nt.r.append(r2.r[lp][p])
            nt.U.append(np.vstack([st.PU[c] for c in cs]) if cs else np.zeros((0, r2.r[lp][p])))
            nt.V.append(np.vstack([st.PV[c] for c in cs]) if cs else np.zeros((0, r2.r[lp][p])))
            nt.SU.append(r2.SU[lp][p].copy())
            nt.SV.append(r2.SV[lp][p].copy())
        for p in range(levp.nb):
            for q in levp.nbrs[p]:
                B = np.zeros((nt.m[p], nt.m[q]))
                for c in levp.children[p]:
                    for c2 in levp.children[q]:
                        if (c, c2) in st.K:
                            oc, oc2 = offs[c], offs[c2]
                            B[oc[0]:oc[1], oc2[0]:oc2[1]] = st.K[(c, c2)]
                nt.S[(p, q)] = B
        nt.setK_all(r2.K[lp])
        if lp > 2:
            nt.PU = [B.copy() for B in r2.PU[lp]]
            nt.PV = [B.copy() for B in r2.PV[lp]]
        self.merge_offsets = getattr(self, "merge_offsets", {})
        self.merge_offsets[lp] = offs
        # recompression of the merged bases
        nbasis = {}
        for p in range(levp.nb):
            nbasis[p] = self._recompress(nt.U[p] * nt.SU[p][None, :], nt.V[p] * nt.SV[p][None, :], nt.m[p])
        self._apply_basis_change(nt, nbasis)
        return nt

    def _top(self, st: LevelState) -> None:
        """Dense system of y^(2) (Alg. 1, solve for y^(2))."""
        lev = self.tree.levels[st.l]
        rs = st.r
        offs = np.concatenate([[0], np.cumsum(rs)]).astype(int)
        n = int(offs[-1])
        D = np.zeros((n, n))
        for i in range(lev.nb):
            for j in range(lev.nb):
                if (i, j) in st.K:
                    D[offs[i]:offs[i + 1], offs[j]:offs[j + 1]] = st.K[(i, j)]
        self.top_offs = offs
        self.top_D = D
        if n > 0:
            self.top_lu = sla.lu_factor(D, check_finite=True)

    # ------------------------------------------------------------- solve
    def _solve_tree(self, B: np.ndarray) -> np.ndarray:
        tr = self.tree
        L = tr.L
        k = B.shape[1]
        bx = {L: [B[tr.leaf_points(i)].copy() for i in range(tr.levels[L].nb)]}
        by = {}
        cP = {}
        for l in range(L, 1, -1):
            lev = tr.levels[l]
            by[l] = [np.zeros((self.final_r[l][i], k)) for i in range(lev.nb)]
            cl = []
            for e in self.elims[l]:
                bP = np.vstack([bx[l][e.i], np.zeros((e.r, k))])
                c = sla.lu_solve((e.lu, e.piv), bP) if e.m + e.r > 0 else bP
                cl.append(c)
                upd = e.EFP @ c
                o = 0
                for (t, b), dim in e.F:
                    if t == "x":
                        bx[l][b] -= upd[o:o + dim]
                    else:
                        by[l][b] -= upd[o:o + dim]
                    o += dim
            cP[l] = cl
            if l > 2:
                levp = tr.levels[l - 1]
                bx[l - 1] = [np.vstack([by[l][c] for c in levp.children[p]]) if levp.children[p]
                             else np.zeros((0, k)) for p in range(levp.nb)]
        # top
        lev2 = tr.levels[2]
        rhs = np.vstack(by[2]) if lev2.nb else np.zeros((0, k))
        y2 = sla.lu_solve(self.top_lu, rhs) if rhs.shape[0] > 0 else rhs
        sy = {2: [y2[self.top_offs[i]:self.top_offs[i + 1]] for i in range(lev2.nb)]}
        sx = {}
        for l in range(2, L + 1):
            lev = tr.levels[l]
            sx[l] = [None] * lev.nb
            for e, c in zip(reversed(self.elims[l]), reversed(cP[l])):
                parts = []
                for (t, b), dim in e.F:
                    parts.append(sx[l][b] if t == "x" else sy[l][b])
                xF = np.vstack(parts) if parts else np.zeros((0, k))
                xP = c - e.W @ xF
                sx[l][e.i] = xP[:e.m]
            if l < L:
                levc = tr.levels[l + 1]
                offs = self.merge_offsets[l]
                sy[l + 1] = [None] * levc.nb
                for p in range(lev.nb):
                    for cidx in lev.children[p]:
                        o0, o1 = offs[cidx]
                        sy[l + 1][cidx] = sx[l][p][o0:o1]
        X = np.zeros((tr.n, k))
        for i in range(tr.levels[L].nb):
            X[tr.leaf_points(i)] = sx[L][i]
        return X
