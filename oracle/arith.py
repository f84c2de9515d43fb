"""Product recursion, block substitution and Cholesky factorisation
(Section 3 "Algebraic operations", Section 6 "Complexity of the LR
factorization", Section 7 for the Cholesky variant).

The factor L overwrites the lower triangle of an H^2-matrix stored with
``lower=True`` (row basis V, column basis W); every operation below is
expressed through the local low-rank update of ``update.addlr``, dense
operations on inadmissible leaves and products with sub-blocks.

chol(t) (recursion of Section 3 with R = L^*):
    leaf t:  N_tt <- lower Cholesky factor of N_tt (standard elimination).
    else:    chol(t1); solve X L_{t1 t1}^* = A_{t2 t1} (block substitution);
             A_{t2 t2} -= L_{t2 t1} L_{t2 t1}^* (product); chol(t2).

rsolve(c, (r, c)) solves X L_cc^* = Y on the block (r, c) in place
(substitution X R = Y of Section 3 with R = L^*):
    inadmissible leaf: dense triangular solve;
    admissible leaf Y = V_r S W_c^*: the exact solution is
        V_r S (L_cc^{-1} W_c)^*, applied as the low-rank update
        (V_r S)(L_cc^{-1} W_c - W_c)^*  because W_c is shared (reading);
    subdivided with c a leaf: every son (r', c);
    subdivided with sons c1, c2: for all r' in sons+(r) solve with c1, then
        for all r' update (r', c2) -= X(r', c1) L(c2, c1)^*, then for all r'
        solve with c2 (the order of the forward substitution in Section 6).

mm(t, s, r, alpha): Z(t, r) += alpha X(t, s) Y(r, s)^* with X, Y, Z blocks of
the same factor (Section 3; Section 6, Cases 1 and 2):
    Case 1, (t,s) and (r,s) subdivided:
        target subdivided: recursion over s' (outer), t', r' in sons+ (the
            order of the eight updates printed in Section 3); targets above
            the diagonal are skipped (lower storage);
        target inadmissible leaf: dense product added to N_tr;
        target admissible leaf: one temporary low-rank matrix per son pair
            (t', r') receives the recursion by truncated addition, then each
            is extended by zero and added with a low-rank update, in the
            order (t1,r1), (t1,r2), (t2,r1), (t2,r2).
    Case 2, a factor is a leaf (precedence in this order, a reading):
        (r,s) admissible: X~ = X(t,s) W_s by products with the sub-block,
            emit U = alpha X~ S_rs^*, V = V_r;
        (t,s) admissible: emit U = alpha V_t S_ts, V = Y(r,s) W_s;
        (t,s) inadmissible: emit U = alpha N_ts, V = Y(r,s) densely;
        (r,s) inadmissible: emit U = alpha X(t,s) densely, V = N_rs.
    An emission is added to the enclosing temporary (truncated addition),
    to N_tr for an inadmissible target, otherwise by addlr on (t, r).

tinv(c) overwrites the factor L with an approximation of L^{-1} (Remark
"Inversion" at the end of Section 6, specialised to A_12 = 0, so the Schur
complement is A_22 and C_12 = 0):
    leaf c:  N_cc <- (N_cc)^{-1} (dense lower triangular inverse).
    else:    tinv(c1); B_21 = A_21 A_11^{-1} (in place, rmul_tri);
             tinv(c2); C_21 = -C_22 B_21 (in place, lmul_tri, then negation).
    The products with the triangular diagonal blocks run in place by
    recursion over the sons of the triangular factor, with the product
    Z(t, r) += X(t, s) Y(s, r) of Section 3 (mm_n) for the off-diagonal part
    and, for an admissible leaf, the exact result applied as a low-rank update
    of the shared basis (as in rsolve; reading).

Truncated addition of low-rank matrices (the H-matrix rule recalled at the
end of Section 3): QR of both stacked factors, SVD of the small core, drop
singular values <= eps * ||core||_F (block_rel), <= eps * sigma_1
(const_rel), or only exact zeros (none).
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .h2 import H2Matrix, TruncParams, block_apply, block_dense
from .trees import ADM, INNER, NEAR
from .update import addlr


class NotSPDError(RuntimeError):
    def __init__(self, leaf: int):
        super().__init__(f"leaf block of cluster {leaf} is not positive definite")
        self.leaf = leaf


def _rk_truncate(A: np.ndarray, B: np.ndarray, tp: TruncParams):
    if A.shape[1] == 0:
        return A, B
    Qa, Ra = np.linalg.qr(A)
    Qb, Rb = np.linalg.qr(B)
    P, sig, QT = np.linalg.svd(Ra @ Rb.T)
    if tp.mode == "block_rel":
        tau = tp.eps * np.sqrt(np.sum(sig ** 2))
    elif tp.mode == "const_rel":
        tau = tp.eps * (sig[0] if len(sig) else 0.0)
    else:
        tau = 0.0
    r = int(np.count_nonzero(sig > tau))
    return Qa @ (P[:, :r] * sig[:r]), Qb @ QT[:r].T


class RkTemp:
    """Temporary low-rank matrix U V^* on the index pair (t, r)."""

    def __init__(self, ct, t: int, r: int):
        self.ct, self.t, self.r = ct, t, r
        self.U = np.zeros((int(ct.size[t]), 0))
        self.V = np.zeros((int(ct.size[r]), 0))

    def add(self, U2, V2, t2, r2, tp):
        ct = self.ct
        a = int(ct.offset[t2] - ct.offset[self.t])
        c = int(ct.offset[r2] - ct.offset[self.r])
        k2 = U2.shape[1]
        Ue = np.zeros((self.U.shape[0], k2)); Ue[a:a + U2.shape[0]] = U2
        Ve = np.zeros((self.V.shape[0], k2)); Ve[c:c + V2.shape[0]] = V2
        self.U, self.V = _rk_truncate(np.hstack([self.U, Ue]), np.hstack([self.V, Ve]), tp)


MAX_UPDATE_RANK = 32     # columns of one local update factor


def flush_temps(ct, bZ: int, t: int, r: int, temps, tp: TruncParams, add):
    """Add the temporaries of an admissible product target Z|_(t, r) (one per
    pair of sons, each placed at its rows of t and r) by local updates: one
    update each, in pair order; or, with tp.accumulate, consecutive
    temporaries concatenated while their total rank stays within
    MAX_UPDATE_RANK, one local update per group."""
    placed = []
    for tm in temps:
        U = np.zeros((int(ct.size[t]), tm.U.shape[1]))
        V = np.zeros((int(ct.size[r]), tm.V.shape[1]))
        a = int(ct.offset[tm.t] - ct.offset[t])
        c = int(ct.offset[tm.r] - ct.offset[r])
        U[a:a + tm.U.shape[0]] = tm.U
        V[c:c + tm.V.shape[0]] = tm.V
        placed.append((U, V))
    if not getattr(tp, "accumulate", False):
        for U, V in placed:
            add(bZ, U, V)
        return
    i = 0
    while i < len(placed):
        j, kt = i, 0
        while j < len(placed) and kt + placed[j][0].shape[1] <= MAX_UPDATE_RANK:
            kt += placed[j][0].shape[1]
            j += 1
        j = max(j, i + 1)
        add(bZ, np.hstack([u for u, _ in placed[i:j]]), np.hstack([v for _, v in placed[i:j]]))
        i = j


class _Chol:
    def __init__(self, L: H2Matrix, tp: TruncParams, stats: dict | None):
        assert L.lower
        self.L, self.tp = L, tp
        self.ct, self.bt = L.ct, L.bt
        self.stats = stats if stats is not None else {}

    def _count(self, key, inc=1):
        self.stats[key] = self.stats.get(key, 0) + inc

    # ---------------------------------------------------------------- update
    def _addlr(self, b, U, V):
        self._count("addlr_calls")
        # optional diagnostics: stats["margins"] (a list) receives the
        # threshold margins of every recompression (no effect on the result)
        if addlr(self.L, b, U, V, self.tp, self.stats.get("margins")):
            self._count("addlr_done")

    def _emit_block(self, t, r, U, V):
        bZ = self.bt.find(t, r)
        if self.bt.kind[bZ] == NEAR:
            self._count("near_add")
            self.L.N[bZ] = self.L.N[bZ] + U @ V.T
        else:
            self._addlr(bZ, U, V)

    # ---------------------------------------------------------------- product
    def mm(self, t, s, r, alpha, tmp=None):
        L, ct, bt = self.L, self.ct, self.bt
        bX, bY = bt.find(t, s), bt.find(r, s)
        if bt.kind[bX] == INNER and bt.kind[bY] == INNER:
            triples = [(t2, s2, r2) for s2 in ct.sons_plus(s)
                       for t2 in ct.sons_plus(t) for r2 in ct.sons_plus(r)]
            if tmp is not None:
                for (t2, s2, r2) in triples:
                    self.mm(t2, s2, r2, alpha, tmp)
                return
            bZ = bt.find(t, r)
            if bt.kind[bZ] == INNER:
                for (t2, s2, r2) in triples:
                    if ct.offset[t2] < ct.offset[r2]:
                        continue              # above the diagonal: not stored
                    self.mm(t2, s2, r2, alpha)
            elif bt.kind[bZ] == NEAR:
                self._count("near_dense_product")
                cache = {}
                P = block_dense(L, bX, cache) @ block_dense(L, bY, cache).T
                L.N[bZ] = L.N[bZ] + alpha * P
            else:
                self._count("temp_targets")
                pairs = [(t2, r2) for t2 in ct.sons_plus(t) for r2 in ct.sons_plus(r)]
                temps = {p: RkTemp(ct, p[0], p[1]) for p in pairs}
                for (t2, s2, r2) in triples:
                    self.mm(t2, s2, r2, alpha, temps[(t2, r2)])
                flush_temps(ct, bZ, t, r, [temps[p] for p in pairs], self.tp, self._addlr)
            return
        # Case 2: at least one factor is a leaf -> low-rank emission
        cache = {}
        if bt.kind[bY] == ADM:
            self._count("emit_R3")
            Xt = block_apply(L, bX, L.basis(1, s, cache), cache=cache)
            U = alpha * (Xt @ L.S[bY].T)
            V = L.basis(0, r, cache)
        elif bt.kind[bX] == ADM:
            self._count("emit_R4")
            U = alpha * (L.basis(0, t, cache) @ L.S[bX])
            V = block_apply(L, bY, L.basis(1, s, cache), cache=cache)
        elif bt.kind[bX] == NEAR:
            self._count("emit_R5")
            U = alpha * L.N[bX]
            V = block_dense(L, bY, cache)
        else:
            self._count("emit_R6")
            U = alpha * block_dense(L, bX, cache)
            V = L.N[bY]
        if tmp is not None:
            self._count("temp_add")
            tmp.add(U, V, t, r, self.tp)
        else:
            self._emit_block(t, r, U, V)

    # ----------------------------------------------------------- substitution
    def fsolve(self, c, w):
        """Solve L_cc y = w (rows of w in cluster order of c)."""
        L, ct, bt = self.L, self.ct, self.bt
        if ct.is_leaf(c):
            return sla.solve_triangular(L.N[bt.find(c, c)], w, lower=True)
        c1, c2 = ct.sons(c)
        n1 = int(ct.size[c1])
        y1 = self.fsolve(c1, w[:n1])
        y2 = self.fsolve(c2, w[n1:] - block_apply(L, bt.find(c2, c1), y1))
        return np.concatenate([y1, y2])

    def bsolve(self, c, w):
        """Solve L_cc^* y = w."""
        L, ct, bt = self.L, self.ct, self.bt
        if ct.is_leaf(c):
            return sla.solve_triangular(L.N[bt.find(c, c)], w, lower=True, trans="T")
        c1, c2 = ct.sons(c)
        n1 = int(ct.size[c1])
        y2 = self.bsolve(c2, w[n1:])
        y1 = self.bsolve(c1, w[:n1] - block_apply(L, bt.find(c2, c1), y2, trans=True))
        return np.concatenate([y1, y2])

    def rsolve(self, c, b):
        L, ct, bt = self.L, self.ct, self.bt
        r = int(bt.row[b])
        assert int(bt.col[b]) == c
        if bt.kind[b] == INNER:
            if ct.is_leaf(c):
                for r2 in ct.sons(r):
                    self.rsolve(c, bt.find(r2, c))
                return
            c1, c2 = ct.sons(c)
            rs = ct.sons_plus(r)
            for r2 in rs:
                self.rsolve(c1, bt.find(r2, c1))
            for r2 in rs:
                self.mm(r2, c1, c2, -1.0)
            for r2 in rs:
                self.rsolve(c2, bt.find(r2, c2))
        elif bt.kind[b] == NEAR:
            self._count("near_trsm")
            Lcc = L.N[bt.find(c, c)]
            L.N[b] = sla.solve_triangular(Lcc, L.N[b].T, lower=True).T
        else:
            self._count("adm_solve")
            cache = {}
            Wc = L.basis(1, c, cache)
            Wp = self.fsolve(c, Wc.copy())
            U = L.basis(0, r, cache) @ L.S[b]
            self._addlr(b, U, Wp - Wc)

    # ----------------------------------------------------- triangular inverse
    def trmv(self, c, w, trans=False):
        """L_cc w (L_cc^* w for trans) for the lower triangular diagonal block
        (c, c): dense lower triangle on a leaf, otherwise the sons' diagonal
        blocks and the block (c2, c1)."""
        L, ct, bt = self.L, self.ct, self.bt
        if ct.is_leaf(c):
            T = np.tril(L.N[bt.find(c, c)])
            return (T.T if trans else T) @ w
        c1, c2 = ct.sons(c)
        n1 = int(ct.size[c1])
        b = bt.find(c2, c1)
        if not trans:
            y1 = self.trmv(c1, w[:n1])
            y2 = self.trmv(c2, w[n1:]) + block_apply(L, b, w[:n1])
        else:
            y1 = self.trmv(c1, w[:n1], True) + block_apply(L, b, w[n1:], trans=True)
            y2 = self.trmv(c2, w[n1:], True)
        return np.concatenate([y1, y2])

    def mm_n(self, t, s, r, alpha, tmp=None):
        """Z(t, r) += alpha X(t, s) Y(s, r), X = block (t, s), Y = block
        (s, r) used as stored (not adjoint); all three lie strictly below the
        diagonal.  Same recursion as mm: Case 1 over s' (outer), t', r' with
        one temporary per son pair for an admissible leaf target; Case 2
        precedence (s,r) admissible, (t,s) admissible, (t,s) inadmissible,
        (s,r) inadmissible."""
        L, ct, bt = self.L, self.ct, self.bt
        bX, bY = bt.find(t, s), bt.find(s, r)
        if bt.kind[bX] == INNER and bt.kind[bY] == INNER:
            triples = [(t2, s2, r2) for s2 in ct.sons_plus(s)
                       for t2 in ct.sons_plus(t) for r2 in ct.sons_plus(r)]
            if tmp is not None:
                for (t2, s2, r2) in triples:
                    self.mm_n(t2, s2, r2, alpha, tmp)
                return
            bZ = bt.find(t, r)
            if bt.kind[bZ] == INNER:
                for (t2, s2, r2) in triples:
                    self.mm_n(t2, s2, r2, alpha)
            elif bt.kind[bZ] == NEAR:
                self._count("near_dense_product")
                cache = {}
                P = block_dense(L, bX, cache) @ block_dense(L, bY, cache)
                L.N[bZ] = L.N[bZ] + alpha * P
            else:
                self._count("temp_targets")
                pairs = [(t2, r2) for t2 in ct.sons_plus(t) for r2 in ct.sons_plus(r)]
                temps = {p: RkTemp(ct, p[0], p[1]) for p in pairs}
                for (t2, s2, r2) in triples:
                    self.mm_n(t2, s2, r2, alpha, temps[(t2, r2)])
                flush_temps(ct, bZ, t, r, [temps[p] for p in pairs], self.tp, self._addlr)
            return
        cache = {}
        if bt.kind[bY] == ADM:          # Y = V_s S W_r^*
            U = alpha * (block_apply(L, bX, L.basis(0, s, cache), cache=cache) @ L.S[bY])
            V = L.basis(1, r, cache)
        elif bt.kind[bX] == ADM:        # X = V_t S W_s^*
            U = alpha * (L.basis(0, t, cache) @ L.S[bX])
            V = block_apply(L, bY, L.basis(1, s, cache), trans=True, cache=cache)
        elif bt.kind[bX] == NEAR:
            U = alpha * L.N[bX]
            V = block_dense(L, bY, cache).T
        else:
            U = alpha * block_dense(L, bX, cache)
            V = L.N[bY].T
        if tmp is not None:
            self._count("temp_add")
            tmp.add(U, V, t, r, self.tp)
        else:
            self._emit_block(t, r, U, V)

    def rmul_tri(self, c, b):
        """X(r, c) <- X(r, c) L_cc in place on the block b = (r, c), with the
        diagonal block already inverted.  Sons c1, c2 of c split X into
        [X1 X2]: X1 <- X1 L_11 + X2 L_21 (recursion, then product with the
        untouched X2), X2 <- X2 L_22."""
        L, ct, bt = self.L, self.ct, self.bt
        r = int(bt.row[b])
        if bt.kind[b] == INNER:
            if ct.is_leaf(c):
                for r2 in ct.sons(r):
                    self.rmul_tri(c, bt.find(r2, c))
                return
            c1, c2 = ct.sons(c)
            rs = ct.sons_plus(r)
            for r2 in rs:
                self.rmul_tri(c1, bt.find(r2, c1))
            for r2 in rs:
                self.mm_n(r2, c2, c1, 1.0)
            for r2 in rs:
                self.rmul_tri(c2, bt.find(r2, c2))
        elif bt.kind[b] == NEAR:
            L.N[b] = L.N[b] @ np.tril(L.N[bt.find(c, c)])
        else:
            # V_r S W_c^* L_cc = V_r S (L_cc^* W_c)^*, added as the update
            # (V_r S)(L_cc^* W_c - W_c)^* (W_c is shared)
            cache = {}
            Wc = L.basis(1, c, cache)
            Wp = self.trmv(c, Wc, trans=True)
            self._addlr(b, L.basis(0, r, cache) @ L.S[b], Wp - Wc)

    def lmul_tri(self, c, b):
        """Y(c, r) <- L_cc Y(c, r) in place on the block b = (c, r).  Sons
        split Y into [Y1; Y2]: Y2 <- L_22 Y2 + L_21 Y1 (recursion, then
        product with the untouched Y1), Y1 <- L_11 Y1."""
        L, ct, bt = self.L, self.ct, self.bt
        r = int(bt.col[b])
        if bt.kind[b] == INNER:
            if ct.is_leaf(c):
                for r2 in ct.sons(r):
                    self.lmul_tri(c, bt.find(c, r2))
                return
            c1, c2 = ct.sons(c)
            rs = ct.sons_plus(r)
            for r2 in rs:
                self.lmul_tri(c2, bt.find(c2, r2))
            for r2 in rs:
                self.mm_n(c2, c1, r2, 1.0)
            for r2 in rs:
                self.lmul_tri(c1, bt.find(c1, r2))
        elif bt.kind[b] == NEAR:
            L.N[b] = np.tril(L.N[bt.find(c, c)]) @ L.N[b]
        else:
            # L_cc V_c S W_r^*, added as the update (L_cc V_c - V_c)(W_r S^*)^*
            cache = {}
            Vc = L.basis(0, c, cache)
            Vp = self.trmv(c, Vc)
            self._addlr(b, Vp - Vc, L.basis(1, r, cache) @ L.S[b].T)

    def neg(self, b):
        for l in self.bt.leaves_below(b):
            if self.bt.kind[l] == ADM:
                self.L.S[l] = -self.L.S[l]
            else:
                self.L.N[l] = -self.L.N[l]

    def tinv(self, c):
        """Remark "Inversion" with A_12 = 0: the Schur complement is A_22, so
        C_22 = A_22^{-1}, C_12 = 0, C_11 = A_11^{-1} and
        C_21 = -C_22 (A_21 A_11^{-1}); both products overwrite the block
        (c2, c1) in place."""
        L, ct, bt = self.L, self.ct, self.bt
        if ct.is_leaf(c):
            b = bt.find(c, c)
            self._count("leaf_trtri")
            L.N[b] = sla.solve_triangular(np.tril(L.N[b]), np.eye(int(ct.size[c])), lower=True)
            return
        c1, c2 = ct.sons(c)
        b = bt.find(c2, c1)
        self.tinv(c1)
        self.rmul_tri(c1, b)
        self.tinv(c2)
        self.lmul_tri(c2, b)
        self.neg(b)

    def chol(self, t):
        L, ct, bt = self.L, self.ct, self.bt
        if ct.is_leaf(t):
            b = bt.find(t, t)
            self._count("leaf_potrf")
            try:
                L.N[b] = sla.cholesky(L.N[b], lower=True)
            except np.linalg.LinAlgError:
                raise NotSPDError(t) from None
            return
        t1, t2 = ct.sons(t)
        self.chol(t1)
        self.rsolve(t1, bt.find(t2, t1))
        self.mm(t2, t1, t2, -1.0)
        self.chol(t2)


def cholesky(A: H2Matrix, tp: TruncParams, stats: dict | None = None) -> H2Matrix:
    """Approximate Cholesky factor L ~ A (A stored with lower=True).  A is
    overwritten in place and returned."""
    _Chol(A, tp, stats).chol(0)
    return A


def tri_invert(L: H2Matrix, tp: TruncParams, stats: dict | None = None) -> H2Matrix:
    """Approximate inverse G ~ L^{-1} of a lower triangular factor, in place
    (same block tree and storage; diagonal leaves hold dense lower
    triangular inverses)."""
    _Chol(L, tp, stats).tinv(0)
    return L


def tri_apply(G: H2Matrix, w: np.ndarray, trans: bool = False) -> np.ndarray:
    """G w (or G^* w) for a lower triangular H^2-matrix, cluster order, by
    the plain definition: sum over the stored leaves."""
    return block_apply(G, 0, np.asarray(w, dtype=np.float64), trans=trans)


def precond_apply_inverse(G: H2Matrix, r: np.ndarray) -> np.ndarray:
    """z = G^* G r with G ~ L^{-1}, r and z in original index order."""
    perm = G.ct.perm
    rc = np.asarray(r, dtype=np.float64)[perm]
    z = tri_apply(G, tri_apply(G, rc), trans=True)
    out = np.empty_like(z)
    out[perm] = z
    return out


def forward_solve(L: H2Matrix, w: np.ndarray) -> np.ndarray:
    """L y = w, both in cluster order (vector substitution of Section 3)."""
    return _Chol(L, TruncParams(), None).fsolve(0, np.asarray(w, dtype=np.float64))


def backward_solve(L: H2Matrix, w: np.ndarray) -> np.ndarray:
    """L^* y = w, both in cluster order."""
    return _Chol(L, TruncParams(), None).bsolve(0, np.asarray(w, dtype=np.float64))


def precond_apply(L: H2Matrix, r: np.ndarray) -> np.ndarray:
    """z = (L L^*)^{-1} r with r, z in original index order."""
    perm = L.ct.perm
    rc = np.asarray(r, dtype=np.float64)[perm]
    z = backward_solve(L, forward_solve(L, rc))
    out = np.empty_like(z)
    out[perm] = z
    return out
