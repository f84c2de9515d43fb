"""H^2 product of three matrices and the LR factorisation (Section 3
"Algebraic operations"; Section 6, Cases 1 and 2).  Test infrastructure:
plain NumPy/SciPy in FP64, not part of the product path.

product(Z, alpha, X, Y): Z|_{t x r} += alpha X|_{t x s} Y|_{s x r} for three
H^2-matrices on one block tree (full storage), by the recursion of
Section 3 started at the root triple:
    Case 1, (t,s) and (s,r) subdivided:
        target subdivided: recursion over s' (outer), t', r' in sons+
            (the order of the eight products printed in Section 3);
        target inadmissible leaf: dense product added to N_tr;
        target admissible leaf: one temporary low-rank matrix per son pair
            (t', r') receives the recursion by truncated addition, then each
            is extended by zero and added by a local low-rank update, in the
            order (t1,r1), (t1,r2), (t2,r1), (t2,r2).
    Case 2, a factor is a leaf (precedence in this order, a reading):
        (s,r) admissible, Y|_{s x r} = V^Y_s S W^Y_r^*:
            U = alpha (X|_{t x s} V^Y_s) S, V = W^Y_r;
        (t,s) admissible, X|_{t x s} = V^X_t S W^X_s^*:
            U = alpha V^X_t S, V = (Y|_{s x r})^* W^X_s;
        (t,s) inadmissible: U = alpha N^X_ts, V = (Y|_{s x r})^* densely;
        (s,r) inadmissible: U = alpha X|_{t x s} densely, V = (N^Y_sr)^*.
    An emission goes to the enclosing temporary (truncated addition), to
    N_tr for an inadmissible target, otherwise to the local update on (t, r).

lr(A): A = L R in place with L unit lower triangular (strict lower part
stored) and R upper triangular, no pivoting (Section 3):
    leaf t:  standard Gaussian elimination of the dense block;
    else:    lr(t1); L_11 R_12 = A_12 (lsolve); L_21 R_11 = A_21 (rsolve);
             A_22 -= L_21 R_12 (product); lr(t2).
lsolve(c, (c, r)): L_cc X = Y in place (block forward substitution):
    inadmissible leaf: dense unit lower triangular solve;
    admissible leaf Y = V_c S W_r^*: the exact solution L_cc^{-1} V_c S W_r^*
        is applied as the update (L_cc^{-1} V_c - V_c)(W_r S^*)^* because
        V_c is shared (reading, as for the Cholesky substitution);
    subdivided with c a leaf: every son (c, r');
    subdivided with sons c1, c2: for all r' solve with c1, then for all r'
        update (c2, r') -= L(c2, c1) X(c1, r'), then for all r' solve with c2.
rsolve(c, (r, c)): X R_cc = Y in place, the mirror image:
    admissible leaf: update (V_r S)(R_cc^{-*} W_c - W_c)^*;
    subdivided: solve with c1, update (r', c2) -= X(r', c1) R(c1, c2), solve
        with c2.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .arith import RkTemp, flush_temps
from .h2 import H2Matrix, TruncParams, block_apply, block_dense, to_dense
from .trees import ADM, INNER, NEAR
from .update import addlr


class ZeroPivotError(RuntimeError):
    def __init__(self, leaf: int):
        super().__init__(f"zero pivot in the leaf block of cluster {leaf}")
        self.leaf = leaf


class _Prod:
    """Z += alpha X Y on sub-blocks; X, Y, Z may be the same matrix (the
    Schur product of the LR factorisation) or three different ones."""

    def __init__(self, Z: H2Matrix, X: H2Matrix, Y: H2Matrix, tp: TruncParams, stats: dict):
        assert not Z.lower and not X.lower and not Y.lower
        assert X.bt is Z.bt and Y.bt is Z.bt
        self.Z, self.X, self.Y, self.tp, self.stats = Z, X, Y, tp, stats
        self.ct, self.bt = Z.ct, Z.bt

    def _count(self, key):
        self.stats[key] = self.stats.get(key, 0) + 1

    def _addlr(self, b, U, V):
        self._count("addlr_calls")
        if addlr(self.Z, b, U, V, self.tp, self.stats.get("margins")):
            self._count("addlr_done")

    def mm(self, t, s, r, alpha, tmp=None):
        X, Y, Z, ct, bt = self.X, self.Y, self.Z, self.ct, self.bt
        bX, bY = bt.find(t, s), bt.find(s, r)
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
                    self.mm(t2, s2, r2, alpha)
            elif bt.kind[bZ] == NEAR:
                self._count("near_dense_product")
                P = block_dense(X, bX, {}) @ block_dense(Y, bY, {})
                Z.N[bZ] = Z.N[bZ] + alpha * P
            else:
                self._count("temp_targets")
                pairs = [(t2, r2) for t2 in ct.sons_plus(t) for r2 in ct.sons_plus(r)]
                temps = {p: RkTemp(ct, p[0], p[1]) for p in pairs}
                for (t2, s2, r2) in triples:
                    self.mm(t2, s2, r2, alpha, temps[(t2, r2)])
                flush_temps(ct, bZ, t, r, [temps[p] for p in pairs], self.tp, self._addlr)
            return
        cx, cy = {}, {}
        if bt.kind[bY] == ADM:
            U = alpha * (block_apply(X, bX, Y.basis(0, s, cy), cache=cx) @ Y.S[bY])
            V = Y.basis(1, r, cy)
        elif bt.kind[bX] == ADM:
            U = alpha * (X.basis(0, t, cx) @ X.S[bX])
            V = block_apply(Y, bY, X.basis(1, s, cx), trans=True, cache=cy)
        elif bt.kind[bX] == NEAR:
            U = alpha * X.N[bX]
            V = block_dense(Y, bY, cy).T
        else:
            U = alpha * block_dense(X, bX, cx)
            V = Y.N[bY].T
        if tmp is not None:
            self._count("temp_add")
            tmp.add(U, V, t, r, self.tp)
            return
        bZ = bt.find(t, r)
        if bt.kind[bZ] == NEAR:
            self._count("near_add")
            Z.N[bZ] = Z.N[bZ] + U @ V.T
        else:
            self._addlr(bZ, U, V)


def product(Z: H2Matrix, alpha: float, X: H2Matrix, Y: H2Matrix, tp: TruncParams,
            stats: dict | None = None) -> H2Matrix:
    """Z += alpha X Y in place (all three full-storage matrices of one block
    tree, Z distinct from X and Y); returns Z."""
    assert Z is not X and Z is not Y
    _Prod(Z, X, Y, tp, stats if stats is not None else {}).mm(0, 0, 0, alpha)
    return Z


def _getrf_nopiv(A: np.ndarray, leaf: int) -> np.ndarray:
    """Gaussian elimination without pivoting: returns L - I + R packed in one
    array (L unit lower, R upper)."""
    A = np.array(A, dtype=np.float64)
    n = A.shape[0]
    for k in range(n):
        if A[k, k] == 0.0:
            raise ZeroPivotError(leaf)
        A[k + 1:, k] /= A[k, k]
        A[k + 1:, k + 1:] -= np.outer(A[k + 1:, k], A[k, k + 1:])
    return A


class _LR:
    def __init__(self, M: H2Matrix, tp: TruncParams, stats: dict):
        assert not M.lower
        self.M, self.tp, self.stats = M, tp, stats
        self.ct, self.bt = M.ct, M.bt
        self.prod = _Prod(M, M, M, tp, stats)

    def _addlr(self, b, U, V):
        self.prod._addlr(b, U, V)

    # vector solves with the factors of the diagonal block (c, c)
    def fsolve_unit(self, c, w):
        """L_cc y = w, L unit lower (cluster order of c)."""
        M, ct, bt = self.M, self.ct, self.bt
        if ct.is_leaf(c):
            return sla.solve_triangular(M.N[bt.find(c, c)], w, lower=True, unit_diagonal=True)
        c1, c2 = ct.sons(c)
        n1 = int(ct.size[c1])
        y1 = self.fsolve_unit(c1, w[:n1])
        y2 = self.fsolve_unit(c2, w[n1:] - block_apply(M, bt.find(c2, c1), y1))
        return np.concatenate([y1, y2])

    def bsolve_upper(self, c, w):
        """R_cc y = w, R upper."""
        M, ct, bt = self.M, self.ct, self.bt
        if ct.is_leaf(c):
            return sla.solve_triangular(M.N[bt.find(c, c)], w, lower=False)
        c1, c2 = ct.sons(c)
        n1 = int(ct.size[c1])
        y2 = self.bsolve_upper(c2, w[n1:])
        y1 = self.bsolve_upper(c1, w[:n1] - block_apply(M, bt.find(c1, c2), y2))
        return np.concatenate([y1, y2])

    def fsolve_upper_adj(self, c, w):
        """R_cc^* y = w (R^* lower)."""
        M, ct, bt = self.M, self.ct, self.bt
        if ct.is_leaf(c):
            return sla.solve_triangular(M.N[bt.find(c, c)], w, lower=False, trans="T")
        c1, c2 = ct.sons(c)
        n1 = int(ct.size[c1])
        y1 = self.fsolve_upper_adj(c1, w[:n1])
        y2 = self.fsolve_upper_adj(c2, w[n1:] - block_apply(M, bt.find(c1, c2), y1, trans=True))
        return np.concatenate([y1, y2])

    # block substitutions
    def lsolve(self, c, b):
        M, ct, bt = self.M, self.ct, self.bt
        r = int(bt.col[b])
        assert int(bt.row[b]) == c
        if bt.kind[b] == INNER:
            if ct.is_leaf(c):
                for r2 in ct.sons(r):
                    self.lsolve(c, bt.find(c, r2))
                return
            c1, c2 = ct.sons(c)
            rs = ct.sons_plus(r)
            for r2 in rs:
                self.lsolve(c1, bt.find(c1, r2))
            for r2 in rs:
                self.prod.mm(c2, c1, r2, -1.0)
            for r2 in rs:
                self.lsolve(c2, bt.find(c2, r2))
        elif bt.kind[b] == NEAR:
            M.N[b] = sla.solve_triangular(M.N[bt.find(c, c)], M.N[b], lower=True, unit_diagonal=True)
        else:
            cache = {}
            Vc = M.basis(0, c, cache)
            Vp = self.fsolve_unit(c, Vc.copy())
            self._addlr(b, Vp - Vc, M.basis(1, r, cache) @ M.S[b].T)

    def rsolve(self, c, b):
        M, ct, bt = self.M, self.ct, self.bt
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
                self.prod.mm(r2, c1, c2, -1.0)
            for r2 in rs:
                self.rsolve(c2, bt.find(r2, c2))
        elif bt.kind[b] == NEAR:
            Rcc = M.N[bt.find(c, c)]
            M.N[b] = sla.solve_triangular(Rcc, M.N[b].T, lower=False, trans="T").T
        else:
            cache = {}
            Wc = M.basis(1, c, cache)
            Wp = self.fsolve_upper_adj(c, Wc.copy())
            self._addlr(b, M.basis(0, r, cache) @ M.S[b], Wp - Wc)

    def lr(self, t):
        M, ct, bt = self.M, self.ct, self.bt
        if ct.is_leaf(t):
            b = bt.find(t, t)
            self.prod._count("leaf_getrf")
            M.N[b] = _getrf_nopiv(M.N[b], t)
            return
        t1, t2 = ct.sons(t)
        self.lr(t1)
        self.lsolve(t1, bt.find(t1, t2))
        self.rsolve(t1, bt.find(t2, t1))
        self.prod.mm(t2, t1, t2, -1.0)
        self.lr(t2)


def lr(A: H2Matrix, tp: TruncParams, stats: dict | None = None) -> H2Matrix:
    """LR factorisation of A (full storage) in place; returns A holding the
    strict lower part of L (unit diagonal implied) and R."""
    _LR(A, tp, stats if stats is not None else {}).lr(0)
    return A


def lr_solve(F: H2Matrix, r: np.ndarray) -> np.ndarray:
    """z = R^{-1} L^{-1} r for the factors held in F, r and z in original
    index order."""
    perm = F.ct.perm
    op = _LR(F, TruncParams(), {})
    rc = np.asarray(r, dtype=np.float64)[perm]
    z = op.bsolve_upper(0, op.fsolve_unit(0, rc))
    out = np.empty_like(z)
    out[perm] = z
    return out


def lr_dense(F: H2Matrix):
    """Dense L (unit lower) and R (upper) held in F, cluster order."""
    D = to_dense(F)
    return np.tril(D, -1) + np.eye(D.shape[0]), np.triu(D)
