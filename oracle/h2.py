"""H^2-matrix state (Section 2, Def. "Cluster basis" with eq. (nested),
Def. "H^2-matrix" with eq. (vsw)) and its plain evaluation.

A matrix is stored by

* row cluster basis V: leaf matrices V_t (#t x k_t) and transfer matrices
  E_t (k_t x k_{father}) for every non-root cluster, so that
  V_father|_t = V_t E_t (eq. (nested));
* column cluster basis W with transfers E^W in the same way;
* coupling matrices S_b (k_t x k_s) for admissible leaves b = (t, s), so that
  G|_{t x s} = V_t S_b W_s^* (eq. (vsw));
* dense nearfield matrices N_b for inadmissible leaves;
* R-factors rho^V_t, rho^W_s of the (expanded) basis matrices, i.e. upper
  triangular/trapezoidal matrices with rho^* rho = V_t^* V_t.  They are the
  matrices R_{W,s} of Section 4 that the weight construction needs; here
  they are kept for every cluster and refreshed after each update.

All index arithmetic uses cluster order (``ct.perm``); the public helpers take
vectors in original order where stated.

A square matrix uses one cluster tree for rows and columns (Section 3).  A
lower triangular factor stores only the blocks on or below the diagonal
(``lower=True``).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .trees import ADM, NEAR, BlockTree, ClusterTree


@dataclass
class TruncParams:
    """Recompression accuracy.

    mode 'block_rel': every block entering a weight stack is scaled by the
        inverse of its Frobenius norm and singular values sigma_{r+1} <= eps
        are dropped (blockwise relative accuracy, Section 4 last paragraph and
        Section 7).
    mode 'const_rel': unit block scales, drop sigma_{r+1} <= eps * sigma_1.
    mode 'none': keep every numerically non-zero singular value (exact
        arithmetic up to rounding).
    In every mode a basis recompression also drops singular values at the
    rounding level, sigma <= max(m, n) * eps_mach * sigma_1 for an m x n
    matrix (the usual numerical rank): they are indistinguishable from zero
    and their singular vectors are not determined by the data.
    rank_cap: an update that would create a rank above this raises.
    level_factor: see level_scale (cluster-basis recompression only).
    accumulate: in products (hence Cholesky, LR, triangular inverse), add the
        temporaries of one admissible target by accumulated updates: the
        temporaries, in pair order, are concatenated into as few local
        updates as the update rank MAX_UPDATE_RANK allows (greedy) instead
        of one update each (a truncation strategy of the kind named at the
        end of Section 4; a reading).
    """
    eps: float = 1e-6
    mode: str = "block_rel"
    rank_cap: int = 64
    accumulate: bool = False
    level_factor: float = 1.0

    def level_scale(self, level: int, depth: int) -> float:
        """Variable-order weighting of the cluster-basis recompression (the
        level-dependent accuracy the last paragraph of Section 4 names, a
        reading): the threshold of a cluster at level l of a tree of depth p
        is multiplied by q^(p - l), q = level_factor in (0, 1], so that larger
        clusters are approximated more accurately (higher rank), as in a
        variable-order scheme.  q = 1: no change.  Repeated products (not a
        power function) so that the GPU path can form the same number."""
        s = 1.0
        for _ in range(int(depth) - int(level)):
            s *= self.level_factor
        return s

    def tau(self, sig: np.ndarray) -> float:
        if self.mode == "block_rel":
            return self.eps
        if self.mode == "const_rel":
            return self.eps * (sig[0] if len(sig) else 0.0)
        if self.mode == "none":
            return 0.0
        raise ValueError(self.mode)

    def rank(self, sig: np.ndarray, shape: tuple[int, int] | None = None, scale: float = 1.0) -> int:
        """r = min{ r : sigma_{r+1} <= tau } for descending sig, tau the
        mode's threshold times scale (the level scale of the cluster); with
        the matrix shape, tau is at least the rounding level
        max(m, n) * eps_mach * sigma_1."""
        if len(sig) == 0:
            return 0
        tau = self.tau(sig) * scale
        if shape is not None:
            tau = max(tau, max(shape) * np.finfo(np.float64).eps * sig[0])
        return int(np.count_nonzero(sig > tau))


class RankCapError(RuntimeError):
    pass


class H2Matrix:
    def __init__(self, ct: ClusterTree, bt: BlockTree, lower: bool = False):
        self.ct, self.bt, self.lower = ct, bt, lower
        leaves = [b for b in range(bt.nb) if bt.kind[b] != 0 and (not lower or bt.is_lower(b))]
        self.leaves = leaves
        self.adm = [b for b in leaves if bt.kind[b] == ADM]
        self.near = [b for b in leaves if bt.kind[b] == NEAR]
        self.row_blocks = [[] for _ in range(ct.nc)]
        self.col_blocks = [[] for _ in range(ct.nc)]
        for b in self.adm:
            self.row_blocks[int(bt.row[b])].append(b)
            self.col_blocks[int(bt.col[b])].append(b)
        nc = ct.nc
        z = lambda *s: np.zeros(s)
        # bases: index 0 = row basis V, 1 = column basis W
        self.k = [np.zeros(nc, np.int64), np.zeros(nc, np.int64)]
        self.leafbasis = [dict(), dict()]
        self.E = [dict(), dict()]
        self.rho = [dict(), dict()]
        for side in (0, 1):
            for t in range(nc):
                if ct.is_leaf(t):
                    self.leafbasis[side][t] = z(int(ct.size[t]), 0)
                self.E[side][t] = z(0, 0)
                self.rho[side][t] = z(0, 0)
        self.S = {b: z(0, 0) for b in self.adm}
        self.N = {b: z(int(ct.size[bt.row[b]]), int(ct.size[bt.col[b]])) for b in self.near}

    # ------------------------------------------------------------------ utils
    def copy(self) -> "H2Matrix":
        Z = H2Matrix.__new__(H2Matrix)
        Z.__dict__.update(self.__dict__)
        Z.k = [a.copy() for a in self.k]
        Z.leafbasis = [{t: v.copy() for t, v in d.items()} for d in self.leafbasis]
        Z.E = [{t: v.copy() for t, v in d.items()} for d in self.E]
        Z.rho = [{t: v.copy() for t, v in d.items()} for d in self.rho]
        Z.S = {b: v.copy() for b, v in self.S.items()}
        Z.N = {b: v.copy() for b, v in self.N.items()}
        return Z

    def basis(self, side: int, t: int, cache: dict | None = None) -> np.ndarray:
        """Expanded basis matrix (#t x k_t) through eq. (nested)."""
        if cache is not None and (side, t) in cache:
            return cache[(side, t)]
        ct = self.ct
        if ct.is_leaf(t):
            out = self.leafbasis[side][t]
        else:
            parts = [self.basis(side, s, cache) @ self.E[side][s] for s in ct.sons(t)]
            out = np.vstack(parts)
        if cache is not None:
            cache[(side, t)] = out
        return out

    def storage_values(self) -> int:
        """Number of stored floating point values (bases, transfers, couplings, nearfield)."""
        n = 0
        for side in (0, 1):
            n += sum(v.size for v in self.leafbasis[side].values())
            n += sum(v.size for v in self.E[side].values())
        n += sum(v.size for v in self.S.values()) + sum(v.size for v in self.N.values())
        return n


def from_csr(A: sp.spmatrix, ct: ClusterTree, bt: BlockTree, lower: bool = False) -> H2Matrix:
    """H^2 representation of a sparse matrix whose admissible blocks vanish:
    all ranks are 0 and every inadmissible leaf holds its dense block.
    Raises ValueError if an admissible block holds a non-zero."""
    Ap = sp.csr_matrix(A)[ct.perm][:, ct.perm].tocsr()
    Z = H2Matrix(ct, bt, lower)
    blk = np.full(ct.n, -1, np.int64)
    leaves = [t for t in range(ct.nc) if ct.is_leaf(t)]
    for t in leaves:
        a, b = ct.rng(t)
        blk[a:b] = t
    coo = Ap.tocoo()
    r, c = coo.row, coo.col
    keep = (coo.data != 0)
    r, c, v = r[keep], c[keep], coo.data[keep]
    lt, ls = blk[r], blk[c]
    # every non-zero must fall into an inadmissible leaf (leaf x leaf pair)
    for (tt, ss) in set(zip(lt.tolist(), ls.tolist())):
        b = bt.index.get((tt, ss))
        if b is None or bt.kind[b] != NEAR:
            raise ValueError("non-zero entry in an admissible block")
    for b in Z.near:
        t, s = int(bt.row[b]), int(bt.col[b])
        a0, a1 = ct.rng(t)
        c0, c1 = ct.rng(s)
        Z.N[b] = Ap[a0:a1, c0:c1].toarray()
    return Z


def to_dense(Z: H2Matrix) -> np.ndarray:
    """Dense matrix in cluster order (plain definition, eq. (vsw))."""
    ct, bt = Z.ct, Z.bt
    D = np.zeros((ct.n, ct.n))
    cache = {}
    for b in Z.adm:
        t, s = int(bt.row[b]), int(bt.col[b])
        a0, a1 = ct.rng(t); c0, c1 = ct.rng(s)
        D[a0:a1, c0:c1] = Z.basis(0, t, cache) @ Z.S[b] @ Z.basis(1, s, cache).T
    for b in Z.near:
        t, s = int(bt.row[b]), int(bt.col[b])
        a0, a1 = ct.rng(t); c0, c1 = ct.rng(s)
        D[a0:a1, c0:c1] = Z.N[b]
    return D


def block_apply(Z: H2Matrix, b: int, x: np.ndarray, trans: bool = False,
                cache: dict | None = None) -> np.ndarray:
    """Z|_{t x s} x (or its transpose applied to x) for the block-tree node
    b = (t, s): sum over the stored leaves below b of V S W^* x (admissible)
    and N x (inadmissible), with densely expanded bases."""
    ct, bt = Z.ct, Z.bt
    t, s = int(bt.row[b]), int(bt.col[b])
    ta, _ = ct.rng(t)
    sa, _ = ct.rng(s)
    if cache is None:
        cache = {}
    x = np.asarray(x)
    if not trans:
        y = np.zeros((int(ct.size[t]),) + x.shape[1:])
    else:
        y = np.zeros((int(ct.size[s]),) + x.shape[1:])
    for l in bt.leaves_below(b):
        if Z.lower and not bt.is_lower(l):
            continue
        tl, sl = int(bt.row[l]), int(bt.col[l])
        r0, r1 = ct.rng(tl); c0, c1 = ct.rng(sl)
        r0 -= ta; r1 -= ta; c0 -= sa; c1 -= sa
        if bt.kind[l] == ADM:
            Vt, Ws = Z.basis(0, tl, cache), Z.basis(1, sl, cache)
            if not trans:
                y[r0:r1] += Vt @ (Z.S[l] @ (Ws.T @ x[c0:c1]))
            else:
                y[c0:c1] += Ws @ (Z.S[l].T @ (Vt.T @ x[r0:r1]))
        else:
            if not trans:
                y[r0:r1] += Z.N[l] @ x[c0:c1]
            else:
                y[c0:c1] += Z.N[l].T @ x[r0:r1]
    return y


def block_dense(Z: H2Matrix, b: int, cache: dict | None = None) -> np.ndarray:
    """Dense copy of the sub-block Z|_{t x s} of the block-tree node b."""
    ct, bt = Z.ct, Z.bt
    s = int(bt.col[b])
    return block_apply(Z, b, np.eye(int(ct.size[s])), cache=cache)


def matvec(Z: H2Matrix, x: np.ndarray, trans: bool = False) -> np.ndarray:
    """y = Z x (or Z^* x) with x, y in original index order."""
    ct = Z.ct
    xc = np.asarray(x)[ct.perm]
    yc = block_apply(Z, 0, xc, trans=trans)
    y = np.empty_like(yc)
    y[ct.perm] = yc
    return y
