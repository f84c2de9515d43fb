"""Local low-rank update Z|_{t0 x s0} <- Z|_{t0 x s0} + X Y^* of an H^2-matrix
(Section 4 "Recompression" for the global case, Section 5 "Local updates"
for a block b0 = (t0, s0) of the block tree).

The steps, in the paper's order and notation:

0. Exact extension (eq. (tildeZ_h2)): V~_t = [V_t  X|_t], W~_s = [W_s  Y|_s],
   S~_b = diag(S_b, I), extended transfers diag(E_t, I); at the subtree roots
   E~_{t0} = [E_{t0}; 0] (Section 5, transfer update), so the predecessors of
   t0 are not extended.  Blocks with only t in T_{t0} get S~_b = [S_b; 0],
   blocks with only s in T_{s0} get [S_b  0] (the three coupling rules of
   Section 5).
1. R-factors of the extended bases by the upward recursion the paper cites
   for R_{W,s} (Section 4): leaf R of [W_s Y|_s], inner R of
   [R_{s1} E~_{s1}; R_{s2} E~_{s2}].  Both row and column factors are
   needed (row weights use R_W, column weights use R_V).
2. Block scales omega_b (blockwise relative accuracy): omega_b = 1/||Z~|_b||_F
   = 1/||R_{V,t} S~_b R_{W,s}^*||_F (0 for a zero block); 1 in the other modes.
3. Weight matrices B~_t top-down (eq. (Qt_condensed) and the recursion that
   follows it): B~_t is the R-factor of the stack
   [omega_b R_{W,s} S~_b^* for s in row(t); B~_{t+} E~_t^*].  For a local
   update the weights of the predecessors of t0 are built first from the
   current matrix (all blocks, Section 5), then those of T_{t0}.
4. Nested recompression bottom-up (eq. (Qt_nested), (hatQt_condensed)):
   leaf SVD of V~_t B~_t^*, inner SVD of V^_t B~_t^* with
   V^_t = [R_{t1} E~_{t1}; R_{t2} E~_{t2}]; keep r_t = min{r : sigma_{r+1} <=
   tau} left singular vectors, split Q^_t into F_{t1}, F_{t2}; basis change
   R_t = Q_t^* V~_t = Q^_t^* V^_t.
5. Coupling conversion S_b <- R_t S~_b R_s^* (identity factor for the side
   outside the subtrees).
6. Bases: V_t <- Q_t in T_{t0}, E_{t'} <- F_{t'}, E_{t0} <- R_{t0} [E_{t0}; 0];
   same for columns.
7. Inadmissible leaves inside b0 receive X|_t Y|_s^* densely.

Readings where the paper is silent:

* Row and column bases are both recompressed from the same extended matrix
  Z~; the column basis comes from the same construction applied to the
  adjoint of the extended matrix (Section 4).
* The weights of the predecessors of t0 are recomputed from the current
  state on every call.
* The stored R-factors rho_t (needed for R_{W,s} outside the subtrees and for
  the block scales) are set to the identity on the recompressed subtrees
  (orthonormal Q_t) and recomputed bottom-up along the path from the father
  of t0 to the root, whose bases change through E_{t0}.
* An update whose factor X or Y has no columns or is identically zero leaves
  Z unchanged and is skipped.
"""

from __future__ import annotations

import numpy as np

from .h2 import H2Matrix, RankCapError, TruncParams


def qr_r(A: np.ndarray) -> np.ndarray:
    """R-factor (min(m,n) x n) of a thin QR decomposition."""
    m, n = A.shape
    if m == 0 or n == 0:
        return np.zeros((min(m, n), n))
    return np.linalg.qr(A, mode="r")


def svd_left(M: np.ndarray):
    """Left singular vectors and singular values (descending)."""
    m, n = M.shape
    if m == 0 or n == 0:
        return np.zeros((m, 0)), np.zeros(0)
    U, s, _ = np.linalg.svd(M, full_matrices=False)
    return U, s


def addlr(Z: H2Matrix, b0: int, X: np.ndarray, Y: np.ndarray, tp: TruncParams,
          margins: list | None = None) -> bool:
    """Apply Z|_{t0 x s0} += X Y^* with recompression; returns False if skipped.

    X (#t0 x k), Y (#s0 x k): rows in cluster order restricted to t0 / s0.
    ``margins`` (optional) receives, per recompressed cluster, the relative
    distance of the kept and the first dropped singular value from the
    threshold (block_rel mode), for near-threshold diagnostics."""
    ct, bt = Z.ct, Z.bt
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    kp = X.shape[1]
    assert Y.shape[1] == kp
    if kp == 0 or not np.any(X) or not np.any(Y):
        return False
    r0 = (int(bt.row[b0]), int(bt.col[b0]))
    assert X.shape[0] == ct.size[r0[0]] and Y.shape[0] == ct.size[r0[1]]
    F = (X, Y)
    sub = (ct.subtree(r0[0]), ct.subtree(r0[1]))
    insub = (set(sub[0]), set(sub[1]))
    base = (int(ct.offset[r0[0]]), int(ct.offset[r0[1]]))
    blocks = (Z.row_blocks, Z.col_blocks)

    def K(side, t):
        return int(Z.k[side][t]) + (kp if t in insub[side] else 0)

    def kpar(side, t):
        return int(Z.k[side][ct.parent[t]])

    def Eext(side, t):
        """Transfer of the extended basis (K_t x K_father)."""
        E = Z.E[side][t]
        if t not in insub[side]:
            return E
        if t == r0[side]:
            return np.vstack([E, np.zeros((kp, kpar(side, t)))])
        kt = int(Z.k[side][t])
        out = np.zeros((kt + kp, E.shape[1] + kp))
        out[:kt, :E.shape[1]] = E
        out[kt:, E.shape[1]:] = np.eye(kp)
        return out

    def Vext(side, t):
        a, b = ct.rng(t)
        a -= base[side]; b -= base[side]
        return np.hstack([Z.leafbasis[side][t], F[side][a:b]])

    def Sext(b):
        t, s = int(bt.row[b]), int(bt.col[b])
        S = Z.S[b]
        tin, sin = t in insub[0], s in insub[1]
        kt, ks = S.shape
        if tin and sin:
            out = np.zeros((kt + kp, ks + kp))
            out[:kt, :ks] = S
            out[kt:, ks:] = np.eye(kp)
            return out
        if tin:
            return np.vstack([S, np.zeros((kp, ks))])
        if sin:
            return np.hstack([S, np.zeros((kt, kp))])
        return S

    # -- step 1: R-factors of the extended bases, bottom-up
    rhox = ({}, {})
    for side in (0, 1):
        for t in reversed(sub[side]):
            if ct.is_leaf(t):
                rhox[side][t] = qr_r(Vext(side, t))
            else:
                t1, t2 = ct.sons(t)
                rhox[side][t] = qr_r(np.vstack([rhox[side][t1] @ Eext(side, t1),
                                                rhox[side][t2] @ Eext(side, t2)]))

    def rho(side, t):
        return rhox[side][t] if t in insub[side] else Z.rho[side][t]

    # -- step 2: block scales
    omega_cache = {}

    def omega(b):
        if tp.mode != "block_rel":
            return 1.0
        if b not in omega_cache:
            t, s = int(bt.row[b]), int(bt.col[b])
            nrm = np.linalg.norm(rho(0, t) @ Sext(b) @ rho(1, s).T)
            omega_cache[b] = 1.0 / nrm if nrm > 0 else 0.0
        return omega_cache[b]

    # -- step 3: weights, first along pred(t0) \ {t0}, then through T_{t0}
    Bw = ({}, {})
    for side in (0, 1):
        path = ct.path_to(r0[side])[:-1]
        order = path + sub[side]
        for t in order:
            Kt = K(side, t)
            parts = []
            for b in blocks[side][t]:
                C = Sext(b) if side == 0 else Sext(b).T      # K_t x K_other
                other = int(bt.col[b]) if side == 0 else int(bt.row[b])
                parts.append(omega(b) * (rho(1 - side, other) @ C.T))
            if ct.parent[t] >= 0:
                parts.append(Bw[side][int(ct.parent[t])] @ Eext(side, t).T)
            Bw[side][t] = qr_r(np.vstack(parts)) if parts else np.zeros((0, Kt))

    # -- step 4: recompression, bottom-up
    R = ({}, {})
    newk = ({}, {})
    newleaf = ({}, {})
    newE = ({}, {})
    for side in (0, 1):
        for t in reversed(sub[side]):
            if ct.is_leaf(t):
                Vt = Vext(side, t)
            else:
                t1, t2 = ct.sons(t)
                Vt = np.vstack([R[side][t1] @ Eext(side, t1), R[side][t2] @ Eext(side, t2)])
            M = Vt @ Bw[side][t].T
            U, sig = svd_left(M)
            scale = tp.level_scale(ct.level[t], ct.depth) if getattr(tp, "level_factor", 1.0) != 1.0 else 1.0
            r = tp.rank(sig, M.shape, scale)
            if margins is not None and len(sig) and tp.mode == "block_rel" and tp.eps > 0:
                et = tp.eps * scale
                lo = sig[r - 1] / et - 1.0 if r > 0 else np.inf
                hi = 1.0 - sig[r] / et if r < len(sig) else np.inf
                margins.append(min(lo, hi))
            if r > tp.rank_cap:
                raise RankCapError(f"rank {r} > cap {tp.rank_cap} at cluster {t}")
            Q = U[:, :r]
            R[side][t] = Q.T @ Vt
            newk[side][t] = r
            if ct.is_leaf(t):
                newleaf[side][t] = Q
            else:
                r1 = newk[side][t1]
                newE[side][t1] = Q[:r1].copy()
                newE[side][t2] = Q[r1:].copy()

    # -- step 5: couplings of every admissible leaf touching the subtrees
    affected = []
    seen = set()
    for side in (0, 1):
        for t in sub[side]:
            for b in blocks[side][t]:
                if b not in seen:
                    seen.add(b)
                    affected.append(b)
    newS = {}
    for b in affected:
        t, s = int(bt.row[b]), int(bt.col[b])
        Rt = R[0][t] if t in insub[0] else np.eye(int(Z.k[0][t]))
        Rs = R[1][s] if s in insub[1] else np.eye(int(Z.k[1][s]))
        newS[b] = Rt @ Sext(b) @ Rs.T

    # -- step 7 (uses the old state only through X, Y): nearfield inside b0
    for b in Z.near:
        t, s = int(bt.row[b]), int(bt.col[b])
        if t in insub[0] and s in insub[1]:
            a0, a1 = ct.rng(t); c0, c1 = ct.rng(s)
            Z.N[b] = Z.N[b] + X[a0 - base[0]:a1 - base[0]] @ Y[c0 - base[1]:c1 - base[1]].T

    # -- step 6: write bases, transfers, couplings, ranks, R-factors
    for side in (0, 1):
        t0 = r0[side]
        if ct.parent[t0] >= 0:
            E0 = R[side][t0] @ Eext(side, t0)
        for t in sub[side]:
            if ct.is_leaf(t):
                Z.leafbasis[side][t] = newleaf[side][t]
            if t != t0:
                Z.E[side][t] = newE[side][t]
            Z.k[side][t] = newk[side][t]
            Z.rho[side][t] = np.eye(newk[side][t])
        if ct.parent[t0] >= 0:
            Z.E[side][t0] = E0
            for t in reversed(ct.path_to(t0)[:-1]):
                t1, t2 = ct.sons(t)
                Z.rho[side][t] = qr_r(np.vstack([Z.rho[side][t1] @ Z.E[side][t1],
                                                 Z.rho[side][t2] @ Z.E[side][t2]]))
    for b, S in newS.items():
        Z.S[b] = S
    return True


def common_block(bt, blocks) -> int:
    """The smallest block of the block tree that contains every block in
    ``blocks``: the deepest common ancestor (a block contains its sons'
    index sets, so the ancestors of a block are exactly the blocks that
    contain it)."""
    def ancestors(b):
        out = []
        while b >= 0:
            out.append(int(b))
            b = int(bt.parent[b])
        return out
    common = set(ancestors(blocks[0]))
    for b in blocks[1:]:
        common &= set(ancestors(b))
    # the deepest one: the first ancestor of blocks[0] that is common
    return next(a for a in ancestors(blocks[0]) if a in common)


def addlr_accumulated(Z: H2Matrix, updates, tp: TruncParams, margins: list | None = None):
    """Accumulated local update (the accumulation variant of the truncation
    strategies, last paragraph of Section 4): the updates (b_i, X_i, Y_i) are
    merged into ONE local update of the smallest block b* = (t*, s*)
    containing every target, with the factors placed side by side,
        X* = [P_1 X_1, ..., P_m X_m],   Y* = [Q_1 Y_1, ..., Q_m Y_m],
    P_i (Q_i) putting the rows of t_i (s_i) at their place in t* (s*) and
    zeros elsewhere, so that X* Y*^* = sum_i P_i X_i Y_i^* Q_i^* exactly;
    then one recompression instead of m.  Returns b*.

    Reading: the paper names the truncation strategies without fixing how
    contributions are grouped; merging into the smallest containing block
    with block-placed factors is the reading taken here."""
    ct, bt = Z.ct, Z.bt
    blocks = [int(b) for b, _, _ in updates]
    bs = common_block(bt, blocks)
    ts, ss = int(bt.row[bs]), int(bt.col[bs])
    ks = [np.asarray(X).shape[1] for _, X, _ in updates]
    Xs = np.zeros((int(ct.size[ts]), sum(ks)))
    Ys = np.zeros((int(ct.size[ss]), sum(ks)))
    c = 0
    for (b, X, Y), k in zip(updates, ks):
        t, s = int(bt.row[b]), int(bt.col[b])
        rt = int(ct.offset[t] - ct.offset[ts])
        rs = int(ct.offset[s] - ct.offset[ss])
        Xs[rt:rt + int(ct.size[t]), c:c + k] = X
        Ys[rs:rs + int(ct.size[s]), c:c + k] = Y
        c += k
    addlr(Z, bs, Xs, Ys, tp, margins)
    return bs
