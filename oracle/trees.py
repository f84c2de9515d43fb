"""Cluster tree and block tree (Section 2, Def. "Cluster tree", Def. "Block
tree"; binary trees as assumed at the start of Section 3).

Readings of points the paper leaves open:

* Clustering: geometric bisection.  A cluster is a leaf iff it holds at most
  ``leaf_size`` indices.  Otherwise its (tight, integer) bounding box is split
  at the midpoint of its longest axis (ties go to the lowest axis); son 0
  receives the points with 2*c[d] <= lo[d] + hi[d], son 1 the rest, each in
  the father's order (stable).
* Clusters are numbered breadth first (son 0 before son 1); the indices are
  ordered depth first, so every cluster is a contiguous range
  ``perm[offset : offset + size]``.
* Admissibility (the paper names only the parameter eta, Section 7): (t, s)
  is admissible iff max(diam^2(B_t), diam^2(B_s)) <= eta^2 * dist^2(B_t, B_s)
  and the boxes are at least two grid steps apart along some axis (so that
  no stencil coupling only points within one step per axis reaches across),
  evaluated in exact integer arithmetic on the integer bounding boxes.
* Block tree: starting from (root, root), an admissible pair is an admissible
  leaf, a pair of two leaf clusters is an inadmissible leaf, every other pair
  is subdivided into sons+(t) x sons+(s) (Section 6, Case 1), enumerated with
  t' outer.  Blocks are numbered breadth first.

Domain-decomposition clustering (Section 7 uses a domain decomposition
cluster strategy in the style of Grasedyck, Kriemann and Le Borne; the paper
gives no details, and all trees here stay binary as Section 3 assumes):

* A domain cluster with more than ``leaf_size`` indices is cut by the grid
  hyperplane x_d = m, d its longest axis (lowest on ties) and
  m = floor((lo[d] + hi[d]) / 2), into D1 = {x_d < m}, the interface
  I = {x_d = m} and D2 = {x_d > m}.  Its sons are the union U = D1 u D2 and
  I, in this order, so the indices run D1, D2, I (each stable).  U, if it
  holds more than ``leaf_size`` indices, has the sons D1 and D2, which are
  domain clusters again.  Interface clusters and their descendants are split
  by geometric bisection as above.  If D1, D2 or I would be empty, the
  domain cluster is bisected instead and both sons stay domain clusters.
* Block tree: the pairs (D1, D2) and (D2, D1) below a split union node are
  admissible leaves whatever eta says.  On a stencil of reach 1 the matrix
  vanishes there, and so does its Cholesky factor in this (nested
  dissection) order: no fill ever enters, the blocks keep rank 0.
"""

from __future__ import annotations

from collections import deque
from dataclasses import dataclass, field

import numpy as np

INNER, ADM, NEAR = 0, 1, 2


@dataclass
class ClusterTree:
    n: int
    dim: int
    perm: np.ndarray          # cluster order -> original index
    offset: np.ndarray
    size: np.ndarray
    level: np.ndarray
    son0: np.ndarray          # -1 for leaves
    son1: np.ndarray
    parent: np.ndarray        # -1 for the root
    lo: np.ndarray            # (nc, dim) integer bounding boxes
    hi: np.ndarray
    depth: int = 0
    union: np.ndarray | None = None   # True: sons are two separated domains

    @property
    def nc(self) -> int:
        return len(self.offset)

    def is_leaf(self, t: int) -> bool:
        return self.son0[t] < 0

    def sons(self, t: int):
        return [] if self.son0[t] < 0 else [int(self.son0[t]), int(self.son1[t])]

    def sons_plus(self, t: int):
        """sons+(t) of Section 6: the sons, or {t} for a leaf."""
        return [t] if self.son0[t] < 0 else [int(self.son0[t]), int(self.son1[t])]

    def subtree(self, t: int):
        """Clusters of the subtree rooted at t, top-down (breadth first)."""
        out = [t]
        i = 0
        while i < len(out):
            out.extend(self.sons(out[i]))
            i += 1
        return out

    def path_to(self, t: int):
        """pred(t) ordered from the root down to t (inclusive)."""
        p = []
        while t >= 0:
            p.append(int(t))
            t = int(self.parent[t])
        return p[::-1]

    def rng(self, t: int):
        return int(self.offset[t]), int(self.offset[t] + self.size[t])

    def contains(self, t0: int, t: int) -> bool:
        """True iff t lies in the subtree of t0."""
        a0, b0 = self.rng(t0)
        a, b = self.rng(t)
        return a0 <= a and b <= b0 and self.level[t] >= self.level[t0]


DOMAIN, UNION, OTHER = 0, 1, 2


def build_cluster_tree(coords: np.ndarray, leaf_size: int = 32, dd: bool = False) -> ClusterTree:
    """Geometric bisection (dd=False) or domain decomposition (dd=True)."""
    coords = np.asarray(coords, dtype=np.int64)
    n, dim = coords.shape
    perm = np.arange(n, dtype=np.int64)
    offset, size, level, son0, son1, parent, lo, hi = [], [], [], [], [], [], [], []
    role, cut = [], []
    q = deque()

    def new(off, sz, lev, par, rl, ct=0):
        idx = len(offset)
        offset.append(off); size.append(sz); level.append(lev)
        son0.append(-1); son1.append(-1); parent.append(par)
        role.append(rl); cut.append(ct)
        pts = coords[perm[off:off + sz]]
        lo.append(pts.min(axis=0)); hi.append(pts.max(axis=0))
        q.append(idx)
        return idx

    new(0, n, 0, -1, DOMAIN if dd else OTHER)
    while q:
        t = q.popleft()
        off, sz = offset[t], size[t]
        if sz <= leaf_size:
            continue
        idx = perm[off:off + sz]
        if role[t] == UNION:
            # the father already ordered D1 before D2
            s0 = new(off, cut[t], level[t] + 1, t, DOMAIN)
            s1 = new(off + cut[t], sz - cut[t], level[t] + 1, t, DOMAIN)
            son0[t], son1[t] = s0, s1
            continue
        ext = hi[t] - lo[t]
        d = int(np.argmax(ext))
        if role[t] == DOMAIN:
            m = (int(lo[t][d]) + int(hi[t][d])) // 2
            x = coords[idx, d]
            m1, mi, m2 = x < m, x == m, x > m
            n1, ni, n2 = int(m1.sum()), int(mi.sum()), int(m2.sum())
            if n1 > 0 and ni > 0 and n2 > 0:
                perm[off:off + sz] = np.concatenate([idx[m1], idx[m2], idx[mi]])
                s0 = new(off, n1 + n2, level[t] + 1, t, UNION, n1)
                s1 = new(off + n1 + n2, ni, level[t] + 1, t, OTHER)
                son0[t], son1[t] = s0, s1
                continue
        mask = 2 * coords[idx, d] <= lo[t][d] + hi[t][d]
        n0 = int(mask.sum())
        assert 0 < n0 < sz
        perm[off:off + sz] = np.concatenate([idx[mask], idx[~mask]])
        rs = DOMAIN if role[t] == DOMAIN else OTHER
        s0 = new(off, n0, level[t] + 1, t, rs)
        s1 = new(off + n0, sz - n0, level[t] + 1, t, rs)
        son0[t], son1[t] = s0, s1
    ct = ClusterTree(n, dim, perm, np.array(offset, np.int64), np.array(size, np.int64),
                     np.array(level, np.int64), np.array(son0, np.int64),
                     np.array(son1, np.int64), np.array(parent, np.int64),
                     np.array(lo, np.int64), np.array(hi, np.int64))
    ct.depth = int(ct.level.max())
    ct.union = (np.array(role) == UNION) & (ct.son0 >= 0)
    return ct


def dd_zero_pair(ct: ClusterTree, t: int, s: int) -> bool:
    """(t, s) are the two domains below one split union node."""
    if ct.union is None or t == s:
        return False
    p = int(ct.parent[t])
    return p >= 0 and p == int(ct.parent[s]) and bool(ct.union[p])


def admissible(ct: ClusterTree, t: int, s: int, eta2: float) -> bool:
    lt, ht, ls, hs = ct.lo[t], ct.hi[t], ct.lo[s], ct.hi[s]
    diam_t = int(((ht - lt) ** 2).sum())
    diam_s = int(((hs - ls) ** 2).sum())
    gap = np.maximum(0, np.maximum(ls - ht, lt - hs))
    dist = int((gap ** 2).sum())
    return int(gap.max()) >= 2 and max(diam_t, diam_s) <= eta2 * dist


@dataclass
class BlockTree:
    ct: ClusterTree
    row: np.ndarray
    col: np.ndarray
    kind: np.ndarray          # INNER / ADM / NEAR
    parent: np.ndarray
    first_son: np.ndarray     # -1 for leaves
    nsons: np.ndarray
    index: dict = field(default_factory=dict)   # (t, s) -> block id

    @property
    def nb(self) -> int:
        return len(self.row)

    def find(self, t: int, s: int) -> int:
        return self.index[(t, s)]

    def is_lower(self, b: int) -> bool:
        """Diagonal block or block strictly below the diagonal in cluster order."""
        t, s = int(self.row[b]), int(self.col[b])
        return t == s or self.ct.offset[t] > self.ct.offset[s]

    def sons(self, b: int):
        f = int(self.first_son[b])
        return [] if f < 0 else list(range(f, f + int(self.nsons[b])))

    def leaves_below(self, b: int):
        """Leaf blocks of the subtree rooted at b, breadth first."""
        out, stack = [], [b]
        i = 0
        while i < len(stack):
            x = stack[i]
            i += 1
            if self.kind[x] == INNER:
                stack.extend(self.sons(x))
            else:
                out.append(x)
        return out


def build_block_tree(ct: ClusterTree, eta: float = 2.0) -> BlockTree:
    eta2 = float(eta) ** 2
    row, col, kind, parent, first, nsons = [], [], [], [], [], []
    q = deque()

    def new(t, s, par):
        row.append(t); col.append(s); parent.append(par)
        kind.append(INNER); first.append(-1); nsons.append(0)
        q.append(len(row) - 1)

    new(0, 0, -1)
    while q:
        b = q.popleft()
        t, s = row[b], col[b]
        if admissible(ct, t, s, eta2) or dd_zero_pair(ct, t, s):
            kind[b] = ADM
        elif ct.is_leaf(t) and ct.is_leaf(s):
            kind[b] = NEAR
        else:
            first[b] = len(row)
            cnt = 0
            for t2 in ct.sons_plus(t):
                for s2 in ct.sons_plus(s):
                    new(t2, s2, b)
                    cnt += 1
            nsons[b] = cnt
    bt = BlockTree(ct, np.array(row, np.int64), np.array(col, np.int64),
                   np.array(kind, np.int64), np.array(parent, np.int64),
                   np.array(first, np.int64), np.array(nsons, np.int64))
    bt.index = {(int(r), int(c)): i for i, (r, c) in enumerate(zip(bt.row, bt.col))}
    return bt
