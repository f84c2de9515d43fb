"""Pins of the domain-decomposition cluster tree (Section 7 clusters the
model problem by domain decomposition) and of the H^2 Cholesky factorisation
on it.  The tree is pinned by what nested dissection fixes: the interface
separates the two domains of every cut, the matrix vanishes between them,
and the exact (LAPACK) Cholesky factor of the reordered matrix has exactly
zero entries there, so the zero blocks of the block tree never fill.  At
the setting of Table 1's grid level 7 the oracle is checked against the
values the paper prints for that row."""
import json
import os

import numpy as np
import pytest

import workloads as w
from oracle.arith import cholesky, precond_apply
from oracle.h2 import TruncParams, from_csr, to_dense
from oracle.solve import pcg, power_error
from oracle.trees import ADM, NEAR, admissible, build_block_tree, build_cluster_tree, dd_zero_pair


def _dd(N, dim=2, leaf=32, eta=4.0):
    ct = build_cluster_tree(w.grid_points(N, dim), leaf, dd=True)
    return ct, build_block_tree(ct, eta)


def _matrix(N, dim, seed):
    if dim == 2:
        return w.fem2d_p1(N, w.sigma_subdomains_2d(N, 8, seed))
    return w.fem3d_q1(N, w.sigma_blocks_3d(N, 4, seed))


@pytest.mark.parametrize("N,dim,leaf", [(24, 2, 8), (33, 2, 32), (64, 2, 32), (8, 3, 8), (12, 3, 32)])
def test_dd_tree_structure(N, dim, leaf):
    ct, bt = _dd(N, dim, leaf)
    pts = w.grid_points(N, dim)
    assert sorted(ct.perm.tolist()) == list(range(ct.n))
    nunion = 0
    for t in range(ct.nc):
        if ct.is_leaf(t):
            assert ct.size[t] <= leaf
            continue
        s0, s1 = ct.sons(t)
        a, b = ct.rng(t)
        assert ct.rng(s0)[0] == a and ct.rng(s0)[1] == ct.rng(s1)[0] and ct.rng(s1)[1] == b
        if ct.union[t]:
            nunion += 1
            # the sibling of a union is the interface: one plane x_d = m
            # with the first domain strictly below and the second above
            f = int(ct.parent[t])
            assert ct.sons(f)[0] == t
            I = pts[ct.perm[slice(*ct.rng(ct.sons(f)[1]))]]
            D1 = pts[ct.perm[slice(*ct.rng(s0))]]
            D2 = pts[ct.perm[slice(*ct.rng(s1))]]
            planes = [d for d in range(dim) if (I[:, d] == I[0, d]).all()
                      and D1[:, d].max() < I[0, d] < D2[:, d].min()]
            assert planes, t
    assert nunion > 0
    # block leaves still partition I x I exactly once
    cover = np.zeros((ct.n, ct.n), np.int64)
    nzero = 0
    for b in range(bt.nb):
        if bt.kind[b] == 0:
            continue
        t, s = int(bt.row[b]), int(bt.col[b])
        cover[slice(*ct.rng(t)), slice(*ct.rng(s))] += 1
        if bt.kind[b] == ADM and not admissible(ct, t, s, 16.0):
            assert dd_zero_pair(ct, t, s)
            nzero += 1
        if bt.kind[b] == NEAR:
            assert ct.is_leaf(t) and ct.is_leaf(s)
    assert (cover == 1).all()
    assert nzero > 0


@pytest.mark.parametrize("N,dim,seed", [(24, 2, 3), (40, 2, None), (8, 3, 5), (12, 3, None)])
def test_dd_zero_blocks_have_no_fill(N, dim, seed):
    """A and its exact Cholesky factor (LAPACK) vanish on every admissible
    leaf of the DD block tree; the zero pairs are exactly zero in L."""
    ct, bt = _dd(N, dim, 8 if N < 30 else 32)
    A = _matrix(N, dim, seed).toarray()[ct.perm][:, ct.perm]
    L = np.linalg.cholesky(A)
    checked = 0
    for b in range(bt.nb):
        t, s = int(bt.row[b]), int(bt.col[b])
        if bt.kind[b] != ADM:
            continue
        assert not A[slice(*ct.rng(t)), slice(*ct.rng(s))].any()
        if dd_zero_pair(ct, t, s) and bt.is_lower(b):
            assert not L[slice(*ct.rng(t)), slice(*ct.rng(s))].any()
            checked += 1
    assert checked > 0


def test_bisection_tree_has_fill_where_dd_has_none():
    """Plant check for the test above: in bisection order the factor fills
    the block between the two halves of the root."""
    ct = build_cluster_tree(w.grid_points(24, 2), 8)
    A = _matrix(24, 2, 3).toarray()[ct.perm][:, ct.perm]
    L = np.linalg.cholesky(A)
    s0, s1 = ct.sons(0)
    assert np.abs(L[slice(*ct.rng(s1)), slice(*ct.rng(s0))]).max() > 1e-3


@pytest.mark.parametrize("N,dim,leaf,seed", [(24, 2, 8, 3), (33, 2, 32, None), (8, 3, 8, 5)])
def test_dd_cholesky_exact_equals_lapack(N, dim, leaf, seed):
    ct, bt = _dd(N, dim, leaf)
    A = _matrix(N, dim, seed)
    L = cholesky(from_csr(A, ct, bt, lower=True), TruncParams(0.0, "none", 1000))
    D = np.tril(to_dense(L))
    Lref = np.linalg.cholesky(A.toarray()[ct.perm][:, ct.perm])
    assert np.linalg.norm(D - Lref, 2) / np.linalg.norm(Lref, 2) < 1e-13
    for b in L.adm:
        t, s = int(bt.row[b]), int(bt.col[b])
        if dd_zero_pair(ct, t, s):
            assert L.S[b].size == 0 or not L.S[b].any()


def test_dd_cholesky_truncated_preconditioner():
    """Truncated factor on the DD tree: ||A - LL*|| / ||A|| = O(eps) and PCG
    reaches 1e-8 in a few steps (Table 1 reports m = 3)."""
    N = 48
    ct, bt = _dd(N, 2, 32)
    A = _matrix(N, 2, None)
    eps = 50.0 / N ** 2
    L = cholesky(from_csr(A, ct, bt, lower=True), TruncParams(eps, "block_rel", 32))
    Ap = A.toarray()[ct.perm][:, ct.perm]
    D = np.tril(to_dense(L))
    assert np.linalg.norm(Ap - D @ D.T, 2) / np.linalg.norm(Ap, 2) < 50 * eps
    b = w.gaussian(ct.n, 1, 9)[:, 0]
    x, it, rel = pcg(A, b, lambda r: precond_apply(L, r))
    assert it <= 6 and rel <= 1e-8
    assert np.linalg.norm(A @ x - b) / np.linalg.norm(b) < 1e-7


def test_table1_level7_setting():
    """The setting of Table 1's grid level 7 (Section 7): n = 16,129,
    sigma = 1, domain-decomposition clustering, eta 4, relative accuracy
    3.1e-3 (leaf size 32; the paper gives none).  The paper prints m = 3
    PCG steps, Err 0.06 and 1.0 KB per unknown for its run
    (tests/golden/table1_fem2d_l7.json).  The oracle must need the same
    number of steps, and its factor must be at least as good a
    preconditioner (Err below the printed value) without using more storage
    per unknown.  Measured: m = 3, Err 8e-4, 0.71 KB."""
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1_fem2d_l7.json")))
    ct, bt = _dd(128, 2, 32, g["eta"])
    assert ct.n == g["n"]
    A = _matrix(128, 2, None)
    L = cholesky(from_csr(A, ct, bt, lower=True), TruncParams(g["eps"], "block_rel", 32))

    def prec(r):
        return precond_apply(L, r)
    b = w.gaussian(ct.n, 1, 9)[:, 0]
    _, it, rel = pcg(A, b, prec)
    assert it == g["pcg_steps"] and rel <= 1e-8
    assert power_error(A, prec, ct.n, iters=30) < g["err"]
    assert 8.0 * L.storage_values() / ct.n / 1024.0 < g["mem_per_n_kb"]


def test_near_target_products_equal_recursion(monkeypatch):
    """Products Z|_(t,r) += X|_(t,s) Y|_(r,s)^* whose target is an
    inadmissible leaf pair while both factors are subdivided (s has sons)
    are frequent on DD trees, where interface leaves meet large domains
    (Section 6, the product recursion).  The oracle forms them densely.
    Recursing over the sons of s instead ends in low-rank emissions added to
    the dense target.  The two sums are equal in exact arithmetic, so the
    factors must agree to rounding, with equal ranks; the plain run must
    contain such products for the check to mean anything."""
    import oracle.arith as OA
    from oracle.trees import INNER
    N = 48
    ct, bt = _dd(N, 2, 32)
    A = _matrix(N, 2, None)
    tp = TruncParams(50.0 / N ** 2, "block_rel", 32)
    st0 = {}
    L0 = cholesky(from_csr(A, ct, bt, lower=True), tp, st0)
    assert st0.get("near_dense_product", 0) > 0
    plain = OA._Chol.mm

    def recursed(self, t, s, r, alpha, tmp=None):
        if tmp is None and bt.kind[bt.find(t, s)] == INNER and bt.kind[bt.find(r, s)] == INNER \
                and bt.kind[bt.find(t, r)] == NEAR:
            for s2 in ct.sons_plus(s):
                for t2 in ct.sons_plus(t):
                    for r2 in ct.sons_plus(r):
                        recursed(self, t2, s2, r2, alpha)
            return
        return plain(self, t, s, r, alpha, tmp)
    monkeypatch.setattr(OA._Chol, "mm", recursed)
    st1 = {}
    L1 = cholesky(from_csr(A, ct, bt, lower=True), tp, st1)
    assert st1.get("near_dense_product", 0) == 0
    assert np.array_equal(L1.k[0], L0.k[0]) and np.array_equal(L1.k[1], L0.k[1])
    D0, D1 = np.tril(to_dense(L0)), np.tril(to_dense(L1))
    assert np.linalg.norm(D1 - D0, 2) / np.linalg.norm(D0, 2) < 1e-13
