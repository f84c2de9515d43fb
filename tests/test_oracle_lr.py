"""Pins of the oracle's LR factorisation and three-matrix product (Section 3;
Section 6, Cases 1 and 2)."""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as w
from oracle.h2 import TruncParams, from_csr, to_dense
from oracle.lr import lr, lr_dense, lr_solve, product
from oracle.trees import build_block_tree, build_cluster_tree
from oracle.update import addlr

NONE = TruncParams(0.0, "none", 1000)


def _trees(N, leaf=32):
    ct = build_cluster_tree(w.grid_points(N, 2), leaf)
    return ct, build_block_tree(ct, 2.0)


def _perm(A, ct):
    return A.toarray()[ct.perm][:, ct.perm]


def _nonsym(N, sigma_seed, c=3.0):
    p = w.problem(N, sigma_seed=sigma_seed, rhs_seed=4)
    return p["A"] + w.convection_x(N, c)


@pytest.mark.parametrize("N, leaf, seed", [(16, 8, 3), (16, 16, None), (12, 4, None)])
def test_lr_exact_reproduces_a(N, leaf, seed):
    """Without truncation the stored factors multiply back to A, with L unit
    lower and R upper triangular; an LR factorisation without pivoting is
    unique, so this fixes both factors."""
    ct, bt = _trees(N, leaf)
    A = _nonsym(N, seed)
    F = lr(from_csr(A, ct, bt), NONE)
    Ld, Rd = lr_dense(F)
    Ap = _perm(A, ct)
    assert np.linalg.norm(Ld @ Rd - Ap, 2) / np.linalg.norm(Ap, 2) < 1e-13
    assert np.allclose(np.diag(Ld), 1.0)


def test_lr_of_spd_matches_cholesky():
    """For SPD A: L = L_c D^{-1} and R = D L_c^* with L_c = LAPACK Cholesky
    factor and D its diagonal."""
    ct, bt = _trees(16, 8)
    p = w.problem(16, sigma_seed=7, rhs_seed=4)
    F = lr(from_csr(p["A"], ct, bt), NONE)
    Ld, Rd = lr_dense(F)
    Lc = np.linalg.cholesky(_perm(p["A"], ct))
    D = np.diag(np.diag(Lc))
    assert np.linalg.norm(Ld - Lc @ np.linalg.inv(D), 2) / np.linalg.norm(Ld, 2) < 1e-12
    assert np.linalg.norm(Rd - D @ Lc.T, 2) / np.linalg.norm(Rd, 2) < 1e-12


@pytest.mark.parametrize("eps", [1e-3, 1e-5])
def test_lr_truncated_accuracy(eps):
    """With block-relative truncation ||A - L R|| / ||A|| = O(eps)."""
    ct, bt = _trees(24, 8)
    A = _nonsym(24, 5)
    F = lr(from_csr(A, ct, bt), TruncParams(eps, "block_rel", 64))
    Ld, Rd = lr_dense(F)
    Ap = _perm(A, ct)
    err = np.linalg.norm(Ld @ Rd - Ap, 2) / np.linalg.norm(Ap, 2)
    assert err < 50 * eps
    assert err > 1e-15


def test_lr_solve_exact_is_inverse():
    """z = R^{-1} L^{-1} r equals A^{-1} r for the exact factors."""
    N = 16
    ct, bt = _trees(N, 8)
    A = _nonsym(N, 3)
    F = lr(from_csr(A, ct, bt), NONE)
    r = w.gaussian(A.shape[0], 1, 9)[:, 0]
    z = lr_solve(F, r)
    zref = np.linalg.solve(A.toarray(), r)
    assert np.linalg.norm(z - zref) / np.linalg.norm(zref) < 1e-12


def _h2_with_updates(A, ct, bt, seed, k=3):
    """Full-storage H^2(A) plus exact rank-k updates on the root's son
    blocks (non-trivial bases and couplings); returns it and its dense copy."""
    Z = from_csr(A, ct, bt)
    D = _perm(A, ct)
    sons = [b for b in range(bt.nb) if bt.parent[b] == 0]
    for i, b in enumerate(sons):
        t, s = int(bt.row[b]), int(bt.col[b])
        X = w.gaussian(int(ct.size[t]), k, seed + 2 * i)
        Y = w.gaussian(int(ct.size[s]), k, seed + 2 * i + 1)
        addlr(Z, b, X, Y, NONE)
        a0, a1 = ct.rng(t); c0, c1 = ct.rng(s)
        D[a0:a1, c0:c1] += X @ Y.T
    return Z, D


@pytest.mark.parametrize("N, leaf", [(16, 8), (12, 4)])
def test_product_exact_equals_dense(N, leaf):
    """Without truncation Z + alpha X Y equals the dense product."""
    ct, bt = _trees(N, leaf)
    A = _nonsym(N, 3 if N % 8 == 0 else None)
    X, Xd = _h2_with_updates(A, ct, bt, 100)
    Y, Yd = _h2_with_updates(A.T.tocsr(), ct, bt, 200)
    Z, Zd = _h2_with_updates(A, ct, bt, 300, k=2)
    assert np.linalg.norm(to_dense(X) - Xd) < 1e-10 * np.linalg.norm(Xd)
    product(Z, -0.7, X, Y, NONE)
    ref = Zd - 0.7 * Xd @ Yd
    assert np.linalg.norm(to_dense(Z) - ref, 2) / np.linalg.norm(ref, 2) < 1e-13


@pytest.mark.parametrize("eps", [1e-3, 1e-6])
def test_product_truncated_accuracy(eps):
    ct, bt = _trees(16, 8)
    A = _nonsym(16, 3)
    X, Xd = _h2_with_updates(A, ct, bt, 100)
    Y, Yd = _h2_with_updates(A, ct, bt, 200)
    Z, Zd = _h2_with_updates(A, ct, bt, 300, k=2)
    product(Z, 1.0, X, Y, TruncParams(eps, "block_rel", 64))
    ref = Zd + Xd @ Yd
    err = np.linalg.norm(to_dense(Z) - ref, 2) / np.linalg.norm(ref, 2)
    assert err < 50 * eps


def test_getrf_zero_pivot():
    from oracle.lr import ZeroPivotError
    ct, bt = _trees(8, 64)
    A = _nonsym(8, None)
    A = A.tolil()
    A[ct.perm[0], ct.perm[0]] = 0.0
    with pytest.raises(ZeroPivotError):
        lr(from_csr(A.tocsr(), ct, bt), NONE)
