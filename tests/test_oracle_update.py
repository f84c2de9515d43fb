"""Pins of the oracle's local low-rank update (Sections 4 and 5)."""
import numpy as np
import pytest

import workloads as w
from oracle.h2 import H2Matrix, TruncParams, from_csr, to_dense, block_apply, matvec
from oracle.trees import ADM, build_block_tree, build_cluster_tree
from oracle.update import addlr


@pytest.fixture(scope="module")
def sq32():
    p = w.problem("p1_square_32")
    ct = build_cluster_tree(p["coords"], 32)
    bt = build_block_tree(ct, 2.0)
    return p, ct, bt


def _rel2(A, B):
    return np.linalg.norm(A - B, 2) / max(np.linalg.norm(B, 2), 1e-300)


def test_global_update_exact(sq32):
    """Without truncation the recompressed matrix equals Z + X Y^* (the
    rank-extended representation of eq. (tildeZ_h2) is exact)."""
    p, ct, bt = sq32
    Z = from_csr(p["A"], ct, bt)
    D0 = to_dense(Z)
    X = w.gaussian(ct.n, 8, 1)[ct.perm]
    Y = w.gaussian(ct.n, 8, 101)[ct.perm]
    addlr(Z, 0, X, Y, TruncParams(0.0, "none", 1000))
    assert _rel2(to_dense(Z), D0 + X @ Y.T) < 1e-13
    # a second global update on the now non-trivial bases
    X2 = w.gaussian(ct.n, 5, 2)[ct.perm]
    Y2 = w.gaussian(ct.n, 5, 3)[ct.perm]
    addlr(Z, 0, X2, Y2, TruncParams(0.0, "none", 1000))
    assert _rel2(to_dense(Z), D0 + X @ Y.T + X2 @ Y2.T) < 1e-13


def _local_blocks(ct, bt):
    adm = [b for b in range(bt.nb) if bt.kind[b] == ADM]
    inner = [b for b in range(bt.nb) if bt.kind[b] == 0 and bt.row[b] != bt.col[b]]
    diag = [b for b in range(bt.nb) if bt.kind[b] == 0 and bt.row[b] == bt.col[b] and b != 0]
    return [adm[3], adm[40], inner[2], inner[7], diag[1]]


def test_local_updates_exact_sequence(sq32):
    """A sequence of local updates on admissible leaves, subdivided blocks and
    diagonal blocks stays exact without truncation, and the bases stay nested
    with correct R-factors (rho^* rho = V^* V)."""
    p, ct, bt = sq32
    Z = from_csr(p["A"], ct, bt)
    ref = to_dense(Z)
    for i, b in enumerate(_local_blocks(ct, bt)):
        t, s = int(bt.row[b]), int(bt.col[b])
        X = w.gaussian(int(ct.size[t]), 3 + i, 10 + i)
        Y = w.gaussian(int(ct.size[s]), 3 + i, 20 + i)
        addlr(Z, b, X, Y, TruncParams(0.0, "none", 1000))
        a0, a1 = ct.rng(t); c0, c1 = ct.rng(s)
        ref[a0:a1, c0:c1] += X @ Y.T
        assert _rel2(to_dense(Z), ref) < 1e-13
    cache = {}
    for side in (0, 1):
        for t in range(ct.nc):
            Vt = Z.basis(side, t, cache)
            rho = Z.rho[side][t]
            scale = max(1.0, float(np.abs(Vt).max()) ** 2) if Vt.size else 1.0
            assert np.allclose(rho.T @ rho, Vt.T @ Vt, atol=1e-11 * scale)


def test_untouched_data_bitwise(sq32):
    """Couplings, bases and nearfield outside the subtrees / b0 are unchanged
    (Section 5: only blocks touching T_t0 or T_s0 change)."""
    p, ct, bt = sq32
    Z = from_csr(p["A"], ct, bt)
    X = w.gaussian(ct.n, 6, 1)[ct.perm]
    addlr(Z, 0, X, X, TruncParams(1e-8, "block_rel", 64))
    b = [x for x in range(bt.nb) if bt.kind[x] == ADM][17]
    t, s = int(bt.row[b]), int(bt.col[b])
    Z0 = Z.copy()
    addlr(Z, b, w.gaussian(int(ct.size[t]), 2, 5), w.gaussian(int(ct.size[s]), 2, 6),
          TruncParams(1e-8, "block_rel", 64))
    T0, S0 = set(ct.subtree(t)), set(ct.subtree(s))
    for bb in Z.adm:
        if int(bt.row[bb]) not in T0 and int(bt.col[bb]) not in S0:
            assert np.array_equal(Z.S[bb], Z0.S[bb])
    for bb in Z.near:
        assert np.array_equal(Z.N[bb], Z0.N[bb])
    anc_t, anc_s = set(ct.path_to(t)), set(ct.path_to(s))
    for c in range(ct.nc):
        if c not in T0:
            if ct.is_leaf(c):
                assert np.array_equal(Z.leafbasis[0][c], Z0.leafbasis[0][c])
            if c != t:
                assert np.array_equal(Z.E[0][c], Z0.E[0][c])
            if c not in anc_t:
                assert np.array_equal(Z.rho[0][c], Z0.rho[0][c])
        if c not in S0 and ct.is_leaf(c):
            assert np.array_equal(Z.leafbasis[1][c], Z0.leafbasis[1][c])


def _two_cluster_problem():
    # two well separated 2x2 point groups: the only admissible block is (t1, t2)
    pts = np.array([[0, 0], [1, 0], [0, 1], [1, 1], [10, 0], [11, 0], [10, 1], [11, 1]], np.int32)
    ct = build_cluster_tree(pts, 4)
    bt = build_block_tree(ct, 2.0)
    return ct, bt


def test_single_block_is_eckart_young():
    """When t0 and s0 touch only b0, the update of a zero block is the best
    rank-r approximation of X Y^* with sigma_{r+1} <= eps ||X Y^*||_F."""
    ct, bt = _two_cluster_problem()
    adm = [b for b in range(bt.nb) if bt.kind[b] == ADM]
    b0 = bt.find(1, 2)
    assert adm == [bt.find(1, 2), bt.find(2, 1)]
    rng = np.random.Generator(np.random.PCG64(9))
    U, _ = np.linalg.qr(rng.standard_normal((4, 4)))
    V, _ = np.linalg.qr(rng.standard_normal((4, 4)))
    sig = np.array([3.0, 1.0, 2e-3, 1e-6])
    G = U @ np.diag(sig) @ V.T
    fro = np.linalg.norm(G)
    for eps, r in ((1e-1, 2), (1e-4, 3), (1e-8, 4)):
        Z = H2Matrix(ct, bt)
        for bb in Z.near:
            Z.N[bb][:] = 0.0
        addlr(Z, b0, G, np.eye(4), TruncParams(eps, "block_rel", 8))
        D = to_dense(Z)
        best = U[:, :r] @ np.diag(sig[:r]) @ V[:, :r].T
        assert np.allclose(D[0:4, 4:8], best, atol=1e-13 * fro)
        assert Z.k[0][1] == r and Z.k[1][2] == r
        assert np.count_nonzero(sig > eps * fro) == r


def test_truncation_error_blockwise_bound(sq32):
    """After a truncated global update every admissible block keeps the
    blockwise relative error ||(Z_new - Z~)|_b||_2 <= 2 (p+1) eps ||Z~|_b||_F
    (p = depth; the constant is chosen by this test, the paper prints none),
    and the total error decreases with eps."""
    p, ct, bt = sq32
    base = from_csr(p["A"], ct, bt)
    X0 = w.gaussian(ct.n, 10, 31)[ct.perm] * np.linspace(1, 1e-4, 10)
    Y0 = w.gaussian(ct.n, 10, 32)[ct.perm]
    errs = []
    for eps in (1e-2, 1e-4, 1e-6):
        Z = base.copy()
        addlr(Z, 0, X0, Y0, TruncParams(eps, "block_rel", 64))
        D = to_dense(Z)
        ref = to_dense(base) + X0 @ Y0.T
        for b in Z.adm:
            t, s = int(bt.row[b]), int(bt.col[b])
            a0, a1 = ct.rng(t); c0, c1 = ct.rng(s)
            e = np.linalg.norm(D[a0:a1, c0:c1] - ref[a0:a1, c0:c1], 2)
            assert e <= 2 * (ct.depth + 1) * eps * np.linalg.norm(ref[a0:a1, c0:c1])
        errs.append(_rel2(D, ref))
    assert errs[0] > errs[1] > errs[2]


def test_const_rel_mode(sq32):
    p, ct, bt = sq32
    Z = from_csr(p["A"], ct, bt)
    X = w.gaussian(ct.n, 6, 4)[ct.perm]
    ref = to_dense(Z) + X @ X.T
    addlr(Z, 0, X, X, TruncParams(1e-10, "const_rel", 64))
    assert _rel2(to_dense(Z), ref) < 1e-8


def test_skip_zero_update(sq32):
    p, ct, bt = sq32
    Z = from_csr(p["A"], ct, bt)
    Z0 = Z.copy()
    assert addlr(Z, 0, np.zeros((ct.n, 3)), w.gaussian(ct.n, 3, 1), TruncParams()) is False
    assert addlr(Z, 0, np.zeros((ct.n, 0)), np.zeros((ct.n, 0)), TruncParams()) is False
    assert all(np.array_equal(Z.N[b], Z0.N[b]) for b in Z.near)


def test_rank_cap(sq32):
    from oracle.h2 import RankCapError
    p, ct, bt = sq32
    Z = from_csr(p["A"], ct, bt)
    X = w.gaussian(ct.n, 8, 1)[ct.perm]
    with pytest.raises(RankCapError):
        addlr(Z, 0, X, X, TruncParams(0.0, "none", 4))


def test_matvec_plain_definition(sq32):
    p, ct, bt = sq32
    Z = from_csr(p["A"], ct, bt)
    X = w.gaussian(ct.n, 4, 8)[ct.perm]
    addlr(Z, 0, X, X[::-1].copy(), TruncParams(0.0, "none", 64))
    D = to_dense(Z)
    x = w.gaussian(ct.n, 1, 9)[:, 0]
    y = matvec(Z, x)
    Dorig = np.empty_like(D)
    Dorig[np.ix_(ct.perm, ct.perm)] = D
    assert np.allclose(y, Dorig @ x, rtol=1e-13, atol=1e-13 * np.abs(Dorig @ x).max())
    assert np.allclose(matvec(Z, x, trans=True), Dorig.T @ x, atol=1e-12)
    b = bt.find(2, 1)
    t, s = int(bt.row[b]), int(bt.col[b])
    a0, a1 = ct.rng(t); c0, c1 = ct.rng(s)
    xs = w.gaussian(c1 - c0, 3, 1)
    assert np.allclose(block_apply(Z, b, xs), D[a0:a1, c0:c1] @ xs, atol=1e-12)
