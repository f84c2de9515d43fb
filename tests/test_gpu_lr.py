"""Parity of the LR factorisation (h2_lr, h2_lr_solve) and of the product
of three H^2-matrices (h2_product) with the oracle (Section 3), through the
C ABI on the same seeded inputs.  Bar: represented operators within 1e-12
relative spectral error (dense expansion through h2_matvec), solutions
within 1e-12."""
import numpy as np
import pytest

import workloads as w
from oracle.h2 import TruncParams, from_csr as o_from_csr, to_dense as o_to_dense
from oracle.lr import lr as o_lr, lr_solve as o_lr_solve, product as o_product
from oracle.trees import build_block_tree, build_cluster_tree
from oracle.update import addlr as o_addlr
from tests.helpers import dense_via_matvec, gpu, rel2, to_dev_cols, to_original

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def lib():
    gpu()
    from paper_1402_5056_amd import h2lr
    return h2lr


def _nonsym(N, sigma_seed, c=3.0):
    p = w.problem(N, sigma_seed=sigma_seed, rhs_seed=4)
    return p["A"] + w.convection_x(N, c)


def _trees(lib, N, leaf):
    coords = w.grid_points(N, 2)
    ctx = lib.h2_ctx_create(0)
    bt = lib.h2_btree_build(ctx, lib.h2_ctree_build(ctx, coords, leaf), 2.0)
    oc = build_cluster_tree(coords, leaf)
    return ctx, bt, oc, build_block_tree(oc, 2.0)


def _tp(eps, mode):
    return TruncParams(eps, mode, 32)


@pytest.mark.parametrize("N,leaf,seed,eps,mode", [
    (16, 8, 3, 0.0, "none"),          # exact: L R = A
    (24, 8, 5, 1e-6, "block_rel"),
    (32, 16, 7, 1e-4, "block_rel"),
    (40, 24, None, 1e-5, "block_rel"),  # unbalanced tree (leaves on two levels)
    (32, 8, 9, 1e-8, "const_rel"),
])
def test_lr_parity(lib, N, leaf, seed, eps, mode):
    print(f"case: LR N={N} leaf {leaf} eps={eps} {mode}", flush=True)
    A = _nonsym(N, seed)
    ctx, bt, oc, ob = _trees(lib, N, leaf)
    stats = {"margins": []}
    F = o_lr(o_from_csr(A, oc, ob), _tp(eps, mode), stats)
    if mode == "block_rel" and stats["margins"]:
        assert min(stats["margins"]) > 1e-8, "seed too close to the truncation threshold"
    M = lib.h2_mat_from_csr(ctx, bt, A, lower=False)
    lib.h2_lr(M, lib.trunc(eps, mode, 32))
    D = dense_via_matvec(lib, M, oc.n)
    Dref = to_original(o_to_dense(F), oc.perm)
    err = rel2(D, Dref)
    print(f"  ||F_gpu - F_oracle|| / ||F_oracle|| = {err:.2e}", flush=True)
    assert err < TOL
    # z = R^{-1} L^{-1} r
    torch = gpu()
    r = w.gaussian(oc.n, 3, 11)
    R = torch.tensor(np.ascontiguousarray(r.T), device="cuda")
    Zt = torch.zeros_like(R)
    lib.h2_lr_solve(M, R, Zt)
    zref = np.stack([o_lr_solve(F, r[:, i]) for i in range(3)])
    assert rel2(Zt.cpu().numpy(), zref) < TOL
    if mode == "none":
        zexact = np.linalg.solve(A.toarray(), r).T
        assert rel2(Zt.cpu().numpy(), zexact) < 1e-11


def test_lr_zero_pivot(lib):
    N = 8
    A = _nonsym(N, None).tolil()
    ctx, bt, oc, ob = _trees(lib, N, 32)
    A[oc.perm[0], oc.perm[0]] = 0.0
    M = lib.h2_mat_from_csr(ctx, bt, A.tocsr(), lower=False)
    with pytest.raises(lib.H2Error) as ei:
        lib.h2_lr(M, lib.trunc(0.0, "none", 32))
    assert ei.value.name == "H2_ERR_ZERO_PIVOT"
    with pytest.raises(lib.H2Error) as ei:
        lib.h2_lr(M, lib.trunc(0.0, "none", 32))
    assert ei.value.name == "H2_ERR_STATE"


def test_lr_argument_errors(lib):
    p = w.problem(16, sigma_seed=1, rhs_seed=2)
    ctx, bt, oc, ob = _trees(lib, 16, 8)
    Ml = lib.h2_mat_from_csr(ctx, bt, p["A"], lower=True)
    with pytest.raises(lib.H2Error):
        lib.h2_lr(Ml, lib.trunc(1e-6))
    M = lib.h2_mat_from_csr(ctx, bt, p["A"], lower=False)
    torch = gpu()
    r = torch.zeros(oc.n, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.H2Error):   # not factorised yet
        lib.h2_lr_solve(M, r, r)


def _with_updates(lib, ctx, bt, oc, ob, A, seed, k=3):
    """Full-storage H^2(A) plus exact rank-k updates on the root's son blocks,
    built identically on both sides (oracle and device)."""
    Z = o_from_csr(A, oc, ob)
    M = lib.h2_mat_from_csr(ctx, bt, A, lower=False)
    none = TruncParams(0.0, "none", 32)
    sons = [b for b in range(ob.nb) if ob.parent[b] == 0]
    for i, b in enumerate(sons):
        t, s = int(ob.row[b]), int(ob.col[b])
        X = w.gaussian(int(oc.size[t]), k, seed + 2 * i)
        Y = w.gaussian(int(oc.size[s]), k, seed + 2 * i + 1)
        o_addlr(Z, b, X, Y, none)
        lib.h2_lowrank_update(M, b, to_dev_cols(X), to_dev_cols(Y), lib.trunc(0.0, "none", 32))
    return Z, M


@pytest.mark.parametrize("N,leaf,alpha,eps,mode", [
    (16, 8, -0.7, 0.0, "none"),
    (24, 16, 1.0, 1e-6, "block_rel"),
    (32, 16, 0.5, 1e-3, "block_rel"),
    (24, 16, -1.0, 1e-8, "const_rel"),
])
def test_product_parity(lib, N, leaf, alpha, eps, mode):
    print(f"case: product N={N} leaf {leaf} alpha={alpha} eps={eps} {mode}", flush=True)
    ctx, bt, oc, ob = _trees(lib, N, leaf)
    A = _nonsym(N, 3)
    Xo, Xd = _with_updates(lib, ctx, bt, oc, ob, A, 100)
    Yo, Yd = _with_updates(lib, ctx, bt, oc, ob, A.T.tocsr(), 200)
    Zo, Zd = _with_updates(lib, ctx, bt, oc, ob, A, 300, k=2)
    # the operands agree before the product
    assert rel2(dense_via_matvec(lib, Xd, oc.n), to_original(o_to_dense(Xo), oc.perm)) < TOL
    stats = {"margins": []}
    o_product(Zo, alpha, Xo, Yo, _tp(eps, mode), stats)
    if mode == "block_rel" and stats["margins"]:
        assert min(stats["margins"]) > 1e-8, "seed too close to the truncation threshold"
    lib.h2_product(Zd, alpha, Xd, Yd, lib.trunc(eps, mode, 32))
    D = dense_via_matvec(lib, Zd, oc.n)
    Dref = to_original(o_to_dense(Zo), oc.perm)
    err = rel2(D, Dref)
    print(f"  ||Z_gpu - Z_oracle|| / ||Z_oracle|| = {err:.2e}", flush=True)
    assert err < TOL
    # the factors are unchanged
    assert rel2(dense_via_matvec(lib, Yd, oc.n), to_original(o_to_dense(Yo), oc.perm)) < TOL


def test_product_argument_errors(lib):
    ctx, bt, oc, ob = _trees(lib, 16, 8)
    p = w.problem(16, sigma_seed=1, rhs_seed=2)
    Z = lib.h2_mat_from_csr(ctx, bt, p["A"], lower=False)
    X = lib.h2_mat_from_csr(ctx, bt, p["A"], lower=False)
    L = lib.h2_mat_from_csr(ctx, bt, p["A"], lower=True)
    tr = lib.trunc(1e-6)
    with pytest.raises(lib.H2Error):
        lib.h2_product(Z, 1.0, Z, X, tr)          # target is a factor
    with pytest.raises(lib.H2Error):
        lib.h2_product(Z, 1.0, X, L, tr)          # lower storage
    ctx2, bt2, oc2, ob2 = _trees(lib, 16, 8)
    X2 = lib.h2_mat_from_csr(ctx2, bt2, p["A"], lower=False)
    with pytest.raises(lib.H2Error):
        lib.h2_product(Z, 1.0, X, X2, tr)         # another block tree
