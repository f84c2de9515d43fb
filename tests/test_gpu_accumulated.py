"""Accumulated local updates through the C ABI against the oracle's twins.

* h2_lowrank_update_accumulated against oracle.update.addlr_accumulated:
  several updates merged into one local update of the smallest containing
  block, one recompression.  Bar: the same merged block, equal rank
  vectors, and the H^2 matrices within 1e-12 relative spectral error in
  FP64, exact and truncated, full and lower storage.
* Cholesky and LR with accumulated product temporaries (h2_trunc.accumulate)
  against the oracle with TruncParams.accumulate: equal ranks, factors
  within 1e-12, PCG iteration counts equal."""
import numpy as np
import pytest

import workloads as w
from oracle.h2 import TruncParams, from_csr as o_from_csr, to_dense as o_to_dense
from oracle.trees import ADM, build_block_tree, build_cluster_tree
from oracle.update import addlr_accumulated as o_accumulated, common_block
from tests.helpers import dense_via_matvec, gpu, rel2, to_dev_cols, to_original

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def lib():
    gpu()
    from paper_1402_5056_amd import h2lr
    return h2lr


def _groups(ct, bt, lower):
    adm = [b for b in range(bt.nb) if bt.kind[b] == ADM and (not lower or bt.is_lower(b))]
    diag = next([a, b] for a in adm for b in adm
                if a < b and common_block(bt, [a, b]) != 0
                and bt.row[common_block(bt, [a, b])] == bt.col[common_block(bt, [a, b])])
    return [[adm[5], adm[6], adm[9]], [adm[2], adm[30]], diag]


@pytest.mark.parametrize("lower", [False, True])
@pytest.mark.parametrize("mode,eps", [("none", 0.0), ("block_rel", 1e-6)])
def test_accumulated_parity(lib, lower, mode, eps):
    print(f"case: accumulated update, N=32, lower {lower}, {mode} {eps}", flush=True)
    p = w.problem("p1_square_32")
    oc = build_cluster_tree(p["coords"], 32)
    ob = build_block_tree(oc, 2.0)
    ctx = lib.h2_ctx_create(0)
    bt = lib.h2_btree_build(ctx, lib.h2_ctree_build(ctx, p["coords"], 32), 2.0)
    M = lib.h2_mat_from_csr(ctx, bt, p["A"], lower=lower)
    Z = o_from_csr(p["A"], oc, ob, lower=lower)
    tp = TruncParams(eps, mode, 32)
    tr = lib.trunc(eps, mode, 32)
    for g, group in enumerate(_groups(oc, ob, lower)):
        ups = []
        for i, b in enumerate(group):
            t, s = int(ob.row[b]), int(ob.col[b])
            X = w.gaussian(int(oc.size[t]), 2 + i, 300 + 10 * g + i) * np.logspace(0, -3, 2 + i)
            Y = w.gaussian(int(oc.size[s]), 2 + i, 400 + 10 * g + i)
            ups.append((b, X, Y))
        margins = []
        bo = o_accumulated(Z, ups, tp, margins)
        if mode != "none":
            assert not margins or min(margins) > 1e-8, "seed too close to the truncation threshold"
        bg = lib.h2_lowrank_update_accumulated(M, [(b, to_dev_cols(X), to_dev_cols(Y)) for b, X, Y in ups], tr)
        assert bg == bo
        kr, kc = lib.h2_mat_ranks(M, oc.nc)
        assert np.array_equal(kr, Z.k[0]) and np.array_equal(kc, Z.k[1])
        D = dense_via_matvec(lib, M, oc.n)
        R = to_original(o_to_dense(Z), oc.perm)
        if lower:
            P = oc.perm
            D = np.tril(D[np.ix_(P, P)])
            R = np.tril(R[np.ix_(P, P)])
        err = rel2(D, R)
        print(f"  group {g}: merged block {bg}, ||Z - Z_oracle||_2 / ||Z_oracle||_2 = {err:.2e}", flush=True)
        assert err < TOL


def test_accumulated_errors(lib):
    print("case: accumulated update argument errors", flush=True)
    p = w.problem(16, sigma_seed=7, rhs_seed=1)
    ctx = lib.h2_ctx_create(0)
    bt = lib.h2_btree_build(ctx, lib.h2_ctree_build(ctx, p["coords"], 8), 2.0)
    M = lib.h2_mat_from_csr(ctx, bt, p["A"])
    X = to_dev_cols(w.gaussian(225, 20, 1))
    with pytest.raises(lib.H2Error) as ei:       # 40 columns in all
        lib.h2_lowrank_update_accumulated(M, [(0, X, X), (0, X, X)], lib.trunc(1e-6))
    assert ei.value.name == "H2_ERR_ARG"
    with pytest.raises(lib.H2Error) as ei:
        lib.h2_lowrank_update_accumulated(M, [], lib.trunc(1e-6))
    assert ei.value.name == "H2_ERR_ARG"


# ------------------------------------- accumulated temporaries in the factorisations
@pytest.mark.parametrize("N,leaf,seed,eps", [(16, 8, 7, 0.0), (24, 8, 3, 1e-6), (32, 32, 3, 1e-5),
                                             (48, 32, 5, 1e-4)])
def test_cholesky_accumulated_parity(lib, N, leaf, seed, eps):
    """H^2-Cholesky with accumulated product temporaries (h2_trunc.accumulate
    = 1) against the oracle with the same flag: equal ranks, factor within
    1e-12, PCG iteration counts equal."""
    from oracle.arith import cholesky as o_cholesky, precond_apply as o_precond
    from oracle.solve import pcg as o_pcg
    print(f"case: accumulated Cholesky N={N} leaf {leaf} eps {eps}", flush=True)
    torch = gpu()
    p = w.problem(N, sigma_seed=seed, rhs_seed=N)
    oc = build_cluster_tree(p["coords"], leaf)
    ob = build_block_tree(oc, 2.0)
    mode = "none" if eps == 0.0 else "block_rel"
    stats = {"margins": []}
    L = o_cholesky(o_from_csr(p["A"], oc, ob, lower=True), TruncParams(eps, mode, 32, accumulate=True), stats)
    if mode != "none" and stats["margins"]:
        assert min(stats["margins"]) > 1e-8, "seed too close to the truncation threshold"
    ctx = lib.h2_ctx_create(0)
    bt = lib.h2_btree_build(ctx, lib.h2_ctree_build(ctx, p["coords"], leaf), 2.0)
    M = lib.h2_mat_from_csr(ctx, bt, p["A"], lower=True)
    lib.h2_cholesky(M, lib.trunc(eps, mode, 32, accumulate=True))
    kr, kc = lib.h2_mat_ranks(M, oc.nc)
    assert np.array_equal(kr, L.k[0]) and np.array_equal(kc, L.k[1])
    P = oc.perm
    D = np.tril(dense_via_matvec(lib, M, oc.n)[np.ix_(P, P)])
    err = rel2(D, np.tril(o_to_dense(L)))
    print(f"  ||L - L_oracle||_2 / ||L_oracle||_2 = {err:.2e}, updates {stats.get('addlr_done')}", flush=True)
    assert err < TOL
    A = lib.h2_csr_create(ctx, p["A"])
    b = torch.tensor(p["b"], device="cuda")
    x = torch.zeros_like(b)
    it, rel, ok = lib.h2_pcg(A, M, b, x, 1e-8, 100)
    xo, ito, _ = o_pcg(p["A"], p["b"], lambda v: o_precond(L, v))
    assert ok and it == ito
    assert np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo) < 1e-10


def test_lr_accumulated_parity(lib):
    """LR factorisation (non-symmetric) with accumulated temporaries against
    the oracle with the same flag."""
    from oracle.lr import lr as o_lr
    print("case: accumulated LR N=24 leaf 8 eps 1e-6", flush=True)
    N, leaf = 24, 8
    p = w.problem(N, sigma_seed=5, rhs_seed=4)
    A = p["A"] + w.convection_x(N, 3.0)
    oc = build_cluster_tree(p["coords"], leaf)
    ob = build_block_tree(oc, 2.0)
    F = o_lr(o_from_csr(A, oc, ob), TruncParams(1e-6, "block_rel", 32, accumulate=True), {"margins": []})
    ctx = lib.h2_ctx_create(0)
    bt = lib.h2_btree_build(ctx, lib.h2_ctree_build(ctx, p["coords"], leaf), 2.0)
    M = lib.h2_mat_from_csr(ctx, bt, A, lower=False)
    lib.h2_lr(M, lib.trunc(1e-6, "block_rel", 32, accumulate=True))
    err = rel2(dense_via_matvec(lib, M, oc.n), to_original(o_to_dense(F), oc.perm))
    print(f"  ||F - F_oracle||_2 / ||F_oracle||_2 = {err:.2e}", flush=True)
    assert err < TOL
