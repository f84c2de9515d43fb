"""Accumulated local update (h2_lowrank_update_accumulated) through the C
ABI against the oracle's twin (oracle.update.addlr_accumulated): several
updates merged into one local update of the smallest containing block, one
recompression.  Bar: the same merged block, equal rank vectors, and the
H^2 matrices within 1e-12 relative spectral error in FP64, exact and
truncated, full and lower storage."""
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
