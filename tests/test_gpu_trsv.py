"""Single triangular solves with the H^2 Cholesky factor through the C ABI
(Section 3, block forward substitution with vector right-hand sides):
z = L^{-1} r and z = L^{-*} r against the oracle's substitutions, within
1e-12 relative in FP64; the two in sequence equal h2_precond."""
import numpy as np
import pytest

import workloads as w
from oracle.arith import backward_solve as o_bsolve, cholesky as o_cholesky, forward_solve as o_fsolve
from oracle.h2 import TruncParams, from_csr as o_from_csr
from oracle.trees import build_block_tree, build_cluster_tree
from tests.helpers import gpu

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.mark.parametrize("N,sigma_seed,leaf", [(24, 3, 16), (32, 4, 32)])
def test_trsv_parity(N, sigma_seed, leaf):
    print(f"case: trsv N={N} leaf={leaf}", flush=True)
    torch = gpu()
    from paper_1402_5056_amd import h2lr as lib
    p = w.problem(N, sigma_seed=sigma_seed, rhs_seed=5)
    ctx = lib.h2_ctx_create(0)
    ct = lib.h2_ctree_build(ctx, p["coords"], leaf)
    bt = lib.h2_btree_build(ctx, ct, 2.0)
    M = lib.h2_mat_from_csr(ctx, bt, p["A"], lower=True)
    lib.h2_cholesky(M, lib.trunc(1e-6, "block_rel", 32))
    oc = build_cluster_tree(p["coords"], leaf)
    ob = build_block_tree(oc, 2.0)
    L = o_cholesky(o_from_csr(p["A"], oc, ob, lower=True), TruncParams(1e-6, "block_rel", 32))
    n = oc.n
    r = w.gaussian(n, 3, 17)
    R = torch.tensor(np.ascontiguousarray(r.T), device="cuda")
    Y = torch.zeros_like(R)
    Z = torch.zeros_like(R)
    lib.h2_trsv(M, R, Y)
    lib.h2_trsv(M, Y, Z, trans=True)
    P = torch.zeros_like(R)
    lib.h2_precond(M, R, P)
    torch.cuda.synchronize()
    perm = oc.perm
    for j in range(3):
        y = np.empty(n)
        y[perm] = o_fsolve(L, r[perm, j])
        z = np.empty(n)
        z[perm] = o_bsolve(L, y[perm])
        ey = np.linalg.norm(Y[j].cpu().numpy() - y) / np.linalg.norm(y)
        ez = np.linalg.norm(Z[j].cpu().numpy() - z) / np.linalg.norm(z)
        print(f"  column {j}: forward {ey:.2e}, backward {ez:.2e}", flush=True)
        assert ey < TOL and ez < TOL
    assert torch.allclose(Z, P, rtol=1e-13, atol=0.0)


def test_trsv_errors():
    gpu()
    from paper_1402_5056_amd import h2lr as lib
    p = w.problem(16, rhs_seed=1)
    ctx = lib.h2_ctx_create(0)
    ct = lib.h2_ctree_build(ctx, p["coords"], 8)
    bt = lib.h2_btree_build(ctx, ct, 2.0)
    full = lib.h2_mat_from_csr(ctx, bt, p["A"], lower=False)
    import torch
    r = torch.zeros(p["A"].shape[0], dtype=torch.float64, device="cuda")
    with pytest.raises(lib.H2Error) as ei:
        lib.h2_trsv(full, r, r)
    assert ei.value.name == "H2_ERR_ARG"
