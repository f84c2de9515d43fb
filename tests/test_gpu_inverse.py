"""Parity of the triangular inverse G ~ L^{-1} (inversion remark at the end of
Section 6, upper off-diagonal block zero) and of the preconditioner G^* G
with the CPU oracle, through the C ABI.  Bar: represented operators within
1e-12 relative spectral error in FP64; PCG iteration counts equal."""
import numpy as np
import pytest

import workloads as w
from oracle.arith import cholesky as o_cholesky, precond_apply_inverse as o_precond_inv, tri_invert as o_tri_invert
from oracle.h2 import TruncParams, from_csr as o_from_csr, to_dense as o_to_dense
from oracle.solve import pcg as o_pcg
from oracle.trees import build_block_tree, build_cluster_tree
from tests.helpers import dense_via_matvec, gpu, rel2, to_original

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def lib():
    gpu()
    from paper_1402_5056_amd import h2lr
    return h2lr


def _factor(lib, N, sigma_seed, eps, leaf, mode="block_rel", eta=2.0, dd=False, dim=2):
    p = w.problem(N, dim=dim, sigma_seed=sigma_seed, rhs_seed=5)
    ctx = lib.h2_ctx_create(0)
    ct = (lib.h2_ctree_build_dd if dd else lib.h2_ctree_build)(ctx, p["coords"], leaf)
    bt = lib.h2_btree_build(ctx, ct, eta)
    M = lib.h2_mat_from_csr(ctx, bt, p["A"], lower=True)
    oc = build_cluster_tree(p["coords"], leaf, dd=dd)
    ob = build_block_tree(oc, eta)
    tp = TruncParams(eps, mode, 32)
    L = o_cholesky(o_from_csr(p["A"], oc, ob, lower=True), tp)
    lib.h2_cholesky(M, lib.trunc(eps, mode, 32))
    return p, ctx, M, oc, L, tp


@pytest.mark.parametrize("N,sigma_seed,eps,leaf,mode", [
    (32, None, 1e-12, 32, "block_rel"), (16, 7, 1e-6, 8, "block_rel"), (32, 3, 1e-4, 32, "block_rel"),
    (24, 3, 1e-6, 16, "block_rel"), (40, 7, 1e-5, 24, "block_rel"), (32, 4, 1e-8, 32, "const_rel")])
def test_tri_invert_parity(lib, N, sigma_seed, eps, leaf, mode):
    """Balanced and unbalanced trees (24 x 24 leaf 16 and 40 x 40 leaf 24
    have leaves on two levels)."""
    print(f"case: tri_invert N={N} sigma={sigma_seed} eps={eps} leaf={leaf} mode={mode}", flush=True)
    p, ctx, M, oc, L, tp = _factor(lib, N, sigma_seed, eps, leaf, mode)
    G = o_tri_invert(L, tp)
    assert not lib.h2_mat_is_inverse(M)
    lib.h2_tri_invert(M, lib.trunc(eps, mode, 32))
    assert lib.h2_mat_is_inverse(M)
    D = dense_via_matvec(lib, M, oc.n)
    Gd = np.tril(o_to_dense(G))
    Dref = to_original(Gd, oc.perm)
    err = rel2(D, Dref)
    print(f"  ||G_gpu - G_oracle||_2 / ||G_oracle||_2 = {err:.3e}", flush=True)
    assert err < TOL
    # nothing above the diagonal (in cluster order)
    Dc = D[np.ix_(oc.perm, oc.perm)]
    assert np.all(np.triu(Dc, 1) == 0.0)
    _, kr, kc = lib.h2_mat_stats(M)
    assert (kr, kc) == (int(G.k[0].max()), int(G.k[1].max()))
    if eps <= 1e-12:   # nearly exact: the dense inverse of LAPACK's factor
        Ap = p["A"].toarray()[oc.perm][:, oc.perm]
        Gref = np.linalg.inv(np.linalg.cholesky(Ap))
        assert rel2(Dc, Gref) < 1e-9


def test_tri_invert_parity_dd(lib):
    print("case: tri_invert dd N=33 eta 4", flush=True)
    p, ctx, M, oc, L, tp = _factor(lib, 33, None, 1e-4, 32, eta=4.0, dd=True)
    G = o_tri_invert(L, tp)
    lib.h2_tri_invert(M, lib.trunc(1e-4, "block_rel", 32))
    D = dense_via_matvec(lib, M, oc.n)
    err = rel2(D, to_original(np.tril(o_to_dense(G)), oc.perm))
    print(f"  ||G_gpu - G_oracle||_2 / ||G_oracle||_2 = {err:.3e}", flush=True)
    assert err < TOL


def test_precond_inverse_and_pcg(lib):
    print("case: precond G^*G + pcg N=32", flush=True)
    torch = gpu()
    p, ctx, M, oc, L, tp = _factor(lib, 32, 3, 1e-4, 32)
    G = o_tri_invert(L, tp)
    lib.h2_tri_invert(M, lib.trunc(1e-4, "block_rel", 32))
    r = w.gaussian(oc.n, 3, 9)
    R = torch.tensor(np.ascontiguousarray(r.T), device="cuda")
    Zt = torch.zeros_like(R)
    lib.h2_precond(M, R, Zt)
    zref = np.stack([o_precond_inv(G, r[:, i]) for i in range(3)])
    assert rel2(Zt.cpu().numpy(), zref) < TOL
    A = lib.h2_csr_create(ctx, p["A"])
    b = torch.tensor(p["b"], device="cuda")
    x = torch.zeros_like(b)
    it, rel, ok = lib.h2_pcg(A, M, b, x, 1e-8, 100)
    xo, ito, relo = o_pcg(p["A"], p["b"], lambda v: o_precond_inv(G, v))
    print(f"  pcg iterations gpu {it} oracle {ito}", flush=True)
    assert ok and it == ito
    assert np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo) < 1e-10


def test_tri_invert_errors(lib):
    print("case: tri_invert argument errors", flush=True)
    p = w.problem(16, rhs_seed=1)
    ctx = lib.h2_ctx_create(0)
    ct = lib.h2_ctree_build(ctx, p["coords"], 8)
    bt = lib.h2_btree_build(ctx, ct, 2.0)
    full = lib.h2_mat_from_csr(ctx, bt, p["A"], lower=False)
    with pytest.raises(lib.H2Error) as ei:
        lib.h2_tri_invert(full, lib.trunc(1e-6))
    assert ei.value.name == "H2_ERR_ARG"
    M = lib.h2_mat_from_csr(ctx, bt, p["A"], lower=True)
    lib.h2_cholesky(M, lib.trunc(1e-6))
    lib.h2_tri_invert(M, lib.trunc(1e-6))
    with pytest.raises(lib.H2Error) as ei:
        lib.h2_tri_invert(M, lib.trunc(1e-6))
    assert ei.value.name == "H2_ERR_ARG"
    # a copy keeps the form; assigning the factor back restores it
    C = lib.h2_mat_copy(M)
    assert lib.h2_mat_is_inverse(C)
    F = lib.h2_mat_from_csr(ctx, bt, p["A"], lower=True)
    lib.h2_mat_assign(C, F)
    assert not lib.h2_mat_is_inverse(C)
