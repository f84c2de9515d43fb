"""The mixed-precision form (h2_trunc.precision = H2_PREC_MIXED): coupling
projections and transfer / basis-change products of every local update in
float on the matrix cores, QR / SVD / weights / nearfield / vector solves
in FP64.  Its factor is compared with the FP64 oracle (an error report, not
a parity claim), PCG in FP64 must reach the same iteration count and the
1e-8 residual.

Bar for the factor: float products carry a relative rounding error of about
K u_f (K <= 64 terms, u_f = 2^-24 = 6e-8), i.e. <= 4e-6 per product; the
recompressions that follow are FP64 and the truncation tolerance (1e-4 to
1e-6 here) is larger, so the factor must stay within 1e-4 of the FP64
oracle's in relative spectral norm (measured values are printed).  The
trial form H2_PREC_MIXED_BF16 also stores leaf bases at bfloat16 precision;
its error is reported and only bounded by 5e-2."""
import numpy as np
import pytest

import workloads as w
from oracle.arith import cholesky as o_cholesky, precond_apply as o_precond
from oracle.h2 import TruncParams, from_csr as o_from_csr, to_dense as o_to_dense
from oracle.solve import pcg as o_pcg
from oracle.trees import build_block_tree, build_cluster_tree
from tests.helpers import dense_via_matvec, gpu, rel2, to_original

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    gpu()
    from paper_1402_5056_amd import h2lr
    return h2lr


@pytest.mark.parametrize("N,seed,eps,leaf", [(32, 3, 1e-4, 32), (48, 5, 1e-6, 16)])
def test_mixed_cholesky_error_and_pcg(lib, N, seed, eps, leaf):
    print(f"case: mixed precision Cholesky N={N} eps={eps} leaf {leaf}", flush=True)
    torch = gpu()
    p = w.problem(N, sigma_seed=seed, rhs_seed=7)
    oc = build_cluster_tree(p["coords"], leaf)
    ob = build_block_tree(oc, 2.0)
    Lo = o_cholesky(o_from_csr(p["A"], oc, ob, lower=True), TruncParams(eps, "block_rel", 32))
    ctx = lib.h2_ctx_create(0)
    bt = lib.h2_btree_build(ctx, lib.h2_ctree_build(ctx, p["coords"], leaf), 2.0)
    out = {}
    for prec in ("fp64", "mixed", "mixed_bf16"):
        L = lib.h2_mat_from_csr(ctx, bt, p["A"], lower=True)
        lib.h2_cholesky(L, lib.trunc(eps, "block_rel", 32, precision=prec))
        D = np.tril(dense_via_matvec(lib, L, oc.n)[np.ix_(oc.perm, oc.perm)])
        Dref = np.tril(o_to_dense(Lo))
        A = lib.h2_csr_create(ctx, p["A"])
        b = torch.tensor(p["b"], device="cuda")
        x = torch.zeros_like(b)
        it, rel, ok = lib.h2_pcg(A, L, b, x, 1e-8, 100)
        res = np.linalg.norm(p["b"] - p["A"] @ x.cpu().numpy()) / np.linalg.norm(p["b"])
        out[prec] = (rel2(D, Dref), it, ok, res)
        print(f"  {prec}: ||L - L_oracle|| / ||L_oracle|| = {out[prec][0]:.2e}, PCG {it} iterations, "
              f"true residual {res:.2e}", flush=True)
    xo, ito, _ = o_pcg(p["A"], p["b"], lambda r: o_precond(Lo, r))
    assert out["fp64"][0] < 1e-12
    assert out["mixed"][0] < 1e-4
    assert out["mixed"][0] > out["fp64"][0]          # the float products are really used
    assert out["mixed"][2] and out["mixed"][1] == ito == out["fp64"][1]
    assert out["mixed"][3] < 1e-8
    # trial form with leaf bases at bfloat16 precision (u = 2^-9): its factor
    # error is of the order of that unit roundoff; PCG in FP64 still reaches
    # the tolerance, possibly in more steps
    assert out["mixed_bf16"][0] > out["mixed"][0]
    assert out["mixed_bf16"][0] < 5e-2
    assert out["mixed_bf16"][2] and out["mixed_bf16"][3] < 1e-8
