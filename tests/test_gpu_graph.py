"""Batched PCG replayed from a captured HIP graph (h2_pcg_batched_graph)
through the C ABI.  The graph form must give every column the iterates of
the launch-by-launch form (h2_pcg_batched) bit for bit: the same solutions,
iteration counts, residuals and statuses, including a zero right-hand side,
several right-hand sides per system and columns stopped by the iteration
limit.  The graph is replayed once per iteration with host reads in between
and the solve is repeated after other eager work; each repetition is checked.
One system is also checked against the oracle's PCG with the oracle's factor
(Section 7 protocol: same iteration count, solution within 1e-10)."""
import numpy as np
import pytest

import workloads as w
from oracle.arith import cholesky as o_cholesky, precond_apply as o_precond
from oracle.h2 import TruncParams, from_csr as o_from_csr
from oracle.solve import pcg as o_pcg
from oracle.trees import build_block_tree, build_cluster_tree
from tests.helpers import gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    gpu()
    from paper_1402_5056_amd import h2lr
    return h2lr


@pytest.fixture(scope="module")
def systems(lib):
    torch = gpu()
    ctx = lib.h2_ctx_create(0)
    tr = lib.trunc(1e-4, "block_rel", 32)
    out = []
    for side, sg, leaf, k in ((16, 7, 8, 1), (24, 3, 16, 3), (32, 4, 32, 2), (48, 5, 32, 4)):
        p = w.problem(side, sigma_seed=sg, rhs_seed=side)
        ct = lib.h2_ctree_build(ctx, p["coords"], leaf)
        bt = lib.h2_btree_build(ctx, ct, 2.0)
        M = lib.h2_mat_from_csr(ctx, bt, p["A"], lower=True)
        n = p["A"].shape[0]
        B = w.gaussian(n, k, 900 + side).T.copy()
        if side == 24:
            B[1] = 0.0                          # a zero right-hand side
        out.append({"p": p, "M": M, "csr": lib.h2_csr_create(ctx, p["A"]), "leaf": leaf,
                    "b": torch.tensor(B if k > 1 else B[0], device="cuda")})
    lib.h2_cholesky_batched([q["M"] for q in out], tr)
    return out


def _solve(lib, systems, rtol, maxit, graph):
    torch = gpu()
    xs = [torch.full_like(q["b"], 7.0) for q in systems]   # the solver clears x
    its, rels, codes = lib.h2_pcg_batched([q["csr"] for q in systems], [q["M"] for q in systems],
                                          [q["b"] for q in systems], xs, rtol, maxit, check=False, graph=graph)
    return xs, its, rels, codes


def test_graph_equals_eager(lib, systems):
    print("case: batched PCG, graph vs launch-by-launch, 4 systems, 10 columns", flush=True)
    torch = gpu()
    xe, ite, rele, ce = _solve(lib, systems, 1e-10, 200, False)
    assert ce == [0] * 10
    for rep in range(2):
        xg, itg, relg, cg = _solve(lib, systems, 1e-10, 200, True)
        print(f"  replay set {rep}: iterations {itg} (eager {ite})", flush=True)
        assert cg == ce and itg == ite and relg == rele
        for a, b in zip(xg, xe):
            assert torch.equal(a, b)
        # eager work between the repetitions
        q = systems[3]
        z = torch.empty_like(q["b"])
        lib.h2_precond(q["M"], q["b"], z)
        torch.cuda.synchronize()
    assert ite[2] == 0 and rele[2] == 0.0       # the zero right-hand side: x = 0 at once
    assert torch.count_nonzero(xe[1][1]) == 0


def test_graph_iteration_limit(lib, systems):
    print("case: batched PCG graph form, iteration limit 2", flush=True)
    torch = gpu()
    xe, ite, rele, ce = _solve(lib, systems, 1e-14, 2, False)
    xg, itg, relg, cg = _solve(lib, systems, 1e-14, 2, True)
    assert cg == ce and itg == ite and relg == rele
    assert -7 in cg                              # H2_ERR_NOT_CONVERGED
    for a, b in zip(xg, xe):
        assert torch.equal(a, b)


def test_graph_against_oracle(lib, systems):
    print("case: batched PCG graph form vs oracle PCG, side 32", flush=True)
    q = systems[2]
    p = q["p"]
    xg, itg, _, cg = _solve(lib, systems, 1e-8, 200, True)
    oc = build_cluster_tree(p["coords"], q["leaf"])
    L = o_cholesky(o_from_csr(p["A"], oc, build_block_tree(oc, 2.0), lower=True),
                   TruncParams(1e-4, "block_rel", 32))
    b = q["b"].cpu().numpy()
    for c in range(b.shape[0]):
        xo, ito, _ = o_pcg(p["A"], b[c], lambda v: o_precond(L, v))
        err = np.linalg.norm(xg[2][c].cpu().numpy() - xo) / np.linalg.norm(xo)
        print(f"  column {c}: iterations {itg[4 + c]} (oracle {ito}), x vs oracle {err:.2e}", flush=True)
        assert cg[4 + c] == 0 and itg[4 + c] == ito and err < 1e-10
