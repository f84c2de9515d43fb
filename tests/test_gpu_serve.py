"""Serving loop (continuous batching): every request's result is the same
alone and in the mix, the HBM budget is respected, oversized requests are
rejected.  Results are compared with the single-request run (same arithmetic,
so equal within 1e-12 relative, expected bit for bit) and with the CPU
oracle's PCG solution (1e-10 relative)."""
import numpy as np
import pytest

import workloads as w
from oracle.arith import cholesky as o_cholesky, precond_apply as o_precond
from oracle.h2 import TruncParams, from_csr as o_from_csr
from oracle.solve import pcg as o_pcg
from oracle.trees import build_block_tree, build_cluster_tree
from tests.helpers import gpu

pytestmark = pytest.mark.gpu
TOL_MIX = 1e-12


@pytest.fixture(scope="module")
def serve():
    gpu()
    from paper_1402_5056_amd import serve as s
    return s


def _requests(serve, specs, rids=None):
    out = []
    for i, (arrival, side, sg, nrhs) in enumerate(specs):
        rid = i if rids is None else rids[i]
        p = w.problem(side, sigma_seed=sg, rhs_seed=100 + rid)
        B = w.gaussian(p["A"].shape[0], nrhs, 200 + rid)
        out.append(serve.Request(rid, arrival, p["A"], p["coords"], B))
    return out


SPECS = [(0.0, 16, 7, 1), (0.0, 24, 3, 2), (0.01, 32, 4, 3), (0.02, 16, 5, 2), (0.05, 40, 7, 1),
         (0.06, 24, None, 3), (0.3, 32, 1, 1)]


def test_serve_mix_equals_alone(serve):
    print("case: serving mix of 7 requests, 2 slots", flush=True)
    server = serve.Server(8 << 30, eps=1e-5, leaf=16, rtol=1e-10, slots=2, max_batch=3)
    reqs = server.run(_requests(serve, SPECS), log=lambda m: print("  " + m, flush=True))
    assert all(r.status == "done" for r in reqs), [(r.rid, r.status, r.error) for r in reqs]
    print(f"  launches {server.launches}, max in flight {server.max_inflight}, latency "
          f"{serve.latency_summary(reqs)}", flush=True)
    assert server.launches >= 2
    assert server.max_inflight >= 2
    assert server.used == 0
    for r in reqs:
        alone = serve.Server(8 << 30, eps=1e-5, leaf=16, rtol=1e-10, slots=1)
        (a,) = alone.run(_requests(serve, [(0.0,) + SPECS[r.rid][1:]], rids=[r.rid]))
        a_rel = np.linalg.norm(r.result - a.result) / np.linalg.norm(a.result)
        print(f"  request {r.rid}: n={r.A.shape[0]} nrhs={r.B.shape[1]} iters {r.iters}, "
              f"||x_mix - x_alone|| / ||x_alone|| = {a_rel:.2e}", flush=True)
        assert a.status == "done" and a.iters == r.iters
        assert a_rel <= TOL_MIX
        # the oracle: same factor and PCG on the CPU
        oc = build_cluster_tree(r.coords, 16)
        ob = build_block_tree(oc, 2.0)
        L = o_cholesky(o_from_csr(r.A, oc, ob, lower=True), TruncParams(1e-5, "block_rel", 32))
        for j in range(r.B.shape[1]):
            xo, ito, _ = o_pcg(r.A, r.B[:, j], lambda v: o_precond(L, v), rtol=1e-10)
            assert ito == r.iters[j]
            assert np.linalg.norm(r.result[:, j] - xo) / np.linalg.norm(xo) < 1e-10


def test_serve_admits_while_running(serve):
    """Continuous batching: a large request occupies one launch slot; small
    requests arriving later are admitted, factorised, solved and released on
    the other slot while the large launch is still running."""
    print("case: small requests served while a large one runs", flush=True)
    specs = [(0.0, 96, 1, 1), (0.05, 16, 2, 1), (0.1, 16, 3, 2), (0.15, 24, 4, 1)]
    server = serve.Server(8 << 30, leaf=32, slots=2, max_batch=1)
    reqs = server.run(_requests(serve, specs), log=lambda m: print("  " + m, flush=True))
    assert all(r.status == "done" for r in reqs), [(r.rid, r.status, r.error) for r in reqs]
    big = reqs[0]
    early = [r.rid for r in reqs[1:] if r.t_done < big.t_done]
    print(f"  large request done at {big.t_done:.2f}s; small ones done before it: {early}; "
          f"admitted while a launch ran: {server.admitted_in_flight}", flush=True)
    assert len(early) >= 2
    assert server.admitted_in_flight >= 2 and server.max_inflight == 2
    assert server.used == 0
    for r in reqs:
        for j in range(r.B.shape[1]):
            x = r.result[:, j]
            assert np.linalg.norm(r.B[:, j] - r.A @ x) / np.linalg.norm(r.B[:, j]) < 1e-8


def test_serve_budget_and_rejection(serve):
    print("case: serving under a budget that holds one request", flush=True)
    specs = [(0.0, 24, 3, 1), (0.0, 24, 5, 1), (0.0, 16, 7, 2), (0.0, 64, 1, 1)]
    probe = serve.Server(1 << 40, leaf=16, slots=1)
    reqs = _requests(serve, specs)
    est = [probe._estimate(r) for r in reqs]
    budget = max(est[:3]) + 1
    assert est[3] > budget
    server = serve.Server(budget, leaf=16, slots=2, max_batch=4)
    reqs = server.run(_requests(serve, specs))
    assert [r.status for r in reqs] == ["done", "done", "done", "rejected"]
    assert server.peak <= budget
    assert server.launches == 3     # one request held at a time
    for r in reqs[:3]:
        x = r.result[:, 0]
        assert np.linalg.norm(r.B[:, 0] - r.A @ x) / np.linalg.norm(r.B[:, 0]) < 1e-7


def test_estimate_equals_allocation():
    """h2_estimate_bytes (used for admission) equals the device bytes a new
    matrix holds; task lists and PCG vectors come on top afterwards."""
    print("case: byte estimate vs allocation", flush=True)
    torch = gpu()
    from paper_1402_5056_amd import h2lr
    ctx = h2lr.h2_ctx_create(0)
    for side, leaf, lower in ((24, 16, True), (32, 32, False)):
        p = w.problem(side, sigma_seed=3, rhs_seed=1)
        ct = h2lr.h2_ctree_build(ctx, p["coords"], leaf)
        bt = h2lr.h2_btree_build(ctx, ct, 2.0)
        est = h2lr.h2_estimate_bytes(bt, lower)
        M = h2lr.h2_mat_from_csr(ctx, bt, p["A"], lower=lower)
        assert h2lr.h2_mat_bytes(M) == est
        if lower:
            h2lr.h2_cholesky(M, h2lr.trunc(1e-4))
            after = h2lr.h2_mat_bytes(M)
            assert after > est
            b = torch.tensor(p["b"], device="cuda")
            x = torch.zeros_like(b)
            h2lr.h2_pcg(h2lr.h2_csr_create(ctx, p["A"]), M, b, x, 1e-8, 100)
            assert h2lr.h2_mat_bytes(M) > after
