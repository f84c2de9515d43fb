"""Launch-shape autotuner of the substitutions with a Cholesky factor
(h2_autotune_precond, h2_precond_config) through the C ABI.  The shape
(threads per workgroup) changes the time only: every shape gives the
default's result bit for bit, and that result equals the oracle's
preconditioner (Section 3 block substitutions) within 1e-12.  The tuning
cache reproduces the choice without timing for the same key."""
import numpy as np
import pytest

import workloads as w
from oracle.arith import cholesky as o_cholesky, precond_apply as o_precond
from oracle.h2 import TruncParams, from_csr as o_from_csr
from oracle.trees import build_block_tree, build_cluster_tree
from tests.helpers import gpu, rel2

pytestmark = pytest.mark.gpu
TOL = 1e-12
SHAPES = (128, 256, 512)


@pytest.fixture(scope="module")
def lib():
    gpu()
    from paper_1402_5056_amd import h2lr
    return h2lr


@pytest.fixture(scope="module")
def factor(lib):
    p = w.problem(48, sigma_seed=5, rhs_seed=48)
    ctx = lib.h2_ctx_create(0)
    ct = lib.h2_ctree_build(ctx, p["coords"], 32)
    bt = lib.h2_btree_build(ctx, ct, 2.0)
    M = lib.h2_mat_from_csr(ctx, bt, p["A"], lower=True)
    lib.h2_cholesky(M, lib.trunc(1e-4, "block_rel", 32))
    oc = build_cluster_tree(p["coords"], 32)
    L = o_cholesky(o_from_csr(p["A"], oc, build_block_tree(oc, 2.0), lower=True),
                   TruncParams(1e-4, "block_rel", 32))
    return p, ctx, M, L


def _apply(lib, torch, M, r):
    R = torch.tensor(np.ascontiguousarray(r.T), device="cuda")
    Z = torch.zeros_like(R)
    lib.h2_precond(M, R, Z)
    return Z.cpu().numpy()


def test_every_shape_gives_the_same_result(lib, factor):
    print("case: substitution launch shapes 128/256/512, nrhs 1 and 8, N=48", flush=True)
    torch = gpu()
    p, ctx, M, L = factor
    n = p["A"].shape[0]
    for nrhs in (1, 8):
        r = w.gaussian(n, nrhs, 70 + nrhs)
        lib.h2_precond_config(M, nrhs, 0)
        z0 = _apply(lib, torch, M, r)
        zref = np.stack([o_precond(L, r[:, i]) for i in range(nrhs)])
        err = rel2(z0, zref)
        print(f"  nrhs {nrhs}: default shape vs oracle {err:.2e}", flush=True)
        assert err < TOL
        for t in SHAPES:
            lib.h2_precond_config(M, nrhs, t)
            assert np.array_equal(_apply(lib, torch, M, r), z0), f"shape {t} changed the result"
        lib.h2_precond_config(M, nrhs, 0)
    with pytest.raises(lib.H2Error) as ei:
        lib.h2_precond_config(M, 1, 64)       # one wave: below the substitutions' two
    assert ei.value.name == "H2_ERR_ARG"


def test_autotune_and_cache(lib, factor, tmp_path):
    print("case: autotune nrhs 1 and 4 with a cache file, N=48", flush=True)
    torch = gpu()
    p, ctx, M, L = factor
    n = p["A"].shape[0]
    cache = str(tmp_path / "tune.txt")
    r = w.gaussian(n, 4, 81)
    lib.h2_precond_config(M, 4, 0)
    z0 = _apply(lib, torch, M, r)
    for nrhs in (1, 4):
        t, ms, cached, by = lib.h2_autotune_precond(M, nrhs, 3, cache)
        print(f"  nrhs {nrhs}: {t} threads, {ms:.3f} ms per application (by shape {by})", flush=True)
        assert t in SHAPES and ms > 0.0 and not cached
        assert set(by) == set(SHAPES) and ms == min(by.values())
    assert np.array_equal(_apply(lib, torch, M, r), z0)
    lines = open(cache).read().splitlines()
    assert len(lines) == 2 and all(len(ln.split()) == 3 for ln in lines)
    # the same key again (also on a copy of the matrix): taken from the cache
    t4 = int(lines[1].split()[1])
    C = lib.h2_mat_copy(M)
    for m in (M, C):
        t, ms, cached, by = lib.h2_autotune_precond(m, 4, 3, cache)
        assert cached and t == t4 and by == {}
    assert len(open(cache).read().splitlines()) == 2
    # PCG with the tuned shape: iterations and solution as with the default
    A = lib.h2_csr_create(ctx, p["A"])
    b = torch.tensor(p["b"], device="cuda")
    x1, x2 = torch.zeros_like(b), torch.zeros_like(b)
    it1, _, ok1 = lib.h2_pcg(A, M, b, x1, 1e-8, 100)
    lib.h2_precond_config(M, 1, 0)
    it2, _, ok2 = lib.h2_pcg(A, M, b, x2, 1e-8, 100)
    assert ok1 and ok2 and it1 == it2 and torch.equal(x1, x2)
