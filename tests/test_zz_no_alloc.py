"""h2_pcg_noalloc (PCG with the library's fixed device work area) against
h2_pcg on the same factor, through the C ABI: two calls in a row, the second
with a smaller system, so the second call runs on an area that still holds
the first call's (longer) vectors.  Both entries run the same kernels in the
same order, so iteration counts, residuals and solutions must agree."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as w
from tests.helpers import gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    gpu()
    from paper_1402_5056_amd import h2lr
    return h2lr


def _factor(lib, N, sigma_seed, rhs_seed):
    p = w.problem(N, sigma_seed=sigma_seed, rhs_seed=rhs_seed)
    ctx = lib.h2_ctx_create(0)
    ct = lib.h2_ctree_build(ctx, p["coords"], 32)
    bt = lib.h2_btree_build(ctx, ct, 2.0)
    L = lib.h2_mat_from_csr(ctx, bt, p["A"], lower=True)
    lib.h2_cholesky(L, lib.trunc(1e-4, "block_rel", 32))
    A = lib.h2_csr_create(ctx, p["A"])
    return p, ctx, A, L


def test_noalloc_equals_pcg_two_calls(lib):
    torch = gpu()
    results = []
    for N, ss, rs in ((48, 3, 4), (24, 5, 6)):          # n = 2209, then 529
        print(f"case: h2_pcg_noalloc vs h2_pcg, N={N}", flush=True)
        p, ctx, A, L = _factor(lib, N, ss, rs)
        b = torch.tensor(p["b"], device="cuda")
        x_ref = torch.zeros_like(b)
        it_ref, rel_ref, ok_ref = lib.h2_pcg(A, L, b, x_ref, 1e-8, 200)
        x = torch.full_like(b, 7.0)                          # cleared by the call
        it, rel, ok = lib.h2_pcg_noalloc(A, L, b, x, 1e-8, 200)
        torch.cuda.synchronize()
        assert ok and ok_ref
        assert it == it_ref and rel == rel_ref
        xr, xn = x_ref.cpu().numpy(), x.cpu().numpy()
        assert np.linalg.norm(xn - xr) / np.linalg.norm(xr) <= 1e-12
        assert np.linalg.norm(p["b"] - p["A"] @ xn) / np.linalg.norm(p["b"]) < 1e-8
        results.append((N, it, float(np.max(np.abs(xn - xr)))))
    print("noalloc results (N, iterations, max |x - x_pcg|):", results, flush=True)


def test_noalloc_requires_planned_preconditioner(lib):
    torch = gpu()
    p, ctx, A, L = _factor(lib, 16, 1, 2)
    b = torch.tensor(p["b"], device="cuda")
    x = torch.zeros_like(b)
    with pytest.raises(lib.H2Error) as ei:
        lib.h2_pcg_noalloc(A, L, b, x, 1e-8, 50)
    assert ei.value.status == -1 and "not planned" in str(ei.value)
    lib.h2_pcg(A, L, b, x, 1e-8, 50)                         # plans it
    it, rel, ok = lib.h2_pcg_noalloc(A, L, b, x, 1e-8, 50)
    assert ok and rel <= 1e-8


def test_noalloc_rejects_too_large_system(lib):
    """A 1-D system one unknown larger than the work area: the size check
    fails before any device work."""
    torch = gpu()
    n = lib.NOALLOC_MAX_N + 1
    coords = np.arange(1, n + 1, dtype=np.int32).reshape(n, 1)
    A = sp.diags([-np.ones(n - 1), 2.0 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="csr")
    ctx = lib.h2_ctx_create(0)
    ct = lib.h2_ctree_build(ctx, coords, 32)
    bt = lib.h2_btree_build(ctx, ct, 2.0)
    L = lib.h2_mat_from_csr(ctx, bt, A, lower=True)
    Ad = lib.h2_csr_create(ctx, A)
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    with pytest.raises(lib.H2Error) as ei:
        lib.h2_pcg_noalloc(Ad, L, b, x, 1e-8, 10)
    assert ei.value.status == -1 and "H2_NOALLOC_MAX_N" in str(ei.value)
