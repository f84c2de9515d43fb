"""Batched H^2-Cholesky: independent problems of different sizes factorised
in one launch (one workgroup each) through the C ABI.  Each factor must equal
the one h2_cholesky makes alone (same arithmetic, bit for bit) and the CPU
oracle's within 1e-12 relative spectral error in FP64."""
import numpy as np
import pytest

import workloads as w
from oracle.arith import cholesky as o_cholesky
from oracle.h2 import TruncParams, from_csr as o_from_csr, to_dense as o_to_dense
from oracle.solve import pcg as o_pcg
from oracle.arith import precond_apply as o_precond
from oracle.trees import build_block_tree, build_cluster_tree
from tests.helpers import dense_via_matvec, gpu, rel2, to_original

pytestmark = pytest.mark.gpu
TOL = 1e-12

# (grid side, coefficient seed, leaf size, eta, domain decomposition): balanced,
# unbalanced (leaves on two levels) and domain-decomposition trees
CASES = [(16, 7, 8, 2.0, False), (24, 3, 16, 2.0, False), (32, None, 32, 2.0, False),
         (40, 7, 24, 2.0, False), (33, None, 32, 4.0, True), (48, 5, 32, 2.0, False)]


@pytest.fixture(scope="module")
def lib():
    gpu()
    from paper_1402_5056_amd import h2lr
    return h2lr


def _problem(lib, ctx, side, sigma_seed, leaf, eta, dd, negate=False):
    p = w.problem(side, sigma_seed=sigma_seed, rhs_seed=side)
    A = -p["A"] if negate else p["A"]
    ct = (lib.h2_ctree_build_dd if dd else lib.h2_ctree_build)(ctx, p["coords"], leaf)
    bt = lib.h2_btree_build(ctx, ct, eta)
    return p, A, bt


def test_batched_equals_single_and_oracle(lib):
    print("case: batched cholesky of 6 problems (sides 16..48)", flush=True)
    ctx = lib.h2_ctx_create(0)
    eps = 1e-5
    tr = lib.trunc(eps, "block_rel", 32)
    probs, batch, single = [], [], []
    for side, sg, leaf, eta, dd in CASES:
        p, A, bt = _problem(lib, ctx, side, sg, leaf, eta, dd)
        probs.append((p, A, side, sg, leaf, eta, dd))
        batch.append(lib.h2_mat_from_csr(ctx, bt, A, lower=True))
        single.append(lib.h2_mat_from_csr(ctx, bt, A, lower=True))
    codes = lib.h2_cholesky_batched(batch, tr)
    assert codes == [0] * len(CASES)
    for (p, A, side, sg, leaf, eta, dd), Mb, Ms in zip(probs, batch, single):
        lib.h2_cholesky(Ms, tr)
        n = A.shape[0]
        Db = dense_via_matvec(lib, Mb, n)
        Ds = dense_via_matvec(lib, Ms, n)
        assert np.array_equal(Db, Ds), f"side {side}: batched factor differs from the single one"
        assert lib.h2_mat_stats(Mb) == lib.h2_mat_stats(Ms)
        oc = build_cluster_tree(p["coords"], leaf, dd=dd)
        ob = build_block_tree(oc, eta)
        L = o_cholesky(o_from_csr(A, oc, ob, lower=True), TruncParams(eps, "block_rel", 32))
        err = rel2(Db, to_original(np.tril(o_to_dense(L)), oc.perm))
        print(f"  side {side} leaf {leaf} dd {dd}: ||L_batch - L_oracle||_2 / ||L_oracle||_2 = {err:.3e}",
              flush=True)
        assert err < TOL


def test_batched_pcg(lib):
    print("case: pcg with batched factors (sides 24, 32)", flush=True)
    torch = gpu()
    ctx = lib.h2_ctx_create(0)
    tr = lib.trunc(1e-4, "block_rel", 32)
    items = []
    for side, sg, leaf in ((24, 3, 16), (32, 4, 32)):
        p, A, bt = _problem(lib, ctx, side, sg, leaf, 2.0, False)
        items.append((p, A, leaf, lib.h2_mat_from_csr(ctx, bt, A, lower=True)))
    lib.h2_cholesky_batched([m for *_, m in items], tr)
    for p, A, leaf, M in items:
        oc = build_cluster_tree(p["coords"], leaf)
        ob = build_block_tree(oc, 2.0)
        L = o_cholesky(o_from_csr(A, oc, ob, lower=True), TruncParams(1e-4, "block_rel", 32))
        csr = lib.h2_csr_create(ctx, A)
        b = torch.tensor(p["b"], device="cuda")
        x = torch.zeros_like(b)
        it, rel, ok = lib.h2_pcg(csr, M, b, x, 1e-8, 100)
        xo, ito, _ = o_pcg(A, p["b"], lambda v: o_precond(L, v))
        print(f"  n={A.shape[0]}: pcg iterations batched {it} oracle {ito}", flush=True)
        assert ok and it == ito
        assert np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo) < 1e-10


def test_batched_failure_is_per_matrix(lib):
    """A matrix that is not positive definite fails alone: its status is
    H2_ERR_NOT_SPD and it is poisoned; the others are factorised."""
    print("case: batched cholesky with one negated (not SPD) matrix", flush=True)
    ctx = lib.h2_ctx_create(0)
    tr = lib.trunc(1e-6, "block_rel", 32)
    mats, ref = [], []
    for i, (side, sg, leaf) in enumerate(((16, 7, 8), (24, 3, 16), (16, 5, 8))):
        p, A, bt = _problem(lib, ctx, side, sg, leaf, 2.0, False, negate=(i == 1))
        mats.append(lib.h2_mat_from_csr(ctx, bt, A, lower=True))
        ref.append((A, lib.h2_mat_from_csr(ctx, bt, A, lower=True)))
    with pytest.raises(lib.H2Error) as ei:
        lib.h2_cholesky_batched(mats, tr)
    assert ei.value.name == "H2_ERR_NOT_SPD"
    assert "matrix 1" in str(ei.value)
    for i in (0, 2):
        A, Ms = ref[i]
        lib.h2_cholesky(Ms, tr)
        n = A.shape[0]
        assert np.array_equal(dense_via_matvec(lib, mats[i], n), dense_via_matvec(lib, Ms, n))
    with pytest.raises(lib.H2Error) as ei:
        lib.h2_cholesky(mats[1], tr)
    assert ei.value.name == "H2_ERR_STATE"


def test_batched_argument_errors(lib):
    print("case: batched cholesky argument errors", flush=True)
    ctx = lib.h2_ctx_create(0)
    p, A, bt = _problem(lib, ctx, 16, 7, 8, 2.0, False)
    M = lib.h2_mat_from_csr(ctx, bt, A, lower=True)
    full = lib.h2_mat_from_csr(ctx, bt, A, lower=False)
    tr = lib.trunc(1e-6)
    for mats in ([M, M], [full], []):
        with pytest.raises(lib.H2Error) as ei:
            lib.h2_cholesky_batched(mats, tr)
        assert ei.value.name == "H2_ERR_ARG"


def test_pcg_batched_equals_single(lib):
    """Batched PCG (one preconditioner launch for all unconverged systems)
    gives each system the iterates of its single solve."""
    print("case: batched pcg of 4 systems vs single solves", flush=True)
    torch = gpu()
    ctx = lib.h2_ctx_create(0)
    tr = lib.trunc(1e-4, "block_rel", 32)
    probs = []
    for side, sg, leaf in ((16, 7, 8), (24, 3, 16), (32, 4, 32), (48, 5, 32)):
        p, A, bt = _problem(lib, ctx, side, sg, leaf, 2.0, False)
        M = lib.h2_mat_from_csr(ctx, bt, A, lower=True)
        probs.append((p, A, M, lib.h2_csr_create(ctx, A)))
    lib.h2_cholesky_batched([q[2] for q in probs], tr)
    bs = [torch.tensor(q[0]["b"], device="cuda") for q in probs]
    xs = [torch.zeros_like(b) for b in bs]
    its, rels, codes = lib.h2_pcg_batched([q[3] for q in probs], [q[2] for q in probs], bs, xs, 1e-10, 200)
    assert codes == [0] * len(probs)
    for (p, A, M, csr), b, x, it, rel in zip(probs, bs, xs, its, rels):
        x1 = torch.zeros_like(b)
        it1, rel1, ok = lib.h2_pcg(csr, M, b, x1, 1e-10, 200)
        print(f"  n={A.shape[0]}: iterations batched {it} single {it1}", flush=True)
        assert ok and it == it1 and rel == rel1
        assert torch.equal(x, x1)
        xr = x.cpu().numpy()
        assert np.linalg.norm(p["b"] - A @ xr) / np.linalg.norm(p["b"]) < 1e-9


def test_pcg_batched_not_converged(lib):
    print("case: batched pcg with maxit 1", flush=True)
    torch = gpu()
    ctx = lib.h2_ctx_create(0)
    p, A, bt = _problem(lib, ctx, 24, 3, 16, 2.0, False)
    M = lib.h2_mat_from_csr(ctx, bt, A, lower=True)
    lib.h2_cholesky(M, lib.trunc(1e-2, "block_rel", 32))
    b = torch.tensor(p["b"], device="cuda")
    x = torch.zeros_like(b)
    its, rels, codes = lib.h2_pcg_batched([lib.h2_csr_create(ctx, A)], [M], [b], [x], 1e-14, 1, check=False)
    assert its == [1] and codes == [-7]


def test_launch_overlapping_streams(lib):
    """Two launches on two streams are in flight together; their matrices
    are busy until finish; each factor equals the single one."""
    print("case: two launched batches on two streams", flush=True)
    torch = gpu()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    c1 = lib.h2_ctx_create(0, s1.cuda_stream)
    c2 = lib.h2_ctx_create(0, s2.cuda_stream)
    c0 = lib.h2_ctx_create(0)
    tr = lib.trunc(1e-5, "block_rel", 32)
    groups = []
    for ctx, sides in ((c1, ((32, 4, 32), (16, 7, 8))), (c2, ((24, 3, 16), (40, 7, 24)))):
        g = []
        for side, sg, leaf in sides:
            p, A, bt = _problem(lib, ctx, side, sg, leaf, 2.0, False)
            p0, A0, bt0 = _problem(lib, c0, side, sg, leaf, 2.0, False)
            g.append((A, lib.h2_mat_from_csr(ctx, bt, A, lower=True), lib.h2_mat_from_csr(c0, bt0, A0, lower=True)))
        groups.append(g)
    torch.cuda.synchronize()
    j1 = lib.h2_cholesky_launch([q[1] for q in groups[0]], tr)
    j2 = lib.h2_cholesky_launch([q[1] for q in groups[1]], tr)
    with pytest.raises(lib.H2Error) as ei:
        lib.h2_cholesky(groups[0][0][1], tr)
    assert ei.value.name == "H2_ERR_ARG"
    j1.done()
    j2.done()
    assert j2.finish() == [0, 0]
    assert j1.finish() == [0, 0]
    for g in groups:
        for A, M, Ms in g:
            lib.h2_cholesky(Ms, tr)
            n = A.shape[0]
            assert np.array_equal(dense_via_matvec(lib, M, n), dense_via_matvec(lib, Ms, n))


def test_pcg_batched_multi_rhs(lib):
    """Several right-hand sides per system: one CG iteration per column, the
    columns of a system share its preconditioner launches; each column
    matches the single-column solve (iteration count, solution within
    1e-12 relative)."""
    print("case: batched pcg with 1, 5 and 16 right-hand sides", flush=True)
    torch = gpu()
    ctx = lib.h2_ctx_create(0)
    tr = lib.trunc(1e-4, "block_rel", 32)
    probs = []
    for (side, sg, leaf), k in zip(((16, 7, 8), (24, 3, 16), (32, 4, 32)), (1, 5, 16)):
        p, A, bt = _problem(lib, ctx, side, sg, leaf, 2.0, False)
        M = lib.h2_mat_from_csr(ctx, bt, A, lower=True)
        B = w.gaussian(A.shape[0], k, 50 + side)
        probs.append((A, M, lib.h2_csr_create(ctx, A), B))
    lib.h2_cholesky_batched([q[1] for q in probs], tr)
    bs = [torch.tensor(np.ascontiguousarray(q[3].T), device="cuda") for q in probs]
    xs = [torch.zeros_like(b) for b in bs]
    its, rels, codes = lib.h2_pcg_batched([q[2] for q in probs], [q[1] for q in probs], bs, xs, 1e-10, 200)
    assert len(its) == 22 and codes == [0] * 22
    pos = 0
    for (A, M, csr, B), b, x in zip(probs, bs, xs):
        X = x.cpu().numpy().T
        for c in range(B.shape[1]):
            b1 = torch.tensor(B[:, c], device="cuda")
            x1 = torch.zeros_like(b1)
            it1, _, ok = lib.h2_pcg(csr, M, b1, x1, 1e-10, 200)
            x1 = x1.cpu().numpy()
            err = np.linalg.norm(X[:, c] - x1) / np.linalg.norm(x1)
            assert ok and its[pos] == it1, (pos, its[pos], it1)
            assert err < 1e-12, (pos, err)
            assert np.linalg.norm(B[:, c] - A @ X[:, c]) / np.linalg.norm(B[:, c]) < 1e-9
            pos += 1
    print(f"  iterations per column {its}", flush=True)


def test_update_batched_equals_single_and_oracle(lib):
    """Up to four local updates per matrix, all matrices in one launch: each
    result equals the single h2_lowrank_update calls in the same order bit
    for bit, and the oracle's sequence of updates within 1e-12."""
    from oracle.update import addlr as o_addlr
    from tests.helpers import to_dev_cols
    print("case: batched low-rank updates (sides 24, 32, 40; 4, 3, 4 updates)", flush=True)
    ctx = lib.h2_ctx_create(0)
    eps = 1e-6
    tr = lib.trunc(eps, "block_rel", 32)
    tp = TruncParams(eps, "block_rel", 32)
    mats, singles, updates, refs = [], [], [], []
    for (side, sg, leaf), nup in zip(((24, 3, 16), (32, 4, 32), (40, 7, 24)), (4, 3, 4)):
        p, A, bt = _problem(lib, ctx, side, sg, leaf, 2.0, False)
        mats.append(lib.h2_mat_from_csr(ctx, bt, A))
        singles.append(lib.h2_mat_from_csr(ctx, bt, A))
        oc = build_cluster_tree(p["coords"], leaf)
        ob = build_block_tree(oc, 2.0)
        sons = [b for b in range(ob.nb) if ob.parent[b] == 0]
        ups, Z = [], o_from_csr(A, oc, ob)
        for j in range(nup):
            b = sons[j % len(sons)]
            t, s = int(ob.row[b]), int(ob.col[b])
            X = w.gaussian(int(oc.size[t]), 3 + j, 300 + side + j) * np.logspace(0, -3, 3 + j)
            Y = w.gaussian(int(oc.size[s]), 3 + j, 400 + side + j)
            margins = []
            o_addlr(Z, b, X, Y, tp, margins)
            assert not margins or min(margins) > 1e-8, "seed too close to the truncation threshold"
            ups.append((b, to_dev_cols(X), to_dev_cols(Y)))
        updates.append(ups)
        refs.append((A.shape[0], oc, Z))
    codes = lib.h2_lowrank_update_batched(mats, updates, tr)
    assert codes == [0, 0, 0]
    for M, Ms, ups, (n, oc, Z) in zip(mats, singles, updates, refs):
        for b, X, Y in ups:
            lib.h2_lowrank_update(Ms, b, X, Y, tr)
        D = dense_via_matvec(lib, M, n)
        assert np.array_equal(D, dense_via_matvec(lib, Ms, n))
        err = rel2(D, to_original(o_to_dense(Z), oc.perm))
        print(f"  n={n}: ||Z_batch - Z_oracle||_2 / ||Z_oracle||_2 = {err:.3e}", flush=True)
        assert err < TOL


def test_update_batched_argument_errors(lib):
    print("case: batched update argument errors", flush=True)
    from tests.helpers import to_dev_cols
    ctx = lib.h2_ctx_create(0)
    p, A, bt = _problem(lib, ctx, 16, 7, 8, 2.0, False)
    M = lib.h2_mat_from_csr(ctx, bt, A)
    L = lib.h2_mat_from_csr(ctx, bt, A, lower=True)
    X = to_dev_cols(w.gaussian(225, 2, 1))
    tr = lib.trunc(1e-6)
    bad = [([M], [[(10 ** 6, X, X)]]),                 # block out of range
           ([M], [[(0, X, X)] * 5]),                   # more than four updates
           ([M, M], [[(0, X, X)], [(0, X, X)]])]      # same matrix twice
    for mats, ups in bad:
        with pytest.raises(lib.H2Error) as ei:
            lib.h2_lowrank_update_batched(mats, ups, tr)
        assert ei.value.name == "H2_ERR_ARG"
    # above the diagonal of a lower-stored matrix
    ex = lib.h2_btree_export(bt)
    above = next(b for b in range(len(ex["row"])) if ex["row"][b] < ex["col"][b])
    with pytest.raises(lib.H2Error) as ei:
        lib.h2_lowrank_update_batched([L], [[(above, X, X)]], tr)
    assert ei.value.name == "H2_ERR_ARG"


def test_update_and_cholesky_one_launch(lib):
    """Local updates of full-storage matrices and Cholesky factorisations of
    other matrices in one launch (h2_update_cholesky_launch): every result
    equals the separate batched calls bit for bit (same task lists, same
    arithmetic), and the factors equal the oracle's within 1e-12."""
    from tests.helpers import to_dev_cols
    print("case: updates + Cholesky in one launch (sides 24, 32, 40)", flush=True)
    ctx = lib.h2_ctx_create(0)
    eps = 1e-6
    tr = lib.trunc(eps, "block_rel", 32)
    U, Us, L, Ls, updates, refs = [], [], [], [], [], []
    for (side, sg, leaf), nup in zip(((24, 3, 16), (32, 4, 32), (40, 7, 24)), (4, 3, 2)):
        p, A, bt = _problem(lib, ctx, side, sg, leaf, 2.0, False)
        U.append(lib.h2_mat_from_csr(ctx, bt, A))
        Us.append(lib.h2_mat_from_csr(ctx, bt, A))
        L.append(lib.h2_mat_from_csr(ctx, bt, A, lower=True))
        Ls.append(lib.h2_mat_from_csr(ctx, bt, A, lower=True))
        ex = lib.h2_btree_export(bt)
        tree = lib.h2_ctree_export(lib.h2_ctree_build(ctx, p["coords"], leaf))
        sons = [b for b in range(len(ex["parent"])) if ex["parent"][b] == 0]
        ups = []
        for j in range(nup):
            b = sons[j % len(sons)]
            X = w.gaussian(int(tree["size"][ex["row"][b]]), 4, 500 + side + j)
            Y = w.gaussian(int(tree["size"][ex["col"][b]]), 4, 600 + side + j)
            ups.append((b, to_dev_cols(X), to_dev_cols(Y)))
        updates.append(ups)
        oc = build_cluster_tree(p["coords"], leaf)
        refs.append((A.shape[0], oc, o_from_csr(A, oc, build_block_tree(oc, 2.0), lower=True)))
    job = lib.h2_update_cholesky_launch(U, updates, L, tr)
    assert job.finish() == [0] * 6
    assert lib.h2_lowrank_update_batched(Us, updates, tr) == [0, 0, 0]
    assert lib.h2_cholesky_batched(Ls, tr) == [0, 0, 0]
    tp = TruncParams(eps, "block_rel", 32)
    for M, Ms, F, Fs, (n, oc, H) in zip(U, Us, L, Ls, refs):
        assert np.array_equal(dense_via_matvec(lib, M, n), dense_via_matvec(lib, Ms, n))
        D = dense_via_matvec(lib, F, n)
        assert np.array_equal(D, dense_via_matvec(lib, Fs, n))
        err = rel2(D, to_original(o_to_dense(o_cholesky(H, tp)), oc.perm))
        print(f"  n={n}: updates equal, factor equal, ||L - L_oracle||_2 / ||L_oracle||_2 = {err:.3e}", flush=True)
        assert err < TOL
    # argument errors: a matrix in both lists, nothing to do
    with pytest.raises(lib.H2Error) as ei:
        lib.h2_update_cholesky_launch([L[0]], [[]], [L[0]], tr)
    assert ei.value.name == "H2_ERR_ARG"
    with pytest.raises(lib.H2Error) as ei:
        lib.h2_update_cholesky_launch([], [], [], tr)
    assert ei.value.name == "H2_ERR_ARG"
