"""Pins of the accumulated local update (oracle.update.addlr_accumulated):
several updates merged into one local update of the smallest block that
contains all targets (the accumulation variant of the truncation
strategies, last paragraph of Section 4; the grouping is a reading).

* The merge block is the smallest block of the block tree containing every
  target, against a brute-force search over all blocks by index ranges.
* Without truncation the result is exactly Z + sum_i X_i Y_i^* on the
  targets' index ranges (and unchanged elsewhere), for full and
  lower-stored matrices, and equal to the sequence of single updates.
* With truncation every admissible block stays within the blockwise
  relative bound of the exact sum, and the error falls with eps.
* A planted misplacement of the merged factor's rows (rolled by one row)
  breaks the exactness pin.
* In products (Cholesky): accumulated temporaries (TruncParams.accumulate)
  keep the exact factor without truncation with fewer updates, keep the
  O(eps) accuracy and the PCG count with truncation, and group by rank as
  stated."""
import numpy as np
import pytest

import workloads as w
import oracle.update as U
from oracle.h2 import TruncParams, from_csr, to_dense
from oracle.trees import ADM, build_block_tree, build_cluster_tree
from oracle.update import addlr, addlr_accumulated, common_block


@pytest.fixture(scope="module")
def sq32():
    p = w.problem("p1_square_32")
    ct = build_cluster_tree(p["coords"], 32)
    bt = build_block_tree(ct, 2.0)
    return p, ct, bt


def _rel2(A, B):
    return np.linalg.norm(A - B, 2) / max(np.linalg.norm(B, 2), 1e-300)


def _contains(ct, bt, a, b):
    """Block a contains block b (index ranges)."""
    ta, sa, tb, sb = int(bt.row[a]), int(bt.col[a]), int(bt.row[b]), int(bt.col[b])
    (a0, a1), (c0, c1) = ct.rng(ta), ct.rng(sa)
    (b0, b1), (d0, d1) = ct.rng(tb), ct.rng(sb)
    return a0 <= b0 and b1 <= a1 and c0 <= d0 and d1 <= c1


def test_common_block_brute_force(sq32):
    p, ct, bt = sq32
    rng = np.random.default_rng(5)
    for _ in range(40):
        m = int(rng.integers(1, 5))
        blocks = [int(b) for b in rng.choice(bt.nb, size=m, replace=False)]
        cands = [a for a in range(bt.nb) if all(_contains(ct, bt, a, b) for b in blocks)]
        best = min(cands, key=lambda a: int(ct.size[bt.row[a]]) * int(ct.size[bt.col[a]]))
        assert common_block(bt, blocks) == best


def _targets(ct, bt, lower):
    adm = [b for b in range(bt.nb) if bt.kind[b] == ADM and (not lower or bt.is_lower(b))]
    # three admissible leaves below one off-diagonal block, two far apart,
    # and a pair whose smallest common block is a diagonal block below the root
    diag = next([a, b] for a in adm for b in adm
                if a < b and common_block(bt, [a, b]) != 0
                and bt.row[common_block(bt, [a, b])] == bt.col[common_block(bt, [a, b])])
    return [adm[5], adm[6], adm[9]], [adm[2], adm[30]], diag


def _updates(ct, bt, blocks, seed):
    ups = []
    for i, b in enumerate(blocks):
        t, s = int(bt.row[b]), int(bt.col[b])
        ups.append((b, w.gaussian(int(ct.size[t]), 2 + i, seed + i), w.gaussian(int(ct.size[s]), 2 + i, seed + 50 + i)))
    return ups


def _dense_sum(ct, bt, D0, ups):
    ref = D0.copy()
    for b, X, Y in ups:
        a0, a1 = ct.rng(int(bt.row[b]))
        c0, c1 = ct.rng(int(bt.col[b]))
        ref[a0:a1, c0:c1] += X @ Y.T
    return ref


@pytest.mark.parametrize("lower", [False, True])
def test_accumulated_exact(sq32, lower):
    p, ct, bt = sq32
    for group in _targets(ct, bt, lower):
        Z = from_csr(p["A"], ct, bt, lower=lower)
        Zs = Z.copy()
        D0 = to_dense(Z)
        ups = _updates(ct, bt, group, 40)
        bs = addlr_accumulated(Z, ups, TruncParams(0.0, "none", 1000))
        assert all(_contains(ct, bt, bs, b) for b in group)
        ref = _dense_sum(ct, bt, D0, ups)
        D = to_dense(Z)
        if lower:
            D, ref = np.tril(D), np.tril(ref)
        assert _rel2(D, ref) < 1e-13
        for b, X, Y in ups:
            addlr(Zs, b, X, Y, TruncParams(0.0, "none", 1000))
        Ds = np.tril(to_dense(Zs)) if lower else to_dense(Zs)
        assert _rel2(D, Ds) < 1e-13


def test_accumulated_truncated_bound(sq32):
    p, ct, bt = sq32
    group = _targets(ct, bt, False)[0]
    errs = []
    for eps in (1e-2, 1e-4, 1e-6):
        Z = from_csr(p["A"], ct, bt)
        D0 = to_dense(Z)
        ups = [(b, X * np.logspace(0, -4, X.shape[1]), Y) for b, X, Y in _updates(ct, bt, group, 70)]
        addlr_accumulated(Z, ups, TruncParams(eps, "block_rel", 64))
        D = to_dense(Z)
        ref = _dense_sum(ct, bt, D0, ups)
        for b in Z.adm:
            t, s = int(bt.row[b]), int(bt.col[b])
            a0, a1 = ct.rng(t); c0, c1 = ct.rng(s)
            e = np.linalg.norm(D[a0:a1, c0:c1] - ref[a0:a1, c0:c1], 2)
            assert e <= 2 * (ct.depth + 1) * eps * np.linalg.norm(ref[a0:a1, c0:c1]) + 1e-14
        errs.append(_rel2(D, ref))
    assert errs[0] > errs[1] > errs[2]


def test_planted_misplacement_fails(sq32, monkeypatch):
    """Roll the merged factor's rows by one: the exactness pin must notice."""
    p, ct, bt = sq32
    group = _targets(ct, bt, False)[0]
    orig = U.addlr

    def shifted(Z, b, X, Y, tp, margins=None):
        return orig(Z, b, np.roll(X, 1, axis=0), Y, tp, margins)
    monkeypatch.setattr(U, "addlr", shifted)
    Z = from_csr(p["A"], ct, bt)
    D0 = to_dense(Z)
    ups = _updates(ct, bt, group, 40)
    addlr_accumulated(Z, ups, TruncParams(0.0, "none", 1000))
    assert _rel2(to_dense(Z), _dense_sum(ct, bt, D0, ups)) > 1e-3


# ------------------------------------------------ accumulated updates in products

def _chol_setup(N, sigma_seed, leaf=32):
    p = w.problem(N, sigma_seed=sigma_seed, rhs_seed=5)
    ct = build_cluster_tree(p["coords"], leaf)
    return p, ct, build_block_tree(ct, 2.0)


def test_accumulated_cholesky_exact():
    """Without truncation the Cholesky factor with accumulated updates is
    LAPACK's, as with one update per temporary, and fewer updates run."""
    from oracle.arith import cholesky
    p, ct, bt = _chol_setup(24, 3, leaf=8)
    Ap = p["A"].toarray()[ct.perm][:, ct.perm]
    Lref = np.linalg.cholesky(Ap)
    calls = {}
    for acc in (False, True):
        st = {}
        L = cholesky(from_csr(p["A"], ct, bt, lower=True), TruncParams(0.0, "none", 1000, accumulate=acc), st)
        assert _rel2(np.tril(to_dense(L)), Lref) < 1e-12
        calls[acc] = st["addlr_done"]
    assert calls[True] < calls[False]


@pytest.mark.parametrize("eps", [1e-4, 1e-6])
def test_accumulated_cholesky_truncated(eps):
    """With truncation: ||A - L L^*|| / ||A|| = O(eps) as for one update per
    temporary, and PCG keeps its iteration count within one."""
    from oracle.arith import cholesky, precond_apply
    from oracle.solve import pcg
    p, ct, bt = _chol_setup(32, 3)
    Ap = p["A"].toarray()[ct.perm][:, ct.perm]
    its = {}
    for acc in (False, True):
        L = cholesky(from_csr(p["A"], ct, bt, lower=True), TruncParams(eps, "block_rel", 32, accumulate=acc))
        D = np.tril(to_dense(L))
        assert np.linalg.norm(Ap - D @ D.T, 2) / np.linalg.norm(Ap, 2) < 50 * eps
        _, its[acc], rel = pcg(p["A"], p["b"], lambda v: precond_apply(L, v))
        assert rel <= 1e-8
    assert abs(its[True] - its[False]) <= 1


def test_flush_groups_by_rank():
    """The grouping rule: consecutive temporaries while the total rank stays
    within MAX_UPDATE_RANK, greedy in pair order (ranks 20, 10, 5, 30 give
    the groups {20, 10}, {5}, {30}), each group one update with the
    concatenated factors, whose sum equals that of one update each."""
    from oracle.arith import MAX_UPDATE_RANK, RkTemp, flush_temps
    assert MAX_UPDATE_RANK == 32
    p, ct, bt = _chol_setup(32, None)
    t = int(ct.son0[0]); r = t
    sons = ct.sons(t)
    temps = []
    for i, (k, (a, b)) in enumerate(zip((20, 10, 5, 30), [(sons[0], sons[0]), (sons[0], sons[1]),
                                                           (sons[1], sons[0]), (sons[1], sons[1])])):
        tm = RkTemp(ct, a, b)
        tm.U = w.gaussian(int(ct.size[a]), k, 60 + i)
        tm.V = w.gaussian(int(ct.size[b]), k, 70 + i)
        temps.append(tm)
    got = []
    flush_temps(ct, 7, t, r, temps, TruncParams(1e-6, "block_rel", 32, accumulate=True),
                lambda b, U, V: got.append((b, U.shape[1], U @ V.T)))
    assert [g[1] for g in got] == [30, 5, 30]
    total = sum(g[2] for g in got)
    one = []
    flush_temps(ct, 7, t, r, temps, TruncParams(1e-6, "block_rel", 32),
                lambda b, U, V: one.append(U @ V.T))
    assert len(one) == 4 and np.allclose(total, sum(one), atol=1e-12)
