"""Pins of the variable-order weighting of the recompression
(TruncParams.level_factor q; the level-dependent accuracy named in the last
paragraph of Section 4, a reading): the threshold of a cluster at level l of
a tree of depth p is scaled by q^(p - l).

* q = 1 leaves every result unchanged (bit for bit).
* q < 1 makes every threshold above the leaves stricter, so no rank falls
  below the q = 1 rank, the clusters above the leaves gain rank while the
  leaves (scale q^0 = 1) keep theirs, and the update error falls.
* The scaling direction: the planted reversal q^l (leaves strictest) gives
  the leaves a rank gain.
* In the Cholesky factorisation the accuracy stays O(eps) and PCG needs
  no more steps than with q = 1."""
import numpy as np
import pytest

import workloads as w
from oracle.arith import cholesky, precond_apply
from oracle.h2 import TruncParams, from_csr, to_dense
from oracle.solve import pcg
from oracle.trees import build_block_tree, build_cluster_tree
from oracle.update import addlr


@pytest.fixture(scope="module")
def sq32():
    p = w.problem(32, sigma_seed=4, rhs_seed=5)
    ct = build_cluster_tree(p["coords"], 16)
    bt = build_block_tree(ct, 2.0)
    return p, ct, bt


def _update(p, ct, bt, tp):
    Z = from_csr(p["A"], ct, bt)
    X = w.gaussian(ct.n, 16, 91)[ct.perm] * np.logspace(0, -6, 16)
    Y = w.gaussian(ct.n, 16, 92)[ct.perm]
    addlr(Z, 0, X, Y, tp)
    return Z, to_dense(from_csr(p["A"], ct, bt)) + X @ Y.T


def _gain_by_level(ct, Z1, Zq):
    g = np.zeros(ct.depth + 1)
    for side in (0, 1):
        for t in range(ct.nc):
            g[int(ct.level[t])] += int(Zq.k[side][t]) - int(Z1.k[side][t])
    return g


def test_factor_one_is_identity(sq32):
    p, ct, bt = sq32
    Z1, _ = _update(p, ct, bt, TruncParams(1e-3, "block_rel", 64))
    Zq, _ = _update(p, ct, bt, TruncParams(1e-3, "block_rel", 64, level_factor=1.0))
    assert np.array_equal(to_dense(Z1), to_dense(Zq))


def test_stricter_toward_the_root(sq32):
    p, ct, bt = sq32
    Z1, ref = _update(p, ct, bt, TruncParams(1e-3, "block_rel", 64))
    Zq, _ = _update(p, ct, bt, TruncParams(1e-3, "block_rel", 64, level_factor=0.3))
    for side in (0, 1):
        assert np.all(Zq.k[side] >= Z1.k[side])
    g = _gain_by_level(ct, Z1, Zq)
    # leaves keep their threshold (q^0 = 1) and rank; the clusters above
    # (the coarsest have no far field at all) gain
    assert g[ct.depth] == 0 and g[:ct.depth].sum() > 0
    e1 = np.linalg.norm(to_dense(Z1) - ref, 2)
    eq = np.linalg.norm(to_dense(Zq) - ref, 2)
    assert eq < e1


def test_planted_reversal_moves_the_gain(sq32, monkeypatch):
    p, ct, bt = sq32
    Z1, _ = _update(p, ct, bt, TruncParams(1e-3, "block_rel", 64))
    Zq, _ = _update(p, ct, bt, TruncParams(1e-3, "block_rel", 64, level_factor=0.3))
    good = _gain_by_level(ct, Z1, Zq)
    monkeypatch.setattr(TruncParams, "level_scale",
                        lambda self, level, depth: self.level_factor ** int(level))
    Zr, _ = _update(p, ct, bt, TruncParams(1e-3, "block_rel", 64, level_factor=0.3))
    bad = _gain_by_level(ct, Z1, Zr)
    assert bad[ct.depth] > 0                        # now the leaves are the strictest
    assert not np.array_equal(good, bad)


def test_cholesky_variable_order(sq32):
    p, ct, bt = sq32
    Ap = p["A"].toarray()[ct.perm][:, ct.perm]
    its = {}
    for q in (1.0, 0.5):
        L = cholesky(from_csr(p["A"], ct, bt, lower=True), TruncParams(1e-3, "block_rel", 32, level_factor=q))
        D = np.tril(to_dense(L))
        assert np.linalg.norm(Ap - D @ D.T, 2) / np.linalg.norm(Ap, 2) < 50 * 1e-3
        _, its[q], rel = pcg(p["A"], p["b"], lambda v: precond_apply(L, v))
        assert rel <= 1e-8
    assert its[0.5] <= its[1.0]
