"""Pins of the oracle's trees (Def. "Cluster tree", Def. "Block tree",
Section 2) and of the FEM inputs (Section 7 model problem)."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as w
from oracle.trees import ADM, NEAR, build_block_tree, build_cluster_tree, admissible

GOLD = os.path.join(os.path.dirname(__file__), "golden", "tree_counts.json")


def _trees(N, dim=2, leaf=32, eta=2.0):
    ct = build_cluster_tree(w.grid_points(N, dim), leaf)
    return ct, build_block_tree(ct, eta)


@pytest.mark.parametrize("case", json.load(open(GOLD))["cases"])
def test_tree_counts_golden(case):
    ct, bt = _trees(case["N"], case["dim"], 32, case["eta"])
    leaves = [t for t in range(ct.nc) if ct.is_leaf(t)]
    assert ct.nc == case["clusters"]
    assert len(leaves) == case["leaves"]
    assert ct.size[leaves].min() == case["leaf_min"] and ct.size[leaves].max() == case["leaf_max"]
    assert ct.depth == case["depth"]
    assert int((bt.kind == ADM).sum()) == case["adm"]
    assert int((bt.kind == NEAR).sum()) == case["near"]
    assert np.bincount(bt.row[bt.kind == ADM]).max() == case["csp_adm_row"]


@pytest.mark.parametrize("N,leaf,eta", [(12, 8, 2.0), (17, 5, 1.0), (20, 16, 4.0)])
def test_partition_and_admissibility(N, leaf, eta):
    ct, bt = _trees(N, 2, leaf, eta)
    n = ct.n
    # cluster tree: sons partition the father (Def. "Cluster tree")
    assert sorted(ct.perm.tolist()) == list(range(n))
    for t in range(ct.nc):
        if not ct.is_leaf(t):
            a, b = ct.rng(t)
            s0, s1 = ct.sons(t)
            assert ct.rng(s0) == (a, a + ct.size[s0]) and ct.rng(s1)[1] == b
            assert ct.size[s0] > 0 and ct.size[s1] > 0
        else:
            assert ct.size[t] <= leaf
    # block tree leaves partition I x I exactly once (remark after Def. "Block tree")
    cover = np.zeros((n, n), np.int64)
    for b in range(bt.nb):
        t, s = int(bt.row[b]), int(bt.col[b])
        if bt.kind[b] != 0:
            a0, a1 = ct.rng(t); c0, c1 = ct.rng(s)
            cover[a0:a1, c0:c1] += 1
            if bt.kind[b] == ADM:
                assert admissible(ct, t, s, eta * eta)
            else:
                assert ct.is_leaf(t) and ct.is_leaf(s)
                assert not admissible(ct, t, s, eta * eta)
        else:
            assert len(bt.sons(b)) == len(ct.sons_plus(t)) * len(ct.sons_plus(s))
    assert (cover == 1).all()


def test_admissibility_brute_force():
    """Box distance and diameter against brute-force point sets (tiny grid)."""
    ct, bt = _trees(9, 2, 4, 2.0)
    pts = w.grid_points(9, 2)
    for b in range(bt.nb):
        if bt.kind[b] != ADM:
            continue
        t, s = int(bt.row[b]), int(bt.col[b])
        P = pts[ct.perm[slice(*ct.rng(t))]]
        Q = pts[ct.perm[slice(*ct.rng(s))]]
        # every point pair is at least the box distance apart
        d2 = ((P[:, None, :] - Q[None, :, :]) ** 2).sum(-1).min()
        lo_t, hi_t = P.min(0), P.max(0)
        assert ((hi_t - lo_t) ** 2).sum() <= 4 * d2


def test_fem2d_closed_form_eigenvalues():
    N = 12
    A = w.fem2d_p1(N, np.ones((N, N))).toarray()
    assert np.allclose(A, A.T)
    p = np.arange(1, N)
    lam = (4 - 2 * np.cos(p[:, None] * np.pi / N) - 2 * np.cos(p[None, :] * np.pi / N)).ravel()
    assert np.allclose(np.sort(np.linalg.eigvalsh(A)), np.sort(lam), atol=1e-12)
    # eigenvector sin(p pi x) sin(q pi y)
    pts = w.grid_points(N, 2)
    v = np.sin(2 * np.pi * pts[:, 0] / N) * np.sin(3 * np.pi * pts[:, 1] / N)
    assert np.allclose(A @ v, (4 - 2 * np.cos(2 * np.pi / N) - 2 * np.cos(3 * np.pi / N)) * v)


def test_fem2d_piecewise_sigma_entries():
    N = 16
    sig = w.sigma_subdomains_2d(N, 8, seed=3)
    A = w.fem2d_p1(N, sig)
    assert abs(A - A.T).max() == 0
    # node (i, j) = (2, 3): right neighbour edge touches cells (2,2), (2,3)
    i, j = 2, 3
    idx = (i - 1) + (N - 1) * (j - 1)
    assert np.isclose(A[idx, idx + 1], -(sig[2, 2] + sig[2, 3]) / 2)
    # full Neumann row sums vanish, so interior rows not touching the boundary sum to 0
    i, j = 5, 6
    idx = (i - 1) + (N - 1) * (j - 1)
    assert abs(A[idx].sum()) < 1e-12
    # subdomain draws are log-uniform in [1e-2, 1e2]
    assert sig.min() >= 1e-2 and sig.max() <= 1e2


def test_fem3d_q1_closed_form_eigenvalues():
    N = 6
    h = 1.0 / N
    A = w.fem3d_q1(N, np.ones((N, N, N))).toarray()
    assert np.allclose(A, A.T)
    th = np.arange(1, N) * np.pi / N
    k1 = (2 - 2 * np.cos(th)) / h
    m1 = h * (2.0 / 3.0 + np.cos(th) / 3.0)
    K, M = k1, m1
    lam = (K[:, None, None] * M[None, :, None] * M[None, None, :]
           + M[:, None, None] * K[None, :, None] * M[None, None, :]
           + M[:, None, None] * M[None, :, None] * K[None, None, :]).ravel()
    assert np.allclose(np.sort(np.linalg.eigvalsh(A)), np.sort(lam), atol=1e-12)


def test_fem_far_blocks_vanish():
    """A is zero on every admissible block at the experiment grids (so H^2(A)
    has rank 0 everywhere); checked on the 32 x 32 grid and a 3D grid."""
    from oracle.h2 import from_csr, to_dense
    for N, dim in ((32, 2), (16, 3)):
        pb = w.problem(N, dim=dim, sigma_seed=4)
        ct = build_cluster_tree(pb["coords"], 32)
        bt = build_block_tree(ct, 2.0)
        Z = from_csr(pb["A"], ct, bt)
        Ap = pb["A"].toarray()[ct.perm][:, ct.perm]
        assert np.array_equal(to_dense(Z), Ap)


def test_nonzero_far_block_rejected():
    """A matrix with a coupling inside an admissible block is rejected."""
    from oracle.h2 import from_csr
    pb = w.problem(32, dim=2, sigma_seed=4)
    ct = build_cluster_tree(pb["coords"], 32)
    bt = build_block_tree(ct, 2.0)
    b = int(np.flatnonzero(bt.kind == ADM)[0])
    i = int(ct.perm[ct.offset[bt.row[b]]])
    j = int(ct.perm[ct.offset[bt.col[b]]])
    A = pb["A"].tolil()
    A[i, j] = A[j, i] = -0.5
    with pytest.raises(ValueError):
        from_csr(A.tocsr(), ct, bt)


def test_stencil_neighbours_never_admissible():
    """Clusters one grid step apart are never admissible, whatever eta: the
    Q1 stencil on a 12^3 grid with leaf 32 reaches across such a pair."""
    pb = w.problem(12, dim=3, sigma_seed=4)
    ct = build_cluster_tree(pb["coords"], 32)
    bt = build_block_tree(ct, 2.0)
    Ap = abs(pb["A"]).toarray()[ct.perm][:, ct.perm]
    for b in np.flatnonzero(bt.kind == ADM):
        t, s = int(bt.row[b]), int(bt.col[b])
        assert not Ap[slice(*ct.rng(t)), slice(*ct.rng(s))].any()
