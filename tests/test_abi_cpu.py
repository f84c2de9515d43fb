"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every symbol the header declares, and its integer tree construction is
bit-identical to the oracle's (Def. "Cluster tree", Def. "Block tree")."""
import os
import re
import subprocess

import numpy as np
import pytest

import workloads as w
from oracle.trees import build_block_tree, build_cluster_tree

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "h2lr.h")
LIB = os.path.join(ROOT, "paper_1402_5056_amd", "libh2lr.so")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:h2_status|const char \*)\s*(h2_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "library not built"
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (h2_\w+)", out))
    declared = _declared()
    assert len(declared) >= 20
    missing = [s for s in declared if s not in exported]
    assert not missing, missing


def test_binding_covers_header():
    from paper_1402_5056_amd import h2lr
    assert set(_declared()) <= set(h2lr.EXPORTED)


@pytest.mark.parametrize("N,dim,leaf,eta", [(32, 2, 32, 2.0), (256, 2, 32, 2.0), (29, 2, 7, 1.0),
                                             (16, 3, 32, 2.0), (45, 2, 16, 4.0)])
def test_trees_bit_exact_vs_oracle(N, dim, leaf, eta):
    from paper_1402_5056_amd import h2lr
    ctx = h2lr.h2_ctx_create(-1)
    c = w.grid_points(N, dim)
    ct = h2lr.h2_ctree_build(ctx, c, leaf)
    bt = h2lr.h2_btree_build(ctx, ct, eta)
    oc = build_cluster_tree(c, leaf)
    ob = build_block_tree(oc, eta)
    e = h2lr.h2_ctree_export(ct)
    for k in ("perm", "offset", "size", "level", "son0", "son1", "parent"):
        assert np.array_equal(e[k], getattr(oc, k)), k
    b = h2lr.h2_btree_export(bt)
    for k in ("row", "col", "kind", "parent"):
        assert np.array_equal(b[k], getattr(ob, k)), k
    nb, na, nn, csp = h2lr.h2_btree_info(bt)
    assert (nb, na, nn) == (ob.nb, int((ob.kind == 1).sum()), int((ob.kind == 2).sum()))
    assert h2lr.h2_btree_find(bt, 1, 2) == ob.find(1, 2)
    assert h2lr.h2_btree_find(bt, 0, 5) == -1


@pytest.mark.parametrize("N,dim,leaf,eta", [(32, 2, 32, 4.0), (256, 2, 32, 4.0), (29, 2, 7, 2.0),
                                             (16, 3, 32, 2.0), (13, 3, 8, 4.0), (45, 2, 16, 4.0)])
def test_dd_trees_bit_exact_vs_oracle(N, dim, leaf, eta):
    from paper_1402_5056_amd import h2lr
    ctx = h2lr.h2_ctx_create(-1)
    c = w.grid_points(N, dim)
    ct = h2lr.h2_ctree_build_dd(ctx, c, leaf)
    bt = h2lr.h2_btree_build(ctx, ct, eta)
    oc = build_cluster_tree(c, leaf, dd=True)
    ob = build_block_tree(oc, eta)
    e = h2lr.h2_ctree_export(ct)
    for k in ("perm", "offset", "size", "level", "son0", "son1", "parent"):
        assert np.array_equal(e[k], getattr(oc, k)), k
    b = h2lr.h2_btree_export(bt)
    for k in ("row", "col", "kind", "parent"):
        assert np.array_equal(b[k], getattr(ob, k)), k


def test_abi_argument_errors():
    from paper_1402_5056_amd import h2lr
    ctx = h2lr.h2_ctx_create(-1)
    with pytest.raises(h2lr.H2Error) as ei:
        h2lr.h2_ctree_build(ctx, w.grid_points(8, 2), 0)
    assert ei.value.name == "H2_ERR_ARG"
    ct = h2lr.h2_ctree_build(ctx, w.grid_points(8, 2), 4)
    bt = h2lr.h2_btree_build(ctx, ct, 2.0)
    with pytest.raises(h2lr.H2Error) as ei:
        h2lr.h2_mat_from_csr(ctx, bt, w.fem2d_p1(8, np.ones((8, 8))))
    assert ei.value.name == "H2_ERR_ARG"      # host-only context holds no matrices
