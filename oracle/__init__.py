"""CPU oracle for the H^2 low-rank update, product, Cholesky and PCG path.

TEST INFRASTRUCTURE ONLY.  Nothing in the library (``paper_1402_5056_amd``)
imports, links or calls this package; only ``tests/``, the smoke check in
``__graft_entry__.py`` and the ``cpu_baseline`` leg of ``bench.py`` use it.

It is a plain, slow FP64 implementation written from the paper (Boerm &
Reimer, "Efficient arithmetic operations for rank-structured matrices based
on hierarchical low-rank updates"):

* ``trees``   cluster tree (Def. "Cluster tree", Section 2), block tree
              (Def. "Block tree"), admissible / inadmissible leaves.
* ``h2``      H^2-matrix state (Def. "Cluster basis", eq. (nested);
              Def. "H^2-matrix", eq. (vsw)), dense expansion, matvec.
* ``update``  the local low-rank update Z|t0 x s0 += X Y^* (Sections 4 and 5).
* ``arith``   product recursion (Sections 3 and 6, Cases 1 and 2),
              block substitution and the recursive Cholesky factorisation.
* ``solve``   preconditioned CG and the power-iteration error estimate
              (Section 7).

Small dense kernels (QR, SVD, triangular solves, Cholesky of leaf blocks) are
LAPACK calls through NumPy/SciPy.  Every reading of a passage where the paper
is silent or ambiguous is listed in the docstring of the function that makes
it.
"""

from .trees import ClusterTree, BlockTree, build_cluster_tree, build_block_tree  # noqa: F401
from .h2 import H2Matrix, from_csr, TruncParams  # noqa: F401
from .update import addlr  # noqa: F401
from .arith import cholesky, forward_solve, backward_solve, precond_apply  # noqa: F401
from .solve import pcg, power_error  # noqa: F401
