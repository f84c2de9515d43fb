"""Writes the stored oracle results of the full-size workloads.

Calls only ``oracle/`` and ``workloads/`` (the seeded input generators):
P1 FEM on the unit square, sigma piecewise constant on 8 x 8 subdomains
(log10 sigma ~ U[-2, 2]), geometric-bisection tree with leaf 32, eta 2,
block-relative accuracy 1e-4, H^2-Cholesky factor L, one Gaussian
right-hand side b, PCG to ||r|| <= 1e-8 ||b|| (x0 = 0).  Stored per
workload: the iteration count and residual of PCG, the largest ranks,
the smallest truncation margin over all recompressions of the
factorisation, norms of z = (L L^*)^{-1} b and of the PCG solution x, and
z, x at 512 seeded sample indices (original index order).

With --spread the factorisation is repeated with LAPACK's gesvd instead of
gesdd in the recompression SVDs (same definition, other rounding) and the
relative differences of z and x that this causes are stored as well: the
rounding sensitivity of the method itself at this size, against which
another implementation's deviation is judged.

    python tests/golden/make_full_size.py 256 10 11 --spread
    python tests/golden/make_full_size.py 512 20 21 --spread
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as w  # noqa: E402
from oracle.arith import cholesky, precond_apply  # noqa: E402
from oracle.h2 import TruncParams, from_csr  # noqa: E402
from oracle.solve import pcg  # noqa: E402
from oracle.trees import build_block_tree, build_cluster_tree  # noqa: E402

NSAMPLE = 512


def _gesvd(M):
    import scipy.linalg as sl
    if M.shape[0] == 0 or M.shape[1] == 0:
        return np.zeros((M.shape[0], 0)), np.zeros(0)
    U, sig, _ = sl.svd(M, full_matrices=False, lapack_driver="gesvd")
    return U, sig


def main(side: int, sseed: int, rseed: int, spread: bool = False):
    p = w.problem(side, sigma_seed=sseed, rhs_seed=rseed)
    ct = build_cluster_tree(p["coords"], 32)
    bt = build_block_tree(ct, 2.0)
    L = from_csr(p["A"], ct, bt, lower=True)
    stats = {"margins": []}
    t0 = time.perf_counter()
    cholesky(L, TruncParams(1e-4, "block_rel", 32), stats)
    t1 = time.perf_counter()
    z = precond_apply(L, p["b"])
    x, it, rel = pcg(p["A"], p["b"], lambda r: precond_apply(L, r), rtol=1e-8)
    t2 = time.perf_counter()
    n = int(ct.n)
    idx = np.sort(np.random.Generator(np.random.PCG64(777)).choice(n, NSAMPLE, replace=False))
    out = {
        "_source": "oracle/ (H^2-Cholesky of Sections 3-6, PCG), written by tests/golden/make_full_size.py",
        "workload": f"P1 FEM unit square {side}x{side} grid, sigma 8x8 subdomains seed {sseed}, "
                    f"bisection leaf 32, eta 2, block_rel 1e-4, Gaussian b seed {rseed}",
        "side": side, "n": n, "sigma_seed": sseed, "rhs_seed": rseed,
        "pcg_iters": int(it), "pcg_relres": float(rel),
        "max_rank": [int(L.k[0].max()), int(L.k[1].max())],
        "min_margin": float(min(stats["margins"])) if stats["margins"] else None,
        "addlr_done": int(stats.get("addlr_done", 0)),
        "z_norm": float(np.linalg.norm(z)), "x_norm": float(np.linalg.norm(x)),
        "z_inf": float(np.max(np.abs(z))), "x_inf": float(np.max(np.abs(x))),
        "idx": [int(i) for i in idx],
        "z": [float(v) for v in z[idx]],
        "x": [float(v) for v in x[idx]],
        "oracle_setup_s": t1 - t0, "oracle_solve_s": t2 - t1,
    }
    if spread:
        import oracle.update as o_update
        saved = o_update.svd_left
        o_update.svd_left = _gesvd
        try:
            L2 = cholesky(from_csr(p["A"], ct, bt, lower=True), TruncParams(1e-4, "block_rel", 32), {})
        finally:
            o_update.svd_left = saved
        z2 = precond_apply(L2, p["b"])
        x2, it2, _ = pcg(p["A"], p["b"], lambda r: precond_apply(L2, r), rtol=1e-8)
        out["spread_svd_routine"] = {
            "what": "relative change of z and x when the recompression SVDs use gesvd instead of gesdd",
            "z": float(np.linalg.norm(z2 - z) / np.linalg.norm(z)),
            "z_sampled": float(np.linalg.norm((z2 - z)[idx]) / np.linalg.norm(z[idx])),
            "x": float(np.linalg.norm(x2 - x) / np.linalg.norm(x)),
            "x_sampled": float(np.linalg.norm((x2 - x)[idx]) / np.linalg.norm(x[idx])),
            "pcg_iters": int(it2),
            "ranks_equal": bool(np.array_equal(L.k[0], L2.k[0]) and np.array_equal(L.k[1], L2.k[1])),
        }
    path = os.path.join(HERE, f"p1_square_{side}_sigma.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print(path, f"setup {t1 - t0:.1f}s solve {t2 - t1:.1f}s iters {it}")


if __name__ == "__main__":
    main(int(sys.argv[1]), int(sys.argv[2]), int(sys.argv[3]), "--spread" in sys.argv[4:])
