"""Pins of the oracle's Cholesky factorisation, vector substitutions and PCG
(Sections 3, 6, 7)."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import workloads as w
from oracle.arith import RkTemp, backward_solve, cholesky, forward_solve, precond_apply
from oracle.h2 import TruncParams, from_csr, to_dense
from oracle.solve import pcg, power_error
from oracle.trees import build_block_tree, build_cluster_tree


def _setup(N, sigma_seed=None, leaf=32):
    p = w.problem(N, sigma_seed=sigma_seed, rhs_seed=5)
    ct = build_cluster_tree(p["coords"], leaf)
    bt = build_block_tree(ct, 2.0)
    return p, ct, bt


def test_cholesky_exact_equals_lapack():
    """Without truncation the H^2 Cholesky factor is the Cholesky factor."""
    p, ct, bt = _setup(32)
    L = cholesky(from_csr(p["A"], ct, bt, lower=True), TruncParams(0.0, "none", 1000))
    D = np.tril(to_dense(L))
    Ap = p["A"].toarray()[ct.perm][:, ct.perm]
    Lref = np.linalg.cholesky(Ap)
    assert np.linalg.norm(D - Lref, 2) / np.linalg.norm(Lref, 2) < 1e-13


def test_cholesky_exact_piecewise_sigma_small_leaves():
    p, ct, bt = _setup(16, sigma_seed=7, leaf=8)
    L = cholesky(from_csr(p["A"], ct, bt, lower=True), TruncParams(0.0, "none", 1000))
    Ap = p["A"].toarray()[ct.perm][:, ct.perm]
    D = np.tril(to_dense(L))
    assert np.linalg.norm(D - np.linalg.cholesky(Ap), 2) / np.linalg.norm(D, 2) < 1e-12


@pytest.mark.parametrize("eps", [1e-4, 1e-6])
def test_cholesky_truncated_accuracy(eps):
    """||A - L L^*|| / ||A|| = O(eps) and the preconditioner is good."""
    p, ct, bt = _setup(32, sigma_seed=3)
    L = cholesky(from_csr(p["A"], ct, bt, lower=True), TruncParams(eps, "block_rel", 64))
    Ap = p["A"].toarray()[ct.perm][:, ct.perm]
    D = np.tril(to_dense(L))
    rel = np.linalg.norm(Ap - D @ D.T, 2) / np.linalg.norm(Ap, 2)
    assert rel < 50 * eps
    assert L.k[0].max() <= 32 and L.k[1].max() <= 32


def test_vector_substitution_matches_dense():
    p, ct, bt = _setup(32, sigma_seed=3)
    L = cholesky(from_csr(p["A"], ct, bt, lower=True), TruncParams(1e-6, "block_rel", 64))
    D = np.tril(to_dense(L))
    rhs = w.gaussian(ct.n, 2, 4)
    y = forward_solve(L, rhs)
    assert np.allclose(y, sla.solve_triangular(D, rhs, lower=True), rtol=1e-11, atol=1e-11)
    z = backward_solve(L, rhs)
    assert np.allclose(z, sla.solve_triangular(D, rhs, lower=True, trans="T"), rtol=1e-11, atol=1e-11)


def test_pcg_exact_factor_one_step():
    p, ct, bt = _setup(32)
    L = cholesky(from_csr(p["A"], ct, bt, lower=True), TruncParams(0.0, "none", 1000))
    x, it, rel = pcg(p["A"], p["b"], lambda r: precond_apply(L, r))
    assert it == 1 and rel < 1e-12


def test_pcg_identity_is_plain_cg():
    p, ct, bt = _setup(32)
    x, it, rel = pcg(p["A"], p["b"], lambda r: r.copy(), rtol=1e-8)
    count = [0]
    def cb(_):
        count[0] += 1
    xs, info = spla.cg(p["A"], p["b"], rtol=1e-8, atol=0.0, callback=cb, maxiter=1000)
    assert info == 0
    assert abs(count[0] - it) <= 1
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-7


def test_pcg_truncated_factor_and_err():
    """Table 1 behaviour (qualitative; the settings differ): few CG steps to
    1e-8 and ||I - B A|| < 1."""
    p, ct, bt = _setup(32, sigma_seed=3)
    L = cholesky(from_csr(p["A"], ct, bt, lower=True), TruncParams(1e-4, "block_rel", 64))
    x, it, rel = pcg(p["A"], p["b"], lambda r: precond_apply(L, r))
    assert rel <= 1e-8 and it <= 5
    assert np.linalg.norm(p["b"] - p["A"] @ x) / np.linalg.norm(p["b"]) <= 1e-8
    assert power_error(p["A"], lambda r: precond_apply(L, r), ct.n) < 0.5


def test_not_spd_detected():
    from oracle.arith import NotSPDError
    p, ct, bt = _setup(16, leaf=8)
    A = p["A"].tolil()
    A[5, 5] = -1.0
    with pytest.raises(NotSPDError):
        cholesky(from_csr(A.tocsr(), ct, bt, lower=True), TruncParams(1e-6, "block_rel", 64))


def test_rk_truncated_addition():
    """Truncated low-rank addition = best approximation of the sum."""
    ct = build_cluster_tree(w.grid_points(8, 2), 4)
    t, r = 1, 2
    tmp = RkTemp(ct, t, r)
    rng = np.random.Generator(np.random.PCG64(3))
    nt, nr = int(ct.size[t]), int(ct.size[r])
    total = np.zeros((nt, nr))
    tp = TruncParams(1e-12, "block_rel", 64)
    for i in range(3):
        U = rng.standard_normal((nt, 2)); V = rng.standard_normal((nr, 2))
        tmp.add(U, V, t, r, tp)
        total += U @ V.T
    assert np.allclose(tmp.U @ tmp.V.T, total, atol=1e-12)
    assert tmp.U.shape[1] == 6
    # zero-extended contribution of a son pair
    s0 = ct.sons(t)[0]
    U = rng.standard_normal((int(ct.size[s0]), 1)); V = rng.standard_normal((nr, 1))
    tmp.add(U, V, s0, r, tp)
    total[:int(ct.size[s0])] += U @ V.T
    assert np.allclose(tmp.U @ tmp.V.T, total, atol=1e-12)



@pytest.mark.parametrize("mode, kept, err", [("block_rel", 16, 0.15), ("const_rel", 17, 0.09)])
def test_rk_truncation_rule_prescribed_spectrum(mode, kept, err):
    """Truncated addition of the product temporaries (the H-matrix rule at the
    end of Section 3): with a prescribed spectrum of the sum, exactly the
    singular values above eps * ||sum||_F (block_rel) or eps * sigma_1
    (const_rel) are kept, and the spectral error is the first dropped singular
    value (Eckart-Young).  The spectrum makes the two thresholds select
    different ranks (||sum||_F = 4.004, sigma_1 = 1, eps = 0.1)."""
    ct = build_cluster_tree(w.grid_points(16, 2), 32)
    t, r = 1, 2
    nt, nr = int(ct.size[t]), int(ct.size[r])
    rng = np.random.Generator(np.random.PCG64(11))
    Q, _ = np.linalg.qr(rng.standard_normal((nt, 20)))
    P, _ = np.linalg.qr(rng.standard_normal((nr, 20)))
    sig = np.array([1.0] * 16 + [0.15, 0.09, 0.05, 0.01])
    tp = TruncParams(0.1, mode, 64)
    tmp = RkTemp(ct, t, r)
    # first term: the leading 16 directions (nothing below either threshold)
    tmp.add(Q[:, :16] * sig[:16], P[:, :16], t, r, tp)
    assert tmp.U.shape[1] == 16
    # second term: the sum now has the singular values sig
    tmp.add(Q[:, 16:] * sig[16:], P[:, 16:], t, r, tp)
    exact = (Q * sig) @ P.T
    assert tmp.U.shape[1] == kept
    e2 = np.linalg.norm(tmp.U @ tmp.V.T - exact, 2)
    assert abs(e2 - err) < 1e-12
    # the kept part is the best approximation of that rank
    best = (Q[:, :kept] * sig[:kept]) @ P[:, :kept].T
    assert np.linalg.norm(tmp.U @ tmp.V.T - best, 2) < 1e-12

# ------------------------------------------------------- triangular inverse
# Remark "Inversion" (end of Section 6) specialised to a lower triangular
# factor.  Pins: without truncation the result is the dense inverse of the
# Cholesky factor (LAPACK), on balanced and unbalanced trees; one leaf is a
# dense inverse; with truncation ||I - G L|| = O(eps); the preconditioner
# G^* G with an exact G makes PCG converge in one step.

def _inverse(p, ct, bt, eps, mode, cap):
    from oracle.arith import tri_invert
    tp = TruncParams(eps, mode, cap)
    L = cholesky(from_csr(p["A"], ct, bt, lower=True), tp)
    Ld = np.tril(to_dense(L))
    G = tri_invert(L.copy(), tp)
    return Ld, np.tril(to_dense(G)), G


@pytest.mark.parametrize("N,sigma_seed,leaf", [(32, None, 32), (16, 7, 8), (24, 3, 16)])
def test_tri_inverse_exact_equals_dense_inverse(N, sigma_seed, leaf):
    """24 x 24 with leaf 16 has leaves on two levels (subdivided blocks that
    pair a leaf with a cluster that has sons)."""
    p, ct, bt = _setup(N, sigma_seed=sigma_seed, leaf=leaf)
    Ld, Gd, _ = _inverse(p, ct, bt, 0.0, "none", 1000)
    Ap = p["A"].toarray()[ct.perm][:, ct.perm]
    Lref = np.linalg.cholesky(Ap)
    Gref = sla.solve_triangular(Lref, np.eye(ct.n), lower=True)
    assert np.linalg.norm(Gd - Gref, 2) / np.linalg.norm(Gref, 2) < 1e-12
    assert np.linalg.norm(Gd @ Ld - np.eye(ct.n), 2) < 1e-11


def test_tri_inverse_single_leaf():
    p, ct, bt = _setup(6)
    assert ct.nc == 1
    Ld, Gd, _ = _inverse(p, ct, bt, 1e-4, "block_rel", 32)
    assert np.allclose(Gd, np.linalg.inv(Ld), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("eps", [1e-4, 1e-6])
def test_tri_inverse_truncated_accuracy(eps):
    p, ct, bt = _setup(32, sigma_seed=3)
    Ld, Gd, G = _inverse(p, ct, bt, eps, "block_rel", 64)
    rel = np.linalg.norm(np.eye(ct.n) - Gd @ Ld, 2)
    assert rel < 200 * eps
    assert G.k[0].max() <= 32 and G.k[1].max() <= 32
    # the upper triangle stays empty: zero couplings above the diagonal are
    # not stored, diagonal leaves are lower triangular
    assert np.all(np.triu(to_dense(G), 1) == 0.0)


def test_precond_inverse_pcg():
    from oracle.arith import precond_apply_inverse
    p, ct, bt = _setup(32)
    _, _, G = _inverse(p, ct, bt, 0.0, "none", 1000)
    x, it, rel = pcg(p["A"], p["b"], lambda r: precond_apply_inverse(G, r))
    assert it == 1 and rel < 1e-12
    p, ct, bt = _setup(32, sigma_seed=3)
    _, _, G = _inverse(p, ct, bt, 1e-4, "block_rel", 64)
    x, it, rel = pcg(p["A"], p["b"], lambda r: precond_apply_inverse(G, r))
    assert rel <= 1e-8 and it <= 6
    assert power_error(p["A"], lambda r: precond_apply_inverse(G, r), ct.n) < 0.5


def test_cholesky_2d_insensitive_to_svd_routine(monkeypatch):
    """The 2-D factor does not depend on rounding inside the recompression
    SVDs: replacing LAPACK's gesdd by gesvd (same definition) changes it by
    rounding only.  This is what makes a 1e-12 parity bar meaningful in 2-D
    (in 3-D the same change moves the factor far more; the 3-D GPU test
    measures that spread)."""
    import scipy.linalg as sl
    import oracle.update as o_update

    def gesvd(M):
        if M.shape[0] == 0 or M.shape[1] == 0:
            return np.zeros((M.shape[0], 0)), np.zeros(0)
        U, sig, _ = sl.svd(M, full_matrices=False, lapack_driver="gesvd")
        return U, sig

    p = w.problem(24, sigma_seed=3, rhs_seed=1)
    ct = build_cluster_tree(p["coords"], 16)
    bt = build_block_tree(ct, 2.0)
    tp = TruncParams(1e-6, "block_rel", 32)
    L1 = np.tril(to_dense(cholesky(from_csr(p["A"], ct, bt, lower=True), tp)))
    monkeypatch.setattr(o_update, "svd_left", gesvd)
    L2 = np.tril(to_dense(cholesky(from_csr(p["A"], ct, bt, lower=True), tp)))
    assert np.linalg.norm(L1 - L2, 2) / np.linalg.norm(L1, 2) < 1e-14
