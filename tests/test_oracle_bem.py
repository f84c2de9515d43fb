"""Pins of the boundary element model problem (second model problem of
Section 7) and of the oracle on it.

* The Galerkin matrix of the single layer operator on the circle of radius
  rho is circulant; its eigenvalues (the FFT of the first row) approximate
  h times the eigenvalues of the continuous operator, rho / (2|k|) for the
  Fourier mode k != 0 and -rho log(rho) for the constants (closed forms of
  the logarithmic potential on a circle), with second-order convergence in
  h: a wrong factor, sign or term fails this.
* The closed-form segment integral and the closed-form self term against
  adaptive quadrature.
* The H^2 matrix built from the nearfield by local updates reproduces A;
  without truncation its Cholesky factor is LAPACK's; with eps ~ h PCG
  converges in a few steps (Table 2 reports 3-4)."""
import numpy as np
import pytest
import scipy.integrate as si

import workloads as w
from oracle.arith import cholesky, precond_apply
from oracle.h2 import TruncParams, from_csr, to_dense
from oracle.solve import pcg
from oracle.trees import ADM, NEAR, build_block_tree, build_cluster_tree
from oracle.update import addlr

RHO = w.bem.RADIUS


def _spectrum_errors(n):
    lam = np.fft.fft(w.bem.circulant_row(n)).real
    h = 2.0 * np.pi * RHO / n
    e0 = lam[0] / (h * (-RHO * np.log(RHO))) - 1.0
    ek = [lam[k] / (h * RHO / (2.0 * k)) - 1.0 for k in (1, 2, 3)]
    return e0, ek, lam


def test_spectrum_matches_continuous_operator():
    e0a, eka, lam = _spectrum_errors(256)
    e0b, ekb, _ = _spectrum_errors(512)
    assert lam.min() > 0.0                       # symmetric positive definite
    assert abs(e0a) < 1e-4 and max(abs(e) for e in eka) < 1e-3
    # second order in h: halving h divides the errors by about four
    assert 3.0 < e0a / e0b < 5.0
    for a, b in zip(eka, ekb):
        assert 3.0 < a / b < 5.0


def test_segment_integral_closed_form():
    a, b = np.array([0.1, -0.2]), np.array([0.4, 0.2])
    L = np.hypot(*(b - a))
    for x in (np.array([1.0, 0.3]), np.array([0.25, 0.0]), a + 0.3 * (b - a), b.copy()):
        ref, _ = si.quad(lambda s: np.log(np.hypot(*(x - a - s * (b - a) / L))), 0.0, L, limit=200,
                         points=None)
        got = float(w.bem._segment_log_integral(x[None, :], a, b)[0])
        assert abs(got - ref) < 1e-9 * max(1.0, abs(ref))


def test_self_term_closed_form():
    L = 0.05
    ref, _ = si.dblquad(lambda t, s: np.log(abs(s - t)) if s != t else 0.0, 0.0, L, 0.0, L,
                        epsabs=1e-13, epsrel=1e-10)
    assert abs(L * L * (np.log(L) - 1.5) - ref) < 1e-6 * abs(ref)


def _h2_by_updates(n, tol):
    p = w.bem.problem(n, rhs_seed=3)
    ct = build_cluster_tree(p["coords"], 32)
    bt = build_block_tree(ct, 2.0)

    def rng(t):
        return int(ct.offset[t]), int(ct.size[t])
    near = [b for b in range(bt.nb) if bt.kind[b] == NEAR]
    far = [b for b in range(bt.nb)
           if bt.kind[b] == ADM and int(ct.offset[bt.row[b]]) > int(ct.offset[bt.col[b]])]
    N = w.bem.nearfield_csr(p["c"], ct.perm, [rng(bt.row[b]) + rng(bt.col[b]) for b in near])
    F = w.bem.far_factors(p["c"], ct.perm, [rng(bt.row[b]) + rng(bt.col[b]) for b in far], tol)
    H = from_csr(N, ct, bt, lower=True)
    for b, (X, Y) in zip(far, F):
        addlr(H, b, X, Y, TruncParams(tol, "block_rel", 64))
    return p, ct, H


def test_h2_by_updates_reproduces_a_and_exact_cholesky():
    p, ct, H = _h2_by_updates(256, 1e-12)
    A = w.bem.dense(p["c"])[np.ix_(ct.perm, ct.perm)]
    D = np.tril(to_dense(H))
    assert np.linalg.norm(D - np.tril(A), 2) / np.linalg.norm(A, 2) < 1e-11
    L = cholesky(H, TruncParams(0.0, "none", 64))
    Lc = np.linalg.cholesky(A)
    assert np.linalg.norm(np.tril(to_dense(L)) - Lc, 2) / np.linalg.norm(Lc, 2) < 1e-10


@pytest.mark.parametrize("n", [256, 1024])
def test_truncated_preconditioner_converges(n):
    p, ct, H = _h2_by_updates(n, 1e-10)
    L = cholesky(H, TruncParams(1.0 / n, "block_rel", 32))
    x, it, rel = pcg(w.bem.dense(p["c"]), p["b"], lambda r: precond_apply(L, r))
    assert rel <= 1e-8 and it <= 6
