"""Preconditioned CG and the preconditioner-quality estimate (Section 1:
preconditioned cg iteration; Section 7: relative residual below 1e-8,
convergence factor ||I - A~^{-1} A||_2 by power iteration).

Readings: x_0 = 0; stop when the Euclidean norm of the recursive residual
satisfies ||r||_2 <= rtol ||b||_2; the iteration count m counts products
with A.  Err is estimated by 30 power iterations on M = I - B A (B the
preconditioner) from a seeded Gaussian start, reporting ||M v_30|| / ||v_30||;
M is similar to the symmetric I - L^{-1} A L^{-*}, so this approximates its
spectral radius.
"""

from __future__ import annotations

import numpy as np


def pcg(A, b, prec, rtol: float = 1e-8, maxit: int = 1000):
    """Textbook preconditioned conjugate gradients (Hestenes-Stiefel).

    A: sparse matrix or callable, prec: callable r -> B r.
    Returns (x, iterations, relative recursive residual)."""
    mul = A if callable(A) else (lambda v: A @ v)
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    nb = np.linalg.norm(b)
    if nb == 0:
        return x, 0, 0.0
    z = prec(r)
    p = z.copy()
    rz = float(r @ z)
    it = 0
    while it < maxit:
        q = mul(p)
        it += 1
        alpha = rz / float(p @ q)
        x += alpha * p
        r -= alpha * q
        rel = np.linalg.norm(r) / nb
        if rel <= rtol:
            return x, it, rel
        z = prec(r)
        rz_new = float(r @ z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it, np.linalg.norm(r) / nb


def power_error(A, prec, n: int, seed: int = 7, iters: int = 30) -> float:
    mul = A if callable(A) else (lambda v: A @ v)
    v = np.random.Generator(np.random.PCG64(seed)).standard_normal(n)
    est = 0.0
    for _ in range(iters):
        v = v / np.linalg.norm(v)
        w = v - prec(mul(v))
        est = np.linalg.norm(w)
        v = w
    return float(est)
