"""Boundary element model problem of the numerical experiments (Section 7,
second model problem): the single layer potential operator on a circle,
discretised by the Galerkin method with piecewise constant basis functions
on a regular mesh.  This module only generates the problem data.

Readings (the paper names the operator, the curve, the regular mesh and the
piecewise constant basis, nothing more):

* the curve is the circle of radius 1/2 (diameter one).  On the circle of
  radius one the logarithmic single layer operator maps constants to zero
  (logarithmic capacity one); on smaller circles it is positive definite;
* kernel g(x, y) = -log|x - y| / (2 pi);
* the mesh is the regular n-gon inscribed in the circle, vertex i at angle
  2 pi i / n, panel i the straight segment from vertex i to vertex i + 1
  (length L = sin(pi / n)); panel i has the original index i;
* entry A_ij = int_{P_i} int_{P_j} g(x, y) ds_y ds_x.  The inner integral
  over a straight segment is evaluated in closed form; the outer one by
  Gauss-Legendre quadrature on P_i (16 points on the two neighbours of a
  panel, where the integrand has a logarithmic singularity at the shared
  vertex, 4 points elsewhere); the diagonal in closed form,
  int_0^L int_0^L log|s - t| ds dt = L^2 (log L - 3/2).  By the rotation
  symmetry of the mesh A_ij depends only on (j - i) mod n: the matrix is
  defined as the circulant of the first row c, symmetrised by
  c_k <- (c_k + c_{n-k}) / 2 (the mesh is also reflection symmetric);
* coordinates for the cluster tree: panel midpoints, shifted to [0, 1]^2,
  scaled by 30000 and rounded to integers (squared box sizes stay below
  2^31).
"""

from __future__ import annotations

import numpy as np

RADIUS = 0.5
COORD_SCALE = 30000


def vertices(n: int) -> np.ndarray:
    ang = 2.0 * np.pi * np.arange(n + 1) / n
    return RADIUS * np.stack([np.cos(ang), np.sin(ang)], axis=1)


def _segment_log_integral(x: np.ndarray, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """int over the segment [a, b] of log|x - y| ds_y, closed form, for
    points x (... x 2) and one segment."""
    L = float(np.hypot(*(b - a)))
    tau = (b - a) / L
    nu = np.array([-tau[1], tau[0]])
    r = x - a
    p = r @ tau
    d = np.abs(r @ nu)

    def G(u):
        # antiderivative of log(u^2 + d^2) / 2 in u
        with np.errstate(divide="ignore", invalid="ignore"):
            lg = np.where((u == 0.0) & (d == 0.0), 0.0, np.log(u * u + d * d))
        return 0.5 * u * lg - u + d * np.arctan2(u, d)
    return G(L - p) - G(-p)


def first_row(n: int) -> np.ndarray:
    """c_k = A_{0k} for k = 0..n-1 (before symmetrisation)."""
    V = vertices(n)
    L = float(np.hypot(*(V[1] - V[0])))
    c = np.empty(n)
    for k in range(n):
        q = 16 if k in (1, n - 1) else 4
        t, w = np.polynomial.legendre.leggauss(q)
        s = 0.5 * (t + 1.0)                               # points on [0, 1]
        xq = V[0][None, :] + s[:, None] * (V[1] - V[0])[None, :]
        if k == 0:
            c[k] = -(L * L * (np.log(L) - 1.5)) / (2.0 * np.pi)
        else:
            inner = _segment_log_integral(xq, V[k], V[k + 1])
            c[k] = -(0.5 * L * np.dot(w, inner)) / (2.0 * np.pi)
    return c


def circulant_row(n: int) -> np.ndarray:
    """Symmetrised first row: the matrix is A_ij = c[(j - i) mod n]."""
    c = first_row(n)
    return 0.5 * (c + np.roll(c[::-1], 1))


def block(c: np.ndarray, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """A[rows][:, cols] of the circulant with first row c."""
    n = len(c)
    return c[(np.asarray(cols)[None, :] - np.asarray(rows)[:, None]) % n]


def dense(c: np.ndarray) -> np.ndarray:
    idx = np.arange(len(c))
    return block(c, idx, idx)


def midpoint_coords(n: int) -> np.ndarray:
    V = vertices(n)
    mid = 0.5 * (V[:-1] + V[1:]) + 0.5
    return np.rint(mid * COORD_SCALE).astype(np.int32)


def problem(n: int, rhs_seed: int = 0):
    """dict(coords, c (first row), n, b) of the BEM model problem with n
    panels; b is a Gaussian right-hand side (seeded)."""
    from .fem import gaussian
    return {"coords": midpoint_coords(n), "c": circulant_row(n), "n": n,
            "b": gaussian(n, 1, rhs_seed)[:, 0]}


def far_factors(c: np.ndarray, perm: np.ndarray, blocks, rel_tol: float = 1e-10):
    """Low-rank factors of far-field blocks of the circulant matrix, as input
    for building its H^2 representation by local updates.  blocks: list of
    (row offset, row size, column offset, column size) in cluster order (the
    index ranges of an admissible block under the permutation perm).
    Returns [(X, Y)] with A|_block ~= X Y^T, X = U_r Sigma_r, Y = V_r from the
    SVD of the dense block, keeping sigma > rel_tol * sigma_1 (the kernel
    approximation the paper leaves open; here simply the truncated SVD)."""
    out = []
    for (ro, rn, co, cn) in blocks:
        D = block(c, perm[ro:ro + rn], perm[co:co + cn])
        U, s, Vt = np.linalg.svd(D, full_matrices=False)
        r = int(np.count_nonzero(s > rel_tol * s[0])) if s.size and s[0] > 0 else 0
        out.append((np.ascontiguousarray(U[:, :r] * s[:r]), np.ascontiguousarray(Vt[:r].T)))
    return out


def nearfield_csr(c: np.ndarray, perm: np.ndarray, blocks):
    """CSR (original order) holding A on the given inadmissible leaves,
    blocks as for far_factors."""
    import scipy.sparse as sp
    rows, cols, vals = [], [], []
    for (ro, rn, co, cn) in blocks:
        r = perm[ro:ro + rn]
        cc = perm[co:co + cn]
        D = block(c, r, cc)
        rows.append(np.repeat(r, cn))
        cols.append(np.tile(cc, rn))
        vals.append(D.ravel())
    n = len(c)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
