"""Finite element model problems of the numerical experiments (Section 7).

The model problem is -div(sigma grad u) = f on the unit square (or cube) with
homogeneous Dirichlet data (Section 1), discretised by nodal piecewise linear
(2D, right-isosceles triangles) or trilinear (3D, Q1 bricks) elements on a
regular grid with N cells per axis, h = 1/N.  The unknowns are the interior
grid nodes; node (i, j[, l]) with 1 <= i, j, l <= N-1 has the original index
(i-1) + (N-1)(j-1) [+ (N-1)^2 (l-1)] (x fastest).

sigma is piecewise constant: log10(sigma) ~ U[-2, 2], one value per subdomain
of cells, drawn from numpy's PCG64 generator in subdomain-lexicographic order
(x fastest).  All random draws in this package use numpy.random.Generator
(PCG64(seed)).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def grid_points(N: int, dim: int) -> np.ndarray:
    """Integer coordinates of the interior nodes, shape (n, dim), x fastest."""
    ax = np.arange(1, N, dtype=np.int32)
    if dim == 2:
        j, i = np.meshgrid(ax, ax, indexing="ij")
        return np.stack([i.ravel(), j.ravel()], axis=1).astype(np.int32)
    if dim == 3:
        l, j, i = np.meshgrid(ax, ax, ax, indexing="ij")
        return np.stack([i.ravel(), j.ravel(), l.ravel()], axis=1).astype(np.int32)
    raise ValueError("dim must be 2 or 3")


def sigma_subdomains_2d(N: int, nsub: int = 8, seed: int | None = None) -> np.ndarray:
    """Cell coefficients sigma[ci, cj] (shape N x N): constant on nsub x nsub
    equal subdomains, 10**U[-2,2] each; sigma == 1 when seed is None."""
    if seed is None:
        return np.ones((N, N))
    if N % nsub:
        raise ValueError("grid side must be a multiple of the subdomain count")
    u = _rng(seed).uniform(-2.0, 2.0, size=nsub * nsub)
    vals = 10.0 ** u.reshape(nsub, nsub)          # vals[sj, si], x fastest
    w = N // nsub
    ci = np.arange(N) // w
    return vals[ci[None, :], ci[:, None]]           # sigma[ci, cj] = vals[cj//w, ci//w]


def sigma_blocks_3d(N: int, block: int = 4, seed: int | None = None) -> np.ndarray:
    """Cell coefficients sigma[ci, cj, ck] constant on block^3 cell blocks."""
    if seed is None:
        return np.ones((N, N, N))
    if N % block:
        raise ValueError("grid side must be a multiple of the block size")
    nb = N // block
    u = _rng(seed).uniform(-2.0, 2.0, size=nb ** 3)
    vals = 10.0 ** u.reshape(nb, nb, nb)             # vals[bk, bj, bi]
    c = np.arange(N) // block
    return vals[c[None, None, :], c[None, :, None], c[:, None, None]]   # sigma[ci,cj,ck]=vals[ck,cj,ci]


def fem2d_p1(N: int, sigma: np.ndarray) -> sp.csr_matrix:
    """P1 stiffness matrix on the interior nodes of the N x N grid.

    For a right-isosceles triangulation every axis edge is a leg of both
    triangles that share it, whose opposite angles are 45 degrees, and every
    diagonal edge is opposite a right angle.  The elementwise formula
    a_ij = -1/2 sum_T sigma_T cot(theta_T) therefore gives -(sigma_a+sigma_b)/2
    on axis edges (a, b the two cells touching the edge) and 0 on diagonals,
    independent of the diagonal direction; the diagonal entry is minus the sum
    of the off-diagonal entries including those to Dirichlet nodes."""
    m = N - 1
    n = m * m
    sig = np.asarray(sigma, dtype=np.float64)
    I, J = np.meshgrid(np.arange(1, N), np.arange(1, N), indexing="xy")  # I[j-1, i-1] = i
    I = I.ravel(); J = J.ravel()
    idx = (I - 1) + m * (J - 1)
    # edge coefficients towards +x, -x, +y, -y
    cxp = 0.5 * (sig[I, J - 1] + sig[I, J])
    cxm = 0.5 * (sig[I - 1, J - 1] + sig[I - 1, J])
    cyp = 0.5 * (sig[I - 1, J] + sig[I, J])
    cym = 0.5 * (sig[I - 1, J - 1] + sig[I, J - 1])
    rows = [idx]; cols = [idx]; vals = [cxp + cxm + cyp + cym]
    mask = I < m
    rows.append(idx[mask]); cols.append(idx[mask] + 1); vals.append(-cxp[mask])
    mask = I > 1
    rows.append(idx[mask]); cols.append(idx[mask] - 1); vals.append(-cxm[mask])
    mask = J < m
    rows.append(idx[mask]); cols.append(idx[mask] + m); vals.append(-cyp[mask])
    mask = J > 1
    rows.append(idx[mask]); cols.append(idx[mask] - m); vals.append(-cym[mask])
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    A.sort_indices()
    return A


_K1 = np.array([[1.0, -1.0], [-1.0, 1.0]])
_M1 = np.array([[1.0 / 3.0, 1.0 / 6.0], [1.0 / 6.0, 1.0 / 3.0]])


def fem3d_q1(N: int, sigma: np.ndarray) -> sp.csr_matrix:
    """Q1 stiffness matrix on the interior nodes of the N^3 grid.

    The element matrix of a brick of side h with coefficient sigma_e is
    sigma_e * h * (K^M^M + M^K^M + M^M^K) with the 1D reference stiffness
    K = [[1,-1],[-1,1]] and mass M = [[1/3,1/6],[1/6,1/3]] (^ = Kronecker
    product over the axes), which follows from integrating products of 1D hat
    functions."""
    m = N - 1
    h = 1.0 / N
    sig = np.asarray(sigma, dtype=np.float64)
    loc = [(a, b, c) for c in (0, 1) for b in (0, 1) for a in (0, 1)]
    Ke = np.zeros((8, 8))
    for p, (a, b, c) in enumerate(loc):
        for q, (a2, b2, c2) in enumerate(loc):
            Ke[p, q] = (_K1[a, a2] * _M1[b, b2] * _M1[c, c2]
                        + _M1[a, a2] * _K1[b, b2] * _M1[c, c2]
                        + _M1[a, a2] * _M1[b, b2] * _K1[c, c2])
    ci, cj, ck = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    ci = ci.ravel(); cj = cj.ravel(); ck = ck.ravel()
    se = sig[ci, cj, ck] * h
    rows = []; cols = []; vals = []
    for p, (a, b, c) in enumerate(loc):
        xp, yp, zp = ci + a, cj + b, ck + c
        okp = (xp >= 1) & (xp <= m) & (yp >= 1) & (yp <= m) & (zp >= 1) & (zp <= m)
        ip = (xp - 1) + m * (yp - 1) + m * m * (zp - 1)
        for q, (a2, b2, c2) in enumerate(loc):
            xq, yq, zq = ci + a2, cj + b2, ck + c2
            ok = okp & (xq >= 1) & (xq <= m) & (yq >= 1) & (yq <= m) & (zq >= 1) & (zq <= m)
            iq = (xq - 1) + m * (yq - 1) + m * m * (zq - 1)
            rows.append(ip[ok]); cols.append(iq[ok]); vals.append(se[ok] * Ke[p, q])
    n = m ** 3
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.eliminate_zeros()
    A.sort_indices()
    return A


def convection_x(N: int, c: float) -> sp.csr_matrix:
    """First-order upwind difference c (u_i - u_{i-1}) along +x on the
    interior nodes of the N x N grid (zero Dirichlet values): added to the
    stiffness matrix it gives a non-symmetric matrix with the same stencil
    reach, diagonally dominant for c >= 0."""
    m = N - 1
    I, J = np.meshgrid(np.arange(1, N), np.arange(1, N), indexing="xy")
    I = I.ravel(); J = J.ravel()
    idx = (I - 1) + m * (J - 1)
    mask = I > 1
    rows = np.concatenate([idx, idx[mask]])
    cols = np.concatenate([idx, idx[mask] - 1])
    vals = np.concatenate([np.full(idx.size, c), np.full(int(mask.sum()), -c)])
    B = sp.coo_matrix((vals, (rows, cols)), shape=(m * m, m * m)).tocsr()
    B.sort_indices()
    return B


def gaussian(n: int, k: int, seed: int) -> np.ndarray:
    """n x k standard normal matrix, drawn row by row in original index order."""
    return _rng(seed).standard_normal((n, k))


_CONFIGS = {
    # name: (dim, N, sigma seed or None, rhs seed)
    "p1_square_32": (2, 32, None, 2),            # P1, 32 x 32 grid, sigma = 1
    "p1_square_256_sigma": (2, 256, 10, 11),     # P1, 256 x 256, sigma on 8 x 8 subdomains
    "p1_square_512_sigma": (2, 512, 20, 21),     # P1, 512 x 512, sigma on 8 x 8 subdomains
    "q1_cube_64_sigma": (3, 64, 30, 31),         # Q1, 64^3, sigma on 4 x 4 x 4 cell blocks
}


def problem(name_or_side, dim: int = 2, sigma_seed: int | None = None, rhs_seed: int = 0):
    """Return dict(coords, A (CSR, original order), b, N, dim) for a named
    workload (keys of _CONFIGS) or for a grid side."""
    if isinstance(name_or_side, str):
        dim, N, sigma_seed, rhs_seed = _CONFIGS[name_or_side]
    else:
        N = int(name_or_side)
    coords = grid_points(N, dim)
    if dim == 2:
        sig = sigma_subdomains_2d(N, 8, sigma_seed)
        A = fem2d_p1(N, sig)
    else:
        sig = sigma_blocks_3d(N, 4, sigma_seed)
        A = fem3d_q1(N, sig)
    b = gaussian(A.shape[0], 1, rhs_seed)[:, 0]
    return {"coords": coords, "A": A, "b": b, "N": N, "dim": dim}
