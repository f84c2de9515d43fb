"""Shared test helpers: dense expansion through the HIP matvec and the
near-threshold check of the oracle.  No method arithmetic lives here."""
import numpy as np


def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a visible HIP device"
    return torch


def to_dev_cols(a):
    """numpy (m x k) -> torch float64 device tensor, column-major (m x k view)."""
    torch = gpu()
    a = np.asarray(a, dtype=np.float64)
    return torch.tensor(np.ascontiguousarray(a.T), device="cuda").t()


def dense_via_matvec(h2lr, M, n, trans=False):
    """Dense matrix (original order) of an H^2 matrix by products with unit
    vectors, 64 at a time, on the device."""
    torch = gpu()
    D = np.zeros((n, n))
    for c0 in range(0, n, 64):
        nc = min(64, n - c0)
        X = torch.zeros((nc, n), dtype=torch.float64, device="cuda")
        X[torch.arange(nc), torch.arange(c0, c0 + nc)] = 1.0
        Y = torch.zeros_like(X)
        torch.cuda.synchronize()      # the matrix may live on another stream
        h2lr.h2_matvec(M, X, Y, trans=trans)
        torch.cuda.synchronize()
        D[:, c0:c0 + nc] = Y.cpu().numpy().T
    return D


def to_original(Dc, perm):
    D = np.empty_like(Dc)
    D[np.ix_(perm, perm)] = Dc
    return D


def rel2(A, B):
    return np.linalg.norm(A - B, 2) / max(np.linalg.norm(B, 2), 1e-300)
