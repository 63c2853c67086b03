"""Shared helpers of the GPU parity tests (imported by tests only)."""
from __future__ import annotations

import math

import numpy as np


def device():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need an MI355X; none is visible")
    return torch.device("cuda:0")


def run_factor(A_np, k, p, q, dtype="f64", omega=None, seed=0, flags=0, lda_pad=0, **kw):
    """Run the HIP path through the C ABI on a numpy matrix; returns numpy
    (U, S, V, info)."""
    import torch
    from paper_1607_01649_amd import RSVD
    dev = device()
    tdt = torch.float64 if dtype == "f64" else torch.float32
    m, n = A_np.shape
    if lda_pad:
        big = torch.zeros(m, n + lda_pad, dtype=tdt, device=dev)
        big[:, :n] = torch.from_numpy(np.ascontiguousarray(A_np)).to(tdt)
        A = big[:, :n]
    else:
        A = torch.from_numpy(np.ascontiguousarray(A_np)).to(dev, tdt)
    om = None if omega is None else torch.from_numpy(np.ascontiguousarray(omega, dtype=np.float64)).to(dev)
    solver = RSVD(m, n, k, p, q, dtype=dtype, device=dev, seed=seed, flags=flags, **kw)
    U, S, V, info = solver(A, om, allow_not_certified=True)
    torch.cuda.synchronize()
    return U.double().cpu().numpy(), S.cpu().numpy(), V.double().cpu().numpy(), info


def max_rel_sigma(s_gpu, s_ref, k):
    return float(np.max(np.abs(s_gpu[:k] - s_ref[:k]) / np.abs(s_ref[:k])))


def subspace_sin(Ua, Ub):
    """sine of the largest principal angle between span(Ua) and span(Ub)
    (orthonormal columns), computed as ||(I - Ua Ua^T) Ub||_2, which stays
    accurate for tiny angles."""
    return float(np.linalg.norm(Ub - Ua @ (Ua.T @ Ub), 2))


def column_errors(Xa, Xb):
    """max over columns of ||xa_j - xb_j|| (same sign convention on both sides)."""
    return float(np.max(np.linalg.norm(Xa - Xb, axis=0)))


def orth_error(X):
    return float(np.linalg.norm(X.T @ X - np.eye(X.shape[1]), 2))
