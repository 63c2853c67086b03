"""Eigenvalue decomposition of a symmetric positive semidefinite matrix by the
Nystrom method (Section 9 and its figure).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Steps, in the paper's order and notation (l = k + p):
  1. G = randn(n, l)                      (the test matrix of Figure 5, same stream)
  2. Y = A G
  3. Q = orth(Y)                          (with q >= 1: Q from Figure 5's power steps;
                                           q = 0 is the figure as printed)
  4. B1 = A Q, B2 = Q^T B1
  5. B2 = C^T C                           (Cholesky, C upper triangular)
  6. F = B1 C^-1                          (triangular solve)
  7. [U, Sigma, ~] = svd(F, 'econ')
  8. Lambda = Sigma^2                     A ~= U Lambda U^T

Readings where the paper is silent: B2 is symmetric in exact arithmetic and is
made exactly symmetric, (B2 + B2^T) / 2, before step 5; a pivot of step 5 at
or below tau times the corresponding diagonal entry of B2 (tau = l u of the
data precision: B2 is the Gram matrix of A^(1/2) Q, accurate to u relative to
its diagonal) is dropped: its row of C and column of C^-1 are zero, so that a
rank-deficient A gives zero columns of F instead of a failure.  Columns of U
are signed by the rule of ``rsvd.svd_small`` (the SVD is taken of F^T).
"""
from __future__ import annotations

import numpy as np

from . import philox
from .rsvd import orth, svd_small


def chol_drop(B: np.ndarray, tau: float):
    """C (upper triangular, C^T C = B up to the dropped pivots) and C^-1, by the
    right-looking elimination one pivot at a time: pivot j (the current B_jj)
    is kept when it exceeds tau times the original B_jj, else its row of C and
    its column of C^-1 are zero and it takes no part in later eliminations.
    Returns (C, Cinv, dropped)."""
    B = np.array(B, dtype=np.float64)
    n = B.shape[0]
    d0 = np.diag(B).copy()
    C = np.zeros_like(B)
    keep = np.zeros(n, dtype=bool)
    W = B.copy()
    for j in range(n):
        piv = W[j, j]
        if piv > tau * d0[j] and piv > 0.0:
            keep[j] = True
            C[j, j:] = W[j, j:] / np.sqrt(piv)
            W[j + 1:, j + 1:] -= np.outer(C[j, j + 1:], C[j, j + 1:])
    # inverse of C on the kept index set (zero rows and columns elsewhere)
    Cinv = np.zeros_like(C)
    idx = np.flatnonzero(keep)
    if idx.size:
        Ck = C[np.ix_(idx, idx)]
        Cinv[np.ix_(idx, idx)] = np.linalg.solve(Ck, np.eye(idx.size))
    return C, Cinv, int(n - idx.size)


def nystrom(A: np.ndarray, G: np.ndarray, q: int = 0, tau: float = None):
    """Steps 2-8 for the given test matrix G (n x l).  Returns (U, Lam, dropped)
    with U (n x l) and Lam (l) in descending order."""
    A = np.asarray(A, dtype=np.float64)
    n, l = G.shape
    Q = orth(A @ G)
    for _ in range(q):
        W = orth(A.T @ Q)
        Q = orth(A @ W)
    B1 = A @ Q
    B2 = Q.T @ B1
    B2 = 0.5 * (B2 + B2.T)
    if tau is None:
        tau = l * 1.1102230246251565e-16
    C, Cinv, dropped = chol_drop(B2, tau)
    F = B1 @ Cinv
    uh, s, v = svd_small(F.T)          # F^T = uh diag(s) v^T, so F = v diag(s) uh^T
    return v, s ** 2, dropped


def nystrom_seeded(A: np.ndarray, k: int, p: int, q: int, seed: int, tau: float = None):
    """The figure with G drawn from ``seed`` (the stream of Figure 5's test matrix)."""
    n = A.shape[1]
    G = philox.gaussian(n, k + p, seed, philox.STREAM_OMEGA)
    return nystrom(A, G, q, tau)
