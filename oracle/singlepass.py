"""Single-pass randomized factorisations of Section 5: every entry of A is
read once (for a general matrix, the two sketches A G_c and A^T G_r come from
the same pass).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Symmetric matrices (Section 5.1 and its figure), A = A^T (n x n), l = k + p:
  1. G = randn(n, l)
  2. Y = A G
  3. Q = the k dominant left singular vectors of Y (the extra over-sampling
     remark of Section 5.1: a k x k core determined by k l equations)
  4. C (k x k, symmetric) = the least-squares solution of C (Q^T G) = Q^T Y
     over symmetric C
  5. C = U_hat D U_hat^T, the eigendecomposition of C
  6. U = Q U_hat                                  A ~= U D U^T

General matrices (Section 5.2 and its figure), A (m x n):
  1. G_c = randn(n, l), G_r = randn(m, l)
  2. Y_c = A G_c, Y_r = A^T G_r
  3. Q_c, Q_r = the k dominant left singular vectors of Y_c, Y_r
  4. C (k x k) = the least-squares solution of the joint system
        (G_r^T Q_c) C = Y_r^T Q_r   and   C (Q_r^T G_c) = Q_c^T Y_c
     (both residuals weighted equally)
  5. C = U_hat D V_hat^T, the SVD of C
  6. U = Q_c U_hat, V = Q_r V_hat                 A ~= U D V^T

Both least-squares problems are solved as written, by a library least-squares
routine on the vectorised system (k^2 unknowns for the joint system, k(k+1)/2
for the symmetric one: its entries on and above the diagonal); where the
solution is not unique the routine's minimum-norm solution is taken.
Gaussians come from ``oracle.philox`` with the seed: G and G_c from the
stream of Figure 5's test matrix, G_r from ``STREAM_GR``.

Readings where the paper is silent: D of the symmetric form keeps the signs
of the eigenvalues (A may be indefinite) and is ordered by decreasing
magnitude; singular vectors and eigenvectors are unique up to sign, so
results are compared per column pair up to a common sign.
"""
from __future__ import annotations

import numpy as np

from . import philox

STREAM_GR = 11      # the row-space test matrix G_r of the general single-pass method


def dominant_left(Y: np.ndarray, k: int) -> np.ndarray:
    """The k dominant left singular vectors of Y (full SVD of Y, the last columns discarded)."""
    u, s, vt = np.linalg.svd(np.asarray(Y, dtype=np.float64), full_matrices=False)
    return u[:, :k]


def lstsq_symmetric(M: np.ndarray, N: np.ndarray) -> np.ndarray:
    """Symmetric C (k x k) minimising ||C M - N||_F for M, N of shape k x l: the unknowns are C's entries on
    and above the diagonal; entry (i, j) moves row i of C M by C_ij M[j, :] and, for i != j, row j by
    C_ij M[i, :]."""
    M = np.asarray(M, dtype=np.float64)
    N = np.asarray(N, dtype=np.float64)
    k, l = M.shape
    iu, ju = np.triu_indices(k)
    D = np.zeros((k, l, iu.size))
    for t, (i, j) in enumerate(zip(iu, ju)):
        D[i, :, t] += M[j]
        if i != j:
            D[j, :, t] += M[i]
    x = np.linalg.lstsq(D.reshape(k * l, -1), N.reshape(-1), rcond=None)[0]
    C = np.zeros((k, k))
    C[iu, ju] = x
    C[ju, iu] = x
    return C


def lstsq_joint(M1: np.ndarray, N1: np.ndarray, M2: np.ndarray, N2: np.ndarray) -> np.ndarray:
    """C (k x k) minimising ||M1 C - N1||_F^2 + ||C M2 - N2||_F^2 (M1, N1: l x k; M2, N2: k x l), on the
    vectorised system: with c = vec(C) column-major, vec(M1 C) = (I kron M1) c and vec(C M2) = (M2^T kron I) c."""
    M1, N1, M2, N2 = (np.asarray(X, dtype=np.float64) for X in (M1, N1, M2, N2))
    k = M1.shape[1]
    I = np.eye(k)
    D = np.vstack([np.kron(I, M1), np.kron(M2.T, I)])
    rhs = np.concatenate([N1.reshape(-1, order="F"), N2.reshape(-1, order="F")])
    c = np.linalg.lstsq(D, rhs, rcond=None)[0]
    return c.reshape(k, k, order="F")


def eig_by_magnitude(C: np.ndarray):
    """Eigendecomposition of symmetric C, eigenvalues ordered by decreasing magnitude (signs kept)."""
    lam, W = np.linalg.eigh(0.5 * (C + C.T))
    order = np.argsort(-np.abs(lam), kind="stable")
    return lam[order], W[:, order]


def single_pass_sym(A: np.ndarray, G: np.ndarray, k: int):
    """Section 5.1's figure for symmetric A and test matrix G (n x l).  Returns (U (n x k), D (k), C)."""
    A = np.asarray(A, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    Y = A @ G
    Q = dominant_left(Y, k)
    C = lstsq_symmetric(Q.T @ G, Q.T @ Y)
    D, Uh = eig_by_magnitude(C)
    return Q @ Uh, D, C


def single_pass_gen(A: np.ndarray, Gc: np.ndarray, Gr: np.ndarray, k: int):
    """Section 5.2's figure for A (m x n) and test matrices Gc (n x l), Gr (m x l).  Returns
    (U (m x k), D (k), V (n x k), C)."""
    A = np.asarray(A, dtype=np.float64)
    Gc = np.asarray(Gc, dtype=np.float64)
    Gr = np.asarray(Gr, dtype=np.float64)
    Yc = A @ Gc
    Yr = A.T @ Gr
    Qc = dominant_left(Yc, k)
    Qr = dominant_left(Yr, k)
    C = lstsq_joint(Gr.T @ Qc, Yr.T @ Qr, Qr.T @ Gc, Qc.T @ Yc)
    u, d, vt = np.linalg.svd(C)
    return Qc @ u, d, Qr @ vt.T, C


def single_pass_sym_seeded(A: np.ndarray, k: int, p: int, seed: int):
    n = A.shape[0]
    return single_pass_sym(A, philox.gaussian(n, k + p, seed, philox.STREAM_OMEGA), k)


def single_pass_gen_seeded(A: np.ndarray, k: int, p: int, seed: int):
    m, n = A.shape
    return single_pass_gen(A, philox.gaussian(n, k + p, seed, philox.STREAM_OMEGA),
                           philox.gaussian(m, k + p, seed, STREAM_GR), k)
