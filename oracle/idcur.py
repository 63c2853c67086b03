"""Interpolative and CUR decompositions of Sections 10-11.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Partial column-pivoted QR (Section 10.3), k steps on a matrix Y (r x N):
  at step j the pivot is the column whose residual after projecting out the
  j columns already chosen has the largest norm (lowest index on ties); its
  normalised residual is q_j, and S = Q^T Y (k x N).  The chosen columns in
  order form J_s, and S(:, J_s) = S11 is upper triangular.

Column ID (the deterministic figure of Section 10.3): Y ~= Y(:, J_s) Z with
  Z = S11^-1 S (so Z(:, J_s) = I_k and Z holds T = S11^-1 S12 elsewhere).
Row ID: the column ID of Y^T: Y ~= X Y(I_s, :), X = Z^T.

Randomized row ID (Section 10.4 with q power steps): the row ID of a matrix
  whose columns span the range of A is a row ID of A (the paper's
  Observation); the sample must keep A's scaling (its k-step pivoted QR is
  what finds the k dominant directions).  Y = A G for q = 0, as printed; for
  q >= 1 the power steps carry the re-orthonormalisation that the figure's
  caption asks for when accuracy beyond eps^(1/(2q+1)) is wanted: Y is
  Figure 5's last sketch before its final orthonormalisation, Y = A W with W =
  orth(A^T orth(Y_prev)) (the same span as (A A^T)^q A G).
  [I_s, X] = ID_row(Y, k), A ~= X A(I_s, :).
Randomized CUR (Section 11, its figure): the same sample for A^T gives the
  row sketch: Y = (the sample of A^T with G of size m x l)^T (l x n);
  [J_s, Z] = ID_col(Y, k); [I_s, ~] = ID_row(A(:, J_s), k) (all k steps of
  the k x m matrix A(:, J_s)^T); U = the least-squares solution of
  U A(I_s, :) = Z (minimum norm, a library least-squares routine);
  A ~= A(:, J_s) U A(I_s, :).
"""
from __future__ import annotations

import numpy as np

from . import philox
from .rsvd import orth


def cpqr(Y: np.ndarray, k: int):
    """k steps of column-pivoted QR of Y (r x N) by pivoted Gram-Schmidt with residual norms recomputed from
    their definition at every step.  Returns (J (k pivots), Q (r x k), S = Q^T Y (k x N))."""
    Y = np.asarray(Y, dtype=np.float64)
    r, N = Y.shape
    k = min(k, r, N)
    Q = np.zeros((r, k))
    J = []
    for j in range(k):
        Res = Y - Q[:, :j] @ (Q[:, :j].T @ Y)
        nrm = np.linalg.norm(Res, axis=0)
        nrm[J] = -1.0
        p = int(np.argmax(nrm))           # first index of the largest norm
        v = Res[:, p]
        v = v - Q[:, :j] @ (Q[:, :j].T @ v)   # second projection (classical Gram-Schmidt, twice)
        Q[:, j] = v / np.linalg.norm(v)
        J.append(p)
    return np.array(J, dtype=np.int64), Q, Q.T @ Y


def id_col(Y: np.ndarray, k: int):
    """Column ID: (J_s, Z) with Y ~= Y(:, J_s) Z, Z = S11^-1 S."""
    J, Q, S = cpqr(Y, k)
    S11 = S[:, J]
    Z = np.linalg.solve(np.triu(S11), S)
    return J, Z


def id_row(Y: np.ndarray, k: int):
    """Row ID: (I_s, X) with Y ~= X Y(I_s, :)."""
    I, Z = id_col(np.asarray(Y).T, k)
    return I, Z.T


def sample(A: np.ndarray, G: np.ndarray, q: int) -> np.ndarray:
    """Y = A G, then q times Y = A orth(A^T orth(Y)): the last sketch of Figure 5 before its final
    orthonormalisation (for q = 0 the figure's Y = A G)."""
    Y = A @ G
    for _ in range(q):
        Y = A @ orth(A.T @ orth(Y))
    return Y


def randomized_row_id(A: np.ndarray, G: np.ndarray, k: int, q: int = 0):
    """(I_s, X) with A ~= X A(I_s, :), from the test matrix G (n x l)."""
    A = np.asarray(A, dtype=np.float64)
    return id_row(sample(A, G, q), k)


def randomized_cur(A: np.ndarray, G: np.ndarray, k: int, q: int = 0):
    """(J_s, U, I_s) with A ~= A(:, J_s) U A(I_s, :), from the test matrix G (m x l) of the row sketch."""
    A = np.asarray(A, dtype=np.float64)
    Js, Z = id_col(sample(A.T, G, q).T, k)
    Is, _ = id_row(A[:, Js], k)
    R = A[Is, :]
    U = np.linalg.lstsq(R.T, Z.T, rcond=None)[0].T
    return Js, U, Is


def randomized_row_id_seeded(A: np.ndarray, k: int, p: int, q: int, seed: int):
    return randomized_row_id(A, philox.gaussian(A.shape[1], k + p, seed, philox.STREAM_OMEGA), k, q)


def randomized_cur_seeded(A: np.ndarray, k: int, p: int, q: int, seed: int):
    return randomized_cur(A, philox.gaussian(A.shape[0], k + p, seed, philox.STREAM_OMEGA), k, q)
