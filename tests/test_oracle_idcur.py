"""Pins of the ID / CUR oracle (Sections 10-11): the pivoted QR against
LAPACK's column-pivoted QR (same pivots, same |S|), its tie rule; the column
ID's identity block and the paper's error identity ||Y - Y(:, J_s) Z|| =
||S22||; exactness of the column, row, randomized row ID and CUR
decompositions on matrices of rank k; the Observation of Section 10.4 (a row
ID of any matrix spanning A's columns is one of A)."""
import numpy as np
import pytest
import scipy.linalg

from oracle import idcur, philox
from workloads import gen


@pytest.mark.parametrize("r,N,k", [(6, 40, 6), (12, 300, 9), (30, 500, 25)])
def test_cpqr_matches_lapack(r, N, k):
    Y = np.random.default_rng(r + N).standard_normal((r, N)) * np.logspace(0, -2, N)
    J, Q, S = idcur.cpqr(Y, k)
    _, R, P = scipy.linalg.qr(Y, pivoting=True, mode="economic")
    assert np.array_equal(J, P[:k])
    assert np.allclose(np.abs(S[:, P]), np.abs(R[:k]), atol=1e-12)
    assert np.allclose(Q.T @ Q, np.eye(k), atol=1e-13)
    assert np.allclose(np.tril(S[:, J], -1), 0.0, atol=1e-12)


def test_cpqr_takes_the_lowest_index_on_ties():
    Y = np.array([[1.0, 0.0, 3.0, 0.0], [0.0, 3.0, 0.0, 1.0]])
    J, _, _ = idcur.cpqr(Y, 2)
    assert list(J) == [1, 2]


def test_column_id_identity_block_and_error_identity():
    r, N, k = 20, 200, 12
    Y = np.random.default_rng(4).standard_normal((r, N)) @ np.diag(np.logspace(0, -3, N))
    J, Z = idcur.id_col(Y, k)
    assert np.allclose(Z[:, J], np.eye(k), atol=1e-12)
    _, Q, S = idcur.cpqr(Y, k)
    e_id = np.linalg.norm(Y - Y[:, J] @ Z, 2)
    e_qr = np.linalg.norm(Y - Q @ S, 2)
    assert abs(e_id - e_qr) <= 1e-9 * e_qr


@pytest.mark.parametrize("m,n,k", [(60, 80, 5), (200, 150, 12)])
def test_ids_are_exact_at_rank_k(m, n, k):
    A = gen.low_rank_matrix(m, n, np.logspace(0, -4, k), 0.0, seed=m)
    J, Z = idcur.id_col(A, k)
    assert np.abs(A - A[:, J] @ Z).max() <= 1e-11
    I, X = idcur.id_row(A, k)
    assert np.allclose(X[I, :], np.eye(k), atol=1e-12)
    assert np.abs(A - X @ A[I, :]).max() <= 1e-11


@pytest.mark.parametrize("q", [0, 1])
def test_randomized_row_id_and_cur_are_exact_at_rank_k(q):
    m, n, k, p = 300, 220, 10, 6
    A = gen.low_rank_matrix(m, n, np.logspace(0, -3, k), 0.0, seed=7)
    I, X = idcur.randomized_row_id_seeded(A, k, p, q, seed=2)
    assert len(set(I.tolist())) == k
    assert np.abs(A - X @ A[I, :]).max() <= 1e-10
    Js, U, Is = idcur.randomized_cur_seeded(A, k, p, q, seed=3)
    assert np.abs(A - A[:, Js] @ U @ A[Is, :]).max() <= 1e-9


def test_row_id_of_a_spanning_matrix_is_a_row_id_of_a():
    """Section 10.4's Observation: with A = Y F, [I_s, X] = ID_row(Y, k) gives A = X A(I_s, :)."""
    g = np.random.default_rng(11)
    m, n, k = 120, 90, 7
    Y = g.standard_normal((m, k))
    F = g.standard_normal((k, n))
    A = Y @ F
    I, X = idcur.id_row(Y, k)
    assert np.abs(A - X @ A[I, :]).max() <= 1e-11 * np.abs(A).max()


def test_randomized_row_id_error_is_near_the_optimum_on_a_decaying_spectrum():
    """The ID's error is within a modest factor of sigma_{k+1} (the paper reports the ID error as that of the
    pivoted QR it comes from)."""
    m, n, k, p = 400, 300, 15, 10
    sig = gen.spectrum("exp", 120, tau=4.0)
    A = gen.low_rank_matrix(m, n, sig, 0.0, seed=12)
    I, X = idcur.randomized_row_id_seeded(A, k, p, 1, seed=4)
    err = np.linalg.norm(A - X @ A[I, :], 2)
    assert sig[k] <= err <= 30 * sig[k]


def test_cpqr_never_repeats_a_pivot_past_the_rank():
    """k beyond the rank of Y: every residual is at rounding level, and columns already chosen (residual
    exactly projected out) must not come back."""
    g = np.random.default_rng(3)
    Y = g.standard_normal((8, 2)) @ g.standard_normal((2, 30))
    J, Q, S = idcur.cpqr(Y, 6)
    assert len(set(J.tolist())) == 6


def test_cur_index_sets_are_the_pivots_lapack_picks():
    """J_s: the pivots of the row sample's column-pivoted QR; I_s: those of A(:, J_s)^T."""
    m, n, k, p = 150, 120, 8, 6
    A = gen.low_rank_matrix(m, n, gen.spectrum("poly", 60, alpha=1.0), 1e-3, seed=21)
    G = philox.gaussian(m, k + p, 5, philox.STREAM_OMEGA)
    Js, U, Is = idcur.randomized_cur(A, G, k, 0)
    Y = G.T @ A
    _, _, P = scipy.linalg.qr(Y, pivoting=True, mode="economic")
    assert np.array_equal(Js, P[:k])
    _, _, P2 = scipy.linalg.qr(A[:, Js].T, pivoting=True, mode="economic")
    assert np.array_equal(Is, P2[:k])
