"""Pins of the Nystrom oracle (Section 9) against facts fixed by the
mathematics: the dropping Cholesky against LAPACK and on a singular matrix of
known rank, exact recovery at rank <= l, the error A - U Lambda U^T positive
semidefinite (so the eigenvalues interlace from below), the printed formula
(AQ)(Q^T A Q)^-1 (AQ)^T, and the paper's claim that it beats the plain
Q (Q^T A Q) Q^T on average."""
import numpy as np
import pytest

from oracle import nystrom as nys, philox, rsvd as orc
from workloads import gen


def _psd(n, lam, seed):
    U = gen.orthonormal_factor(n, len(lam), seed, 1)
    return (U * np.asarray(lam)) @ U.T


@pytest.mark.parametrize("n", [1, 7, 40])
def test_chol_drop_is_cholesky_on_spd(n):
    X = np.random.default_rng(n).standard_normal((3 * n + 2, n))
    B = X.T @ X
    C, Cinv, dropped = nys.chol_drop(B, 1e-14)
    assert dropped == 0
    assert np.allclose(C, np.linalg.cholesky(B).T, rtol=1e-12, atol=1e-12 * np.abs(B).max())
    assert np.allclose(Cinv @ C, np.eye(n), atol=1e-10)


def test_chol_drop_on_a_singular_matrix_drops_the_dependent_pivots():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((30, 6))
    X[:, 2] = X[:, 0] + 3 * X[:, 1]
    X[:, 5] = X[:, 3] - X[:, 4]
    B = X.T @ X
    C, Cinv, dropped = nys.chol_drop(B, 1e-10)
    assert dropped == 2
    assert np.allclose(C.T @ C, B, atol=1e-9 * np.abs(B).max())
    assert np.allclose(C[[2, 5]], 0) and np.allclose(Cinv[:, [2, 5]], 0)


def test_exact_rank_is_recovered():
    n, r, k, p = 300, 12, 10, 6
    lam = np.logspace(0, -4, r)
    A = _psd(n, lam, 3)
    U, L, dropped = nys.nystrom_seeded(A, k, p, 0, seed=5)
    assert np.allclose(L[:r], lam, rtol=1e-9)
    assert np.allclose(L[r:], 0, atol=1e-12)
    assert np.abs(A - (U[:, :r] * L[:r]) @ U[:, :r].T).max() <= 1e-12
    assert dropped == k + p - r


def test_error_is_psd_and_eigenvalues_interlace_from_below():
    n, k, p = 200, 10, 5
    lam = np.arange(1, n + 1, dtype=float) ** -1.0
    A = _psd(n, lam, 4)
    for seed in range(3):
        U, L, _ = nys.nystrom_seeded(A, k, p, 0, seed)
        E = A - (U * L) @ U.T
        assert np.linalg.eigvalsh(0.5 * (E + E.T)).min() >= -1e-12
        assert np.all(L <= lam[:k + p] * (1 + 1e-12))
        assert np.allclose(U.T @ U, np.eye(k + p), atol=1e-12)
        assert np.all(np.diff(L) <= 0) and L.min() >= 0


def test_factor_reproduces_the_printed_formula():
    n, l = 150, 12
    lam = np.arange(1, n + 1, dtype=float) ** -2.0
    A = _psd(n, lam, 6)
    G = philox.gaussian(n, l, 2, philox.STREAM_OMEGA)
    U, L, _ = nys.nystrom(A, G, 0)
    Q = orc.orth(A @ G)
    AQ = A @ Q
    ref = AQ @ np.linalg.inv(Q.T @ AQ) @ AQ.T
    assert np.allclose((U * L) @ U.T, ref, atol=1e-10 * np.abs(ref).max())


def test_nystrom_beats_the_plain_projection_on_average():
    """Section 9: the same two applications of A, a more accurate result."""
    n, k, p = 400, 15, 5
    lam = np.arange(1, n + 1, dtype=float) ** -1.0
    A = _psd(n, lam, 7)
    e_n, e_p = [], []
    for seed in range(8):
        G = philox.gaussian(n, k + p, seed, philox.STREAM_OMEGA)
        U, L, _ = nys.nystrom(A, G, 0)
        Q = orc.orth(A @ G)
        e_n.append(np.linalg.norm(A - (U * L) @ U.T, 2))
        e_p.append(np.linalg.norm(A - Q @ (Q.T @ A @ Q) @ Q.T, 2))
    assert np.mean(e_n) < np.mean(e_p)
