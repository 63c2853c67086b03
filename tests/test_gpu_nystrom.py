"""GPU parity of the Nystrom eigendecomposition (Section 9) through the C ABI
against the oracle on the same test matrix: FP64 and FP32 data, q = 0 (the
figure as printed) and q = 1, a rank-deficient input (a valid count of dropped
pivots, the unique results compared), the structured first sketch of Section 6,
and the full 20000 x 20000 PSD workload."""
import math

import numpy as np
import pytest

from oracle import nystrom as nys, philox, srft
from tests.gpu_helpers import device, max_rel_sigma, run_factor, subspace_sin
from workloads import gen

pytestmark = pytest.mark.gpu


def _psd(n, lam, seed):
    U = gen.orthonormal_factor(n, len(lam), seed, 1)
    A = (U * np.asarray(lam)) @ U.T
    return 0.5 * (A + A.T)


def _flags(extra=0):
    from paper_1607_01649_amd import RSVD_NYSTROM
    return RSVD_NYSTROM | extra


@pytest.mark.parametrize("n,k,p,q", [(600, 20, 10, 0), (900, 30, 10, 1), (517, 7, 9, 0)])
def test_nystrom_f64_matches_the_oracle(n, k, p, q):
    lam = np.arange(1, n + 1, dtype=float) ** -1.5
    A = _psd(n, lam, n)
    seed = 11 + q
    U, S, V, info = run_factor(A, k, p, q, "f64", seed=seed, flags=_flags())
    Ur, Lr, dropped = nys.nystrom_seeded(A, k, p, q, seed)
    assert info.status == 0 and info.dropped_cols == dropped == 0
    assert max_rel_sigma(S, Lr, k) <= 1e-10
    assert np.max(np.linalg.norm(U - Ur[:, :k], axis=0)) <= 1e-8
    assert np.array_equal(U, V)
    assert np.all(np.diff(S) <= 0) and S.min() >= 0


def test_nystrom_f32_matches_the_oracle():
    n, k, p, q, seed = 1500, 40, 20, 1, 3
    lam = np.arange(1, n + 1, dtype=float) ** -1.0
    A = _psd(n, lam, 8).astype(np.float32)
    A = 0.5 * (A + A.T)
    U, S, V, info = run_factor(A, k, p, q, "f32", seed=seed, flags=_flags())
    Ur, Lr, _ = nys.nystrom_seeded(A.astype(np.float64), k, p, q, seed)
    assert info.status == 0
    assert max_rel_sigma(S, Lr, k) <= 1e-4
    gap = Lr[k - 1] - Lr[k]
    assert subspace_sin(Ur[:, :k], U) <= 10 * 1e-4 * Lr[0] / gap


def test_nystrom_rank_deficient_input():
    """A of exact rank r < l: B2 is singular up to rounding.  Which of the l - r noise columns of Q get
    dropped is a rounding decision (their own diagonals are at rounding level), so the count is checked
    for validity on both sides, and the unique quantities (eigenvalues, reconstruction) are compared."""
    n, r, k, p, seed = 400, 12, 12, 8, 5
    lam = np.logspace(0, -3, r)
    A = _psd(n, lam, 9)
    U, S, V, info = run_factor(A, k, p, 0, "f64", seed=seed, flags=_flags())
    Ur, Lr, dropped = nys.nystrom_seeded(A, k, p, 0, seed)
    assert info.status == 0
    assert 0 <= dropped <= k + p - r and 0 <= info.dropped_cols <= k + p - r
    assert max_rel_sigma(S, lam, k) <= 1e-9 and max_rel_sigma(Lr, lam, k) <= 1e-9
    assert np.abs(A - (U * S) @ U.T).max() <= 1e-11
    assert np.allclose(U.T @ U, np.eye(k), atol=1e-10)


def test_nystrom_with_the_structured_sketch_matches_the_oracle():
    from paper_1607_01649_amd import RSVD_SKETCH_SRHT
    n, k, p, seed = 700, 15, 10, 21
    lam = np.arange(1, n + 1, dtype=float) ** -2.0
    A = _psd(n, lam, 10)
    U, S, V, info = run_factor(A, k, p, 0, "f64", seed=seed, flags=_flags(RSVD_SKETCH_SRHT))
    Ur, Lr, _ = nys.nystrom(A, srft.omega(n, k + p, seed), 0)
    assert info.status == 0
    assert max_rel_sigma(S, Lr, k) <= 1e-10
    assert np.max(np.linalg.norm(U - Ur[:, :k], axis=0)) <= 1e-8


def test_nystrom_at_the_full_psd_workload():
    """20000 x 20000 PSD (rank 2000, lambda_j = 1/j), k = 100, p = 10, q = 0 in FP32, the launch the bench
    times, against the oracle in FP64 on the same matrix and G.  FP32 products over n terms carry an error
    of about sqrt(n) u_32 relative to lambda_1 per eigenvalue; the test allows 4 times that.  Properties
    that hold at any size: U orthonormal, eigenvalues descending, interlaced from below by the planted
    spectrum (the Nystrom error A - U Lambda U^T is positive semidefinite)."""
    import torch
    from paper_1607_01649_amd import RSVD
    cfg = gen.config("psd_20000")
    A = cfg.matrix(seed=1, device=str(device()))
    n, k, p = cfg.n, cfg.k, cfg.p
    solver = RSVD(n, n, k, p, cfg.q, dtype="f32", device=device(), seed=1, flags=_flags())
    U, S, V, info = solver(A)
    torch.cuda.synchronize()
    assert info.status == 0 and info.dropped_cols == 0
    S = S.cpu().numpy()
    U = U.double().cpu().numpy()
    Ur, Lr, _ = nys.nystrom_seeded(A.double().cpu().numpy(), k, p, cfg.q, 1)
    tol = 4.0 * math.sqrt(n) * 5.96e-8 * Lr[0]
    err = np.abs(S - Lr[:k]).max()
    print(f"max |Lambda - oracle| = {err:.3e} (tol {tol:.3e})")
    assert err <= tol
    assert np.linalg.norm(U.T @ U - np.eye(k), 2) <= 1e-4
    assert np.all(np.diff(S) <= 0)
    lam = cfg.sigma()
    assert np.all(S <= lam[:k] * (1 + 1e-4))


def test_nystrom_past_128_columns():
    """l = 200: the blocked Cholesky (with its drop rule) for B2 and the block Jacobi of the small SVD."""
    n, k, p = 1000, 160, 40
    lam = np.arange(1, n + 1, dtype=float) ** -1.5
    A = _psd(n, lam, 14)
    U, S, V, info = run_factor(A, k, p, 0, "f64", seed=6, flags=_flags())
    Ur, Lr, dropped = nys.nystrom_seeded(A, k, p, 0, 6)
    assert info.status == 0 and info.dropped_cols == dropped == 0
    assert max_rel_sigma(S, Lr, k) <= 1e-9
    assert np.abs((U * S) @ U.T - (Ur[:, :k] * Lr[:k]) @ Ur[:, :k].T).max() <= 1e-10
