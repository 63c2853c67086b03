"""Pins of the single-pass oracle (Section 5) against facts fixed by the
mathematics: the two least-squares solvers recover a consistent system's
solution exactly, satisfy the normal equations (derived from the gradient, not
from the solver) and cannot be improved by any perturbation; with one equation
set removed the joint solver is the textbook least-squares routine; the
dominant left singular vectors satisfy the eigen-relation of Y Y^T; both
methods reproduce a matrix of rank <= k exactly (an indefinite one for the
symmetric form); and the paper's two remarks hold on average: the single-pass
result is less accurate than the two-pass one, and more over-sampling helps."""
import numpy as np
import pytest

from oracle import philox, rsvd as orc, singlepass as sp
from workloads import gen


def _rng(s):
    return np.random.default_rng(s)


@pytest.mark.parametrize("k,l", [(1, 1), (3, 5), (6, 6), (7, 12)])
def test_symmetric_lstsq_recovers_a_consistent_system(k, l):
    g = _rng(k + l)
    C0 = g.standard_normal((k, k))
    C0 = C0 + C0.T
    M = g.standard_normal((k, l))
    C = sp.lstsq_symmetric(M, C0 @ M)
    assert np.allclose(C, C0, atol=1e-11)
    assert np.array_equal(C, C.T)


@pytest.mark.parametrize("k,l", [(2, 4), (5, 9), (8, 10)])
def test_symmetric_lstsq_meets_the_normal_equations_and_is_optimal(k, l):
    g = _rng(10 * k + l)
    M = g.standard_normal((k, l))
    N = g.standard_normal((k, l))
    C = sp.lstsq_symmetric(M, N)
    # gradient over symmetric directions: (C M - N) M^T + M (C M - N)^T = 0
    R = (C @ M - N) @ M.T
    assert np.abs(R + R.T).max() <= 1e-11 * np.abs(N).max() * np.abs(M).max()
    f0 = np.linalg.norm(C @ M - N) ** 2
    for t in range(20):
        E = g.standard_normal((k, k))
        E = 1e-3 * (E + E.T)
        assert np.linalg.norm((C + E) @ M - N) ** 2 >= f0
    # the unconstrained minimiser is not symmetric in general, and does better
    Cu = np.linalg.lstsq(M.T, N.T, rcond=None)[0].T
    assert np.linalg.norm(Cu @ M - N) <= np.sqrt(f0) + 1e-12


@pytest.mark.parametrize("k,l", [(1, 1), (3, 5), (7, 12)])
def test_joint_lstsq_recovers_a_consistent_system(k, l):
    g = _rng(k * l + 3)
    C0 = g.standard_normal((k, k))
    M1 = g.standard_normal((l, k))
    M2 = g.standard_normal((k, l))
    C = sp.lstsq_joint(M1, M1 @ C0, M2, C0 @ M2)
    assert np.allclose(C, C0, atol=1e-11)


@pytest.mark.parametrize("k,l", [(2, 4), (6, 9)])
def test_joint_lstsq_meets_the_normal_equations_and_is_optimal(k, l):
    g = _rng(7 * k + l)
    M1, N1 = g.standard_normal((l, k)), g.standard_normal((l, k))
    M2, N2 = g.standard_normal((k, l)), g.standard_normal((k, l))
    C = sp.lstsq_joint(M1, N1, M2, N2)
    # M1^T (M1 C - N1) + (C M2 - N2) M2^T = 0
    grad = M1.T @ (M1 @ C - N1) + (C @ M2 - N2) @ M2.T
    assert np.abs(grad).max() <= 1e-11 * 10 * l
    f = lambda X: np.linalg.norm(M1 @ X - N1) ** 2 + np.linalg.norm(X @ M2 - N2) ** 2
    f0 = f(C)
    for t in range(20):
        assert f(C + 1e-3 * g.standard_normal((k, k))) >= f0


def test_joint_lstsq_with_one_equation_set_is_the_textbook_solution():
    g = _rng(5)
    k, l = 4, 9
    M1, N1 = g.standard_normal((l, k)), g.standard_normal((l, k))
    M2, N2 = g.standard_normal((k, l)), g.standard_normal((k, l))
    Z = np.zeros((k, l))
    assert np.allclose(sp.lstsq_joint(M1, N1, Z, Z), np.linalg.lstsq(M1, N1, rcond=None)[0], atol=1e-12)
    Zt = np.zeros((l, k))
    assert np.allclose(sp.lstsq_joint(Zt, Zt, M2, N2), np.linalg.lstsq(M2.T, N2.T, rcond=None)[0].T, atol=1e-12)


def test_dominant_left_vectors_satisfy_the_eigen_relation():
    g = _rng(9)
    Y = g.standard_normal((60, 12)) @ np.diag(np.logspace(0, -2, 12))
    Q = sp.dominant_left(Y, 5)
    lam = np.linalg.svd(Y, compute_uv=False)[:5] ** 2
    assert np.allclose(Q.T @ Q, np.eye(5), atol=1e-13)
    assert np.allclose((Y @ (Y.T @ Q)), Q * lam, atol=1e-12)


@pytest.mark.parametrize("n,r,k,p", [(80, 6, 6, 6), (120, 5, 8, 10)])
def test_symmetric_method_is_exact_at_rank_at_most_k(n, r, k, p):
    lam = np.array([3.0, -2.0, 1.5, -1.0, 0.5, 0.25][:r])
    U0 = gen.orthonormal_factor(n, r, n, 1)
    A = (U0 * lam) @ U0.T
    A = 0.5 * (A + A.T)
    U, D, C = sp.single_pass_sym_seeded(A, k, p, seed=3)
    order = np.argsort(-np.abs(lam))
    assert np.allclose(D[:r], lam[order], atol=1e-12)
    assert np.allclose(D[r:], 0.0, atol=1e-12)
    assert np.abs(A - (U * D) @ U.T).max() <= 1e-12
    assert np.allclose(U.T @ U, np.eye(k), atol=1e-12)


@pytest.mark.parametrize("m,n,r,k,p", [(90, 70, 7, 7, 7), (150, 110, 4, 9, 6)])
def test_general_method_is_exact_at_rank_at_most_k(m, n, r, k, p):
    sig = np.logspace(0, -3, r)
    A = gen.low_rank_matrix(m, n, sig, 0.0, seed=m)
    U, D, V, C = sp.single_pass_gen_seeded(A, k, p, seed=4)
    assert np.allclose(D[:r], sig, rtol=1e-10)
    assert np.allclose(D[r:], 0.0, atol=1e-12)
    assert np.abs(A - (U * D) @ V.T).max() <= 1e-12
    assert np.allclose(U.T @ U, np.eye(k), atol=1e-12) and np.allclose(V.T @ V, np.eye(k), atol=1e-12)


def _noisy(m, n, seed):
    sig = gen.spectrum("poly", 60, alpha=1.0)
    return gen.low_rank_matrix(m, n, sig, 1e-3, seed=seed)


def test_single_pass_is_less_accurate_than_two_passes_on_average():
    """Section 5: the single-pass factorisation tends to be less accurate than Figure 1's."""
    m, n, k, p = 300, 200, 10, 10
    A = _noisy(m, n, 1)
    e1, e2 = [], []
    for seed in range(6):
        U, D, V, _ = sp.single_pass_gen_seeded(A, k, p, seed)
        e1.append(np.linalg.norm(A - (U * D) @ V.T, 2))
        ref = orc.rsvd_seeded(A, k, p, 0, seed).truncate(k)
        e2.append(np.linalg.norm(A - (ref.U * ref.D) @ ref.V.T, 2))
    assert np.mean(e1) > np.mean(e2)


@pytest.mark.parametrize("method", ["gen", "sym"])
def test_more_over_sampling_helps_on_average(method):
    """Section 5.1's remark: over-sampling more aggressively (up to p = k) improves the single-pass result."""
    n, k = 240, 12
    sig = gen.spectrum("poly", 80, alpha=1.0)
    U0 = gen.orthonormal_factor(n, 80, 2, 1)
    A = (U0 * sig) @ U0.T
    A = 0.5 * (A + A.T)
    err = {}
    for p in (2, k):
        e = []
        for seed in range(6):
            if method == "gen":
                U, D, V, _ = sp.single_pass_gen_seeded(A, k, p, seed)
                e.append(np.linalg.norm(A - (U * D) @ V.T, 2))
            else:
                U, D, _ = sp.single_pass_sym_seeded(A, k, p, seed)
                e.append(np.linalg.norm(A - (U * D) @ U.T, 2))
        err[p] = np.mean(e)
    assert err[k] < err[2]
