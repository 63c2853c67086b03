"""Pins of the structured sketch oracle (Section 6, Omega = D F S, in its
real form D H S / sqrt(N)) against facts fixed by the mathematics: the
Hadamard matrix against Sylvester's Kronecker construction and the butterfly
transform, orthogonality, the first step of the shuffle in closed form,
uniformity of the subset, exact range recovery at rank <= l, and the
Section 14 certificate on a result built with it."""
import math

import numpy as np
import pytest

from oracle import philox, rsvd as orc, srft
from workloads import gen


def _fwht(x):
    """Walsh-Hadamard transform by butterflies over the bits (no matrix)."""
    y = np.array(x, dtype=np.float64, copy=True)
    N = y.shape[0]
    h = 1
    while h < N:
        y = y.reshape(N // (2 * h), 2, h, *y.shape[1:])
        a = y[:, 0].copy()
        b = y[:, 1].copy()
        y[:, 0] = a + b
        y[:, 1] = a - b
        y = y.reshape(N, *y.shape[3:])
        h *= 2
    return y


@pytest.mark.parametrize("N", [1, 2, 4, 8, 64, 256])
def test_hadamard_is_sylvester_kronecker_power(N):
    H = np.ones((1, 1))
    while H.shape[0] < N:
        H = np.kron(np.array([[1.0, 1.0], [1.0, -1.0]]), H)
    assert np.array_equal(srft.hadamard(N), H)
    assert np.array_equal(H @ H.T, N * np.eye(N))


@pytest.mark.parametrize("N", [2, 16, 512])
def test_butterfly_transform_equals_the_matrix(N):
    x = np.random.default_rng(N).standard_normal((N, 3))
    assert np.allclose(_fwht(x), srft.hadamard(N) @ x, atol=1e-12 * N)


@pytest.mark.parametrize("n", [1, 5, 64, 100, 1000, 1024, 1025])
def test_padded_size_is_the_next_power_of_two(n):
    N = srft.padded_size(n)
    assert N >= n and N & (N - 1) == 0 and (N == 1 or N // 2 < n)


@pytest.mark.parametrize("n,l", [(256, 30), (1024, 110)])
def test_omega_has_orthonormal_columns_without_padding(n, l):
    Om = srft.omega(n, l, seed=7)
    assert np.abs(Om.T @ Om - np.eye(l)).max() < 1e-13


def test_signs_are_balanced_and_independent_of_the_subset_stream():
    d = srft.signs(200000, seed=3)
    assert set(np.unique(d)) == {-1.0, 1.0}
    assert abs(d.mean()) < 5.0 / math.sqrt(200000)
    # the subset stream uses counter word 1 = 1: a different draw than the signs
    d2 = srft.signs(64, seed=3)
    assert np.array_equal(d2, d[:64])          # prefix-stable in n


def test_first_pick_in_closed_form():
    for seed in range(20):
        key = (seed & 0xFFFFFFFF, seed >> 32)
        u0 = int(philox.philox4x32_10(np.array([[0, 1, srft.STREAM_SRHT, 0]], dtype=np.uint32), key)[0, 0])
        N = 1000 + 37 * seed
        assert srft.subset(N, 1, seed)[0] == (u0 * N) >> 32


@pytest.mark.parametrize("N,l", [(16, 5), (1024, 110), (64, 64)])
def test_subset_is_distinct_and_prefix_stable(N, l):
    s = srft.subset(N, l, seed=11)
    assert len(set(s.tolist())) == l and s.min() >= 0 and s.max() < N
    assert np.array_equal(srft.subset(N, l // 2, seed=11), s[: l // 2])
    if l == N:
        assert np.array_equal(np.sort(s), np.arange(N))


def test_subset_is_uniform_over_seeds():
    """Each index is picked with probability l / N: chi-square over 4000 seeds."""
    N, l, T = 8, 3, 4000
    cnt = np.zeros(N)
    for seed in range(T):
        cnt[srft.subset(N, l, seed)] += 1
    exp = T * l / N
    chi2 = ((cnt - exp) ** 2 / exp).sum()
    assert chi2 < 24.3          # 7 degrees of freedom, p = 0.001


def test_sketch_spans_the_range_of_an_exact_rank_matrix():
    """Property (2) of Section 6 in its exact case: rank(A) = r <= l."""
    m, n, r, l = 300, 200, 12, 20
    A = gen.low_rank_matrix(m, n, np.logspace(0, -4, r), 0.0, seed=2)
    Q = orc.orth(srft.sketch(A, l, seed=5))
    assert np.linalg.norm(A - Q @ (Q.T @ A), 2) <= 1e-12 * np.linalg.norm(A, 2)


def test_srht_rsvd_exact_rank_recovers_sigma_and_meets_the_floor():
    m, n, k, p = 400, 300, 10, 10
    sig = np.logspace(0, -3, 12)
    A = gen.low_rank_matrix(m, n, sig, 0.0, seed=4)
    res = srft.rsvd_srht(A, k, p, q=0, seed=9).truncate(k)
    assert np.allclose(res.D, sig[:k], rtol=1e-10)
    # Eckart-Young: the rank-k error cannot beat sigma_{k+1}, and with l >= rank it attains it
    E = A - (res.U * res.D) @ res.V.T
    assert np.linalg.norm(E, 2) >= sig[k] * (1 - 1e-9)
    assert np.linalg.norm(E, 2) <= sig[k] * (1 + 1e-8)


def test_srht_error_is_close_to_the_gaussian_error_on_a_decaying_spectrum():
    """Section 6: in practice the structured sketch is about as accurate as the Gaussian one."""
    m, n, k, p, q = 500, 512, 20, 20, 0
    sig = np.arange(1, 401, dtype=float) ** -1.5
    A = gen.low_rank_matrix(m, n, sig, 0.0, seed=6)
    e_s, e_g = [], []
    for seed in range(5):
        rs = srft.rsvd_srht(A, k, p, q, seed).truncate(k)
        rg = orc.rsvd_seeded(A, k, p, q, seed).truncate(k)
        e_s.append(np.linalg.norm(A - (rs.U * rs.D) @ rs.V.T, 2))
        e_g.append(np.linalg.norm(A - (rg.U * rg.D) @ rg.V.T, 2))
    assert np.mean(e_s) <= 2.0 * np.mean(e_g)
    assert min(e_s) >= sig[k] * (1 - 1e-9)


def test_certificate_bounds_the_srht_result():
    """Section 14 item (1): the Gaussian-probe certificate judges the structured result."""
    m, n, k, p = 400, 256, 10, 5
    sig = np.arange(1, 201, dtype=float) ** -1.0
    A = gen.low_rank_matrix(m, n, sig, 0.0, seed=8)
    for seed in range(10):
        r = srft.rsvd_srht(A, k, p, 0, seed).truncate(k)
        Gc = philox.gaussian(n, 10, seed, philox.STREAM_CERT)
        bound = orc.certificate(A, r.U, r.D, r.V, Gc)
        true = np.linalg.norm(A - (r.U * r.D) @ r.V.T, 2)
        assert true <= bound


def test_random_signs_center_every_entry():
    """Row 0 of H is all ones, so without D the first row of Omega would be 1/sqrt(N) in every column;
    with D every entry has mean zero over seeds."""
    n, l, T = 64, 8, 800
    acc = np.zeros((n, l))
    for seed in range(T):
        acc += srft.omega(n, l, seed) * math.sqrt(srft.padded_size(n))
    assert np.abs(acc / T).max() < 5.0 / math.sqrt(T)


@pytest.mark.parametrize("n,l", [(1, 1), (37, 10), (256, 40), (1000, 110)])
def test_row_by_row_sketch_equals_the_definition(n, l):
    A = np.random.default_rng(n).standard_normal((23, n))
    assert np.allclose(srft.sketch_rows(A, l, seed=3), srft.sketch(A, l, seed=3), atol=1e-12, rtol=0)
