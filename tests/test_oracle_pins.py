"""Pins of the CPU oracle against facts the paper and the mathematics fix.

None of these re-types the oracle's own formula: each checks a property,
special case, published known answer or theorem that a plausible mistake in
the oracle (a dropped term, a wrong sign or index, a transposed operand)
would violate.
"""
import math
import os

import numpy as np
import pytest

from oracle import philox, rsvd as orc
from workloads import gen


def _low_rank(m, n, sigma, seed, noise=0.0):
    return gen.low_rank_matrix(m, n, np.asarray(sigma, float), noise, seed)


# ---------------------------------------------------------------- generator

def test_philox_known_answers(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(w, 16) for w in line.split()])
    for r in rows:
        out = philox.philox4x32_10(np.array(r[0:4], dtype=np.uint32), (r[4], r[5]))
        assert [int(x) for x in out] == r[6:10]


def test_gaussian_moments_and_prefix_stability():
    g = philox.gaussian(200_001, 10, seed=12345, stream=philox.STREAM_OMEGA)
    x = g.ravel()
    n = x.size
    assert abs(x.mean()) < 5 / math.sqrt(n)
    assert abs(x.var() - 1.0) < 5 * math.sqrt(2.0 / n)
    kurt = np.mean(x ** 4)
    assert abs(kurt - 3.0) < 5 * math.sqrt(96.0 / n)
    # columns are independent of how many are drawn; rows of a shorter draw
    # are a prefix of a longer one (odd row counts included)
    a = philox.gaussian(37, 9, seed=7, stream=4)
    b = philox.gaussian(38, 4, seed=7, stream=4, col0=5)
    assert np.array_equal(a[:, 5:9], b[:37])
    # different streams and seeds differ
    assert not np.allclose(philox.gaussian(8, 2, 7, 4), philox.gaussian(8, 2, 7, 6))
    assert not np.allclose(philox.gaussian(8, 2, 7, 4), philox.gaussian(8, 2, 8, 4))
    # columns uncorrelated
    c = np.corrcoef(g[:, :4].T)
    assert np.max(np.abs(c - np.eye(4))) < 5 / math.sqrt(g.shape[0])


# ---------------------------------------------------------------- primitives

def test_orth_is_an_unpivoted_qr_with_positive_diagonal():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((120, 17))
    Q = orc.orth(X)
    assert np.linalg.norm(Q.T @ Q - np.eye(17)) < 1e-13
    R = Q.T @ X
    assert np.linalg.norm(np.tril(R, -1)) < 1e-12 * np.linalg.norm(X)
    assert np.all(np.diag(R) > 0)
    assert np.linalg.norm(Q @ R - X) < 1e-13 * np.linalg.norm(X)
    # special case: an orthonormal, upper-trapezoidal X is returned unchanged
    E = np.eye(30)[:, :6]
    assert np.array_equal(orc.orth(E), E)
    # unpivoted: the first column of Q is the normalised first column of X
    assert np.allclose(Q[:, 0], X[:, 0] / np.linalg.norm(X[:, 0]), atol=1e-14)


def test_svd_small_recovers_a_planted_factorisation():
    rng = np.random.default_rng(1)
    U0 = orc.orth(rng.standard_normal((25, 25)))
    V0 = orc.orth(rng.standard_normal((90, 25)))
    d0 = np.sort(rng.uniform(0.1, 3.0, 25))[::-1]
    B = (U0 * d0) @ V0.T
    uh, d, v = orc.svd_small(B)
    assert np.allclose(d, d0, rtol=1e-13, atol=0)
    for j in range(25):
        s = np.sign(U0[np.argmax(np.abs(U0[:, j])), j])
        assert np.allclose(uh[:, j], s * U0[:, j], atol=1e-12)
        assert np.allclose(v[:, j], s * V0[:, j], atol=1e-12)
        assert uh[np.argmax(np.abs(uh[:, j])), j] > 0
    # a diagonal matrix with known entries
    D = np.diag([1.0, 5.0, 3.0])
    uh, d, v = orc.svd_small(np.hstack([D, np.zeros((3, 2))]))
    assert np.array_equal(d, [5.0, 3.0, 1.0])
    assert np.array_equal(np.abs(uh), np.eye(3)[:, [1, 2, 0]])


# ---------------------------------------------------------------- Section 3/4

def test_exact_rank_is_recovered_exactly():
    """Section 4: when A has exact rank k, A G spans its range with probability 1."""
    sigma = np.array([3.0, 2.0, 1.0, 0.5, 0.25, 0.1])
    A = _low_rank(200, 150, sigma, seed=3)
    G = gen.gaussian_matrix(150, 8, seed=4)
    r = orc.rsvd_basic(A, G)
    assert np.allclose(r.D[:6], sigma, rtol=1e-12)
    assert np.all(r.D[6:] < 1e-13)
    assert np.linalg.norm(A - (r.U * r.D) @ r.V.T, 2) < 1e-13


def test_full_width_sketch_equals_the_full_svd():
    """Brute force on a tiny input: with l = n the RSVD is the exact SVD."""
    rng = np.random.default_rng(5)
    A = rng.standard_normal((14, 9))
    r = orc.rsvd(A, gen.gaussian_matrix(9, 9, seed=6), q=1)
    s = np.linalg.svd(A, compute_uv=False)
    assert np.allclose(r.D, s, rtol=1e-12)
    assert np.linalg.norm(A - (r.U * r.D) @ r.V.T) < 1e-12


def test_eckart_young_floor_and_stage_b_identity():
    """Section 2.2: sigma_{k+1} (spectral) and the tail norm (Frobenius) are the
    smallest rank-k errors.  Remark in Section 3: Stage B adds no error, so at
    rank l the factorisation error equals ||A - Q Q^T A||.  Second remark:
    |sigma_i - D_ii| <= ||A - Q Q^T A||."""
    sigma = gen.spectrum("poly", 60, alpha=1.0)
    A = _low_rank(300, 220, sigma, seed=9)
    k, p = 12, 6
    r = orc.rsvd(A, gen.gaussian_matrix(220, k + p, seed=10), q=0)
    t = r.truncate(k)
    err_k = np.linalg.norm(A - (t.U * t.D) @ t.V.T, 2)
    assert err_k >= sigma[k] * (1 - 1e-12)
    assert np.linalg.norm(A - (t.U * t.D) @ t.V.T) >= np.sqrt(np.sum(sigma[k:] ** 2)) * (1 - 1e-12)
    resid = A - r.Q @ (r.Q.T @ A)
    e_qq = np.linalg.norm(resid, 2)
    e_full = np.linalg.norm(A - (r.U * r.D) @ r.V.T, 2)
    assert abs(e_full - e_qq) < 1e-12
    assert abs(np.linalg.norm(A - (r.U * r.D) @ r.V.T) - np.linalg.norm(resid)) < 1e-12
    assert np.all(np.abs(sigma[:k + p] - r.D) <= e_qq * (1 + 1e-12))
    # U and V orthonormal
    assert np.linalg.norm(r.U.T @ r.U - np.eye(k + p)) < 1e-13
    assert np.linalg.norm(r.V.T @ r.V - np.eye(k + p)) < 1e-13


# ---------------------------------------------------------------- Section 7, 8

def _errors(A, k, p, q, seeds, fig=orc.rsvd):
    fro, spec = [], []
    for s in seeds:
        G = gen.gaussian_matrix(A.shape[1], k + p, seed=1000 + s)
        r = fig(A, G, q)
        R = A - r.Q @ (r.Q.T @ A)
        fro.append(np.linalg.norm(R))
        spec.append(np.linalg.norm(R, 2))
    return np.array(fro), np.array(spec)


def test_expectation_bounds_q0():
    """Theorem of Section 7.1 (both norms) at q = 0, mean over 200 draws."""
    sigma = gen.spectrum("poly", 150, alpha=1.0)
    A = _low_rank(260, 180, sigma, seed=21)
    k, p = 10, 5
    fro, spec = _errors(A, k, p, 0, range(200))
    bf = orc.thm_expectation_frobenius(sigma, k, p)
    bs = orc.thm_expectation_spectral(sigma, k, p, 0)
    assert fro.mean() + 3 * fro.std() / math.sqrt(len(fro)) <= bf
    assert spec.mean() + 3 * spec.std() / math.sqrt(len(spec)) <= bs
    # and never below the Eckart-Young floor
    assert spec.min() >= sigma[k] * (1 - 1e-12)
    assert fro.min() >= math.sqrt(np.sum(sigma[k:] ** 2)) * (1 - 1e-12)


@pytest.mark.parametrize("q", [1, 2])
def test_expectation_bound_with_power_steps(q):
    """Theorem of Section 8.2 for the power scheme (the re-orthonormalised
    Figure 5 spans the same space in exact arithmetic)."""
    sigma = gen.spectrum("poly", 150, alpha=0.5)
    A = _low_rank(260, 180, sigma, seed=22)
    k, p = 10, 4
    _, spec = _errors(A, k, p, q, range(150))
    assert spec.mean() + 3 * spec.std() / math.sqrt(len(spec)) <= orc.thm_expectation_spectral(sigma, k, p, q)
    # more power steps, smaller mean error on a slowly decaying spectrum
    _, spec0 = _errors(A, k, p, 0, range(150))
    assert spec.mean() < spec0.mean()


def test_tail_bound_frequency():
    """Section 7.2: the deviation bound fails with probability <= 3 e^-p."""
    sigma = gen.spectrum("poly", 120, alpha=0.7)
    A = _low_rank(200, 150, sigma, seed=23)
    k, p = 8, 4
    _, spec = _errors(A, k, p, 0, range(300))
    bound = orc.thm_tail_spectral(sigma, k, p)
    freq = np.mean(spec > bound)
    assert freq <= 3 * math.exp(-p) + 3 * math.sqrt(3 * math.exp(-p) / 300)


def test_power_scheme_targets_the_spectrum_of_A_q():
    """Section 8.1: (A A^T)^q A = U D^(2q+1) V^T.  Build A^(q) from the
    generator's factors (no product with A) and check that the oracle's
    Figure 5 basis spans orth(A^(q) G) for the same G."""
    r_ = 40
    sigma = gen.spectrum("exp", r_, tau=8.0)
    m, n = 180, 140
    U = gen.orthonormal_factor(m, r_, 31, 1)
    V = gen.orthonormal_factor(n, r_, 31, 2)
    A = (U * sigma) @ V.T
    G = gen.gaussian_matrix(n, 12, seed=32)
    for q in (1, 2):
        Aq = (U * sigma ** (2 * q + 1)) @ V.T
        Qref = orc.orth(Aq @ G)
        Q = orc.rsvd(A, G, q).Q
        # principal angles between the two 12-dim subspaces
        cosines = np.linalg.svd(Qref.T @ Q, compute_uv=False)
        assert np.min(cosines) > 1 - 1e-9
        # and Figure 4 (no re-orthonormalisation) agrees in float64 here
        Q4 = orc.rsvd_power(A, G, q).Q
        assert np.min(np.linalg.svd(Q4.T @ Q, compute_uv=False)) > 1 - 1e-9


def test_without_reorthonormalisation_information_is_lost():
    """Remark after Figure 4: directions with sigma_j / sigma_1 <=
    eps_mach^(1/(2q+1)) are lost without re-orthonormalisation; Figure 5
    keeps them."""
    q = 3
    sigma = np.logspace(0, -6, 40)          # reaches 1e-6 << eps^(1/7) ~ 5e-3
    A = _low_rank(150, 120, sigma, seed=41)
    G = gen.gaussian_matrix(120, 40, seed=42)
    good = orc.rsvd(A, G, q)
    bad = orc.rsvd_power(A, G, q)
    j = 30                                   # sigma_j ~ 2.5e-5
    thresh = np.finfo(float).eps ** (1 / (2 * q + 1))
    assert sigma[j] / sigma[0] < thresh
    assert abs(good.D[j] - sigma[j]) / sigma[j] < 1e-6
    assert abs(bad.D[j] - sigma[j]) / sigma[j] > 1e-2


# ---------------------------------------------------------------- Sections 12-14

def test_probe_lemma_failure_rate_and_mean_square():
    """Lemma of Section 13: P(bound < ||T||) <= alpha^r; remark after Figure 14:
    E||T g||^2 = ||T||_F^2."""
    rng = np.random.default_rng(50)
    T = rng.standard_normal((40, 30)) * np.logspace(0, -2, 30)
    t2 = np.linalg.norm(T, 2)
    trials = 4000
    G = rng.standard_normal((30, trials))
    norms = np.linalg.norm(T @ G, axis=0)
    # r = 1, alpha = 1/2: failure probability <= 1/2
    fails = np.mean([orc.probe_bound(norms[i:i + 1], 0.5) < t2 for i in range(trials)])
    assert fails <= 0.5 + 3 * math.sqrt(0.25 / trials)
    # r = 2, alpha = 0.1: <= 0.01
    fails2 = np.mean([orc.probe_bound(norms[i:i + 2], 0.1) < t2 for i in range(0, trials, 2)])
    assert fails2 <= 0.01 + 3 * math.sqrt(0.01 / (trials / 2))
    ms = np.mean(norms ** 2)
    f2 = np.linalg.norm(T) ** 2
    assert abs(ms - f2) < 4 * np.std(norms ** 2) / math.sqrt(trials)


@pytest.mark.parametrize("s", [0, 1, 2])
def test_certificate_bounds_the_true_error(s):
    """Section 14: 10 probes, alpha = 0.1, bound valid w.p. >= 1 - 1e-10; the
    powered variant bounds ||T|| through ||(T T^T)^s T|| = ||T||^(2s+1)."""
    sigma = gen.spectrum("poly", 80, alpha=1.0)
    A = _low_rank(160, 120, sigma, seed=60)
    r = orc.rsvd(A, gen.gaussian_matrix(120, 16, seed=61), 1).truncate(10)
    true = np.linalg.norm(A - (r.U * r.D) @ r.V.T, 2)
    ratios = []
    for t in range(40):
        Gc = gen.gaussian_matrix(120, 10, seed=100 + t)
        b = orc.certificate(A, r.U, r.D, r.V, Gc, s)
        assert b >= true
        ratios.append(b / true)
    if s > 0:   # the powered estimate is tighter on average
        b0 = np.mean([orc.certificate(A, r.U, r.D, r.V, gen.gaussian_matrix(120, 10, seed=100 + t), 0) / true
                      for t in range(40)])
        assert np.mean(ratios) < b0


def test_frobenius_downdating_identity():
    """Section 12.4: ||A - Q B||_F^2 = ||A||_F^2 - ||B||_F^2 for B = Q^T A."""
    rng = np.random.default_rng(70)
    A = rng.standard_normal((90, 70)) @ np.diag(np.logspace(0, -3, 70))
    Q = orc.orth(A @ rng.standard_normal((70, 15)))
    B = Q.T @ A
    direct = np.linalg.norm(A - Q @ B)
    assert abs(orc.frobenius_downdate(np.linalg.norm(A), B) - direct) < 1e-12 * np.linalg.norm(A)


@pytest.mark.parametrize("b", [1, 4])
def test_blocked_growth_spans_the_same_space_as_the_basic_sketch(b):
    """Caption of Figure 13: building Q a few vectors at a time from the
    columns of G gives an orthonormal basis of A G(:, 1:j), as the basic
    RSVD does."""
    sigma = gen.spectrum("poly", 60, alpha=1.0)
    A = _low_rank(150, 100, sigma, seed=80)
    G = gen.gaussian_matrix(100, 24, seed=81)
    Q0 = orc.orth(A @ G[:, :8])
    steps_wanted = 16 // b

    def draw(j):
        return G[:, 8 + j * b: 8 + (j + 1) * b]
    Q, B, steps, hist = orc.blocked_growth(A, Q0, Q0.T @ A, draw,
                                           lambda Q_, B_: Q_.shape[1] >= 24, b, 24)
    assert steps == steps_wanted and Q.shape[1] == 24
    assert np.linalg.norm(Q.T @ Q - np.eye(24)) < 1e-12
    Qref = orc.orth(A @ G)
    assert np.min(np.linalg.svd(Qref.T @ Q, compute_uv=False)) > 1 - 1e-10
    assert np.all(np.diff(hist) <= 1e-12)   # residual never grows


def test_adaptive_vector_finder_meets_its_tolerance():
    """Figure 14: the output Q satisfies ||A - Q Q^T A|| <= eps (w.p. >= 1 -
    min(m,n) 10^-r)."""
    sigma = gen.spectrum("exp", 80, tau=5.0)
    A = _low_rank(120, 100, sigma, seed=90)
    eps = 1e-4
    Q = orc.adaptive_vector(A, eps, r=10, draw=lambda j: gen.gaussian_matrix(100, 1, seed=2000 + j)[:, 0])
    err = np.linalg.norm(A - Q @ (Q.T @ A), 2)
    assert err <= eps
    assert Q.shape[1] < 80
    assert np.linalg.norm(Q.T @ Q - np.eye(Q.shape[1])) < 1e-12


def test_factor_with_fallback_reaches_the_tolerance():
    """The certificate (Section 14) rejects the rank-k result, the blocked
    range finder (Figure 12) grows the basis until the certificate holds, and
    the true error then meets the tolerance."""
    sigma = gen.spectrum("exp", 120, tau=10.0)
    A = _low_rank(200, 160, sigma, seed=95)
    out = orc.factor(A, k=10, p=5, q=1, seed=96, eps=1e-3, block=8, max_rank=120)
    assert out.certified and out.fallback_steps > 0
    assert out.rank > 15
    true = np.linalg.norm(A - (out.U * out.D) @ out.V.T, 2)
    assert true <= 1e-3 * out.sigma1
    assert out.bound >= true
    # the fixed-rank path alone (eps = 0) returns rank k
    plain = orc.factor(A, k=10, p=5, q=1, seed=96)
    assert plain.rank == 10 and plain.U.shape == (200, 10)
    # singular values of Q^T A interlace those of A from below
    assert np.all(plain.D <= sigma[:10] * (1 + 1e-12))
    assert np.allclose(plain.D, sigma[:10], rtol=1e-2)


# ---------------------------------------------------------------- quantisation

def test_bf16_rounding_exhaustive():
    """Every bfloat16 code is a fixed point; the midpoint between neighbouring
    codes rounds to the even one; the result agrees with torch's (CPU) RNE
    conversion on random binary32 values, subnormals, infinities and NaN."""
    import torch
    from oracle import quant
    codes = np.arange(65536, dtype=np.uint32)
    vals = (codes << 16).view(np.float32)
    finite = np.isfinite(vals)
    assert np.array_equal(quant.bf16_bits(vals[finite]), codes[finite].astype(np.uint16))
    # midpoints: code | 0x8000 rounds to the even neighbour
    mids = ((codes << 16) | 0x8000).view(np.float32)
    ok = np.isfinite(mids) & np.isfinite(((codes + 1) << 16).view(np.float32)) & (codes < 0x7F7F) | (
        (codes >= 0x8000) & (codes < 0xFF7F))
    got = quant.bf16_bits(mids[ok]).astype(np.uint32)
    c = codes[ok]
    want = np.where(c % 2 == 0, c, c + 1)
    assert np.array_equal(got, want)
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(200000).astype(np.float32) * np.float32(1e3),
                        (rng.integers(0, 2 ** 32, 200000, dtype=np.uint64).astype(np.uint32)).view(np.float32),
                        np.array([np.inf, -np.inf, 1e-45, -1e-40, 3.4e38], dtype=np.float32)])
    x = x[np.isfinite(x) | np.isinf(x)]
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ref, quant.bf16_round(x))
    assert np.isnan(quant.bf16_round(np.array([np.nan], dtype=np.float32)))[0]


def test_quantised_rsvd_reduces_to_the_plain_oracle_on_representable_data():
    """Integers of magnitude <= 256 are exact in bfloat16; with such A and
    Omega the first product is unchanged, so the quantisation-aware run and
    the plain one share Y exactly and differ only through the rounding of the
    later thin operands, which is small."""
    from oracle import quant
    rng = np.random.default_rng(3)
    A = rng.integers(-8, 9, size=(60, 40)).astype(np.float64)
    G = rng.integers(-4, 5, size=(40, 12)).astype(np.float64)
    a = orc.rsvd(A, G, 0)
    b = quant.rsvd_quantized(A, G, 0, "bf16", "f32")
    assert np.allclose(a.Q, b.Q, atol=1e-12)       # same Y -> same orth
    c = quant.rsvd_quantized(A, G, 0, "f32", "f32")
    assert np.allclose(a.D, c.D, rtol=1e-6)
    d = quant.rsvd_quantized(A, G, 1, "bf16", "bf16")
    assert np.max(np.abs(d.D - orc.rsvd(A, G, 1).D) / orc.rsvd(A, G, 1).D[0]) < 1e-2


def test_fp8_e4m3_codes_and_rounding():
    """OCP E4M3 landmarks (largest 448 = 0x7E, smallest normal 2^-6 = 0x08,
    smallest subnormal 2^-9 = 0x01, 1.0 = 0x38, NaN = 0x7F, no infinities),
    values strictly increasing over the codes, every finite code a fixed point,
    midpoints to the even code, saturation above 448."""
    from oracle import quant
    d = quant.fp8_e4m3_decode(np.arange(256))
    assert d[0x7E] == 448.0 and d[0x08] == 2.0 ** -6 and d[0x01] == 2.0 ** -9 and d[0x38] == 1.0
    assert d[0x07] == 7 * 2.0 ** -9 and d[0x10] == 2.0 ** -5 and d[0x3F] == 1.875
    assert np.isnan(d[0x7F]) and np.isnan(d[0xFF]) and not np.any(np.isinf(d))
    assert np.all(np.diff(d[:0x7F]) > 0)
    assert np.array_equal(d[0x80:0xFF], -d[0x00:0x7F])
    fin = np.arange(256)[np.isfinite(d)]
    assert np.array_equal(quant.fp8_e4m3_bits(d[fin]), fin.astype(np.uint8))
    mids = (d[0:0x7E] + d[1:0x7F]) / 2
    got = quant.fp8_e4m3_bits(mids).astype(int)
    want = np.where(np.arange(0x7E) % 2 == 0, np.arange(0x7E), np.arange(1, 0x7F))
    assert np.array_equal(got, want)
    assert np.all(quant.fp8_e4m3_bits(np.array([449.0, 1e9, -1e30])) == [0x7E, 0x7E, 0xFE])
    # just off the midpoints: nearest wins
    eps = np.diff(d[:0x7F]) * 1e-3
    assert np.array_equal(quant.fp8_e4m3_bits(mids + eps).astype(int), np.arange(1, 0x7F))
    assert np.array_equal(quant.fp8_e4m3_bits(mids - eps).astype(int), np.arange(0, 0x7E))


def test_fp8_block_scale_rule():
    """2^e is the least power of two with amax <= 448 2^e."""
    from oracle import quant
    rng = np.random.default_rng(5)
    a = np.concatenate([[448.0, 224.0, 1.0, 16.0, 1.75, 2.0 ** -30],
                        np.exp(rng.uniform(-40, 40, 5000))]).astype(np.float32).astype(np.float64)
    e = quant.fp8_scale_exponent(a)
    assert np.all(a <= 448.0 * 2.0 ** e) and np.all(a > 448.0 * 2.0 ** (e - 1))
    assert quant.fp8_scale_exponent(0.0) == 0
    # E8M0 range: the least exponent is -127 (only below 448 2^-127 does the limit bite)
    assert quant.fp8_scale_exponent(448.0 * 2.0 ** -127) == -127
    assert quant.fp8_scale_exponent(449.0 * 2.0 ** -127) == -126
    assert quant.fp8_scale_exponent(2.0 ** -140) == -127
    assert quant.fp8_scale_exponent(np.float32(1e-45)) == -127    # smallest subnormal
    # a tiny block keeps scale 2^-127: its values are rounded on that grid (here all to zero or subnormal codes)
    blk = np.full((4, 4), 2.0 ** -140)
    codes, ex, deq = quant.fp8_blocks_matrix(blk, tile=4)
    assert ex[0, 0] == -127 and np.all(codes == quant.fp8_e4m3_bits(blk * 2.0 ** 127))
    codes, ex, deq = quant.fp8_blocks_matrix(rng.standard_normal((300, 200)) * 10, tile=128)
    assert ex.shape == (3, 2)
    assert np.all(np.abs(quant.fp8_e4m3_decode(codes)) <= 448)


def test_fp8_quantised_rsvd_on_representable_data():
    """Integers of magnitude <= 16 times a power of two are exact in E4M3 under
    the block scale, so A is unchanged by its quantisation; with the thin
    operands left in FP32 the quantisation-aware run equals the plain one."""
    from oracle import quant
    rng = np.random.default_rng(7)
    A = rng.integers(-16, 17, size=(200, 150)).astype(np.float64)
    A[0, 0] = 16.0
    assert np.array_equal(quant.fp8_blocks_matrix(A)[2], A)
    G = rng.standard_normal((150, 12))
    a = orc.rsvd(A, G.astype(np.float32).astype(np.float64), 1)
    b = quant.rsvd_quantized(A, G, 1, "f32", "f32")
    assert np.allclose(a.D, b.D, rtol=1e-6)
    c = quant.rsvd_quantized(A, G, 1, "fp8", "fp8")
    assert np.max(np.abs(c.D - a.D) / a.D[0]) < 0.1


# ---------------------------------------------------------------- selector network and rule

def _mlp_case(seed, nb=7):
    from oracle import mlp
    g = np.random.default_rng(seed)
    theta = mlp.init(seed)
    theta[mlp.N_PARAM - 40:] = g.normal(0, 0.1, 40)          # non-zero output biases
    X = g.normal(0, 1, (nb, mlp.N_IN))
    Y = (g.random((nb, mlp.N_OUT)) < 0.4).astype(float)
    M = (g.random((nb, mlp.N_OUT)) < 0.8).astype(float)
    return theta, X, Y, M


def test_mlp_gradient_matches_central_differences():
    from oracle import mlp
    theta, X, Y, M = _mlp_case(5)
    H1, H2, Z = mlp.forward(theta, X)
    g = mlp.backward(theta, X, H1, H2, Z, Y, M)

    def loss(t):
        return mlp.bce_loss(mlp.forward(t, X)[2], Y, M)
    idx = np.random.default_rng(1).choice(mlp.N_PARAM, 400, replace=False)
    idx = np.concatenate([idx, np.arange(mlp.N_PARAM - 40, mlp.N_PARAM), np.arange(1024, 1088)])
    # h = 1e-4: truncation error ~h^2 stays below 1e-7 relative, rounding ~u L / h far below
    h = 1e-4
    worst = 0.0
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        fd = (loss(theta + e) - loss(theta - e)) / (2 * h)
        worst = max(worst, abs(fd - g[i]) / max(abs(g[i]), 1e-3))
    assert worst <= 1e-7


def test_bce_closed_forms_at_zero_logits():
    from oracle import mlp
    theta, X, Y, M = _mlp_case(6)
    theta[-(40 * 64 + 40):] = 0.0                 # W3 = 0, b3 = 0: every logit is 0
    H1, H2, Z = mlp.forward(theta, X)
    assert np.all(Z == 0.0)
    assert abs(mlp.bce_loss(Z, Y, M) - math.log(2.0)) <= 1e-15
    g = mlp.backward(theta, X, H1, H2, Z, Y, M)
    gb3 = g[-40:]
    assert np.allclose(gb3, ((0.5 - Y) * M).sum(0) / M.sum(), rtol=0, atol=1e-15)
    # no signal reaches the hidden layers through W3 = 0
    assert np.all(g[:1024 + 64 + 4096 + 64] == 0.0)


def test_adam_first_step_moves_each_weight_by_lr():
    from oracle import mlp
    g = np.random.default_rng(2).normal(0, 1, 50)
    th, m, v = mlp.adam_step(np.zeros(50), g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    assert np.allclose(th, -1e-3 * np.sign(g), rtol=1e-6)


def test_mlp_fits_a_tiny_set():
    from oracle import mlp
    theta, X, Y, M = _mlp_case(8, nb=8)
    M = np.ones_like(M)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    for t in range(1, 1501):
        H1, H2, Z = mlp.forward(theta, X)
        theta, m, v = mlp.adam_step(theta, mlp.backward(theta, X, H1, H2, Z, Y, M), m, v, t, lr=1e-2)
    assert mlp.bce_loss(mlp.forward(theta, X)[2], Y, M) < 0.02


def test_selector_features_are_scale_invariant_and_reveal_rank():
    from oracle import selector
    A = _low_rank(300, 200, [1.0, 0.5, 0.2, 0.1, 0.05], seed=3)
    s = selector.probe_sigma(A, seed=4)
    x = selector.features(s, 5)
    assert np.allclose(selector.features(selector.probe_sigma(3.0 * A, seed=4), 5), x, atol=1e-12)
    assert np.all(x[4:15] == -2.0)            # sigma_6.. of a rank-5 sketch are clamped at 1e-12
    assert np.all(x[:4] > -1.0) and np.all(np.diff(x[:4]) <= 0)
    assert x[15] == pytest.approx(math.log10(5) / 3)


def test_selector_decision_rule_by_brute_force():
    from oracle import selector
    g = np.random.default_rng(9)
    for trial in range(200):
        m, n = int(g.integers(200, 3000)), int(g.integers(200, 3000))
        k = int(g.integers(1, min(400, m, n) + 1))
        prob = g.random(selector.N_GRID)
        tau = float(g.uniform(0.3, 0.95))
        p, q = selector.choose(prob, m, n, k, tau)
        pts = [(o, pp, qq) for qi, qq in enumerate(selector.Q_GRID) for pi, pp in enumerate(selector.P_GRID)
               for o in [qi * 8 + pi] if k + pp <= min(m, n, 1024)]
        feas = [t for t in pts if prob[t[0]] >= tau]
        o_sel = 8 * selector.Q_GRID.index(q) + selector.P_GRID.index(p)
        if feas:
            best = min(selector.cost_ms(m, n, k, t[1], t[2]) * (2.0 - prob[t[0]]) for t in feas)
            assert selector.cost_ms(m, n, k, p, q) * (2.0 - prob[o_sel]) == best and prob[o_sel] >= tau
        else:
            assert prob[8 * selector.Q_GRID.index(q) + selector.P_GRID.index(p)] == max(prob[t[0]] for t in pts)
    # cost grows with p and with q
    assert selector.cost_ms(4000, 4000, 50, 10, 1) < selector.cost_ms(4000, 4000, 50, 20, 1)
    assert selector.cost_ms(4000, 4000, 50, 10, 1) < selector.cost_ms(4000, 4000, 50, 10, 2)


@pytest.mark.parametrize("q", [0, 2])
def test_prefix_of_the_reorthonormalised_scheme_is_the_shorter_run(q):
    """With prefix-stable Gaussian columns, the first k+p columns of the
    basis of Figure 5 built from k+p_max columns span what the run with k+p
    columns builds (CholeskyQR / QR with positive diagonal keep prefixes), so
    every grid point's certificate follows from one run; checked against the
    separate runs of the definition."""
    from oracle import selector
    sigma = gen.spectrum("polyexp", 150, alpha=1.0, tau=60.0)
    A = _low_rank(400, 300, sigma, seed=21, noise=1e-7)
    k, seed, ps = 12, 3, [0, 5, 10, 20, 40]
    ref = selector.plain_certificates(A, k, q, seed, ps)
    n = A.shape[1]
    G = philox.gaussian(n, k + ps[-1], seed, philox.STREAM_OMEGA)
    Q = orc.orth(A @ G)
    for _ in range(q):
        Q = orc.orth(A @ orc.orth(A.T @ Q))
    Gc = philox.gaussian(n, 10, seed, philox.STREAM_CERT)
    AG = A @ Gc
    for p, r in zip(ps, ref):
        Ql = Q[:, :k + p]
        E = AG - Ql @ (Ql.T @ AG)
        b = orc.probe_bound(np.linalg.norm(E, axis=0), 0.1)
        assert abs(b - r) <= 1e-6 * r + 1e-12
