"""Pins of the oracle's growth-pattern parts and of the theorem helpers.

Each test checks a fact fixed by the paper or by the mathematics, chosen so
that a plausible slip fails it:

* the theorem helpers against the special cases the paper prints (the
  Frobenius sub-optimality factor sqrt(1 + k/9) at p = 10 and sqrt(2) at
  p = k + 1 in Section 7.1; the no-decay simplification of the power-scheme
  bound in Section 8.2; the geometric-tail estimate of Section 7.1's fast-decay
  case);
* the per-block tolerance compression (Sections 12-14) on blocks whose
  singular values are planted, so the kept rank, the singular values and the
  true error are known without running the method;
* the selector's decision rule on probability vectors whose answer is known
  from the rule's statement alone (one feasible point, none, ties, all);
* the FP8 rounding of thin operands on columns whose 128-row segment maxima
  are planted powers of two with different scales either side of each
  segment boundary.
"""
import math

import numpy as np
import pytest

from oracle import batched, quant, rsvd as orc, selector
from workloads import gen


# ------------------------------------------------------------ theorem helpers

@pytest.mark.parametrize("k", [1, 10, 37, 200])
def test_frobenius_bound_factor_at_p10_is_sqrt_1_plus_k_over_9(k):
    sigma = gen.spectrum("poly", k + 500, alpha=0.7)
    tail = math.sqrt(float(np.sum(sigma[k:] ** 2)))     # the Eckart-Young minimum in the Frobenius norm
    assert orc.thm_expectation_frobenius(sigma, k, 10) / tail == pytest.approx(math.sqrt(1 + k / 9), rel=1e-14)
    assert orc.thm_expectation_frobenius(sigma, k, k + 1) / tail == pytest.approx(math.sqrt(2.0), rel=1e-14)


@pytest.mark.parametrize("q", [0, 1, 2, 3])
@pytest.mark.parametrize("k,p,N", [(10, 10, 300), (50, 5, 1000), (3, 2, 40)])
def test_power_bound_with_no_decay_past_k(q, k, p, N):
    """Section 8.2's simplification: sigma_{k+1} = ... = sigma_N gives the
    factor [1 + sqrt(k/(p-1)) + e sqrt(k+p)/p sqrt(N-k)]^(1/(2q+1))."""
    s_k1 = 0.37
    sigma = np.concatenate([np.linspace(5.0, 1.0, k), np.full(N - k, s_k1)])
    factor = (1 + math.sqrt(k / (p - 1)) + math.e * math.sqrt(k + p) / p * math.sqrt(N - k)) ** (1 / (2 * q + 1))
    assert orc.thm_expectation_spectral(sigma, k, p, q) == pytest.approx(factor * s_k1, rel=1e-13)
    # the leading k values do not enter the bound
    sigma2 = sigma.copy()
    sigma2[:k] *= 7.0
    assert orc.thm_expectation_spectral(sigma2, k, p, q) == orc.thm_expectation_spectral(sigma, k, p, q)


def test_power_bound_tends_to_sigma_k1_and_tail_bound_geometric_case():
    """Section 8.2: the factor in front of sigma_{k+1} goes to one as q grows.
    Section 7.1 fast-decay case: with sigma_j = sigma_{k+1} beta^(j-k-1) the
    tail's root sum of squares approaches sigma_{k+1} (1 - beta^2)^(-1/2)."""
    k, p, beta, s_k1 = 20, 10, 0.8, 1e-2
    N = k + 4000
    sigma = np.concatenate([np.ones(k), s_k1 * beta ** np.arange(N - k)])
    vals = [orc.thm_expectation_spectral(sigma, k, p, q) / s_k1 for q in range(8)]
    assert all(a > b for a, b in zip(vals, vals[1:])) and vals[-1] < 1.1 and vals[-1] > 1.0
    frob_tail = s_k1 / math.sqrt(1 - beta ** 2)
    assert orc.thm_expectation_frobenius(sigma, k, p) == pytest.approx(math.sqrt(1 + k / (p - 1)) * frob_tail,
                                                                       rel=1e-12)
    tail = orc.thm_tail_spectral(sigma, k, p)
    assert tail == pytest.approx((1 + 17 * math.sqrt(1 + k / p)) * s_k1 + 8 * math.sqrt(k + p) / (p + 1) * frob_tail,
                                 rel=1e-12)


# ------------------------------------------------------- per-block compression

def _planted_block(m, n, sigma, seed):
    return gen.low_rank_matrix(m, n, np.asarray(sigma, float), 0.0, seed)


@pytest.mark.parametrize("r", [1, 5, 12, 16])
def test_compress_block_exact_rank_is_found_without_growth(r):
    sigma = np.logspace(0, -3, r)
    K = _planted_block(200, 150, sigma, seed=40 + r)
    res = batched.compress_block(K, 1e-6, seed=5, blk=3)
    assert res.certified and res.basis == 16            # l0 = 16 columns suffice: no growth step
    assert res.rank == r
    assert np.max(np.abs(res.S - sigma) / sigma) < 1e-12
    assert res.sigma1 == pytest.approx(sigma[0], rel=1e-12)
    assert np.linalg.norm(K - (res.U * res.S) @ res.V.T, 2) < 1e-12


def test_compress_block_keeps_the_values_above_half_the_tolerance():
    """The tolerance is split in halves: the certificate gets eps/2 and the
    truncation keeps every sigma > eps sigma_hat_1 / 2.  A planted value
    between eps/2 and eps sigma_1 must be kept, one just below eps/2 dropped."""
    eps = 1e-6
    sigma = np.array([1.0, 1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 0.7e-6, 0.3e-6, 1e-8])
    K = _planted_block(180, 220, sigma, seed=77)
    res = batched.compress_block(K, eps, seed=9, blk=0)
    assert res.certified
    assert res.rank == 7                                 # sigma > 0.5e-6: the first seven
    assert np.max(np.abs(res.S - sigma[:7]) / sigma[:7]) < 1e-9
    err = np.linalg.norm(K - (res.U * res.S) @ res.V.T, 2)
    assert err == pytest.approx(0.3e-6, rel=1e-6)        # the first dropped value (Eckart-Young)
    assert err <= eps * res.sigma1


def test_compress_block_grows_by_blocks_until_certified():
    """A block whose tolerance rank exceeds l0 = 16 grows by b = 8 columns per
    step (Figure 12); the grown basis is certified, the first sketch's
    sigma_hat_1 is a lower estimate of sigma_1 from a projection, and the
    brute-force true error is within eps sigma_hat_1."""
    eps = 1e-6
    sigma = 0.6 ** np.arange(60)                        # eps-rank about 28
    K = _planted_block(300, 260, sigma, seed=12)
    res = batched.compress_block(K, eps, seed=4, blk=7)
    assert res.certified and res.basis > 16 and (res.basis - 16) % 8 == 0
    assert res.bound <= 0.5 * eps * res.sigma1          # the certificate's half of the tolerance
    assert res.sigma1 <= sigma[0] * (1 + 1e-12) and res.sigma1 > 0.99 * sigma[0]
    want = int(np.sum(sigma > 0.5 * eps * res.sigma1))
    assert abs(res.rank - want) <= 1                     # the kept values approximate the planted ones
    err = np.linalg.norm(K - (res.U * res.S) @ res.V.T, 2)
    assert err <= eps * res.sigma1
    assert err >= sigma[res.rank] * (1 - 1e-6)           # Eckart-Young floor


@pytest.mark.parametrize("blk", [0, 1, 2])
def test_compress_block_on_kernel_blocks_meets_the_tolerance_by_brute_force(blk):
    K = gen.kernel_block(140 + 60 * blk, 300 - 50 * blk, seed=3, block_id=blk).astype(np.float64)
    res = batched.compress_block(K, 1e-6, seed=11, blk=blk)
    s = np.linalg.svd(K, compute_uv=False)
    assert res.certified and res.bound <= 0.5e-6 * res.sigma1
    err = np.linalg.norm(K - (res.U * res.S) @ res.V.T, 2)
    assert err <= 1e-6 * res.sigma1
    assert res.rank >= int(np.sum(s > 1e-6 * s[0]))      # cannot beat the true eps-rank
    assert res.rank <= int(np.sum(s > 0.25e-6 * s[0]))


def test_compress_block_stops_at_the_rank_cap():
    sigma = np.ones(40)
    K = _planted_block(100, 90, sigma, seed=2)
    res = batched.compress_block(K, 1e-6, seed=1, blk=0, rank_cap=32)
    assert not res.certified and res.basis == 32


# ------------------------------------------------------------ selector rule

def _idx(p, q):
    return 8 * selector.Q_GRID.index(q) + selector.P_GRID.index(p)


def test_choose_single_feasible_point():
    m, n, k = 3000, 2000, 40
    for p, q in [(0, 0), (20, 3), (320, 4), (5, 1)]:
        prob = np.full(selector.N_GRID, 0.1)
        prob[_idx(p, q)] = 0.95
        assert selector.choose(prob, m, n, k, 0.9) == (p, q)


def test_choose_without_feasible_point_takes_the_most_probable():
    m, n, k = 3000, 2000, 40
    prob = np.linspace(0.01, 0.3, selector.N_GRID)[::-1].copy()
    prob[_idx(40, 2)] = 0.45
    assert selector.choose(prob, m, n, k, 0.5) == (40, 2)
    # equal probabilities: the lowest output index (smallest q, then smallest p) wins
    prob = np.full(selector.N_GRID, 0.2)
    assert selector.choose(prob, m, n, k, 0.5) == (0, 0)
    prob[_idx(10, 1)] = prob[_idx(5, 3)] = 0.4
    assert selector.choose(prob, m, n, k, 0.5) == (10, 1)


def test_choose_all_certain_takes_the_cheapest_point():
    """With P = 1 everywhere the expected time is the modelled time, which
    grows with p and with q, so the answer is the smallest p at the smallest q."""
    m, n, k = 3000, 2000, 40
    prob = np.ones(selector.N_GRID)
    assert selector.choose(prob, m, n, k, 0.5) == (0, 0)
    prob[[_idx(p, 0) for p in selector.P_GRID]] = 0.0     # q = 0 never works
    assert selector.choose(prob, m, n, k, 0.5) == (0, 1)


def test_choose_never_picks_a_point_that_does_not_fit():
    m, n, k = 1100, 1000, 900                            # k + p <= 1000: p <= 100 (so 160 and 320 are out)
    prob = np.full(selector.N_GRID, 0.05)
    prob[_idx(320, 0)] = prob[_idx(160, 2)] = 0.99
    prob[_idx(80, 4)] = 0.6
    assert selector.choose(prob, m, n, k, 0.5) == (80, 4)
    assert selector.choose(prob, m, n, k, 0.9) == (80, 4)   # none feasible: the most probable that fits


def test_choose_prefers_certainty_only_when_it_pays():
    """Two feasible points: a cheap one at P = tau and a dear one at P = 1.
    The rule weighs time by (2 - P): the dear point wins only if it costs
    less than (2 - tau) times the cheap one."""
    m, n, k = 6000, 6000, 100
    c_cheap = selector.cost_ms(m, n, k, 10, 1)
    c_dear = selector.cost_ms(m, n, k, 10, 2)
    assert c_dear < (2 - 0.6) * c_cheap                  # one more power step costs less than a 40 % miss
    prob = np.zeros(selector.N_GRID)
    prob[_idx(10, 1)], prob[_idx(10, 2)] = 0.6, 1.0
    assert selector.choose(prob, m, n, k, 0.55) == (10, 2)
    prob[_idx(10, 1)] = 0.99
    assert selector.choose(prob, m, n, k, 0.55) == (10, 1)


# ------------------------------------------------------- FP8 thin operands

def test_fp8_thin_rounding_uses_one_scale_per_128_row_segment():
    """Column j: rows in [128 s, 128 s + 128) hold E4M3-representable values
    times 2^e_s, with the largest magnitude exactly 448 * 2^e_s.  Segment
    scales differ by up to 2^40, so any other segment origin or a column-wide
    scale would flush the small segments' values; the per-segment rule
    reproduces every entry exactly.  K = 300 leaves a ragged last segment."""
    g = np.random.default_rng(5)
    K, cols = 300, 6
    codes = quant.fp8_e4m3_decode(np.arange(256, dtype=np.uint8))
    finite = codes[np.isfinite(codes)]
    X = np.zeros((K, cols))
    exps = [[20, -20, 3], [-9, 9, 0], [0, 0, 0], [-30, 10, -1], [5, 5, -12], [1, -1, 1]]
    for j in range(cols):
        for s, e in enumerate(exps[j]):
            lo, hi = 128 * s, min(K, 128 * s + 128)
            v = g.choice(finite, hi - lo)
            v[g.integers(0, hi - lo)] = 448.0 * (1 if g.random() < 0.5 else -1)
            X[lo:hi, j] = v * 2.0 ** e
    # the largest value of segment 0 sits on row 127 and the smallest scale starts at row 128
    X[127, 0], X[128, 0] = 448.0 * 2.0 ** 20, 448.0 * 2.0 ** -20
    assert np.all(X.astype(np.float32) == X)
    assert np.array_equal(quant.fp8_round_thin(X), X)
    # a column-wide scale loses the small segments
    wide = np.column_stack([quant.fp8_e4m3_round(X[:, j] * 2.0 ** -quant.fp8_scale_exponent(np.max(np.abs(X[:, j]))))
                            * 2.0 ** quant.fp8_scale_exponent(np.max(np.abs(X[:, j]))) for j in range(cols)])
    assert not np.array_equal(wide, X)


def test_fp8_thin_rounding_of_non_representable_values():
    """Each segment is rounded on its own grid: spacing 2^(e-3) below 448 * 2^e
    for normal codes, so the error of every entry is at most half the spacing
    of its binade, and values at a midpoint go to the even code."""
    K = 256
    X = np.zeros((K, 2))
    X[0, 0] = 448.0          # segment scale 1
    X[1, 0] = 1.0 + 2 ** -4  # midpoint of 1 and 1.125: ties to even -> 1
    X[2, 0] = 1.0 + 3 * 2 ** -4  # midpoint of 1.125 and 1.25 -> 1.25
    X[128, 0] = 448.0 * 2 ** -8  # segment scale 2^-8
    X[129, 0] = (1.0 + 2 ** -4) * 2 ** -8
    X[:, 1] = np.linspace(-3.0, 3.0, K)
    X[0, 1] = 448.0 * 4  # scale 4 for segment 0 of column 1
    out = quant.fp8_round_thin(X)
    assert out[1, 0] == 1.0 and out[2, 0] == 1.25 and out[129, 0] == 2 ** -8
    # error bound per binade
    x = X[1:128, 1]
    rel = np.abs(out[1:128, 1] - x) / np.maximum(np.abs(x), 2.0 ** -6 * 4)
    assert np.all(rel <= 2 ** -4 + 1e-15)


def test_compress_block_grows_until_certified_or_capped():
    """Figure 12's loop stops only when the certificate holds or the basis
    cannot grow: over a scan of flat tails whose level moves the first
    certificate across the tolerance, every result is certified or capped."""
    head = np.logspace(0, -2, 10)
    grew = 0
    for t in np.logspace(-9, -6.5, 12):
        sigma = np.concatenate([head, np.full(30, t)])
        K = _planted_block(160, 140, sigma, seed=31)
        res = batched.compress_block(K, 1e-6, seed=2, blk=1, rank_cap=48)
        assert res.certified or res.basis + 8 > 48, (t, res.bound, res.basis)
        grew += res.basis > 16
    assert 0 < grew < 12
