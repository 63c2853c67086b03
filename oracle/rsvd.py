"""Float64 oracle of the randomized range finder and randomized SVD.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Each function follows
one passage of P.-G. Martinsson, "Randomized methods for matrix
computations", named in its docstring.  Matrix products, the unpivoted
Householder QR and the SVD of the small matrix are numpy/LAPACK library
calls, used exactly where the paper calls a packaged routine (Section 2.3
for orth, Section 3 Stage B for the SVD).  There is no blocking, fusion or
reordering beyond what the paper's steps state.

Readings of points the paper leaves open (each also listed in the design
notes):
  * orth is unique only up to column signs; the oracle fixes diag(R) >= 0.
  * the SVD's column order and signs are unspecified; the oracle sorts the
    singular values in descending order and flips each (u_j, v_j) so that the
    entry of largest magnitude of the small-matrix left vector u_hat_j is
    positive (the lowest index wins ties).
  * all matrices are real, so "*" is the transpose.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

from . import philox


# ---------------------------------------------------------------------------
# Primitives
# ---------------------------------------------------------------------------

def orth(X: np.ndarray) -> np.ndarray:
    """Section 2.3: orthonormal basis of the column space of X (m >= l) by an
    unpivoted QR factorisation (Householder, via LAPACK), with the columns
    signed so that diag(R) >= 0."""
    X = np.asarray(X, dtype=np.float64)
    q, r = np.linalg.qr(X, mode="reduced")
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s


def svd_small(B: np.ndarray):
    """Section 3, Stage B step 2 (and Figure 1 step 5): the economy SVD of the
    small matrix B = U_hat diag(D) V^T.  Returns (U_hat, D, V) with D
    descending and the sign rule of the module docstring applied."""
    uh, d, vt = np.linalg.svd(np.asarray(B, dtype=np.float64), full_matrices=False)
    v = vt.T.copy()
    for j in range(uh.shape[1]):
        i = int(np.argmax(np.abs(uh[:, j])))
        if uh[i, j] < 0:
            uh[:, j] = -uh[:, j]
            v[:, j] = -v[:, j]
    return uh, d, v


@dataclass
class RSVDResult:
    """Factors of an RSVD: A ~= U diag(D) V^T, plus the Stage-A basis Q and the
    projected matrix B = Q^T A of Section 3."""
    U: np.ndarray
    D: np.ndarray
    V: np.ndarray
    Q: np.ndarray
    B: np.ndarray
    extra: dict = field(default_factory=dict)

    def truncate(self, k: int) -> "RSVDResult":
        """Remark in Section 4 ("how many basis vectors"): keep the k leading
        terms of the rank-(k+p) factorisation."""
        return RSVDResult(self.U[:, :k], self.D[:k], self.V[:, :k], self.Q, self.B, dict(self.extra))


def stage_b(A: np.ndarray, Q: np.ndarray) -> RSVDResult:
    """Section 3, Stage B: B = Q^T A; B = U_hat D V^T; U = Q U_hat."""
    B = Q.T @ A
    uh, d, v = svd_small(B)
    return RSVDResult(Q @ uh, d, v, Q, B)


# ---------------------------------------------------------------------------
# Figures 1, 4, 5
# ---------------------------------------------------------------------------

def rsvd_basic(A: np.ndarray, G: np.ndarray) -> RSVDResult:
    """Figure 1 (Section 4): Y = A G; Q = orth(Y); then Stage B.  G is the
    n x (k+p) Gaussian test matrix.  Returns the rank-(k+p) factorisation."""
    A = np.asarray(A, dtype=np.float64)
    Q = orth(A @ G)
    return stage_b(A, Q)


def rsvd_power(A: np.ndarray, G: np.ndarray, q: int) -> RSVDResult:
    """Figure 4 (Section 8.1): Y = (A A^T)^q A G formed by alternating
    Z = A^T Y and Y = A Z with no orthonormalisation in between, then
    Q = orth(Y) and Stage B.  Kept as the variant that loses accuracy to
    round-off (Remark after Figure 4)."""
    A = np.asarray(A, dtype=np.float64)
    Y = A @ G
    for _ in range(q):
        Z = A.T @ Y
        Y = A @ Z
    return stage_b(A, orth(Y))


def rsvd(A: np.ndarray, G: np.ndarray, q: int) -> RSVDResult:
    """Figure 5 (Section 8.1): Q = orth(A G); q times { W = orth(A^T Q);
    Q = orth(A W) }; B = Q^T A; SVD of B; U = Q U_hat.  Returns the
    rank-(k+p) factorisation (truncate with ``.truncate(k)``)."""
    A = np.asarray(A, dtype=np.float64)
    Q = orth(A @ G)
    for _ in range(q):
        W = orth(A.T @ Q)
        Q = orth(A @ W)
    return stage_b(A, Q)


def rsvd_seeded(A: np.ndarray, k: int, p: int, q: int, seed: int) -> RSVDResult:
    """Figure 5 with the test matrix drawn from ``seed`` by the counter-based
    generator of ``oracle.philox`` (stream of the test matrix)."""
    n = A.shape[1]
    G = philox.gaussian(n, k + p, seed, philox.STREAM_OMEGA)
    return rsvd(A, G, q)


# ---------------------------------------------------------------------------
# A posteriori estimation (Sections 13 and 14)
# ---------------------------------------------------------------------------

def probe_bound(col_norms: np.ndarray, alpha: float = 0.1) -> float:
    """Lemma of Section 13: ||T|| <= (1/alpha) sqrt(2/pi) max_i ||T g_i||,
    with probability at least 1 - alpha^r for r independent Gaussian g_i."""
    return float(np.max(col_norms)) * math.sqrt(2.0 / math.pi) / alpha


def residual_apply(A: np.ndarray, U: np.ndarray, D: np.ndarray, V: np.ndarray):
    """T = A - U diag(D) V^T as a pair of operators (x -> T x, y -> T^T y),
    never forming T (Section 14 evaluates E = (A - A_approx) G from the thin
    factors)."""
    def fwd(X):
        return A @ X - U @ (D[:, None] * (V.T @ X))

    def adj(Y):
        return A.T @ Y - V @ (D[:, None] * (U.T @ Y))
    return fwd, adj


def certificate(A: np.ndarray, U: np.ndarray, D: np.ndarray, V: np.ndarray, Gc: np.ndarray,
                s: int = 0, alpha: float = 0.1) -> float:
    """Section 14: E = (A - U D V^T) Gc with a thin Gaussian Gc (r columns);
    bound = (1/alpha) sqrt(2/pi) max_i ||E(:, i)||, valid with probability
    >= 1 - alpha^r (Lemma of Section 13).

    With s > 0 the same Lemma is applied to (T T^T)^s T, whose norm is
    ||T||^(2s+1); the returned bound is then the (2s+1)-th root."""
    fwd, adj = residual_apply(A, U, D, V)
    E = fwd(Gc)
    for _ in range(s):
        E = fwd(adj(E))
    b = probe_bound(np.linalg.norm(E, axis=0), alpha)
    return b ** (1.0 / (2 * s + 1))


def certificate_qb(A: np.ndarray, Q: np.ndarray, B: np.ndarray, Gc: np.ndarray, s: int = 0,
                   alpha: float = 0.1) -> float:
    """Section 14 applied to the untruncated pair (Q, B): T = A - Q B."""
    def fwd(X):
        return A @ X - Q @ (B @ X)

    def adj(Y):
        return A.T @ Y - B.T @ (Q.T @ Y)
    E = fwd(Gc)
    for _ in range(s):
        E = fwd(adj(E))
    b = probe_bound(np.linalg.norm(E, axis=0), alpha)
    return b ** (1.0 / (2 * s + 1))


# ---------------------------------------------------------------------------
# Adaptive range finders (Sections 12 and 13)
# ---------------------------------------------------------------------------

def adaptive_vector(A: np.ndarray, eps: float, r: int, draw: Callable[[int], np.ndarray],
                    max_rank: Optional[int] = None) -> np.ndarray:
    """Figure 14 (Section 13): grow Q one vector at a time until r consecutive
    projected samples all have norm <= eps / (10 sqrt(2/pi)).  ``draw(j)``
    returns the j-th Gaussian vector (0-based).  Returns Q."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    cap = min(m, n) if max_rank is None else max_rank
    thresh = eps / (10.0 * math.sqrt(2.0 / math.pi))
    ys = [A @ draw(i) for i in range(r)]
    Q = np.zeros((m, 0))
    j = 0
    while max(np.linalg.norm(y) for y in ys[j:j + r]) > thresh and Q.shape[1] < cap:
        y = ys[j] - Q @ (Q.T @ ys[j])          # the redundant re-projection
        qj = y / np.linalg.norm(y)
        Q = np.column_stack([Q, qj])
        g = draw(j + r)
        ynew = A @ g
        ynew = ynew - Q @ (Q.T @ ynew)
        ys.append(ynew)
        for i in range(j + 1, j + r):
            ys[i] = ys[i] - qj * (qj @ ys[i])
        j += 1
    return Q


def frobenius_downdate(a_fro: float, B: np.ndarray) -> float:
    """Section 12.4: ||A - Q B||_F = sqrt(a^2 - ||B||_F^2) when Q is orthonormal
    and B = Q^T A.  Returned clamped at zero (cancellation)."""
    return math.sqrt(max(a_fro * a_fro - float(np.sum(B * B)), 0.0))


def blocked_growth(A: np.ndarray, Q: np.ndarray, B: np.ndarray, draw_block: Callable[[int], np.ndarray],
                   stop: Callable[[np.ndarray, np.ndarray], bool], b: int, max_rank: int):
    """Figure 12 (Section 12.3), with the residual applied implicitly instead
    of overwriting A: each step draws b Gaussian vectors G, forms
    Y = (A - Q B) G = (I - Q Q^T) A G, projects out Q once more (the redundant
    re-projection of Figure 14), sets Q_new = orth(Y), B_new = Q_new^T A and
    appends both.  ``stop(Q, B)`` is evaluated before every step; growth also
    ends when another block would exceed ``max_rank``.  Returns (Q, B, steps,
    frob_history) where frob_history holds the Section 12.4 downdated
    residual norms."""
    A = np.asarray(A, dtype=np.float64)
    a_fro = float(np.linalg.norm(A))
    steps = 0
    hist = [frobenius_downdate(a_fro, B)]
    while not stop(Q, B) and Q.shape[1] + b <= max_rank:
        G = draw_block(steps)
        Y = A @ G
        Y = Y - Q @ (Q.T @ Y)
        Y = Y - Q @ (Q.T @ Y)
        Qn = orth(Y)
        Bn = Qn.T @ A
        Q = np.column_stack([Q, Qn])
        B = np.vstack([B, Bn])
        steps += 1
        hist.append(frobenius_downdate(a_fro, B))
    return Q, B, steps, hist


# ---------------------------------------------------------------------------
# The complete factorisation with certificate and fallback
# ---------------------------------------------------------------------------

@dataclass
class FactorOutput:
    U: np.ndarray
    D: np.ndarray
    V: np.ndarray
    rank: int
    certified: Optional[bool]
    bound: Optional[float]
    sigma1: float
    fallback_steps: int


def factor(A: np.ndarray, k: int, p: int, q: int, seed: int, eps: float = 0.0, n_probe: int = 10,
           est_power: int = 0, block: int = 32, max_rank: Optional[int] = None,
           G: Optional[np.ndarray] = None) -> FactorOutput:
    """What one call of the library computes, step by step:

    1. l = k + p; Omega from (seed, test-matrix stream) unless ``G`` is given.
    2. Figure 5 (q power steps with re-orthonormalisation) -> Q, B, SVD.
    3. eps == 0: return the rank-k truncation (Remark of Section 4).
    4. eps > 0: certificate of Section 14 on the rank-k residual, relative to
       sigma_hat_1 = D(1).  Certified -> return rank k.
    5. Otherwise the blocked adaptive range finder of Figure 12 grows (Q, B)
       from the rank-l basis, b columns at a time, drawing the next columns
       of the same Gaussian family (prefix extension), until the Section 14
       certificate of A - Q B holds or the rank would exceed ``max_rank``;
       then Stage B on the grown basis, returning all its columns.
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    l = k + p
    if max_rank is None:
        max_rank = l
    if G is None:
        G = philox.gaussian(n, l, seed, philox.STREAM_OMEGA)
    res = rsvd(A, G, q)
    sigma1 = float(res.D[0])
    if eps <= 0:
        t = res.truncate(k)
        return FactorOutput(t.U, t.D, t.V, k, None, None, sigma1, 0)
    Gc = philox.gaussian(n, n_probe, seed, philox.STREAM_CERT)
    t = res.truncate(k)
    bound = certificate(A, t.U, t.D, t.V, Gc, est_power)
    if bound <= eps * sigma1:
        return FactorOutput(t.U, t.D, t.V, k, True, bound, sigma1, 0)

    def draw_block(j):
        return philox.gaussian(n, block, seed, philox.STREAM_OMEGA, col0=l + j * block)

    state = {}

    def stop(Qc, Bc):
        bq = certificate_qb(A, Qc, Bc, Gc, est_power)
        state["bound"] = bq
        return bq <= eps * sigma1

    Q, B, steps, _ = blocked_growth(A, res.Q, res.B, draw_block, stop, block, max(max_rank, l))
    final = stage_b(A, Q)
    bq = state["bound"]
    ok = bq <= eps * sigma1
    return FactorOutput(final.U, final.D, final.V, Q.shape[1], ok, bq, sigma1, steps)


# ---------------------------------------------------------------------------
# Theory used by the pins (Sections 7 and 8.2)
# ---------------------------------------------------------------------------

def thm_expectation_frobenius(sigma: np.ndarray, k: int, p: int) -> float:
    """Theorem of Section 7.1, Frobenius form: E||A - QQ^T A||_F <=
    (1 + k/(p-1))^(1/2) (sum_{j>k} sigma_j^2)^(1/2); needs p >= 2."""
    return math.sqrt(1.0 + k / (p - 1.0)) * math.sqrt(float(np.sum(sigma[k:] ** 2)))


def thm_expectation_spectral(sigma: np.ndarray, k: int, p: int, q: int = 0) -> float:
    """Theorem of Section 7.1 (q = 0, spectral form) and the theorem of
    Section 8.2 (q power steps): E||A - QQ^T A|| <= [(1 + sqrt(k/(p-1)))
    sigma_{k+1}^(2q+1) + e sqrt(k+p)/p (sum_{j>k} sigma_j^(2(2q+1)))^(1/2)]^(1/(2q+1))."""
    e = 2 * q + 1
    t1 = (1.0 + math.sqrt(k / (p - 1.0))) * sigma[k] ** e
    t2 = math.e * math.sqrt(k + p) / p * math.sqrt(float(np.sum(sigma[k:] ** (2 * e))))
    return (t1 + t2) ** (1.0 / e)


def thm_tail_spectral(sigma: np.ndarray, k: int, p: int) -> float:
    """Section 7.2: for p >= 4, ||A - QQ^T A|| <= (1 + 17 sqrt(1 + k/p))
    sigma_{k+1} + 8 sqrt(k+p)/(p+1) (sum_{j>k} sigma_j^2)^(1/2), failing
    with probability at most 3 e^-p."""
    return ((1.0 + 17.0 * math.sqrt(1.0 + k / p)) * sigma[k]
            + 8.0 * math.sqrt(k + p) / (p + 1.0) * math.sqrt(float(np.sum(sigma[k:] ** 2))))
