"""Seeded generators for the five workloads.

Recipes (every draw is seeded; nothing here depends on the GPU library or on
the oracle):

* ``low_rank_matrix`` builds A = U diag(sigma) V^T + N.  U and V are the
  orthonormal Q factors (diagonal of R made positive) of seeded standard
  Gaussian matrices; N has i.i.d. N(0, noise_std^2) entries.
* ``kernel_block`` evaluates K_ij = log|x_i - y_j| for points drawn uniformly
  in the unit box [0,1]^2 (rows) and in the box [3,4] x [0,1] (columns): two
  unit boxes whose centres are three units apart.  Computed in float64 and
  rounded to float32.
* ``selector_item_params`` draws the parameters of one matrix of the stream
  used by the (p, q) selector: m, n uniform in [1000, 8000], alpha uniform in
  [0.5, 3], tau uniform in [10, 500], spectrum sigma_j = j^-alpha *
  exp(-(j-1)/tau).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np

# Stream identifiers used to derive independent seeds for the pieces of one
# workload.  The randomized method's own draws (the test matrix Omega, probe
# and certificate vectors, fallback blocks) are not produced here.
_STREAM_U, _STREAM_V, _STREAM_NOISE, _STREAM_POINTS = 1, 2, 3, 8


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64([int(seed) & 0xFFFFFFFF, int(seed) >> 32, stream]))


def spectrum(kind: str, r: int, **kw) -> np.ndarray:
    """Singular values sigma_1..sigma_r (float64, non-increasing)."""
    j = np.arange(1, r + 1, dtype=np.float64)
    if kind == "poly":
        return j ** (-float(kw["alpha"]))
    if kind == "exp":
        return np.exp(-j / float(kw["tau"]))
    if kind == "polyexp":
        return j ** (-float(kw["alpha"])) * np.exp(-(j - 1.0) / float(kw["tau"]))
    if kind == "flat":
        return np.ones(r)
    raise ValueError(f"unknown spectrum kind {kind!r}")


def gaussian_matrix(rows: int, cols: int, seed: int, stream: int = 0) -> np.ndarray:
    """A seeded standard Gaussian matrix (float64).  Used as an explicit test
    matrix Omega when a test hands the same draw to both implementations."""
    return _rng(seed, 100 + stream).standard_normal((rows, cols))


def orthonormal_factor(rows: int, cols: int, seed: int, stream: int) -> np.ndarray:
    """Orthonormal rows x cols factor: Q of a seeded Gaussian, diag(R) > 0."""
    g = _rng(seed, stream).standard_normal((rows, cols))
    q, r = np.linalg.qr(g, mode="reduced")
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s


def orthonormal_factor_device(rows: int, cols: int, seed: int, stream: int, device: str):
    """Orthonormal rows x cols factor drawn and orthonormalised on a torch
    device (float32 Gaussian from a seeded device generator, Householder QR,
    diag(R) > 0): the recipe of ``orthonormal_factor`` for shapes too large
    for a host QR (not bit-identical to it)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) * 1_000_003 + stream)
    G = torch.randn(rows, cols, generator=g, device=device, dtype=torch.float32)
    Q, R = torch.linalg.qr(G, mode="reduced")
    d = torch.sign(torch.diagonal(R))
    d[d == 0] = 1.0
    return Q * d


def low_rank_matrix(m: int, n: int, sigma: np.ndarray, noise_std: float, seed: int,
                    dtype=np.float64, device: Optional[str] = None, device_factors: bool = False):
    """A = U diag(sigma) V^T + noise.

    With ``device`` None the matrix is formed in float64 with numpy and
    returned as a numpy array of ``dtype``.  With a torch device string the
    orthonormal factors are still drawn with numpy (so they match the CPU
    recipe), but the product and the noise are formed on that device in
    float32 and a torch tensor is returned (large workloads).
    """
    r = len(sigma)
    if device is not None and device_factors:
        import torch
        tu = orthonormal_factor_device(m, r, seed, _STREAM_U, device)
        tu *= torch.from_numpy(np.asarray(sigma, np.float32)).to(device)
        tv = orthonormal_factor_device(n, r, seed, _STREAM_V, device)
        a = tu @ tv.T
        del tu, tv
        if noise_std > 0:
            g = torch.Generator(device=device)
            g.manual_seed(int(seed) * 7919 + _STREAM_NOISE)
            a.add_(torch.randn(a.shape, generator=g, device=device, dtype=torch.float32), alpha=float(noise_std))
        return a
    u = orthonormal_factor(m, r, seed, _STREAM_U)
    v = orthonormal_factor(n, r, seed, _STREAM_V)
    if device is None:
        a = (u * sigma) @ v.T
        if noise_std > 0:
            a += noise_std * _rng(seed, _STREAM_NOISE).standard_normal((m, n))
        return a.astype(dtype)
    import torch
    tu = torch.from_numpy((u * sigma).astype(np.float32)).to(device)
    tv = torch.from_numpy(v.astype(np.float32)).to(device)
    a = tu @ tv.T
    del tu, tv
    if noise_std > 0:
        g = torch.Generator(device=device)
        g.manual_seed(int(seed) * 7919 + _STREAM_NOISE)
        a.add_(torch.randn(a.shape, generator=g, device=device, dtype=torch.float32), alpha=float(noise_std))
    return a


def psd_matrix(n: int, lam: np.ndarray, seed: int, dtype=np.float64, device: Optional[str] = None):
    """A = U diag(lam) U^T, exactly symmetric, U the orthonormal factor of ``low_rank_matrix`` (host
    recipe); on a device the product is formed in float32 and symmetrised there."""
    u = orthonormal_factor(n, len(lam), seed, _STREAM_U)
    if device is None:
        a = (u * lam) @ u.T
        return (0.5 * (a + a.T)).astype(dtype)
    import torch
    tu = torch.from_numpy(u.astype(np.float32)).to(device)
    a = (tu * torch.from_numpy(np.asarray(lam, np.float32)).to(device)) @ tu.T
    del tu
    a.add_(a.T.contiguous()).mul_(0.5)
    return a


def kernel_block(mb: int, nb: int, seed: int, block_id: int) -> np.ndarray:
    """K_ij = log |x_i - y_j| (float64 evaluation, float32 result)."""
    x, y = kernel_points(mb, nb, seed, block_id)
    d = np.sqrt(((x[:, None, :] - y[None, :, :]) ** 2).sum(-1))
    return np.log(d).astype(np.float32)


def kernel_points(mb: int, nb: int, seed: int, block_id: int):
    """The point sets of ``kernel_block`` (float64 arrays of shape (mb, 2) and (nb, 2))."""
    g = _rng(seed * 1_000_003 + block_id, _STREAM_POINTS)
    x = g.random((mb, 2))
    y = g.random((nb, 2))
    y[:, 0] += 3.0
    return x, y


def kernel_blocks_device(ms, ns, seed: int, device: str):
    """All blocks of the batched workload in one float32 device buffer, each
    block row-major with leading dimension n_b, evaluated on the device in
    float64 from the same points as ``kernel_block``.  Returns (buffer, list of
    2-D views)."""
    import torch
    sizes = [int(m) * int(n) for m, n in zip(ms, ns)]
    buf = torch.empty(sum(sizes), dtype=torch.float32, device=device)
    views, off = [], 0
    for b, (m, n) in enumerate(zip(ms, ns)):
        x, y = kernel_points(int(m), int(n), seed, b)
        tx = torch.from_numpy(x).to(device)
        ty = torch.from_numpy(y).to(device)
        d = torch.sqrt(((tx[:, None, :] - ty[None, :, :]) ** 2).sum(-1))
        v = buf[off:off + sizes[b]].view(int(m), int(n))
        v.copy_(torch.log(d).to(torch.float32))
        views.append(v)
        off += sizes[b]
    return buf, views


def batched_blocks(nblk: int, seed: int, lo: int = 64, hi: int = 512):
    """Block shapes for the batched workload: rows and columns i.i.d. uniform
    integers in [lo, hi]."""
    g = _rng(seed, 9)
    ms = g.integers(lo, hi + 1, size=nblk)
    ns = g.integers(lo, hi + 1, size=nblk)
    return ms.astype(np.int32), ns.astype(np.int32)


def selector_item_params(seed: int, item: int):
    """(m, n, alpha, tau) for one matrix of the selector stream."""
    g = _rng(seed * 1_000_033 + item, 10)
    m = int(g.integers(1000, 8001))
    n = int(g.integers(1000, 8001))
    alpha = float(g.uniform(0.5, 3.0))
    tau = float(g.uniform(10.0, 500.0))
    return m, n, alpha, tau


def selector_spectrum(seed: int, item: int):
    """(m, n, sigma, k) of one item of the selector stream: sigma_j = j^-alpha
    exp(-(j-1)/tau) for j = 1..min(m, n) (sigma_1 = 1) and k the number of
    sigma_j above 1e-3 (the target rank for relative tolerance 1e-3)."""
    m, n, alpha, tau = selector_item_params(seed, item)
    s = spectrum("polyexp", min(m, n), alpha=alpha, tau=tau)
    return m, n, s, int(np.sum(s > 1e-3 * s[0]))


def selector_matrix(seed: int, item: int, device: str):
    """A = H_U [diag(sigma); 0] H_V^T for one selector item, float32 on a torch
    device, with H_U = (I - 2 u1 u1^T)(I - 2 u2 u2^T) (and H_V likewise) for
    seeded random unit vectors: orthogonal factors that cost O(mn) to apply.
    Gaussian sketches and probes are orthogonally invariant, so the method's
    error and certificate have the same distribution as for Haar-random
    factors; only sigma, m and n matter.  Returns (A, k)."""
    import torch
    m, n, s, k = selector_spectrum(seed, item)
    g = _rng(seed * 1_000_033 + item, 11)
    A = torch.zeros(m, n, dtype=torch.float64, device=device)
    r = len(s)
    idx = torch.arange(r, device=device)
    A[idx, idx] = torch.from_numpy(s).to(device)
    for _ in range(2):
        u = torch.from_numpy(g.standard_normal(m)).to(device)
        u /= torch.linalg.norm(u)
        A -= 2.0 * torch.outer(u, u @ A)
        v = torch.from_numpy(g.standard_normal(n)).to(device)
        v /= torch.linalg.norm(v)
        A -= 2.0 * torch.outer(A @ v, v)
    return A.to(torch.float32), k


@dataclasses.dataclass(frozen=True)
class WorkloadConfig:
    name: str
    m: int
    n: int
    rank: int
    spectrum: Callable[[int], np.ndarray]
    noise_std: float
    k: int
    p: int
    q: int
    dtype: str            # "f64" or "f32": dtype of A, U, V
    description: str
    psd: bool = False     # A = U diag(sigma) U^T (symmetric positive semidefinite, m == n)

    def sigma(self) -> np.ndarray:
        return self.spectrum(self.rank)

    def scaled(self, m: int, n: int, rank: int, k: int, p: int, q: Optional[int] = None,
               noise_std: Optional[float] = None) -> "WorkloadConfig":
        """Same spectrum family and precision at a smaller shape."""
        return dataclasses.replace(self, name=f"{self.name}@{m}x{n}", m=m, n=n, rank=rank, k=k, p=p,
                                   q=self.q if q is None else q,
                                   noise_std=self.noise_std if noise_std is None else noise_std)

    def matrix(self, seed: int = 0, device: Optional[str] = None):
        """The workload's matrix; on a device, shapes beyond 2^15 rows draw
        their factors on the device (``orthonormal_factor_device``)."""
        dt = np.float64 if self.dtype == "f64" else np.float32
        big = max(self.m, self.n) > 32768
        if self.psd:
            return psd_matrix(self.n, self.sigma(), seed, dt, device)
        return low_rank_matrix(self.m, self.n, self.sigma(), self.noise_std, seed, dt, device,
                               device_factors=big and device is not None)


CONFIGS = {
    # Plain RSVD in float64, 2000 x 2000, sigma_j = j^-2 over 200 modes, noise 1e-8.
    "plain_f64_2000": WorkloadConfig(
        "plain_f64_2000", 2000, 2000, 200, lambda r: spectrum("poly", r, alpha=2.0), 1e-8,
        20, 10, 1, "f64", "A = U diag(j^-2) V^T + N(0,1e-16), 2000x2000, k=20 p=10 q=1"),
    # Precision comparison, 50000 x 20000, rank 2000, sigma_j = j^-0.5, noise 1e-3 sigma_1/sqrt(n).
    "slowdecay_50000x20000": WorkloadConfig(
        "slowdecay_50000x20000", 50000, 20000, 2000, lambda r: spectrum("poly", r, alpha=0.5),
        1e-3 / math.sqrt(20000.0), 100, 10, 2, "f32",
        "A = U diag(j^-0.5) V^T + noise, 50000x20000 rank 2000, k=100 p=10 q=2"),
    # Block-scaled FP8, 65536 x 65536, rank 4096, sigma_j = exp(-j/150).
    "expdecay_65536": WorkloadConfig(
        "expdecay_65536", 65536, 65536, 4096, lambda r: spectrum("exp", r, tau=150.0), 0.0,
        500, 20, 3, "f32", "A = U diag(exp(-j/150)) V^T, 65536^2 rank 4096, k=500 p=20 q=3"),
    # Nystrom eigendecomposition (Section 9), 20000 x 20000 PSD, rank 2000, lambda_j = 1/j (noise-free).
    "psd_20000": WorkloadConfig(
        "psd_20000", 20000, 20000, 2000, lambda r: spectrum("poly", r, alpha=1.0), 0.0,
        100, 10, 0, "f32", "A = U diag(1/j) U^T, 20000^2 PSD rank 2000, k=100 p=10 q=0", psd=True),
}


def config(name: str) -> WorkloadConfig:
    return CONFIGS[name]
