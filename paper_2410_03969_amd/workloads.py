"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only draws points and job descriptions; it holds none of the
factorization's arithmetic.  Every generator is a pure function of its seed.

The workloads mirror the shapes of the paper's kernel experiments (Section 3:
N around 1e5 with k = 1000 and b = 120..150, kernels evaluated from raw points
in dimensions up to a few hundred), scaled to a single GPU:

* ``small``     N=2000 uniform points in [0,1]^3, Gaussian sigma=0.5, k=100, b=20
* ``laplace``   N=1e5 standard normal points / sqrt(20) in R^20, Laplace (l2) sigma=1,
                k=1000, b=120
* ``mixture``   N=1e6 points in R^8 from a 10-component Gaussian mixture (means
                uniform on [-5,5]^8, unit covariance), Gaussian sigma=2, k=2000, b=200
* ``sparse_hd`` N=2e5 points in R^256, 90% zeros, nonzeros N(0,1), Matern-3/2
                length scale 4, k=4000, b=400
* ``serving``   a stream of jobs with Poisson arrivals and uneven N, d, k
* ``grid`` / ``clusters`` special point sets whose kernel matrices are the
  identity or block-diagonal all-ones matrices, exact in every precision.
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np

GAUSSIAN, LAPLACE_L2, MATERN32, MATERN52 = 0, 1, 2, 3
KERNEL_NAMES = {GAUSSIAN: "gaussian", LAPLACE_L2: "laplace_l2",
                MATERN32: "matern32", MATERN52: "matern52"}

FP64, FP32, BF16X3, BF16, FP8 = 0, 1, 2, 3, 4
ACCEL, BLOCK = 0, 1   # pivot rule: accelerated (Alg. 2; b = 1 is simple RPCholesky) or block (Alg. 7)
METHOD_NAMES = {ACCEL: "accel", BLOCK: "block"}
PREC_NAMES = {FP64: "fp64", FP32: "fp32", BF16X3: "bf16x3", BF16: "bf16", FP8: "fp8"}


@dataclass(frozen=True)
class Problem:
    """One factorization request: points X (N x d), kernel, target rank k,
    block size b, algorithm seed and arithmetic mode."""
    N: int
    d: int
    k: int
    b: int
    kernel: int
    sigma: float
    seed: int = 0
    prec: int = FP64
    max_rounds: int = 0  # 0: run until k pivots are held
    method: int = ACCEL

    def with_(self, **kw) -> "Problem":
        return replace(self, **kw)


def small(seed: int = 0):
    rng = np.random.default_rng(seed)
    X = rng.random((2000, 3))
    return X, Problem(N=2000, d=3, k=100, b=20, kernel=GAUSSIAN, sigma=0.5, seed=0)


def laplace(seed: int = 0, N: int = 100_000):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((N, 20)) / np.sqrt(20.0)
    return X, Problem(N=N, d=20, k=1000, b=120, kernel=LAPLACE_L2, sigma=1.0, seed=0)


def mixture(seed: int = 0, N: int = 1_000_000, d: int = 8, components: int = 10):
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-5.0, 5.0, (components, d))
    z = rng.integers(0, components, N)
    X = mu[z] + rng.standard_normal((N, d))
    return X, Problem(N=N, d=d, k=2000, b=200, kernel=GAUSSIAN, sigma=2.0, seed=0)


def sparse_hd(seed: int = 0, N: int = 200_000, d: int = 256):
    rng = np.random.default_rng(seed)
    M = rng.random((N, d)) < 0.1
    X = np.where(M, rng.standard_normal((N, d)), 0.0)
    return X, Problem(N=N, d=d, k=4000, b=400, kernel=MATERN32, sigma=4.0, seed=0)


def grid(d: int, levels: int = 4, spacing: float = 64.0):
    """All points of {0, spacing, ..., (levels-1)*spacing}^d.  With a Gaussian
    kernel of bandwidth 1 every off-diagonal entry underflows to exactly 0, so
    the kernel matrix is the identity in any floating-point format."""
    axes = [np.arange(levels, dtype=np.float64) * spacing] * d
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack([m.reshape(-1) for m in mesh], axis=1)


def clusters(sizes, d: int = 3, spacing: float = 64.0, seed: int = 0):
    """Groups of identical points placed far apart on an integer lattice.  With a
    Gaussian kernel of bandwidth 1 the kernel matrix is block-diagonal with
    all-ones blocks (rank = number of groups), exactly in any format.  Point
    order is shuffled with the seed."""
    rng = np.random.default_rng(seed)
    centers = grid(d, levels=int(np.ceil(len(sizes) ** (1.0 / d))) + 1, spacing=spacing)
    centers = centers[rng.permutation(len(centers))[: len(sizes)]]
    labels = np.concatenate([np.full(n, g) for g, n in enumerate(sizes)])
    perm = rng.permutation(len(labels))
    labels = labels[perm]
    return centers[labels].copy(), labels


def dense_psd(N: int, rank: int, seed: int = 0, scale_spread: float = 3.0):
    """A = B B^T with a non-constant diagonal (rows of B scaled unevenly)."""
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((N, rank))
    B *= np.exp(scale_spread * rng.random((N, 1)) - scale_spread / 2)
    return B @ B.T


@dataclass(frozen=True)
class Job:
    job_id: int
    arrival: float  # seconds after the stream starts
    X: np.ndarray
    problem: Problem


def serving_stream(n_jobs: int = 512, rate: float = 10.0, seed: int = 4,
                   n_min: float = 1e4, n_max: float = 2e5, dims=(3, 8, 32),
                   k_min: int = 200, k_max: int = 1500, prec: int = BF16X3,
                   materialize: bool = True):
    """Poisson arrivals (rate jobs/s), N log-uniform in [n_min, n_max], d drawn
    from dims, k uniform in [k_min, k_max], b = k // 10, Gaussian bandwidth
    sqrt(d), points uniform on [0,1]^d drawn from seed 1000 + job index.  The
    algorithm seed of job j is j."""
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    for j in range(n_jobs):
        t += rng.exponential(1.0 / rate) if rate > 0 else 0.0
        N = int(round(10 ** rng.uniform(np.log10(n_min), np.log10(n_max))))
        d = int(rng.choice(dims))
        k = int(rng.integers(k_min, k_max + 1))
        k = min(k, N)
        b = max(1, k // 10)
        X = np.random.default_rng(1000 + j).random((N, d)) if materialize else None
        jobs.append(Job(j, t, X, Problem(N=N, d=d, k=k, b=b, kernel=GAUSSIAN,
                                         sigma=float(np.sqrt(d)), seed=j, prec=prec)))
    return jobs


def qr_matrix(M: int = 1000, N: int = 100_000, rank: int = 300, decay: float = 0.99, noise: float = 1e-5,
              seed: int = 0):
    """A dense M x N test matrix for the QR method: U diag(decay^i) V^* with
    orthonormal random U (M x rank) and V (N x rank), plus i.i.d. Gaussian
    noise of the given scale; returned column-major as the transpose of a
    C-contiguous N x M array (so B.T is contiguous)."""
    rng = np.random.default_rng(seed)
    U = np.linalg.qr(rng.standard_normal((M, rank)))[0]
    V = np.linalg.qr(rng.standard_normal((N, rank)))[0]
    Bt = (V * decay ** np.arange(rank)) @ U.T          # N x M = B^T
    Bt += noise * rng.standard_normal((N, M))
    return Bt.T
