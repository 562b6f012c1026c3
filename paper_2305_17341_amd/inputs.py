"""Seeded synthetic inputs and workload descriptions.

This module holds no homomorphic arithmetic: it only draws the plaintext
matrices / datasets with numpy's PCG64 and names the CKKS parameter chains of
the workloads.  It is the one module both the HIP path and the CPU oracle's
tests use, so that they start from identical inputs.  It imports nothing else
from this package.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Chain:
    """A CKKS parameter chain: ring degree 2^log_n, prime bit sizes of Q and P."""
    name: str
    log_n: int
    q_bits: tuple
    p_bits: tuple
    log2_scale: float = 40.0
    sigma: float = 3.2

    @property
    def N(self):
        return 1 << self.log_n

    @property
    def top_level(self):
        return len(self.q_bits) - 1


# Plain small: 60-bit q0 + 40-bit primes + one 60-bit special prime at N=2^13.
# The product needs three levels (sigma/tau, column shift, product), so the
# chain carries three 40-bit primes (one more than the two the small workload
# lists; that shorter chain cannot hold a depth-3 product).
SMALL = Chain("n13_small", 13, (60, 40, 40, 40), (60,))
# Plain mid: N=2^14, q0 60-bit + 8 x 40-bit, 2 x 60-bit special primes.
MID = Chain("n14_mid", 14, (60,) + (40,) * 8, (60, 60))
# Batched covariance / PowerMethod: N=2^16, q0 60-bit + 30 x 40-bit, 3 x 60-bit.
LARGE = Chain("n16_large", 16, (60,) + (40,) * 30, (60, 60, 60))
# N=2^15 serving chain: q0 + 14 x 40 + 3 x 60 (the paper's 5-digit / 18-limb key
# geometry at logN=15).
SERVE15 = Chain("n15_serve", 15, (60,) + (40,) * 14, (60, 60, 60))
# a toy chain for fast CPU-only tests
TOY = Chain("n10_toy", 10, (60, 40, 40, 40), (60,))
TOY2 = Chain("n11_toy2", 11, (60, 40, 40, 40, 40), (60, 60))

CHAINS = {c.name: c for c in (SMALL, MID, LARGE, SERVE15, TOY, TOY2)}


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_matrix(seed: int, n: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """n x n FP64 matrix with i.i.d. uniform entries (row-major)."""
    return rng(seed).uniform(lo, hi, size=(n, n))


def dataset(seed: int, s: int, t: int) -> np.ndarray:
    """s x t FP64 dataset, i.i.d. uniform[0,1] (image-pixel-like features in
    [0, 1], the value range of 16x16 greyscale crops divided by 255)."""
    return rng(seed).uniform(0.0, 1.0, size=(s, t))


def planted_dataset(seed: int, s: int, t: int, decay: float = 0.7, noise: float = 0.1) -> np.ndarray:
    """Dataset with a planted spectrum lambda_i ~ decay^i, clipped to [0, 1],
    so that the leading eigenvectors are well separated."""
    g = rng(seed)
    U = g.standard_normal((s, t))
    lam = decay ** np.arange(t)
    Q, _ = np.linalg.qr(g.standard_normal((t, t)))
    X = 0.5 + 0.15 * (U * np.sqrt(lam)) @ Q.T + noise * g.uniform(0.0, 1.0, size=(s, t))
    return np.clip(X, 0.0, 1.0)


def pca_dataset(seed: int, s: int, t: int, top: float = 8.0, decay: float = 0.75) -> np.ndarray:
    """s x t dataset in [0, 1] (pixel-like) whose covariance has a planted
    spectrum close to top * decay^i: the leading eigenvalues stay above the
    contraction coefficient 0.5 the Lazy Normalization schedule assumes (with
    decay 0.75 the eighth, after clipping, is about 0.8 for 256 features)."""
    g = rng(seed)
    lam = top * decay ** np.arange(t)
    Q, _ = np.linalg.qr(g.standard_normal((t, t)))
    Z = (g.standard_normal((s, t)) * np.sqrt(lam)) @ Q.T
    return np.clip(0.5 + Z, 0.0, 1.0)


def centre(X: np.ndarray) -> np.ndarray:
    return X - X.mean(axis=0, keepdims=True)


@dataclass
class ServeJob:
    kind: str
    d: int
    log_n: int
    arrival: float
    seed: int
    extra: dict = field(default_factory=dict)


def poisson_jobs(seed: int, n_jobs: int, rate: float, pairs):
    """Poisson arrivals (exponential gaps at `rate` jobs/s); each job draws a
    (d, log_n) pair uniformly from `pairs`."""
    g = rng(seed)
    t = 0.0
    jobs = []
    for k in range(n_jobs):
        t += g.exponential(1.0 / rate)
        d, log_n = pairs[g.integers(len(pairs))]
        jobs.append(ServeJob("matmul", int(d), int(log_n), t, seed * 1000003 + k))
    return jobs
