"""Privacy-preserving PCA driver (section 6.2, Algorithm Privacy-Preserving
PCA) over the library's calls: block covariance (he_covariance), then for
each of l_E components l_P + 1 rounds of he_power_step (Lazy Normalization
schedule for the Newton counts, the eigenvalue in the last round) and
he_eigen_shift.  Refreshes are the client's (Refresher)."""
from __future__ import annotations

import time

import numpy as np

from . import he


def taylor_point(B2: float) -> float:
    """TaylorInit expands x^-1/2 at the midpoint B^2/2 + 1 of (0, B^2]"""
    return B2 / 2.0 + 1.0


def lazy_schedule(l_p: int, S: float = 0.5, e: float = 1e-5, precision: float = 1e-3, B2: float = 2.0 ** 16,
                  max_tau: int = 200):
    """Newton counts per PowerMethod round (Lazy Normalization, section
    6.1.2): a unit length shrunk by S each round is normalised with the
    fewest Newton steps that keep (l S' S)^2 >= precision, and in the last
    round also 1 - l S' < e."""
    x0 = taylor_point(B2)
    length = 1.0
    out = []
    for t in range(l_p):
        length *= S
        x = length * length
        y = 1.5 * x0 ** -0.5 - 0.5 * x0 ** -1.5 * x
        tau = 0
        while True:
            good = (length * y * S) ** 2 >= precision
            if t == l_p - 1:
                good = good and 1.0 - length * y < e
            if good:
                break
            if tau == max_tau:
                raise ValueError("Lazy Normalization: no Newton count meets the bounds")
            y = y * (1.5 + (-0.5 * x) * (y * y))
            tau += 1
        out.append(tau)
        length *= y
    return out


def replicate(v, k, d, axis):
    """blocks of a replicated vector: axis 0 repeats segments as rows, 1 as columns"""
    blocks = []
    for i in range(k):
        seg = np.asarray(v[i * d:(i + 1) * d], dtype=np.float64)
        blocks.append(np.tile(seg, (d, 1)) if axis == 0 else np.tile(seg[:, None], (1, d)))
    return blocks


def read_vector(ctx, V, d, axis):
    """client side: decrypt a replicated vector"""
    parts = []
    for ct in V:
        b = ctx.decrypt(ct, d * d).reshape(d, d)
        parts.append(b[0, :] if axis == 0 else b[:, 0])
    return np.concatenate(parts)


def power_method(ctx, cov, k, d, V0, axis, taus, x0, refresher):
    """HPowerMethod: len(taus) normalising rounds, then the eigenvalue round.
    Returns (V, axis, lambda, V^T)."""
    V = V0
    for tau in taus:
        V, axis = ctx.power_step(cov, k, d, V, axis, tau, x0, False, refresher)
    return ctx.power_step(cov, k, d, V, axis, 0, x0, True, refresher)


def pppca(ctx, cov, k, d, l_e, l_p, seed=0, B2=2.0 ** 16, nonce0=1 << 40, on_component=None):
    """Algorithm Privacy-Preserving PCA from an encrypted covariance: l_E
    (eigenvalue, eigenvector) pairs by PowerMethod and EigenShift.  The
    random unit start vectors are encrypted by the client (axis 1)."""
    refresher = he.Refresher(ctx, nonce0)
    taus = lazy_schedule(l_p, B2=B2)
    x0 = taylor_point(B2)
    g = np.random.default_rng(seed)
    out = []
    for m in range(l_e):
        v0 = g.standard_normal(k * d)
        v0 /= np.linalg.norm(v0)
        V0 = [ctx.encrypt_matrix(b, nonce=(1 << 50) + m * k + i) for i, b in enumerate(replicate(v0, k, d, 1))]
        t0 = time.perf_counter()
        V, axis, lam, VT = power_method(ctx, cov, k, d, V0, 1, taus, x0, refresher)
        cov = ctx.eigen_shift(cov, k, d, lam, V, VT, axis, refresher)
        ctx.sync()
        out.append((lam, V, VT, axis))
        if on_component is not None:
            on_component(m, time.perf_counter() - t0)
    return out, refresher.count
