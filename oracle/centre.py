"""Oracle of the homomorphic mean and the covariance of a dataset that is not
centred (section 5.2: the mean by Aggregate of the row-block sums, mu^T mu by a
transposition and a coordinate-wise product, Cov = X^T X - mu^T mu; Algorithm
HCovMtrx), plus its plain FP64 definition.

TEST INFRASTRUCTURE ONLY (like the rest of oracle/): written over the
oracle's CKKS primitives and the PowerMethod oracle's circuit helpers, one
operation at a time in the paper's order, with these readings:

  * The mean of feature block j is Aggregate(sum_r X_j[r]; 0) times 1/s: the
    row-block sums added, the column sums spread to every row by adding
    Rot(.; i), i = n, 2n, .. < n^2, and the constant 1/s (true sample count,
    not the padded one; the paper leaves the division implicit) multiplied
    in (encoded at scale q_l, then a rescale).  Block j then holds the means
    of its n features in every row (a row-vector replica); padded feature
    columns hold 0.
  * mu[a]^T is the transposition G of mu[a] (every column holds the means);
    the block (a, b) of mu^T mu is the product (relinearised, rescaled) of
    mu[a]^T and mu[b]: entry (r, c) = mu_a[r] mu_b[c].
  * X^T X / s is the covariance circuit of the library on the raw blocks
    (1/s folded into the transposition); the subtraction brings mu^T mu,
    which sits at a higher level, to the level and scale of the X^T X / s
    blocks first (drop, multiply by the constant 1 encoded at the scale
    ratio, rescale, take the target scale), as the eigen-shift does.

Pins: the decrypted means against the FP64 column means, and the decrypted
blocks against the FP64 covariance (population, 1/s) of the raw data.
"""
from __future__ import annotations

import numpy as np

from .power import Box, HePower


def fp64_mean_and_cov(X):
    """column means and population covariance (1/s) of X"""
    mu = X.mean(axis=0)
    return mu, X.T @ X / X.shape[0] - np.outer(mu, mu)


class HeCentre(HePower):
    def means(self, blocks, rb, k, s):
        """mu[j] for the k feature blocks of the raw dataset blocks[r k + j]"""
        o = self.o
        out = []
        for j in range(k):
            S = blocks[j]
            for r in range(1, rb):
                S = o.add(S, blocks[r * k + j])
            out.append(self.pmul_const(Box(self.aggregate(Box(S), 0)), 1.0 / s))
        return out

    def covariance(self, blocks, rb, k, s, n1z, n1t, n1g, npz=None, npt=None, lazy=False, fused_rescale=False):
        """Cov = X^T X / s - mu^T mu, block (a, b) at index a k + b"""
        o, n = self.o, self.n
        xtx = o.covariance(blocks, rb, k, n, s, n1z, n1t, n1g, npz, npt, lazy=lazy, fused_rescale=fused_rescale)
        mu = self.means(blocks, rb, k, s)
        mut = [o.lt_transpose(m, n, n1g, 1.0) for m in mu]
        out = []
        for a in range(k):
            for b in range(k):
                c = xtx[a * k + b]
                mm = self.mul(Box(mut[a]), Box(mu[b]))
                out.append(o.sub(c, self.match(mm, c.level, c.scale)))
        return out
