"""Packing of a dataset into n x n matrix blocks (section 5.1, padding
methods 1 and 2) and the inverse for a feature x feature result: the client's
side of the covariance path.  Each block is then encrypted row-major as one
ciphertext."""
from __future__ import annotations

import numpy as np


def features_per_block(t: int, n: int, method: int = 1) -> int:
    """Valid features per n x n block (section 5.1): method 1 fills the first
    k - 1 feature blocks and zero-pads the last; method 2 keeps n - p valid
    features in every block, p = floor((k n - t) / k), k = ceil(t / n)."""
    if method == 1:
        return n
    k = -(-t // n)
    return n - (k * n - t) // k


def blocks(X: np.ndarray, n: int, method: int = 1):
    """Split an s x t dataset into ceil(s/n) x ceil(t/n) zero-padded n x n blocks
    (padding method 1 or 2): returns array [row_block][feature_block][n][n].
    Feature f sits in block f // w, column f % w, w = features_per_block."""
    s, t = X.shape
    rb, kb = -(-s // n), -(-t // n)
    w = features_per_block(t, n, method)
    out = np.zeros((rb, kb, n, n))
    for j in range(kb):
        cols = X[:, j * w:min((j + 1) * w, t)]
        for r in range(rb):
            part = cols[r * n:(r + 1) * n]
            out[r, j, :part.shape[0], :part.shape[1]] = part
    return out


def unblock_square(B, t: int, n: int, method: int = 1) -> np.ndarray:
    """t x t matrix from k x k decrypted n x n blocks B[a][b] of a feature x
    feature result (covariance) packed with the given padding method"""
    w = features_per_block(t, n, method)
    M = np.zeros((t, t))
    for a in range(len(B)):
        for b in range(len(B)):
            ra, rb_ = range(a * w, min((a + 1) * w, t)), range(b * w, min((b + 1) * w, t))
            M[ra.start:ra.stop, rb_.start:rb_.stop] = B[a][b][: len(ra), : len(rb_)]
    return M
