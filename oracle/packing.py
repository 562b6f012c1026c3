"""Section 5.1's packing of an s x t dataset into n x n blocks, for the
oracle's tests.

TEST INFRASTRUCTURE ONLY (like the rest of oracle/).  Rows go in blocks of n
(the last zero-padded).  Features go in k = ceil(t / n) blocks:
  * method 1 fills each block's n columns in feature order, and only the
    last block has padding columns;
  * method 2 gives every block p = floor((k n - t) / k) padding columns at
    its end, so each block holds n - p features.
Each feature's (block, column) is computed as divmod(feature, width) and the
data scattered in one indexing step.
"""
from __future__ import annotations

import numpy as np


def width(t: int, n: int, method: int) -> int:
    """features per block"""
    if method == 1:
        return n
    k = -(-t // n)
    return n - (k * n - t) // k


def pack(X: np.ndarray, n: int, method: int = 1) -> np.ndarray:
    """[row block][feature block][n][n]"""
    s, t = X.shape
    w = width(t, n, method)
    fb, fc = np.divmod(np.arange(t), w)
    rb, rr = np.divmod(np.arange(s), n)
    out = np.zeros((-(-s // n), -(-t // n), n, n))
    out[rb[:, None], fb[None, :], rr[:, None], fc[None, :]] = X
    return out


def unpack_square(B, t: int, n: int, method: int = 1) -> np.ndarray:
    """t x t matrix from the k x k blocks B[a][b] of a feature x feature result"""
    w = width(t, n, method)
    fb, fc = np.divmod(np.arange(t), w)
    Bs = np.asarray(B, dtype=np.float64)
    return Bs[fb[:, None], fb[None, :], fc[:, None], fc[None, :]]
