"""Measurement analogue of Table 3 (section 7.1): the transforms Z and T of a
128 x 128 product by double-hoisted BSGS (MaxDiagNo 127) and decomposed by
diagonal convergence (section 4.2, MaxDiagNo 64 and 32), with 8 and 16 baby
steps, on this GPU; and, beside them, dh-BSGS with the simple key
substitution of the baby steps (section 4.2.1, n1 = 16, prefixes 8 and 4).  Ring N = 2^15 with Q = 60 + 14 x 40 bits and P = 3 x 60
bits: a switching key of 5 digits x 18 limbs is 45 MiB, the key geometry of
the paper's table (maximum level 14).  Every transform starts at the level
that makes it end at the baseline level 10 (14 - 4).

Per row: the rotation keys the transform needs (MinRotKeys) and the HBM
bytes of those keys plus the relinearisation key (as the table's Rtk column
counts), the hoisted-ciphertext space of the BSGS (n1 - 1 elements of
R_{Q_l P} at the level of the last factor, one above the baseline: the
factors before it have at most three diagonals and hoist at most two) and
the measured device peak of the call, the time of one transform (median of
`reps` after a warm-up) and of a batch of 8 stacked ciphertexts, the levels
consumed, and the decrypted error against the plaintext permutation."""
from __future__ import annotations

import math
import time

import numpy as np

from . import he
from . import inputs as I

# (matrix, n1, divisor): MaxDiagNo d - 1 (no decomposition), d / 2 and d / 4
# (127, 64 and 32 for d = 128, the table's rows)
ROWS = [(m, n1, div) for m in ("Z", "T") for n1 in (8, 16) for div in (1, 2, 4)]
# (matrix, n1, n1'): the simple key substitution of section 4.2.1 (Table 2's
# SmpKeySub rows; not measured in the paper's Table 3)
SMP_ROWS = [(m, 16, p) for m in ("Z", "T") for p in (8, 4)]
BASELINE = 10


def sigma(A):
    """Z: sigma(A)_{i,j} = A_{i,(i+j) mod n}"""
    n = A.shape[0]
    i, j = np.indices((n, n))
    return A[i, (i + j) % n]


def tau(A):
    """T: tau(A)_{i,j} = A_{(i+j) mod n, j}"""
    n = A.shape[0]
    i, j = np.indices((n, n))
    return A[(i + j) % n, j]


def run(reps: int = 3, d: int = 128, chain=I.SERVE15, seed: int = 5, log=None):
    alpha = len(chain.p_bits)
    L = len(chain.q_bits) - 1
    key_bytes = math.ceil((L + 1) / alpha) * 2 * (L + 1 + alpha) * chain.N * 8
    A = I.uniform_matrix(seed, d)
    rows = []
    cases = [(m, n1, div, 0) for m, n1, div in ROWS] + [(m, n1, 1, p) for m, n1, p in SMP_ROWS]
    for matrix, n1, div, n1p in cases:
        kind = 0 if matrix == "Z" else 1
        maxdiag = d - 1 if div == 1 else d // div
        nprime = 0 if div == 1 else maxdiag
        depth = 1 if nprime == 0 else math.ceil((d - 1) / nprime)
        start = BASELINE + depth
        ctx = he.chain_context(chain, seed=seed)
        if n1p:
            steps = he.smpkeysub_rot_steps(matrix, d, n1, n1p)
            def transform(c):
                return ctx.lintrans_smpkeysub(c, kind, d, n1, n1p)
        else:
            steps = he.lintrans_rot_steps(matrix, d, n1, nprime)
            def transform(c):
                return ctx.lintrans_dcd(c, kind, d, n1, nprime)
        ctx.keygen(steps)
        ct = ctx.encrypt_matrix(A, level=start, nonce=1)
        cts8 = [ctx.encrypt_matrix(A, level=start, nonce=10 + i) for i in range(8)]
        out = transform(ct)      # warm-up: plaintext diagonals cached
        ctx.sync()
        ctx.trim()
        live0, _, _ = ctx.mem_info()
        times = []
        for _ in range(reps):
            t0 = time.perf_counter()
            out = transform(ct)
            ctx.sync()
            times.append(time.perf_counter() - t0)
        _, _, peak = ctx.mem_info()
        want = (sigma if kind == 0 else tau)(A).ravel()
        err = float(np.max(np.abs(ctx.decrypt(out, d * d) - want)))
        # eight ciphertexts through the same transform, one after another
        ctx.sync()
        t0 = time.perf_counter()
        for c in cts8:
            o = transform(c)
        ctx.sync()
        t8 = time.perf_counter() - t0
        qp_ct = 2 * (BASELINE + 1 + 1 + alpha) * chain.N * 8
        scheme = "SmpKeySub" if n1p else "dh-BSGS" if nprime == 0 else "DCDmp"
        row = {"scheme": scheme, "matrix": matrix, "n1": n1, "n1p": n1p or None,
               "max_diag": maxdiag if matrix == "Z" else f"{maxdiag}*{d}",
               # the table's Rtk column counts one key more than the rotations (the
               # relinearisation key)
               "rot_keys": len(steps), "rtk_mib": round((len(steps) + 1) * key_bytes / 2**20, 1),
               "ct_mib_model": round((n1 - 1) * qp_ct / 2**20, 1),
               "peak_mib_measured": round((peak - live0) / 2**20, 1),
               "time_ms": round(1e3 * sorted(times)[len(times) // 2], 2), "time_8_ms": round(1e3 * t8, 2),
               "depth": depth, "level_out": out.level, "max_abs_err": err}
        rows.append(row)
        if log:
            log(f"[table3] {row}")
        del out, o, ct, cts8
        ctx.close()
    return {"workload": f"Z and T of a {d}x{d} product at N=2^{chain.log_n} (Q 60b + {L}x40b, P {alpha}x60b, "
                        f"one key {key_bytes / 2**20:.0f} MiB), ending at level {BASELINE}",
            "rows": rows}
