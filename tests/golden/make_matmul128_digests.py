"""Writes matmul128_digests.json: SHA-256 digests of the residues of 128 x 128
homomorphic products computed by the CPU oracle alone (Algorithm DMatrixMult
with the hoisting of section 4.1: double-hoisted BSGS Z and T, hoisted column
and row shifts, n products, rescale).

Cases (inputs from the seeded generators; keys and encryption randomness are
functions of the context seed and the nonces):
  n15_batch8  N = 2^15, Q = 60 + 14 x 40 bits, P = 3 x 60 bits, context seed 41,
              n1 = 64 for Z, T and the shift blocks, lazy relinearisation and
              ModDown + Rescale of the A side as one rounding; eight products
              A_i B_i, A_i = uniform_matrix(500 + i), B_i = uniform_matrix(600 + i),
              nonces 1 + i and 101 + i.
  n16_default N = 2^16, Q = 60 + 30 x 40 bits, P = 3 x 60 bits, context seed 43,
              n1 = 16 (the default for d = 128), the paper's order
              (relinearisation per product, two roundings); one product
              A = uniform_matrix(700), B = uniform_matrix(701), nonces 1 and 2.

Each digest covers the u64 residues [2][l+1][N] as little-endian bytes; a
digest per limb localises a difference.  The FP64 error of the oracle's own
decryption (exact CRT) against A B is recorded for reference.

This script calls only the oracle and the seeded input generators.  It takes
about 20 minutes on 8 cores and 30 GB of memory:
    python tests/golden/make_matmul128_digests.py
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "matmul128_digests.json")

CASES = {
    "n15_batch8": {"log_n": 15, "q_bits": [60] + [40] * 14, "p_bits": [60, 60, 60], "seed": 41, "n1": 64,
                   "lazy": True, "fused_rescale": True,
                   "members": [{"a_seed": 500 + i, "b_seed": 600 + i, "nonce_a": 1 + i, "nonce_b": 101 + i}
                               for i in range(8)]},
    "n16_default": {"log_n": 16, "q_bits": [60] + [40] * 30, "p_bits": [60, 60, 60], "seed": 43, "n1": 16,
                    "lazy": False, "fused_rescale": False,
                    "members": [{"a_seed": 700, "b_seed": 701, "nonce_a": 1, "nonce_b": 2}]},
}
N_MAT = 128


def rotation_steps(n, n1):
    """Every rotation the product takes (section 4.1 with the BSGS index
    range i in [-n2, n2) for Z and [0, n2) for T): baby steps j and giant
    steps n1 i of Z (diagonals k in (-n, n)); baby steps n j and giant steps
    n n1 i of T (diagonals n k, k in [0, n)); the column shifts j < n1, the
    chain step n1 and the second chain's start -n; the row shifts n j and the
    chain step n n1."""
    s = set(range(1, n1))
    lo, hi = -((n - 1 + n1 - 1) // n1), (n - 1) // n1
    s |= {n1 * i for i in range(lo, hi + 1) if i}
    s |= {n * j for j in range(1, n1)}
    s |= {n * n1 * i for i in range(1, (n - 1) // n1 + 1)}
    s |= {n1, -n, n * n1}
    return sorted(s)


def digest(a):
    return hashlib.sha256(a.astype("<u8").tobytes()).hexdigest()


def run_case(name, member_ids, threads):
    os.environ["OMP_NUM_THREADS"] = str(threads)
    sys.path.insert(0, ROOT)
    import numpy as np

    from oracle import oracle as O
    from paper_2305_17341_amd import inputs as I

    c = CASES[name]
    t0 = time.time()
    o = O.Oracle(c["log_n"], c["q_bits"], c["p_bits"], seed=c["seed"])
    o.keygen(rot_steps=rotation_steps(N_MAT, c["n1"]))
    print(f"[{name}] keys in {time.time() - t0:.0f} s", flush=True)
    out = []
    for i in member_ids:
        m = c["members"][i]
        A, B = I.uniform_matrix(m["a_seed"], N_MAT), I.uniform_matrix(m["b_seed"], N_MAT)
        oa, ob = o.encrypt(A.ravel(), nonce=m["nonce_a"]), o.encrypt(B.ravel(), nonce=m["nonce_b"])
        t1 = time.time()
        r = o.matmul(oa, ob, N_MAT, c["n1"], c["n1"], lazy=c["lazy"], fused_rescale=c["fused_rescale"])
        dt = time.time() - t1
        data = r.data()
        err = float(np.max(np.abs(o.decrypt(r, N_MAT * N_MAT) - (A @ B).ravel())))
        out.append({"member": i, "level": int(r.level), "scale": float(r.scale), "sha256": digest(data),
                    "limb_sha256": [[digest(data[p, k])[:16] for k in range(data.shape[1])] for p in range(2)],
                    "fp64_max_abs_err": err, "oracle_seconds": round(dt, 1), "oracle_threads": threads})
        print(f"[{name}] member {i}: {dt:.0f} s, error {err:.2e}", flush=True)
    return name, out


def main():
    jobs = [("n15_batch8", [0, 1, 2, 3], 3), ("n15_batch8", [4, 5, 6, 7], 3), ("n16_default", [0], 3)]
    res = {name: dict(CASES[name], rotation_steps=rotation_steps(N_MAT, CASES[name]["n1"])) for name in CASES}
    for v in res.values():
        v["results"] = []
    with ProcessPoolExecutor(max_workers=len(jobs)) as ex:
        for name, out in ex.map(run_case, *zip(*jobs)):
            res[name]["results"].extend(out)
    for v in res.values():
        v["results"].sort(key=lambda r: r["member"])
    with open(OUT, "w") as fh:
        json.dump({"about": "oracle residue digests of 128 x 128 products (see make_matmul128_digests.py)",
                   "n": N_MAT, "cases": res}, fh, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
