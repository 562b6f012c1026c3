"""The benchmark's product plan pinned residue for residue at sizes the
oracle cannot run inside a test: the oracle's residues of 128 x 128 products
are stored as SHA-256 digests (tests/golden/matmul128_digests.json, written
by tests/golden/make_matmul128_digests.py, which calls only the oracle).

  * N = 2^15 (q0 + 14 x 40-bit, 3 x 60-bit special primes): the benchmark's
    plan exactly (Algorithm DMatrixMult with n1 = 64 for Z, T and the shifts,
    lazy relinearisation, ModDown + Rescale of the A side as one rounding,
    eight products per launch, replays of the recorded HIP graph, and the
    same launches issued one kernel at a time).  This runs the 63-rotation
    key inner products and the 64-term multiply-sums the headline runs.
  * N = 2^16 (q0 + 30 x 40-bit, 3 x 60-bit): one product with the library's
    defaults (n1 = 16, relinearisation per product, two roundings).
"""
import hashlib
import json
import os

import numpy as np
import pytest

from paper_2305_17341_amd import inputs as I
from tests.fullcrt import FullDecryptor

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden", "matmul128_digests.json")
BATCHED, LAZY, FUSED, GRAPH = 1, 2, 4, 8
N_MAT = 128


def _cases():
    with open(GOLD) as fh:
        return json.load(fh)["cases"]


def _digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).astype("<u8").tobytes()).hexdigest()


def _check(got, want, tag):
    assert got.shape[1] == want["level"] + 1, tag
    if _digest(got) == want["sha256"]:
        return
    bad = [(p, k) for p in range(2) for k in range(got.shape[1])
           if _digest(got[p, k])[:16] != want["limb_sha256"][p][k]]
    raise AssertionError(f"{tag}: residues differ from the oracle's in (poly, limb) {bad}")


def _context(case):
    from paper_2305_17341_amd import he
    ch = I.Chain("pinned", case["log_n"], tuple(case["q_bits"]), tuple(case["p_bits"]))
    ctx = he.chain_context(ch, seed=case["seed"])
    geo = {"n1_z": case["n1"], "n1_t": case["n1"]}
    steps = ctx.matmul_rot_steps(N_MAT, geo)
    assert sorted(steps) == case["rotation_steps"]   # the planner against the oracle script's enumeration
    ctx.keygen(steps)
    return ch, ctx, geo


def _operands(ctx, members):
    As = [I.uniform_matrix(m["a_seed"], N_MAT) for m in members]
    Bs = [I.uniform_matrix(m["b_seed"], N_MAT) for m in members]
    cA = [ctx.encrypt_matrix(a, nonce=m["nonce_a"]) for a, m in zip(As, members)]
    cB = [ctx.encrypt_matrix(b, nonce=m["nonce_b"]) for b, m in zip(Bs, members)]
    return As, Bs, cA, cB


def test_benchmark_plan_n15_batch8_bit_exact(oracle_mod):
    case = _cases()["n15_batch8"]
    ch, ctx, geo = _context(case)
    members = case["members"]
    As, Bs, cA, cB = _operands(ctx, members)
    want = case["results"]
    flags = BATCHED | LAZY | FUSED
    # eager (one kernel at a time), then the recording and two replays
    for rep, f in enumerate([flags, flags | GRAPH, flags | GRAPH, flags | GRAPH]):
        outs = ctx.matmul_batch(cA, cB, [N_MAT] * len(members), dict(geo, flags=f))
        print(f"n15 batch of 8, pass {rep} (flags {f}) done", flush=True)
        for i, o in enumerate(outs):
            assert o.scale == want[i]["scale"]
            _check(o.export(), want[i], f"pass {rep} member {i}")
    fd = FullDecryptor(oracle_mod, ch, case["seed"])
    err = np.max(np.abs(fd.decrypt(outs[0], N_MAT * N_MAT) - (As[0] @ Bs[0]).ravel()))
    assert err < 2.0 ** -15, err
    del outs
    ctx.close()


def test_default_product_n16_bit_exact():
    case = _cases()["n16_default"]
    ch, ctx, geo = _context(case)
    As, Bs, cA, cB = _operands(ctx, case["members"])
    r = ctx.matmul(cA[0], cB[0], N_MAT)
    assert r.scale == case["results"][0]["scale"]
    _check(r.export(), case["results"][0], "N=2^16 default product")
    ctx.close()
