"""Parity at the full-size chain (N = 2^16, q0 60b + 30 x 40b, three 60-bit
special primes): bit-exact rotation and 16 x 16 product against the oracle,
and the 128 x 128 product in the benchmark's launch configuration against
FP64 within 2^-15, decrypted through every limb by the oracle."""
import numpy as np
import pytest

from paper_2305_17341_amd import inputs as I
from tests.fullcrt import FullDecryptor

pytestmark = pytest.mark.gpu

BOUND = 2.0**-15
C = I.LARGE


@pytest.fixture(scope="module")
def gpu_ctx():
    from paper_2305_17341_amd import he
    ctx = he.chain_context(C, seed=31)
    steps = sorted(set(ctx.matmul_rot_steps(16)) | set(ctx.matmul_rot_steps(128)) | {1})
    ctx.keygen(steps)
    return ctx


@pytest.fixture(scope="module")
def oracle16(oracle_mod, gpu_ctx):
    o = oracle_mod.Oracle(C.log_n, C.q_bits, C.p_bits, seed=31)
    o.keygen(rot_steps=sorted(set(gpu_ctx.matmul_rot_steps(16)) | {1}))
    return o


def test_large_rotation_bit_exact(gpu_ctx, oracle16):
    z = np.random.default_rng(1).uniform(-1, 1, oracle16.slots)
    g = gpu_ctx.encrypt(z, nonce=7)
    o = oracle16.encrypt(z, nonce=7)
    assert np.array_equal(g.export(), o.data())
    for step in (1, -16):
        r = gpu_ctx.rotate(g, step)
        assert np.array_equal(r.export(), oracle16.rotate(o, step).data())
        assert np.max(np.abs(gpu_ctx.decrypt(r) - np.roll(z, -step))) < 2.0**-19


def test_large_matmul_16_bit_exact(gpu_ctx, oracle16):
    n = 16
    A, B = I.uniform_matrix(61, n), I.uniform_matrix(62, n)
    r = gpu_ctx.matmul(gpu_ctx.encrypt_matrix(A, nonce=1), gpu_ctx.encrypt_matrix(B, nonce=2), n)
    want = oracle16.matmul(oracle16.encrypt(A.ravel(), nonce=1), oracle16.encrypt(B.ravel(), nonce=2), n, 4, 4)
    assert r.level == C.top_level - 3
    assert np.array_equal(r.export(), want.data())
    err = np.max(np.abs(gpu_ctx.decrypt(r, n * n) - (A @ B).ravel()))
    assert err < BOUND, err


def test_large_matmul_128_accuracy_batched_launch(gpu_ctx, oracle_mod):
    fd = FullDecryptor(oracle_mod, C, 31)
    n = 128
    As = [I.uniform_matrix(100 + i, n) for i in range(2)]
    Bs = [I.uniform_matrix(200 + i, n) for i in range(2)]
    cA = [gpu_ctx.encrypt_matrix(a, nonce=1 + i) for i, a in enumerate(As)]
    cB = [gpu_ctx.encrypt_matrix(b, nonce=1001 + i) for i, b in enumerate(Bs)]
    outs = gpu_ctx.matmul_batch(cA, cB, [n, n])
    for a, b, r in zip(As, Bs, outs):
        assert r.level == C.top_level - 3
        err = np.max(np.abs(fd.decrypt(r, n * n) - (a @ b).ravel()))
        assert err < BOUND, err
    # deterministic: the same inputs give the same residues
    again = gpu_ctx.matmul(cA[0], cB[0], n)
    assert np.array_equal(again.export(), outs[0].export())
