"""The depth-2 product with C^k's masks folded into Z (HE_MM_FOLDED) on the
small workload's literal chain (q0 + two 40-bit primes, one 60-bit special
prime): residue for residue the oracle's folded plan, with and without lazy
relinearisation, batched equal to alone, within 2^-15 of A B at level 0, and
keys for Z, T and the row shifts only."""
import numpy as np
import pytest

from paper_2305_17341_amd import inputs as I

pytestmark = pytest.mark.gpu

LITERAL_SMALL = I.Chain("n13_literal", 13, (60, 40, 40), (60,))
BATCHED, LAZY, FOLDED = 1, 2, 32
BOUND = 2.0 ** -15


@pytest.fixture(scope="module")
def pair(oracle_mod):
    from paper_2305_17341_amd import he
    ch = LITERAL_SMALL
    ctx = he.chain_context(ch, seed=17)
    steps = sorted(set(ctx.matmul_rot_steps(16, {"flags": FOLDED})) |
                   set(ctx.matmul_rot_steps(16, {"n1_z": 16, "n1_t": 16, "flags": FOLDED})))
    ctx.keygen(steps)
    o = oracle_mod.Oracle(ch.log_n, ch.q_bits, ch.p_bits, seed=17)
    o.keygen(rot_steps=steps)
    return ctx, o


def test_folded_plan_keys():
    from paper_2305_17341_amd import he
    n, n1 = 16, 4
    want = set(range(1, n1)) | {n1 * i for i in range(-4, 4) if i} | {n * j for j in range(1, n1)} | \
        {n * n1 * i for i in range(1, 4)}
    ctx = he.chain_context(LITERAL_SMALL, seed=1)
    assert set(ctx.matmul_rot_steps(n, {"flags": FOLDED})) == want
    assert -n in set(ctx.matmul_rot_steps(n))       # the three-level plan's second shift chain


@pytest.mark.parametrize("lazy,n1", [(False, 4), (True, 4), (True, 16)])
def test_folded_product_bit_exact(pair, lazy, n1):
    ctx, o = pair
    n = 16
    A, B = I.uniform_matrix(41, n), I.uniform_matrix(42, n)
    opts = {"n1_z": n1, "n1_t": n1, "flags": FOLDED | (LAZY if lazy else 0)}
    ca, cb = ctx.encrypt_matrix(A, nonce=1), ctx.encrypt_matrix(B, nonce=2)
    r = ctx.matmul(ca, cb, n, opts)
    want = o.matmul(o.encrypt(A.ravel(), nonce=1), o.encrypt(B.ravel(), nonce=2), n, n1, n1, lazy=lazy, folded=True)
    assert r.level == want.level == 0 and r.scale == want.scale
    assert np.array_equal(r.export(), want.data())
    assert np.max(np.abs(ctx.decrypt(r, n * n) - (A @ B).ravel())) < BOUND
    outs = ctx.matmul_batch([ca, cb], [cb, ca], [n, n], dict(opts, flags=opts["flags"] | BATCHED))
    assert np.array_equal(outs[0].export(), r.export())
    assert np.max(np.abs(ctx.decrypt(outs[1], n * n) - (B @ A).ravel())) < BOUND


def test_three_level_plan_refused_on_the_literal_chain(pair):
    from paper_2305_17341_amd import he
    ctx, _ = pair
    a = ctx.encrypt_matrix(I.uniform_matrix(1, 16), nonce=1)
    with pytest.raises(he.HeError) as e:
        ctx.matmul(a, a, 16)
    assert e.value.status == -2
    with pytest.raises(he.HeError) as e:
        ctx.matmul(a, a, 16, {"flags": FOLDED | 4})
    assert e.value.status == -1
