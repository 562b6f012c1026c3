"""Hoisted rotations of a batch of ciphertexts by several steps
(he_rotate_many, section 3.3.1): residue for residue what one rotation at a
time gives, and what the oracle gives."""
import numpy as np
import pytest

from paper_2305_17341_amd import inputs as I

pytestmark = pytest.mark.gpu

C = I.MID
STEPS = [1, -5, 37, 0, 1000, -1]


def test_rotate_many_equals_single_rotations(oracle_mod):
    from paper_2305_17341_amd import he
    ctx = he.chain_context(C, seed=81)
    ctx.keygen([s for s in STEPS if s])
    rng = np.random.default_rng(3)
    zs = [rng.uniform(-1, 1, ctx.N // 2) for _ in range(3)]
    cts = [ctx.encrypt(z, nonce=10 + i) for i, z in enumerate(zs)]
    got = ctx.rotate_many(cts, STEPS)
    for i, c in enumerate(cts):
        for r, s in enumerate(STEPS):
            assert np.array_equal(got[i][r].export(), ctx.rotate(c, s).export()), (i, s)
    o = oracle_mod.Oracle(C.log_n, C.q_bits, C.p_bits, seed=81)
    o.keygen(rot_steps=[37], relin=False)
    assert np.array_equal(got[1][2].export(), o.rotate(o.encrypt(zs[1], nonce=11), 37).data())
    # one ciphertext at a lower level
    low = ctx.drop(cts[0], 3)
    one = ctx.rotate_many([low], STEPS[:3])
    for r, s in enumerate(STEPS[:3]):
        assert np.array_equal(one[0][r].export(), ctx.rotate(low, s).export())
    with pytest.raises(he.HeError) as e:
        ctx.rotate_many(cts, [2])
    assert e.value.status == -4
