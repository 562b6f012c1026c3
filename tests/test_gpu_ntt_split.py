"""The NTT's alternative stage splits (knob ntt_split_<log N>: one stage moved
between the column and block passes) give the oracle's transforms bit for
bit, forward and inverse, with edge values; and a whole product (Decompose,
ModDown and Rescale use the same passes fused with their conversions)
keeps its residues under either split."""
import numpy as np
import pytest

from paper_2305_17341_amd import inputs as I

pytestmark = pytest.mark.gpu

CHAINS = {13: I.SMALL, 14: I.MID, 15: I.SERVE15}


@pytest.mark.parametrize("log_n", [13, 14, 15])
def test_split_transforms_bit_exact(oracle_mod, log_n):
    from paper_2305_17341_amd import he
    ch = CHAINS[log_n]
    ctx = he.chain_context(ch)
    o = oracle_mod.Oracle(ch.log_n, ch.q_bits, ch.p_bits)
    g = np.random.default_rng(log_n + 100)
    mods = list(range(len(o.moduli)))
    limbs = np.stack([g.integers(0, o.moduli[m], o.N, dtype=np.uint64) for m in mods])
    limbs[0, :] = o.moduli[0] - 1
    limbs[1, :] = 0
    knob = f"ntt_split_{log_n}"
    saved = he.knob_get(knob)
    try:
        for split in (1, 0):
            he.knob_set(knob, split)
            fwd = ctx.ntt_limbs(limbs, mods)
            for k, m in enumerate(mods):
                assert np.array_equal(fwd[k], o.ntt(m, limbs[k])), (log_n, split, m)
            assert np.array_equal(ctx.ntt_limbs(fwd, mods, inverse=True), limbs), (log_n, split)
    finally:
        he.knob_set(knob, saved)


@pytest.mark.parametrize("log_n,d", [(13, 16), (14, 32), (15, 64)])
def test_split_keeps_product_residues(log_n, d):
    from paper_2305_17341_amd import he
    ch = CHAINS[log_n]
    ctx = he.chain_context(ch, seed=5)
    ctx.keygen(ctx.matmul_rot_steps(d))
    A, B = I.uniform_matrix(1, d), I.uniform_matrix(2, d)
    ca, cb = ctx.encrypt_matrix(A, nonce=1), ctx.encrypt_matrix(B, nonce=2)
    knob = f"ntt_split_{log_n}"
    saved = he.knob_get(knob)
    try:
        outs = {}
        for split in (0, 1):
            he.knob_set(knob, split)
            outs[split] = [ctx.matmul(ca, cb, d, {"flags": f}).export() for f in (0, 2 | 4)]
        for a, b in zip(outs[0], outs[1]):
            assert np.array_equal(a, b)
    finally:
        he.knob_set(knob, saved)
    with pytest.raises(he.HeError):
        he.knob_set("ntt_split_16", 1)
