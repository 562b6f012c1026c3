"""Z and T alone, by double-hoisted BSGS and decomposed by diagonal
convergence (he_lintrans_dcd): residue for residue equal to the oracle, the
levels consumed as Table 2 counts them, and the Table 3 analogue's
measurement on a small ring (keys, levels, accuracy)."""
import math

import numpy as np
import pytest

from paper_2305_17341_amd import inputs as I

pytestmark = pytest.mark.gpu

DEEP = I.Chain("n11_deep", 11, (60,) + (40,) * 6, (60, 60))


@pytest.mark.parametrize("kind,nprime", [(0, 0), (0, 4), (1, 0), (1, 4), (0, 8), (1, 8)])
def test_dcd_transform_bit_exact(oracle_mod, kind, nprime):
    from paper_2305_17341_amd import he
    n, n1 = 16, 4
    ctx = he.chain_context(DEEP, seed=53)
    steps = he.lintrans_rot_steps("Z" if kind == 0 else "T", n, n1, nprime)
    ctx.keygen(steps)
    o = oracle_mod.Oracle(DEEP.log_n, DEEP.q_bits, DEEP.p_bits, seed=53)
    o.keygen(rot_steps=steps)
    A = I.uniform_matrix(7, n)
    g = ctx.lintrans_dcd(ctx.encrypt_matrix(A, nonce=3), kind, n, n1, nprime)
    w = o.lt_dcd(o.encrypt(A.ravel(), nonce=3), kind, n, n1, nprime if nprime else n - 1)
    depth = 1 if nprime == 0 else math.ceil((n - 1) / nprime)
    assert g.level == DEEP.top_level - depth == w.level and g.scale == w.scale
    assert np.array_equal(g.export(), w.data())
    from paper_2305_17341_amd import table3
    want = (table3.sigma if kind == 0 else table3.tau)(A).ravel()
    assert np.max(np.abs(ctx.decrypt(g, n * n) - want)) < 2.0**-15


def test_table3_analogue_small():
    from paper_2305_17341_amd import table3
    ch = I.Chain("n11_t3", 11, (60,) + (40,) * 14, (60, 60, 60))
    res = table3.run(reps=1, d=16, chain=ch)
    assert len(res["rows"]) == len(table3.ROWS) + len(table3.SMP_ROWS) == 16
    for r in res["rows"]:
        assert r["level_out"] == table3.BASELINE
        assert r["max_abs_err"] < 2.0**-15
        assert r["time_ms"] > 0 and r["rtk_mib"] > 0


@pytest.mark.parametrize("kind,n1,n1p", [(0, 4, 2), (0, 8, 3), (1, 4, 2), (1, 8, 4), (0, 8, 8)])
def test_smpkeysub_transform_bit_exact(oracle_mod, kind, n1, n1p):
    """dh-BSGS with the simple key substitution of the baby steps (section
    4.2.1), keys of the planner only: residues equal to the oracle's"""
    from paper_2305_17341_amd import he
    n = 16
    steps = he.smpkeysub_rot_steps("Z" if kind == 0 else "T", n, n1, n1p)
    ctx = he.chain_context(DEEP, seed=59)
    ctx.keygen(steps)
    o = oracle_mod.Oracle(DEEP.log_n, DEEP.q_bits, DEEP.p_bits, seed=59)
    o.keygen(rot_steps=steps)
    A = I.uniform_matrix(11, n)
    g = ctx.lintrans_smpkeysub(ctx.encrypt_matrix(A, nonce=6), kind, n, n1, n1p)
    w = o.lt_smpkeysub(o.encrypt(A.ravel(), nonce=6), kind, n, n1, n1p)
    assert g.level == DEEP.top_level - 1 == w.level and g.scale == w.scale
    assert np.array_equal(g.export(), w.data())
    if n1p >= n1:   # no prefix: the plain transform, bit for bit
        p = ctx.lintrans(ctx.encrypt_matrix(A, nonce=6), kind, n, n1)
        assert np.array_equal(g.export(), p.export())


def test_smpkeysub_rejects_a_one_step_prefix():
    from paper_2305_17341_amd import he
    ctx = he.chain_context(DEEP, seed=59)
    ctx.keygen([1])
    x = ctx.encrypt_matrix(I.uniform_matrix(11, 16), nonce=6)
    with pytest.raises(he.HeError, match="EINVAL"):
        ctx.lintrans_smpkeysub(x, 0, 16, 4, 1)
