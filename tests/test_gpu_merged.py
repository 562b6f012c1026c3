"""Products of different sizes and levels in one call with their key inner
products merged (HE_MM_MERGED): each merged launch serves a key-switch step
of every product (items of different levels and rotation sets side by side),
and every result is residue for residue the product computed alone, which
the oracle pins for one of them."""
import numpy as np
import pytest

from paper_2305_17341_amd import inputs as I

pytestmark = pytest.mark.gpu

C = I.MID
BATCHED, LAZY, FUSED, MERGED = 1, 2, 4, 64


@pytest.fixture(scope="module")
def ctx():
    from paper_2305_17341_amd import he
    c = he.chain_context(C, seed=83)
    steps = set()
    for d in (8, 16, 32, 64):
        steps |= set(c.matmul_rot_steps(d))
    c.keygen(sorted(steps))
    return c


def _mix(ctx):
    # (d, level): sizes 8 to 64, two products of d = 16 at the top (stacked),
    # one at a lower level
    spec = [(16, 8), (64, 8), (8, 8), (32, 8), (16, 8), (16, 5)]
    As = [I.uniform_matrix(900 + i, d) for i, (d, _) in enumerate(spec)]
    Bs = [I.uniform_matrix(950 + i, d) for i, (d, _) in enumerate(spec)]
    cA = [ctx.encrypt_matrix(a, level=l, nonce=1 + i) for i, (a, (_, l)) in enumerate(zip(As, spec))]
    cB = [ctx.encrypt_matrix(b, level=l, nonce=101 + i) for i, (b, (_, l)) in enumerate(zip(Bs, spec))]
    return spec, As, Bs, cA, cB


@pytest.mark.parametrize("variant", [0, LAZY | FUSED])
def test_merged_mix_equals_alone(ctx, oracle_mod, variant):
    spec, As, Bs, cA, cB = _mix(ctx)
    ds = [d for d, _ in spec]
    outs = ctx.matmul_batch(cA, cB, ds, {"flags": BATCHED | MERGED | variant})
    for i, (d, lvl) in enumerate(spec):
        alone = ctx.matmul(cA[i], cB[i], d, {"flags": variant})
        assert outs[i].level == lvl - 3
        assert np.array_equal(outs[i].export(), alone.export()), (i, d, lvl)
        assert np.max(np.abs(ctx.decrypt(outs[i], d * d) - (As[i] @ Bs[i]).ravel())) < 2.0 ** -15
    if variant == 0:
        o = oracle_mod.Oracle(C.log_n, C.q_bits, C.p_bits, seed=83)
        o.keygen(rot_steps=ctx.matmul_rot_steps(8))
        want = o.matmul(o.encrypt(As[2].ravel(), nonce=3), o.encrypt(Bs[2].ravel(), nonce=103), 8, 4, 4)
        assert np.array_equal(outs[2].export(), want.data())


def test_merged_launches_fewer_key_switch_kernels(ctx):
    spec, As, Bs, cA, cB = _mix(ctx)
    ds = [d for d, _ in spec]
    counts = {}
    for flags in (BATCHED, BATCHED | MERGED):
        ctx.matmul_batch(cA, cB, ds, {"flags": flags})
        ctx.sync()
        ctx.profile_enable(True)
        ctx.matmul_batch(cA, cB, ds, {"flags": flags})
        ctx.sync()
        counts[flags] = ctx.profile_read("multsum_rot")[1] + ctx.profile_read("multsum")[1]
        ctx.profile_enable(False)
    print("key inner product launches, stacked vs merged:", counts, flush=True)
    assert counts[BATCHED | MERGED] < counts[BATCHED]


def test_merged_missing_key_fails_and_context_survives(ctx):
    from paper_2305_17341_amd import he
    a = ctx.encrypt_matrix(I.uniform_matrix(1, 4), nonce=1)          # d = 4: no keys generated for it
    b = ctx.encrypt_matrix(I.uniform_matrix(2, 16), nonce=2)
    with pytest.raises(he.HeError) as e:
        ctx.matmul_batch([a, b], [a, b], [4, 16], {"flags": BATCHED | MERGED})
    assert e.value.status == -4
    r = ctx.matmul_batch([b, b], [b, b], [16, 16], {"flags": BATCHED | MERGED})
    assert np.array_equal(r[0].export(), ctx.matmul(b, b, 16).export())


def test_merged_stacks_of_many_member_counts(ctx):
    """stacks of 1, 2, 3 and 4 members (one merged launch per member count)"""
    spec = [8] + [16] * 2 + [32] * 3 + [64] * 4
    As = [I.uniform_matrix(700 + i, d) for i, d in enumerate(spec)]
    cA = [ctx.encrypt_matrix(a, nonce=300 + i) for i, a in enumerate(As)]
    outs = ctx.matmul_batch(cA, cA, spec, {"flags": BATCHED | MERGED | LAZY})
    for i, d in enumerate(spec):
        alone = ctx.matmul(cA[i], cA[i], d, {"flags": LAZY})
        assert np.array_equal(outs[i].export(), alone.export()), (i, d)
