"""Recorded batched products (HE_MM_GRAPH): the launch sequence of a batch is
captured once as a HIP graph and replayed.  Every replay, with eager work of
the program in between, must give residue for residue the unrecorded
result; dropping the recordings (he_trim) re-records; the recording refuses
to run while the kernel profile is on."""
import numpy as np
import pytest

from paper_2305_17341_amd import inputs as I

pytestmark = pytest.mark.gpu

BATCHED, LAZY, FUSED, GRAPH = 1, 2, 4, 8


@pytest.fixture(scope="module")
def ctx():
    from paper_2305_17341_amd import he
    c = he.chain_context(I.SMALL, seed=41)
    c.keygen(sorted(set(c.matmul_rot_steps(16)) | set(c.matmul_rot_steps(8))))
    return c


def _pairs(ctx, n, count, seed):
    As = [I.uniform_matrix(seed + i, n) for i in range(count)]
    Bs = [I.uniform_matrix(seed + 50 + i, n) for i in range(count)]
    cA = [ctx.encrypt_matrix(a, nonce=seed + i) for i, a in enumerate(As)]
    cB = [ctx.encrypt_matrix(b, nonce=seed + 70 + i) for i, b in enumerate(Bs)]
    return As, Bs, cA, cB


@pytest.mark.parametrize("flags", [BATCHED, BATCHED | LAZY | FUSED])
def test_replays_equal_eager(ctx, flags):
    n = 16
    As, Bs, cA, cB = _pairs(ctx, n, 3, 10)
    eager = [o.export() for o in ctx.matmul_batch(cA, cB, [n] * 3, {"flags": flags})]
    # other operands, eager, between the replays
    _, _, oA, oB = _pairs(ctx, 8, 2, 90)
    for rep in range(4):
        got = ctx.matmul_batch(cA, cB, [n] * 3, {"flags": flags | GRAPH})
        for i in range(3):
            assert np.array_equal(got[i].export(), eager[i]), (rep, i)
        other = ctx.matmul_batch(oA, oB, [8] * 2, {"flags": BATCHED})
        ctx.decrypt(other[0], 64)
        ctx.sync()
    err = np.max(np.abs(ctx.decrypt(got[1], n * n) - (As[1] @ Bs[1]).ravel()))
    assert err < 2.0**-15


def test_several_recordings_and_trim(ctx):
    n = 8
    sets = [_pairs(ctx, n, 2, 200 + 10 * s) for s in range(5)]  # more sets than the recordings kept
    want = [[o.export() for o in ctx.matmul_batch(p[2], p[3], [n] * 2, {"flags": BATCHED | LAZY})] for p in sets]
    for rnd in range(2):
        for s, p in enumerate(sets):
            got = ctx.matmul_batch(p[2], p[3], [n] * 2, {"flags": BATCHED | LAZY | GRAPH})
            for i in range(2):
                assert np.array_equal(got[i].export(), want[s][i]), (rnd, s, i)
        ctx.trim()


def test_recording_refused_while_profiling(ctx):
    from paper_2305_17341_amd import he
    n = 8
    _, _, cA, cB = _pairs(ctx, n, 1, 300)
    ctx.profile_enable(True)
    try:
        with pytest.raises(he.HeError) as e:
            ctx.matmul_batch(cA, cB, [n], {"flags": BATCHED | GRAPH})
        assert e.value.status == -1
    finally:
        ctx.profile_enable(False)
    with pytest.raises(he.HeError):
        ctx.matmul_batch(cA, cB, [n], {"flags": GRAPH})  # must be batched


def test_replay_128_full_size(oracle_mod):
    from tests.fullcrt import FullDecryptor
    from paper_2305_17341_amd import he
    ch = I.LARGE
    n = 128
    c = he.chain_context(ch, seed=43)
    c.keygen(c.matmul_rot_steps(n))
    As, Bs, cA, cB = _pairs(c, n, 2, 700)
    flags = BATCHED | LAZY | FUSED
    eager = [o.export() for o in c.matmul_batch(cA, cB, [n] * 2, {"flags": flags})]
    for rep in range(2):
        got = c.matmul_batch(cA, cB, [n] * 2, {"flags": flags | GRAPH})
        for i in range(2):
            assert np.array_equal(got[i].export(), eager[i]), (rep, i)
    err = np.max(np.abs(FullDecryptor(oracle_mod, ch, 43).decrypt(got[0], n * n) - (As[0] @ Bs[0]).ravel()))
    print(f"recorded 128x128 product: max abs error {err:.3e}", flush=True)
    assert err < 2.0**-15
    c.close()
