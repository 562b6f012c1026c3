"""Batched products (HE_MM_BATCHED): stacking several independent products
into one launch sequence must give, residue for residue, the ciphertexts of
the one-product-at-a-time path, whatever the batch composition (mixed d,
more members than one multsum launch takes, a single member)."""
import numpy as np
import pytest

from paper_2305_17341_amd import inputs as I

pytestmark = pytest.mark.gpu

BATCHED = {"flags": 1}


def _encrypt_pairs(ctx, ds, seed):
    As = [I.uniform_matrix(seed + i, d) for i, d in enumerate(ds)]
    Bs = [I.uniform_matrix(seed + 500 + i, d) for i, d in enumerate(ds)]
    cA = [ctx.encrypt_matrix(a, nonce=seed + i) for i, a in enumerate(As)]
    cB = [ctx.encrypt_matrix(b, nonce=seed + 900 + i) for i, b in enumerate(Bs)]
    return As, Bs, cA, cB


@pytest.fixture(scope="module")
def small_ctx():
    from paper_2305_17341_amd import he
    ctx = he.chain_context(I.SMALL, seed=3)
    ctx.keygen(sorted(set(ctx.matmul_rot_steps(16)) | set(ctx.matmul_rot_steps(8))))
    return ctx


def test_batched_equals_plain_mixed_d(small_ctx):
    # runs of equal d: [16 x 3], [8], [16 x 10] -> batches 3, 1, 8, 2
    ds = [16] * 3 + [8] + [16] * 10
    As, Bs, cA, cB = _encrypt_pairs(small_ctx, ds, 40)
    plain = small_ctx.matmul_batch(cA, cB, ds)
    fused = small_ctx.matmul_batch(cA, cB, ds, opts=BATCHED)
    for i, (p, f) in enumerate(zip(plain, fused)):
        assert p.level == f.level
        assert np.array_equal(p.export(), f.export()), f"member {i} (d={ds[i]})"
    for a, b, f, d in zip(As, Bs, fused, ds):
        err = np.max(np.abs(small_ctx.decrypt(f, d * d) - (a @ b).ravel()))
        assert err < 2.0**-15, err


def test_batched_dcd_equals_plain():
    # decomposed sigma/tau (n' = 4) at N = 2^14: the chains of factors run batched too
    from paper_2305_17341_amd import he
    ctx = he.chain_context(I.MID, seed=5)
    opts = {"nprime_z": 4, "nprime_t": 4}
    ctx.keygen(ctx.matmul_rot_steps(16, opts))
    ds = [16] * 3
    As, Bs, cA, cB = _encrypt_pairs(ctx, ds, 60)
    plain = ctx.matmul_batch(cA, cB, ds, opts=opts)
    fused = ctx.matmul_batch(cA, cB, ds, opts=dict(opts, **BATCHED))
    for i, (p, f) in enumerate(zip(plain, fused)):
        assert np.array_equal(p.export(), f.export()), f"member {i}"
        err = np.max(np.abs(ctx.decrypt(f, 256) - (As[i] @ Bs[i]).ravel()))
        assert err < 2.0**-15, err


@pytest.fixture(scope="module")
def large_ctx():
    from paper_2305_17341_amd import he
    ctx = he.chain_context(I.LARGE, seed=31)
    ctx.keygen(ctx.matmul_rot_steps(128))
    return ctx


def test_batched_equals_plain_large_d128(large_ctx):
    ds = [128] * 3
    As, Bs, cA, cB = _encrypt_pairs(large_ctx, ds, 70)
    fused = large_ctx.matmul_batch(cA, cB, ds, opts=BATCHED)
    for i in range(len(ds)):
        p = large_ctx.matmul(cA[i], cB[i], 128)
        assert np.array_equal(p.export(), fused[i].export()), f"member {i}"
        err = np.max(np.abs(large_ctx.decrypt(fused[i], 128 * 128) - (As[i] @ Bs[i]).ravel()))
        assert err < 2.0**-15, err


def test_knobs_never_change_residues(small_ctx):
    """Every launch-shape knob value (members and rotations per launch, the
    limb visiting order of the NTT block passes and of the multiply-sums,
    rotations per work-group, with a ragged last group; the 60-bit limbs of
    the multi-rotation launch inline or in their own kernel, four or eight
    members a pass; ModDown's lift by int8 matrix products or by FP64
    products, its work-groups in launch order or grouped by XCD; one, two or
    four term streams per thread of the multi-output sums; the A side's two
    masked multi-rotation launches as one or two) gives the residues of the
    default shape."""
    from paper_2305_17341_amd import he
    ds = [16] * 5
    _, _, cA, cB = _encrypt_pairs(small_ctx, ds, 80)
    opts = {"flags": 1 | 2}
    ref = [c.export() for c in small_ctx.matmul_batch(cA, cB, ds, opts=opts)]
    names = ("ms_members", "mr_members", "mr_rotations", "ntt_interleave", "ew_interleave", "mr_group", "mr_int_split",
             "mr_int_pass", "mr_int_chunk", "mr_int_concurrent", "fbc_mfma", "xcd_map", "sum_streams", "mr_pair")
    saved = {n: he.knob_get(n) for n in names}
    try:
        for name, value in [("ms_members", 3), ("mr_members", 2), ("mr_rotations", 5),
                            ("ntt_interleave", 0), ("ew_interleave", 0), ("mr_group", 2), ("mr_group", 1),
                            ("mr_int_split", 0), ("mr_int_split", 1), ("mr_int_pass", 8), ("mr_int_chunk", 3),
                            ("mr_int_chunk", 1), ("mr_int_concurrent", 0), ("mr_int_concurrent", 1),
                            ("fbc_mfma", 0), ("fbc_mfma", 1), ("xcd_map", 0), ("xcd_map", 1),
                            ("sum_streams", 1), ("sum_streams", 2), ("sum_streams", 4),
                            ("mr_pair", 0), ("mr_pair", 1)]:
            he.knob_set(name, value)
            got = small_ctx.matmul_batch(cA, cB, ds, opts=opts)
            for i, g in enumerate(got):
                assert np.array_equal(g.export(), ref[i]), (name, value, i)
        with pytest.raises(he.HeError):
            he.knob_set("ntt_interleave", 2)
    finally:
        for n, v in saved.items():
            he.knob_set(n, v)
