"""Row blocks of the covariance stacked into batches ("cov_row_blocks"): the
residues do not depend on how many row blocks share a batch (the sums over
row blocks are exact), with a ragged last batch, for lazy and per-product
relinearisation."""
import numpy as np
import pytest

from paper_2305_17341_amd import inputs as I
from paper_2305_17341_amd import packing

pytestmark = pytest.mark.gpu

DEEP = I.Chain("n11_deep", 11, (60,) + (40,) * 6, (60, 60))


@pytest.mark.parametrize("flags", [0, 2])
def test_covariance_row_block_batches_keep_residues(flags):
    from paper_2305_17341_amd import he
    n, k, rb = 8, 2, 5
    ctx = he.chain_context(DEEP, seed=61)
    ctx.keygen(sorted(set(ctx.matmul_rot_steps(n, {"n1_z": 2, "n1_t": 2})) | set(ctx.transpose_rot_steps(n))))
    X = I.centre(I.dataset(21, rb * n - 3, k * n - 5))
    blocks = packing.blocks(X, n)
    cts = [ctx.encrypt_matrix(blocks[r, c], nonce=100 + r * k + c) for r in range(rb) for c in range(k)]
    ref = None
    old = he.knob_get("cov_row_blocks")
    try:
        for g in (1, 2, 4, 8):
            he.knob_set("cov_row_blocks", g)
            cov = ctx.covariance(cts, rb, k, n, X.shape[0], {"n1_z": 2, "n1_t": 2, "flags": flags})
            got = [c.export() for c in cov]
            if ref is None:
                ref = got
                P = np.zeros((rb * n, k * n))
                P[: X.shape[0], : X.shape[1]] = X
                want = P.T @ P / X.shape[0]
                for i, c in enumerate(cov):
                    a, b = divmod(i, k)
                    dec = ctx.decrypt(c, n * n).reshape(n, n)
                    assert np.max(np.abs(dec - want[a * n:(a + 1) * n, b * n:(b + 1) * n])) < 2.0 ** -15
            else:
                for x, y in zip(ref, got):
                    assert np.array_equal(x, y), g
    finally:
        he.knob_set("cov_row_blocks", old)


@pytest.mark.parametrize("flags", [0, 2 | 4])
def test_covariance_in_parts_equals_whole(flags):
    """he_covariance_begin/add/end over row blocks split 2 + 1 + 2 (and a
    second dataset through the same state after end) gives he_covariance's
    residues; an uncentred request and a level mismatch are refused."""
    from paper_2305_17341_amd import he
    n, k, rb = 8, 2, 5
    ctx = he.chain_context(DEEP, seed=62)
    geo = {"n1_z": 2, "n1_t": 2, "flags": flags}
    ctx.keygen(sorted(set(ctx.matmul_rot_steps(n, geo)) | set(ctx.transpose_rot_steps(n))))
    for seed in (23, 24):
        X = I.centre(I.dataset(seed, rb * n - 3, k * n - 5))
        blocks = packing.blocks(X, n)
        cts = [ctx.encrypt_matrix(blocks[r, c], nonce=seed * 100 + r * k + c) for r in range(rb) for c in range(k)]
        whole = [c.export() for c in ctx.covariance(cts, rb, k, n, X.shape[0], geo)]
        if seed == 23:
            st = ctx.covariance_begin(k, n, X.shape[0], geo)
        r0 = 0
        for part in (2, 1, 2):
            st.add(cts[r0 * k:(r0 + part) * k], part)
            r0 += part
        parts = st.end()
        for x, y in zip(whole, parts):
            assert np.array_equal(x, y.export())
    # a block one level down does not join the state's level
    st.add(cts[:k], 1)
    low = [ctx.drop(c, cts[0].level - 1) for c in cts[k:2 * k]]
    with pytest.raises(he.HeError):
        st.add(low, 1)
    st.free()
    with pytest.raises(he.HeError):
        ctx.covariance_begin(k, n, 10, {"flags": 16})
