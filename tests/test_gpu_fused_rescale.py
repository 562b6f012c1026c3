"""ModDown and Rescale of the A side as one rounding (HE_MM_FUSED_RESCALE, a
variant of the paper's two roundings): residue for residue equal to the
oracle's fused variant for plain and decomposed products (with and without
lazy relinearisation) and the covariance, batched equal to one-at-a-time, and
the 128 x 128 product at N = 2^16 within 2^-15 of FP64."""
import numpy as np
import pytest

from paper_2305_17341_amd import inputs as I
from paper_2305_17341_amd import packing
from oracle import packing as opacking
from tests.fullcrt import FullDecryptor

pytestmark = pytest.mark.gpu

DEEP = I.Chain("n11_deep", 11, (60,) + (40,) * 6, (60, 60))
BOUND = 2.0 ** -15
BATCHED, LAZY, FUSED = 1, 2, 4


@pytest.fixture(scope="module")
def pair(oracle_mod):
    from paper_2305_17341_amd import he
    n = 16
    ctx = he.chain_context(DEEP, seed=23)
    steps = set(ctx.transpose_rot_steps(8)) | set(ctx.matmul_rot_steps(8, {"n1_z": 2, "n1_t": 2}))
    for npz, npt in [(15, 15), (4, 4)]:
        steps |= set(ctx.matmul_rot_steps(n, {"n1_z": 4, "n1_t": 4, "nprime_z": npz, "nprime_t": npt}))
    steps = sorted(steps)
    ctx.keygen(steps)
    o = oracle_mod.Oracle(DEEP.log_n, DEEP.q_bits, DEEP.p_bits, seed=23)
    o.keygen(rot_steps=steps)
    return ctx, o


@pytest.mark.parametrize("npz,npt,lazy", [(15, 15, False), (15, 15, True), (4, 4, True)])
def test_fused_matmul_bit_exact(pair, npz, npt, lazy):
    ctx, o = pair
    n = 16
    A, B = I.uniform_matrix(31, n), I.uniform_matrix(32, n)
    flags = FUSED | (LAZY if lazy else 0)
    opts = {"n1_z": 4, "n1_t": 4, "nprime_z": npz, "nprime_t": npt, "flags": flags}
    ca, cb = ctx.encrypt_matrix(A, nonce=1), ctx.encrypt_matrix(B, nonce=2)
    r = ctx.matmul(ca, cb, n, opts)
    want = o.matmul(o.encrypt(A.ravel(), nonce=1), o.encrypt(B.ravel(), nonce=2), n, 4, 4, npz, npt, lazy=lazy,
                    fused_rescale=True)
    assert r.level == want.level and r.scale == want.scale
    assert np.array_equal(r.export(), want.data())
    assert np.max(np.abs(ctx.decrypt(r, n * n) - (A @ B).ravel())) < BOUND
    outs = ctx.matmul_batch([ca, cb, ca], [cb, ca, cb], [n] * 3, dict(opts, flags=flags | BATCHED))
    assert np.array_equal(outs[0].export(), r.export())
    assert np.array_equal(outs[2].export(), r.export())
    assert np.array_equal(outs[1].export(), ctx.matmul(cb, ca, n, opts).export())


def test_fused_covariance_bit_exact(pair):
    ctx, o = pair
    n, k, rb = 8, 2, 2
    X = I.centre(I.dataset(6, rb * n - 3, k * n - 5))
    s = X.shape[0]
    blocks = packing.blocks(X, n)
    oblocks = opacking.pack(X, n)
    g = [ctx.encrypt_matrix(blocks[r, j], nonce=200 + r * k + j) for r in range(rb) for j in range(k)]
    oc = [o.encrypt(oblocks[r, j].ravel(), nonce=200 + r * k + j) for r in range(rb) for j in range(k)]
    cov = ctx.covariance(g, rb, k, n, s, {"n1_z": 2, "n1_t": 2, "flags": LAZY | FUSED})
    want = o.covariance(oc, rb, k, n, s, 2, 2, 4, lazy=True, fused_rescale=True)
    P = np.zeros((rb * n, k * n))
    P[: X.shape[0], : X.shape[1]] = X
    ref = P.T @ P / s
    for i in range(k * k):
        assert np.array_equal(cov[i].export(), want[i].data()), i
        a, b = divmod(i, k)
        got = ctx.decrypt(cov[i], n * n).reshape(n, n)
        assert np.max(np.abs(got - ref[a * n:(a + 1) * n, b * n:(b + 1) * n])) < BOUND


def test_fused_needs_at_most_three_special_primes():
    from paper_2305_17341_amd import he
    ctx = he.Context(11, (60,) + (40,) * 6, (50, 50, 50, 50), seed=3)
    ctx.keygen(ctx.matmul_rot_steps(8, {"n1_z": 2, "n1_t": 2}))
    A = I.uniform_matrix(1, 8)
    ca = ctx.encrypt_matrix(A, nonce=1)
    with pytest.raises(he.HeError) as e:
        ctx.matmul(ca, ca, 8, {"n1_z": 2, "n1_t": 2, "flags": FUSED})
    assert e.value.status == -1


def test_fused_matmul_128_full_size(oracle_mod):
    from paper_2305_17341_amd import he
    ch = I.LARGE
    n = 128
    ctx = he.chain_context(ch, seed=37)
    ctx.keygen(ctx.matmul_rot_steps(n))
    As = [I.uniform_matrix(500 + i, n) for i in range(2)]
    Bs = [I.uniform_matrix(600 + i, n) for i in range(2)]
    cA = [ctx.encrypt_matrix(a, nonce=1 + i) for i, a in enumerate(As)]
    cB = [ctx.encrypt_matrix(b, nonce=101 + i) for i, b in enumerate(Bs)]
    outs = ctx.matmul_batch(cA, cB, [n] * 2, {"flags": LAZY | BATCHED | FUSED})
    lazy = ctx.matmul(cA[0], cB[0], n, {"flags": LAZY})
    fd = FullDecryptor(oracle_mod, ch, 37)
    for i in range(2):
        assert outs[i].level == ch.top_level - 3
        err = np.max(np.abs(fd.decrypt(outs[i], n * n) - (As[i] @ Bs[i]).ravel()))
        print(f"fused 128x128 product {i}: max abs error {err:.3e}", flush=True)
        assert err < BOUND
    # one rounding in place of two: the residues agree with rounding twice
    # almost everywhere
    assert np.mean(lazy.export() != outs[0].export()) < 1e-3
