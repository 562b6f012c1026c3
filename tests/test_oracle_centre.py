"""Pins of the homomorphic mean and of the covariance of a dataset that is not
centred (oracle/centre.py): decrypted means against the FP64 column means,
decrypted blocks against the FP64 population covariance, for a ragged
dataset (padded rows and feature columns)."""
import numpy as np
import pytest

from paper_2305_17341_amd import inputs as I
from oracle import packing as opacking

BOUND = 2.0 ** -15
CHAIN = (11, (60,) + (40,) * 7, (60, 60))


@pytest.fixture(scope="module")
def setup(oracle_mod):
    log_n, qb, pb = CHAIN
    o = oracle_mod.Oracle(log_n, qb, pb, seed=17)
    n = 8
    o.keygen(rot_steps=sorted({s for s in range(-n * n + 1, n * n) if s}), relin=True)
    return o, n


def test_means_and_uncentred_covariance(setup):
    from oracle import centre
    o, n = setup
    k, rb = 2, 2
    X = I.dataset(8, rb * n - 3, k * n - 5)          # values in [0, 1], not centred
    s, t = X.shape
    blk = opacking.pack(X, n)
    cts = [o.encrypt(blk[r, j].ravel(), nonce=40 + r * k + j) for r in range(rb) for j in range(k)]
    hc = centre.HeCentre(o, n)
    mu_want, cov_want = centre.fp64_mean_and_cov(X)
    mu = hc.means(cts, rb, k, s)
    got_mu = np.concatenate([o.decrypt(m)[: n * n].reshape(n, n)[0] for m in mu])[:t]
    assert np.max(np.abs(got_mu - mu_want)) < BOUND
    for m in mu:   # every row holds the means
        M = o.decrypt(m)[: n * n].reshape(n, n)
        assert np.max(np.abs(M - M[0])) < BOUND
    cov = hc.covariance(cts, rb, k, s, 4, 4, 4, lazy=True)
    full = np.zeros((k * n, k * n))
    full[:t, :t] = cov_want
    for i in range(k * k):
        a, b = divmod(i, k)
        got = o.decrypt(cov[i])[: n * n].reshape(n, n)
        assert np.max(np.abs(got - full[a * n:(a + 1) * n, b * n:(b + 1) * n])) < BOUND, i
    # the centred covariance is not X^T X / s: the mean path matters here
    assert np.max(np.abs(X.T @ X / s - cov_want)) > 0.1


def test_padding_method_2_packs_and_unpacks():
    """Method 2 (section 5.1): n - p valid features per block,
    p = floor((k n - t) / k); every feature lands once and comes back."""
    n = 8
    for t in (11, 13, 16, 17, 23):
        X = I.dataset(t, 5, t)
        k = -(-t // n)
        w = opacking.width(t, n, 2)
        assert w == n - (k * n - t) // k and k * w >= t and w <= n
        B = opacking.pack(X, n, method=2)
        assert B.shape == (1, k, n, n)
        back = np.concatenate([B[0, j, :5, :w] for j in range(k)], axis=1)[:, :t]
        assert np.array_equal(back, X)
        M = I.dataset(t + 100, t, t)
        Bm = [[np.zeros((n, n)) for _ in range(k)] for _ in range(k)]
        for f in range(t):
            for g in range(t):
                Bm[f // w][g // w][f % w, g % w] = M[f, g]
        assert np.array_equal(opacking.unpack_square(Bm, t, n, 2), M)


def test_uncentred_covariance_padding_method_2(setup):
    """The covariance circuit is unchanged by the packing: with method 2 the
    decrypted blocks, unpacked, give the FP64 covariance."""
    from oracle import centre
    o, n = setup
    X = I.dataset(10, 2 * n - 3, 13)
    s, t = X.shape
    k, rb = -(-t // n), 2
    blk = opacking.pack(X, n, method=2)
    cts = [o.encrypt(blk[r, j].ravel(), nonce=80 + r * k + j) for r in range(rb) for j in range(k)]
    cov = centre.HeCentre(o, n).covariance(cts, rb, k, s, 4, 4, 4, lazy=True)
    B = [[o.decrypt(cov[a * k + b])[: n * n].reshape(n, n) for b in range(k)] for a in range(k)]
    got = opacking.unpack_square(B, t, n, method=2)
    _, want = centre.fp64_mean_and_cov(X)
    assert np.max(np.abs(got - want)) < BOUND


def test_package_packing_equals_the_oracles():
    """The library's client-side packing and the oracle's own give the same
    blocks and the same unpacking, for both padding methods."""
    from paper_2305_17341_amd import packing
    for n in (4, 8):
        for s, t in ((5, 13), (17, 16), (9, 23), (8, 8), (3, 31)):
            X = I.dataset(s * 100 + t, s, t)
            for method in (1, 2):
                assert packing.features_per_block(t, n, method) == opacking.width(t, n, method)
                assert np.array_equal(packing.blocks(X, n, method), opacking.pack(X, n, method))
                k = -(-t // n)
                B = I.rng(t).uniform(-1, 1, (k, k, n, n))
                assert np.array_equal(packing.unblock_square(B, t, n, method),
                                      opacking.unpack_square(B, t, n, method))
