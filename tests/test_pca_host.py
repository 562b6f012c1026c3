"""Host planning of the PCA driver: the Newton schedule of the library's
driver equals the oracle's Lazy Normalization simulation (written apart
from it) and the replication layout round-trips."""
import numpy as np
import pytest

from oracle import power as P
from paper_2305_17341_amd import pca


@pytest.mark.parametrize("l_p", [1, 2, 4, 7, 14, 20])
def test_schedule_matches_oracle_simulation(l_p):
    assert pca.lazy_schedule(l_p) == P.lazy_schedule(l_p)


def test_schedule_other_bounds():
    for S, e in [(0.25, 1e-4), (0.8, 1e-6)]:
        assert pca.lazy_schedule(6, S=S, e=e) == P.lazy_schedule(6, S=S, e=e)


def test_replication_layout():
    v = np.arange(32.0)
    for axis in (0, 1):
        a = pca.replicate(v, 2, 16, axis)
        b = P.replicate(v, 2, 16, axis)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
        assert np.array_equal(P.unreplicate(a, axis), v)


def test_r2_score_matches_scikit_learn():
    from sklearn.metrics import r2_score as sk_r2
    g = np.random.default_rng(4)
    y = g.standard_normal((50, 7)) * np.arange(1, 8)
    yp = y + 0.3 * g.standard_normal((50, 7))
    assert abs(pca.r2_score(y, yp) - sk_r2(y, yp)) < 1e-12
    assert abs(pca.r2_score(y[:, 2], yp[:, 2]) - sk_r2(y[:, 2], yp[:, 2])) < 1e-12


def test_r2_x_limits_and_r2_v_sign():
    g = np.random.default_rng(5)
    X = g.uniform(0, 1, size=(80, 12)) @ g.standard_normal((12, 12))
    w, U = np.linalg.eigh(np.cov(X, rowvar=False, bias=True))
    U = U[:, ::-1]
    assert abs(pca.r2_x(X, U) - 1.0) < 1e-12             # every component: exact reconstruction
    assert abs(pca.r2_x(X, U[:, :0])) < 1e-12              # none: the column means
    r = [pca.r2_x(X, U[:, :m]) for m in range(1, 12)]
    assert all(a < b + 1e-12 for a, b in zip(r, r[1:]))
    flipped = U[:, :4] * np.array([1, -1, -1, 1])
    assert abs(pca.r2_v(U[:, :4], flipped) - 1.0) < 1e-12
    assert pca.r2_v(U[:, :4], U[:, 1:5]) < 0.5


def test_fp64_replay_follows_the_oracle_rounds():
    """pca.fp64_replay takes the oracle's round definition step by
    step (same start vectors, Newton counts, eigen-shift), and on a planted,
    well separated spectrum approaches numpy's eigenpairs"""
    from paper_2305_17341_amd import inputs as I
    X = I.pca_dataset(3, 300, 64)
    cov = np.cov(X, rowvar=False, bias=True)
    l_e, l_p = 3, 14
    lam, V = pca.fp64_replay(cov, l_e, l_p, seed=11)
    taus, x0 = P.lazy_schedule(l_p), 2.0 ** 15 + 1
    g = np.random.default_rng(11)
    shifted = cov.copy()
    for m in range(l_e):
        v = g.standard_normal(64)
        v /= np.linalg.norm(v)
        for tau in taus:
            v, _ = P.fp64_round(shifted, v, tau, x0, False)
        _, lf = P.fp64_round(shifted, v, 0, x0, True)
        assert np.max(np.abs(V[:, m] - v)) < 1e-12 and abs(lam[m] - lf) < 1e-12
        shifted = shifted - lf * np.outer(v, v)
    w, U = np.linalg.eigh(cov)
    assert np.max(np.abs(lam - w[::-1][:l_e]) / w[::-1][:l_e]) < 1e-2
    assert pca.r2_v(U[:, ::-1][:, :l_e], V) > 0.95
