"""Pins of the PowerMethod oracle (section 6.1 and Appendix B): the Lazy
Normalization schedule against the averages printed in section 7, Newton's
monotone convergence from below, Aggregate and AxisFlipping against plain
row/column sums, whole rounds and the eigen-shift against an FP64 replay,
and the eigenvalue bound lambda <= lambda_1."""
import numpy as np
import pytest

from oracle import power as P
from paper_2305_17341_amd import inputs as I

N_BLK, K = 16, 2
X0 = 2.0 ** 15 + 1   # Taylor point B^2/2 + 1 with B^2 = 2^16


def test_lazy_schedule_reproduces_printed_averages():
    # section 7 (vector normalisation): S = 0.5, e = 1e-5, precision 1e-3,
    # linear Taylor at 2^16/2 + 1: on average 14.5 Newton steps for l_P = 4
    # and 13.8 for l_P = 14
    t4 = P.lazy_schedule(4)
    t14 = P.lazy_schedule(14)
    assert np.mean(t4) == 14.5
    assert round(float(np.mean(t14)), 1) == 13.8
    assert len(t4) == 4 and len(t14) == 14


@pytest.mark.parametrize("x", [1e-3, 0.3, 1.0, 7.0, 300.0, 2.0 ** 12, 2.0 ** 16])
def test_newton_increases_towards_inverse_sqrt_from_below(x):
    # Theorem on the iterative InvSRT (statement read as y_{i-1} <= y_i <= x^-1/2)
    y = P.taylor1(x, X0)
    target = x ** -0.5
    assert 0 < y <= target
    for _ in range(60):
        y2 = P.newton(y, x, 1)
        assert y * (1 - 1e-14) <= y2 <= target * (1 + 1e-12)   # monotone up to the last ulp
        y = y2
    if x >= 1.0:
        assert abs(y - target) < 1e-9 * target


def test_newton_order1_taylor_is_tangent():
    # T(x0) = x0^-1/2 and T'(x0) = -x0^-3/2 / 2
    h = 1e-3
    assert P.taylor1(X0, X0) == pytest.approx(X0 ** -0.5, rel=1e-14)
    slope = (P.taylor1(X0 + h, X0) - P.taylor1(X0 - h, X0)) / (2 * h)
    assert slope == pytest.approx(-0.5 * X0 ** -1.5, rel=1e-6)


@pytest.fixture(scope="module")
def ctx(oracle_mod):
    o = oracle_mod.Oracle(11, (60,) + (40,) * 10, (60, 60), seed=3)
    n = N_BLK
    steps = sorted({n << j for j in range(4)} | {1 << j for j in range(4)} | {-(1 << j) for j in range(4)})
    o.keygen(rot_steps=steps)
    return o


def _dec(o, box, n=N_BLK):
    return o.decrypt(box.ct, n * n).reshape(n, n)


def test_aggregate_both_axes(ctx):
    o, n = ctx, N_BLK
    hp = P.HePower(o, n)
    A = I.uniform_matrix(5, n)
    ct = P.Box(o.encrypt(A.ravel(), nonce=1))
    col = _dec(o, P.Box(hp.aggregate(ct, 0)))
    row = _dec(o, P.Box(hp.aggregate(ct, 1)))
    assert np.max(np.abs(col - np.tile(A.sum(axis=0), (n, 1)))) < 1e-6
    assert np.max(np.abs(row - np.tile(A.sum(axis=1)[:, None], (1, n)))) < 1e-6


def test_axis_flipping(ctx):
    o, n = ctx, N_BLK
    hp = P.HePower(o, n)
    v = I.uniform_matrix(6, n)[0]
    for axis in (0, 1):
        V = P.Box(o.encrypt(P.replicate(v, 1, n, axis)[0].ravel(), nonce=2 + axis))
        F = _dec(o, P.Box(hp.axis_flip(V, axis)))
        assert np.max(np.abs(F - P.replicate(v, 1, n, 1 - axis)[0])) < 1e-6


def _planted_cov(seed, t, top=8.0):
    X = I.centre(I.planted_dataset(seed, 64, t))
    cov = X.T @ X / X.shape[0]
    return cov * (top / np.linalg.eigvalsh(cov)[-1])


def test_rounds_eigenvalue_and_shift_match_fp64_replay(ctx):
    o, n, k = ctx, N_BLK, K
    cov = _planted_cov(7, n * k)
    hp = P.HePower(o, n)
    C = [P.Box(o.encrypt(cov[r * n:(r + 1) * n, c * n:(c + 1) * n].ravel(), nonce=100 + r * k + c))
         for r in range(k) for c in range(k)]
    v = np.random.default_rng(1).standard_normal(n * k)
    v /= np.linalg.norm(v)
    axis = 1
    V = [P.Box(o.encrypt(b.ravel(), nonce=200 + i)) for i, b in enumerate(P.replicate(v, k, n, axis))]
    vf = v.copy()
    taus = P.lazy_schedule(4)
    for tau in taus:
        V, axis = hp.step(C, k, V, axis, tau, X0, False)
        vf, _ = P.fp64_round(cov, vf, tau, X0, False)
        got = P.unreplicate([_dec(o, b) for b in V], axis)
        assert np.max(np.abs(got - vf)) < 2.0 ** -15
    assert hp.refreshes > 0
    assert abs(np.linalg.norm(vf) - 1) < 1e-5          # the last round normalises (error bound e)
    V, axis, lam, VT = hp.step(C, k, V, axis, 0, X0, True)
    _, lf = P.fp64_round(cov, vf, 0, X0, True)
    lam_he = o.decrypt(lam.ct, n * n)
    assert np.max(np.abs(lam_he - lf)) < 2.0 ** -15 * max(1.0, abs(lf))
    assert lf <= np.linalg.eigvalsh(cov)[-1] + 1e-12    # Appendix B: lambda <= lambda_1
    vt = P.unreplicate([_dec(o, b) for b in VT], 1 - axis)
    assert np.max(np.abs(vt - vf)) < 2.0 ** -15
    S = hp.eigen_shift(C, k, lam, V, VT, axis)
    ref = cov - lf * np.outer(vf, vf)
    for r in range(k):
        for c in range(k):
            blk = _dec(o, S[r * k + c])
            assert np.max(np.abs(blk - ref[r * n:(r + 1) * n, c * n:(c + 1) * n])) < 2.0 ** -15


@pytest.mark.parametrize("x", [1e-3, 0.3, 1.0, 7.0, 300.0, 2.0 ** 12, 2.0 ** 16])
def test_goldschmidt_iterates_equal_newtons(x):
    # the equivalence the paper proves for the two iterations: 2 h_i = y_i
    y0 = P.taylor1(x, X0)
    for tau in range(0, 40, 3):
        a, b = P.goldschmidt(y0, x, tau), P.newton(y0, x, tau)
        assert abs(a - b) <= 1e-12 * abs(b), (x, tau)


def test_goldschmidt_circuit_two_levels_per_step(ctx):
    """the encrypted Goldschmidt form decrypts to half of Newton's iterate
    and takes 2 tau + 2 levels (Newton's form: 3 tau + 1)"""
    o, n = ctx, N_BLK
    hp = P.HePower(o, n)
    x = np.linspace(1.0, 2.0 ** 16, n * n)
    X = P.Box(o.encrypt(x, nonce=9))
    for tau in (0, 1, 3):
        H = hp.goldschmidt_half(X, X0, tau)
        want = 0.5 * np.array([P.newton(P.taylor1(v, X0), v, tau) for v in x])
        got = o.decrypt(H.ct, n * n)
        assert np.max(np.abs(got - want) / want) < 1e-4, tau
        assert H.ct.level == o.L - (1 if tau == 0 else 2 * tau + 2)
        Y = hp.newton(X, P.Box(hp.taylor(X, X0)), tau)
        assert Y.ct.level == o.L - (3 * tau + 1)
    assert hp.refreshes == 0


def test_goldschmidt_rounds_match_fp64_replay(ctx):
    o, n, k = ctx, N_BLK, K
    cov = _planted_cov(7, n * k)
    hp = P.HePower(o, n, nonce0=1 << 41)
    C = [P.Box(o.encrypt(cov[r * n:(r + 1) * n, c * n:(c + 1) * n].ravel(), nonce=300 + r * k + c))
         for r in range(k) for c in range(k)]
    v = np.random.default_rng(2).standard_normal(n * k)
    v /= np.linalg.norm(v)
    axis = 1
    V = [P.Box(o.encrypt(b.ravel(), nonce=400 + i)) for i, b in enumerate(P.replicate(v, k, n, axis))]
    vf = v.copy()
    for tau in P.lazy_schedule(4):
        V, axis = hp.step(C, k, V, axis, tau, X0, False, goldschmidt=True)
        vf, _ = P.fp64_round(cov, vf, tau, X0, False)
        got = P.unreplicate([_dec(o, b) for b in V], axis)
        assert np.max(np.abs(got - vf)) < 2.0 ** -15


@pytest.mark.parametrize("axis", [0, 1])
def test_pack_then_unpack_restores_blocks(ctx, axis):
    """Appendix C's single-ciphertext refresh of a vector: packed (one
    level), refreshed once, unpacked (one level), the k blocks come back
    replicated in the same form"""
    o, n, k = ctx, N_BLK, K
    hp = P.HePower(o, n, nonce0=1 << 43)
    v = np.random.default_rng(6).standard_normal(n * k)
    reps = P.replicate(v, k, n, axis)
    V = [P.Box(o.encrypt(b.ravel(), level=2, nonce=500 + i)) for i, b in enumerate(reps)]
    Pk = hp.pack(V, axis)
    assert Pk.level == 1
    U = hp.unpack(hp.refresh(Pk), axis, k)
    assert hp.refreshes == 1
    for i in range(k):
        assert U[i].ct.level == o.L - 1
        assert np.max(np.abs(_dec(o, U[i]) - reps[i])) < 2.0 ** -15


def test_pack_refresh_rounds_match_fp64_replay(ctx):
    o, n, k = ctx, N_BLK, K
    cov = _planted_cov(7, n * k)
    for pack in (False, True):
        hp = P.HePower(o, n, nonce0=1 << 44)
        C = [P.Box(o.encrypt(cov[r * n:(r + 1) * n, c * n:(c + 1) * n].ravel(), nonce=600 + r * k + c))
             for r in range(k) for c in range(k)]
        v = np.random.default_rng(3).standard_normal(n * k)
        v /= np.linalg.norm(v)
        axis = 1
        V = [P.Box(o.encrypt(b.ravel(), nonce=700 + i)) for i, b in enumerate(P.replicate(v, k, n, axis))]
        vf = v.copy()
        for tau in [2, 3, 2, 3, 2]:
            V, axis = hp.step(C, k, V, axis, tau, X0, False, pack=pack)
            vf, _ = P.fp64_round(cov, vf, tau, X0, False)
            got = P.unreplicate([_dec(o, b) for b in V], axis)
            assert np.max(np.abs(got - vf)) < 2.0 ** -15
        assert (hp.packs > 0) == pack
