"""The depth-2 product with C^k's masks folded into Z (oracle plan, the
short-chain variant of the product): its permutations satisfy Jiang's
identity, and on the small workload's literal chain (q0 + two 40-bit primes:
two rescales) the product decrypts to A B within 2^-15, using only Z's, T's
and the row shifts' keys."""
import numpy as np
import pytest

from paper_2305_17341_amd import inputs as I

LITERAL_SMALL = I.Chain("n13_literal", 13, (60, 40, 40), (60,))
BOUND = 2.0 ** -15


def _steps(n, n1):
    s = set(range(1, n1))
    lo, hi = -((n - 1 + n1 - 1) // n1), (n - 1) // n1
    s |= {n1 * i for i in range(lo, hi + 1) if i}            # Z (folded A side)
    s |= {n * j for j in range(1, n1)} | {n * n1 * i for i in range(1, (n - 1) // n1 + 1)}   # T, row shifts
    return sorted(s)


@pytest.mark.parametrize("n", [4, 8, 16])
def test_folded_permutations_satisfy_jiang_identity(oracle_mod, n):
    rng = np.random.default_rng(n)
    A, B = rng.uniform(-1, 1, (n, n)), rng.uniform(-1, 1, (n, n))
    tauB = B.ravel()[oracle_mod.perm("tau", n)]
    acc = np.zeros(n * n)
    for k in range(n):
        Ak = A.ravel()[oracle_mod.perm_phi_sigma(n, k)]
        Bk = np.roll(tauB.reshape(n, n), -k, axis=0).ravel()     # psi^k: rows shifted up by k
        acc += Ak * Bk
    assert np.allclose(acc, (A @ B).ravel(), atol=1e-12)
    # k = 0 is Z itself
    assert np.array_equal(oracle_mod.perm_phi_sigma(n, 0), oracle_mod.perm("sigma", n))


@pytest.mark.parametrize("lazy", [False, True])
def test_folded_product_two_levels_on_the_literal_small_chain(oracle_mod, lazy):
    ch = LITERAL_SMALL
    n, n1 = 16, 4
    o = oracle_mod.Oracle(ch.log_n, ch.q_bits, ch.p_bits, seed=13)
    o.keygen(rot_steps=_steps(n, n1))
    A, B = I.uniform_matrix(1, n), I.uniform_matrix(2, n)
    r = o.matmul(o.encrypt(A.ravel(), nonce=1), o.encrypt(B.ravel(), nonce=2), n, n1, n1, lazy=lazy, folded=True)
    assert r.level == ch.top_level - 2 == 0
    err = np.max(np.abs(o.decrypt(r, n * n) - (A @ B).ravel()))
    assert err < BOUND, err


def test_folded_product_rejects_decomposition_and_one_rounding(oracle_mod):
    ch = LITERAL_SMALL
    o = oracle_mod.Oracle(ch.log_n, ch.q_bits, ch.p_bits, seed=13)
    o.keygen(rot_steps=_steps(16, 4))
    a = o.encrypt(I.uniform_matrix(1, 16).ravel(), nonce=1)
    with pytest.raises(RuntimeError):
        o.matmul(a, a, 16, 4, 4, npz=4, folded=True)
    with pytest.raises(RuntimeError):
        o.matmul(a, a, 16, 4, 4, fused_rescale=True, folded=True)
