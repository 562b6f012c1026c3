"""Pins of the CPU oracle against what the mathematics and the paper fix.

Each check is independent of the oracle's own code path: schoolbook products
instead of its NTT, direct evaluation instead of butterflies, big-integer CRT
and division instead of its RNS formulas, a Lucas certificate instead of its
Miller-Rabin, numpy's Philox instead of its Philox, closed forms of the
canonical embedding instead of its FFT encoder.
"""
import math
import random

import numpy as np
import pytest

from oracle import t0
from paper_2305_17341_amd import inputs as I


@pytest.fixture(scope="module")
def toy(oracle_mod):
    o = oracle_mod.Oracle(I.TOY.log_n, I.TOY.q_bits, I.TOY.p_bits, seed=7)
    o.keygen(rot_steps=[1, 2, 3, -1, 5, 16, -16, 100], relin=True)
    return o


@pytest.fixture(scope="module")
def tiny(oracle_mod):
    # N = 16: small enough for schoolbook products and O(N^2) evaluation
    return oracle_mod.Oracle(4, (60, 40, 40), (60,), seed=3)


# ----------------------------------------------------------------- parameters
@pytest.mark.parametrize("chain", [I.TOY, I.SMALL, I.MID, I.LARGE])
def test_primes_are_ntt_friendly_distinct_and_proven(oracle_mod, chain):
    o = oracle_mod.Oracle(chain.log_n, chain.q_bits, chain.p_bits)
    twoN = 2 * chain.N
    bits = list(chain.q_bits) + list(chain.p_bits)
    assert len(set(o.moduli)) == len(o.moduli)
    for q, b in zip(o.moduli, bits):
        assert q % twoN == 1
        assert q.bit_length() == b
        assert t0.proven_prime(q)
    # Q primes of one size are the largest ones, in descending order
    by_size = {}
    for q, b in zip(o.moduli, bits):
        by_size.setdefault(b, []).append(q)
    for b, qs in by_size.items():
        assert qs == sorted(qs, reverse=True)
        top = max(qs)
        # no NTT-friendly prime was skipped above the largest
        cand = top + twoN
        while cand < (1 << b):
            assert not t0.proven_prime(cand)
            cand += twoN


def test_psi_is_primitive_2n_th_root(oracle_mod):
    o = oracle_mod.Oracle(I.SMALL.log_n, I.SMALL.q_bits, I.SMALL.p_bits)
    N = o.N
    for m, q in enumerate(o.moduli):
        psi = o.psi(m)
        assert pow(psi, 2 * N, q) == 1
        assert pow(psi, N, q) == q - 1


# ----------------------------------------------------------------- NTT
def test_ntt_matches_direct_evaluation(tiny):
    rnd = random.Random(1)
    for m, q in enumerate(tiny.moduli):
        a = [rnd.randrange(q) for _ in range(tiny.N)]
        want = t0.ntt_by_evaluation(a, tiny.psi(m), q, tiny.log_n)
        got = [int(x) for x in tiny.ntt(m, np.array(a, dtype=np.uint64))]
        assert got == want
        assert [int(x) for x in tiny.ntt_direct(m, np.array(a, dtype=np.uint64))] == want


@pytest.mark.parametrize("log_n", [4, 6, 8])
def test_ntt_product_is_schoolbook_negacyclic(oracle_mod, log_n):
    o = oracle_mod.Oracle(log_n, (60, 40), (60,), seed=1)
    rnd = random.Random(log_n)
    for m, q in enumerate(o.moduli):
        a = [rnd.randrange(q) for _ in range(o.N)]
        b = [rnd.randrange(q) for _ in range(o.N)]
        A = o.ntt(m, np.array(a, dtype=np.uint64))
        B = o.ntt(m, np.array(b, dtype=np.uint64))
        prod = np.array([(int(x) * int(y)) % q for x, y in zip(A, B)], dtype=np.uint64)
        got = [int(x) for x in o.intt(m, prod)]
        assert got == t0.negacyclic_mul(a, b, q)


def test_intt_inverts_ntt_full_size(oracle_mod):
    o = oracle_mod.Oracle(I.SMALL.log_n, I.SMALL.q_bits, I.SMALL.p_bits)
    g = np.random.default_rng(0)
    for m, q in enumerate(o.moduli):
        a = (g.integers(0, 2**63, o.N, dtype=np.uint64) % np.uint64(q)).astype(np.uint64)
        assert np.array_equal(o.intt(m, o.ntt(m, a)), a)


# ----------------------------------------------------------------- automorphism
def test_automorphism_ntt_equals_signed_coefficient_map(tiny):
    rnd = random.Random(5)
    for m, q in enumerate(tiny.moduli):
        a = [rnd.randrange(q) for _ in range(tiny.N)]
        A = tiny.ntt(m, np.array(a, dtype=np.uint64))
        for g in (5, 25, 2 * tiny.N - 1, 3, 7):
            want = t0.automorph_coef(a, g, q)
            got = [int(x) for x in tiny.intt(m, tiny.automorph_ntt(g, A))]
            assert got == want
            assert [int(x) for x in tiny.automorph_coef(m, g, np.array(a, dtype=np.uint64))] == want


def test_automorphism_composition(toy):
    g = np.random.default_rng(3)
    a = g.integers(0, toy.q[1], toy.N, dtype=np.uint64)
    twoN = 2 * toy.N
    for g1, g2 in ((5, 25), (toy.galois(7), toy.galois(-3)), (5, twoN - 1)):
        lhs = toy.automorph_ntt(g1, toy.automorph_ntt(g2, a))
        rhs = toy.automorph_ntt((g1 * g2) % twoN, a)
        assert np.array_equal(lhs, rhs)


def test_galois_of_step(toy):
    S = toy.slots
    assert toy.galois(0) == 1
    assert toy.galois(1) == 5
    assert toy.galois(-1) == pow(5, S - 1, 2 * toy.N)
    assert toy.galois(S + 3) == toy.galois(3)


# ----------------------------------------------------------------- randomness
def test_philox_matches_numpy(oracle_mod):
    for key, ctr in (((0, 0), (0, 0, 0, 0)), ((5, 7), (10, 20, 30, 40)),
                     ((2**64 - 1, 12345), (2**64 - 1, 2**64 - 1, 3, 9))):
        bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                              counter=np.array(ctr, dtype=np.uint64))
        want = [int(x) for x in bg.random_raw(4)]
        # numpy advances the counter once before its first block
        v = sum(int(x) << (64 * i) for i, x in enumerate(ctr)) + 1
        c = [(v >> (64 * i)) % 2**64 for i in range(4)]
        assert oracle_mod.philox4x64(c, key) == want


def test_gaussian_table_is_the_discrete_gaussian_cdf(oracle_mod):
    sigma = 3.2
    T = oracle_mod.cdt_table(sigma)
    assert T == sorted(T) and len(T) == 38
    rho = [math.exp(-x * x / (2 * sigma * sigma)) for x in range(-19, 20)]
    Z = sum(rho)
    cum = 0.0
    for k in range(38):
        cum += rho[k]
        assert abs(T[k] / 2.0**64 - cum / Z) < 1e-12
    # symmetric about zero
    for k in range(19):
        assert abs(T[k] / 2.0**64 - (1 - T[37 - k] / 2.0**64)) < 1e-12


def test_secret_is_ternary_and_balanced(toy):
    s = toy.secret().astype(int)
    assert set(np.unique(s)) <= {-1, 0, 1}
    for v in (-1, 0, 1):
        assert abs((s == v).mean() - 1 / 3) < 0.06


# ----------------------------------------------------------------- encoding
def test_encode_fft_equals_definition(oracle_mod):
    o = oracle_mod.Oracle(8, (60, 40), (60,))
    g = np.random.default_rng(11)
    for nz in (128, 16, 1):
        z = g.uniform(-1, 1, nz)
        assert np.array_equal(o.encode(z), o.encode(z, direct=True))
    z = (g.uniform(size=128) < 0.5).astype(float)  # a 0/1 mask
    assert np.array_equal(o.encode(z), o.encode(z, direct=True))


def test_encode_matches_exact_decimal_definition(oracle_mod):
    o = oracle_mod.Oracle(4, (60, 40), (60,))
    g = np.random.default_rng(2)
    for z in (g.uniform(-1, 1, 8), np.array([1.0, 0, 0, 1, 1, 0, 1, 0]), np.array([0.5])):
        assert [int(v) for v in o.encode(z)] == t0.encode_exact(list(z), 2.0**40, o.N)


def test_encode_closed_forms(oracle_mod):
    o = oracle_mod.Oracle(10, (60, 40), (60,))
    N = o.N
    # constant message c: m = (round(c Delta), 0, ..., 0)
    m = o.encode(np.array([0.375]))
    assert m[0] == int(0.375 * 2**40) and not m[1:].any()
    # unit vector in slot 0: v_i = (2 Delta / N) cos(pi i / N)
    z = np.zeros(N // 2)
    z[0] = 1.0
    m = o.encode(z)
    v = 2 * 2.0**40 / N * np.cos(np.pi * np.arange(N) / N)
    assert np.max(np.abs(m - v)) <= 0.5 + 1e-3
    # a message replicated with period p lives in X^(N/(2p)): other coefficients vanish
    p = 32
    z = np.random.default_rng(1).uniform(-1, 1, p)
    m = o.encode(z)
    stride = N // (2 * p)
    mask = np.ones(N, dtype=bool)
    mask[::stride] = False
    assert not m[mask].any()


def test_decode_inverts_encode(oracle_mod):
    from oracle.oracle import decode_float
    o = oracle_mod.Oracle(12, (60, 40), (60,))
    z = np.random.default_rng(4).uniform(-1, 1, o.slots)
    m = o.encode(z)
    assert np.max(np.abs(decode_float(m, 2.0**40, o.N) - z)) < 2.0**-30


# ----------------------------------------------------------------- enc / dec
def test_encrypt_decrypt_roundtrip(toy):
    z = np.random.default_rng(9).uniform(-1, 1, toy.slots)
    for lvl in (toy.L, 1, 0):
        ct = toy.encrypt(z, level=lvl, nonce=lvl + 1)
        assert np.max(np.abs(toy.decrypt(ct) - z)) < 2.0**-25


def test_encryption_is_deterministic_in_nonce(toy):
    z = np.linspace(-1, 1, toy.slots)
    a, b, c = toy.encrypt(z, nonce=5), toy.encrypt(z, nonce=5), toy.encrypt(z, nonce=6)
    assert np.array_equal(a.data(), b.data())
    assert not np.array_equal(a.data(), c.data())


# ----------------------------------------------------------------- rescale
def _coef_ints(o, ct, p):
    """CRT-reconstructed centred coefficients of component p of a ciphertext."""
    d = ct.data()[p]
    mods = o.q[: ct.level + 1] + (o.p if ct.nlimbs > ct.level + 1 else [])
    idx = list(range(ct.level + 1)) + ([o.nq + k for k in range(o.alpha)] if ct.nlimbs > ct.level + 1 else [])
    res = [o.intt(m, d[k]) for k, m in enumerate(idx)]
    Q = math.prod(mods)
    return [t0.centred(t0.crt([r[i] for r in res], mods), Q) for i in range(o.N)], Q


def test_rescale_is_rounded_division(toy):
    z = np.random.default_rng(1).uniform(-1, 1, toy.slots)
    ct = toy.encrypt(z, nonce=3)
    r = toy.rescale(ct)
    ql = toy.q[ct.level]
    for p in (0, 1):
        x, _ = _coef_ints(toy, ct, p)
        y, Q2 = _coef_ints(toy, r, p)
        want = [t0.centred(t0.round_div(v, ql), Q2) for v in x]
        assert y == want


# ----------------------------------------------------------------- key switching
def test_decompose_is_exact_lift_up_to_multiple_of_digit_modulus(toy):
    g = np.random.default_rng(8)
    lvl = toy.L
    d = np.stack([g.integers(0, q, toy.N, dtype=np.uint64) for q in toy.q[: lvl + 1]])
    dig = toy.decompose(d, lvl)
    coef = [[int(v) for v in toy.intt(m, d[m])] for m in range(lvl + 1)]
    mods_qp = toy.q[: lvl + 1] + toy.p
    idx_qp = list(range(lvl + 1)) + [toy.nq + k for k in range(toy.alpha)]
    for j in range(toy.beta_at(lvl)):
        src = [k for k in range(j * toy.alpha, (j + 1) * toy.alpha) if k <= lvl]
        D = math.prod(toy.q[k] for k in src)
        outs = [[int(v) for v in toy.intt(m, dig[j][pos])] for pos, m in enumerate(idx_qp)]
        for i in range(0, toy.N, 37):
            x = t0.crt([coef[k][i] for k in src], [toy.q[k] for k in src])
            # the lift y = x + u D, 0 <= u < |src|, is one integer seen mod every prime
            t = mods_qp[-1]
            u = ((outs[-1][i] - x) * pow(D, -1, t)) % t
            assert 0 <= u < len(src)
            y = x + u * D
            for pos, q in enumerate(mods_qp):
                assert outs[pos][i] == y % q


@pytest.mark.parametrize("p_bits", [(60,), (60, 60), (60, 60, 60), (61, 61, 61, 61)])
def test_moddown_is_rounded_division_by_P(oracle_mod, p_bits):
    # KeySwitch (Appendix A) rounds P^{-1} <a, swk> to the nearest integer
    o = oracle_mod.Oracle(10, (60, 40, 40, 40), p_bits, seed=2)
    o.keygen(rot_steps=[1], relin=False)
    z = np.random.default_rng(2).uniform(-1, 1, o.slots)
    ct = o.encrypt(z, nonce=9)
    h = o.hoisted_rotate(ct, 1)
    md = o.moddown(h)
    P = math.prod(o.p)
    for p in (0, 1):
        x, _ = _coef_ints(o, h, p)
        y, Q = _coef_ints(o, md, p)
        assert y == [t0.centred(t0.round_div(v, P), Q) for v in x]


@pytest.mark.parametrize("p_bits", [(60,), (60, 60, 60)])
def test_moddown_rescale_is_one_rounded_division(oracle_mod, p_bits):
    # the variant: ModDown and the Rescale after it as round(x / (P q_l)),
    # against a big-integer division; it differs from rounding twice by at
    # most one per coefficient
    o = oracle_mod.Oracle(10, (60, 40, 40, 40), p_bits, seed=4)
    o.keygen(rot_steps=[1], relin=False)
    z = np.random.default_rng(3).uniform(-1, 1, o.slots)
    ct = o.encrypt(z, nonce=11)
    h = o.hoisted_rotate(ct, 1)
    fused = o.moddown_rescale(h)
    twice = o.rescale(o.moddown(h))
    assert fused.level == ct.level - 1 and fused.scale == twice.scale
    D = math.prod(o.p) * o.q[ct.level]
    for p in (0, 1):
        x, _ = _coef_ints(o, h, p)
        y, Q = _coef_ints(o, fused, p)
        assert y == [t0.centred(t0.round_div(v, D), Q) for v in x]
        y2, _ = _coef_ints(o, twice, p)
        assert max(abs(a - b) for a, b in zip(y, y2)) <= 1


def test_rotation_rotates_slots(toy):
    z = np.random.default_rng(5).uniform(-1, 1, toy.slots)
    ct = toy.encrypt(z, nonce=4)
    for k in (1, 3, -1, 16, 100):
        got = toy.decrypt(toy.rotate(ct, k))
        assert np.max(np.abs(got - np.roll(z, -k))) < 2.0**-20


def test_rotation_composition(toy):
    z = np.random.default_rng(6).uniform(-1, 1, toy.slots)
    ct = toy.encrypt(z, nonce=4)
    two = toy.rotate(toy.rotate(ct, 1), 2)
    one = toy.rotate(ct, 3)
    assert np.max(np.abs(toy.decrypt(two) - toy.decrypt(one))) < 2.0**-20


def test_tensor_decrypts_under_one_s_s2(oracle_mod):
    o = oracle_mod.Oracle(4, (60, 40, 40), (60,), seed=3)
    o.keygen(relin=False)
    g = np.random.default_rng(3)
    a, b = g.uniform(-1, 1, o.slots), g.uniform(-1, 1, o.slots)
    ca, cb = o.encrypt(a, nonce=1), o.encrypt(b, nonce=2)
    t3 = o.tensor(ca, cb)
    q = o.q[0]
    s = [int(v) % q for v in o.secret()]
    s2 = t0.negacyclic_mul(s, s, q)
    comps = [[int(v) for v in o.intt(0, t3[c][0])] for c in range(3)]
    d1s, d2s2 = t0.negacyclic_mul(comps[1], s, q), t0.negacyclic_mul(comps[2], s2, q)
    dec = [t0.centred(comps[0][i] + d1s[i] + d2s2[i], q) for i in range(o.N)]
    ma = [int(v) for v in o.encode(a)]
    mb = [int(v) for v in o.encode(b)]
    want = [t0.centred(v, q) for v in t0.negacyclic_mul(ma, mb, q)]
    # equal up to the encryption noise carried through the product
    assert max(abs(x - y) for x, y in zip(dec, want)) < 2.0**60 * 2.0**-10


def test_mult_relin_rescale(toy):
    g = np.random.default_rng(7)
    a, b = g.uniform(-1, 1, toy.slots), g.uniform(-1, 1, toy.slots)
    ca, cb = toy.encrypt(a, nonce=1), toy.encrypt(b, nonce=2)
    m = toy.rescale(toy.mult(ca, cb))
    assert np.max(np.abs(toy.decrypt(m) - a * b)) < 2.0**-18


def test_pmult_and_add(toy):
    g = np.random.default_rng(8)
    a, w = g.uniform(-1, 1, toy.slots), g.uniform(-1, 1, toy.slots)
    ca = toy.encrypt(a, nonce=1)
    pm = toy.rescale(toy.pmult(ca, toy.encode(w), 2.0**40))
    assert np.max(np.abs(toy.decrypt(pm) - a * w)) < 2.0**-20
    s = toy.add(ca, ca)
    assert np.max(np.abs(toy.decrypt(s) - 2 * a)) < 2.0**-20
