"""Exact big-integer definitions used to pin the C oracle at tiny sizes.

TEST INFRASTRUCTURE ONLY.  Each function is the mathematical definition of a
quantity, written with Python integers, independent of how the C oracle
computes it (schoolbook products instead of transforms, direct evaluation
instead of butterflies, CRT reconstruction instead of fast basis conversion,
a Lucas/Pratt certificate instead of Miller-Rabin).
"""
from __future__ import annotations

import math
import random
from decimal import Decimal, getcontext


def bitrev(x: int, bits: int) -> int:
    r = 0
    for i in range(bits):
        r |= ((x >> i) & 1) << (bits - 1 - i)
    return r


def negacyclic_mul(a, b, q):
    """Schoolbook product in Z_q[X]/(X^N+1)."""
    N = len(a)
    out = [0] * N
    for i in range(N):
        if a[i] == 0:
            continue
        for j in range(N):
            k = i + j
            if k < N:
                out[k] += a[i] * b[j]
            else:
                out[k - N] -= a[i] * b[j]
    return [x % q for x in out]


def eval_at(a, x, q):
    acc = 0
    for c in reversed(a):
        acc = (acc * x + c) % q
    return acc


def ntt_by_evaluation(a, psi, q, log_n):
    """Index i holds a(psi^(2 brv(i) + 1))."""
    N = 1 << log_n
    return [eval_at(a, pow(psi, 2 * bitrev(i, log_n) + 1, q), q) for i in range(N)]


def automorph_coef(a, g, q):
    """a(X) -> a(X^g) in Z_q[X]/(X^N+1)."""
    N = len(a)
    out = [0] * N
    for k, c in enumerate(a):
        e = (g * k) % (2 * N)
        if e < N:
            out[e] = (out[e] + c) % q
        else:
            out[e - N] = (out[e - N] - c) % q
    return out


def crt(residues, primes):
    """Integer in [0, prod) congruent to residues."""
    Q = math.prod(primes)
    x = 0
    for r, q in zip(residues, primes):
        Qi = Q // q
        x += int(r) * Qi * pow(Qi, -1, q)
    return x % Q


def centred(x, Q):
    x %= Q
    return x - Q if x > Q // 2 else x


def round_div(x, d):
    """Nearest integer to x/d for odd d (no ties)."""
    return (2 * x + d) // (2 * d)


# -- primality by certificate (Lucas test with a recursively proven
#    factorisation of q - 1) ------------------------------------------------
def _pollard_rho(n, rng):
    if n % 2 == 0:
        return 2
    while True:
        x = rng.randrange(2, n)
        y, c, d = x, rng.randrange(1, n), 1
        while d == 1:
            x = (x * x + c) % n
            y = (y * y + c) % n
            y = (y * y + c) % n
            d = math.gcd(abs(x - y), n)
        if d != n:
            return d


def _small_prime(n):
    if n < 2:
        return False
    i = 2
    while i * i <= n:
        if n % i == 0:
            return False
        i += 1
    return True


def _factor(n, rng, out):
    if n == 1:
        return
    if n < 1 << 20:
        d = 2
        while d * d <= n:
            while n % d == 0:
                out.append(d)
                n //= d
            d += 1
        if n > 1:
            out.append(n)
        return
    if proven_prime(n, rng):
        out.append(n)
        return
    d = _pollard_rho(n, rng)
    _factor(d, rng, out)
    _factor(n // d, rng, out)


def proven_prime(n, rng=None):
    """Lucas: n is prime iff some a has a^(n-1)=1 and a^((n-1)/f) != 1 for every
    prime f | n-1.  The factors are themselves proven the same way."""
    rng = rng or random.Random(12345)
    if n < 1 << 20:
        return _small_prime(n)
    if pow(2, n - 1, n) != 1:
        return False
    fs = []
    _factor(n - 1, rng, fs)
    fs = sorted(set(fs))
    for a in range(2, 200):
        if pow(a, n - 1, n) != 1:
            return False
        if all(pow(a, (n - 1) // f, n) != 1 for f in fs):
            return True
    return False


# -- high-precision cosine for encoding pins ----------------------------------
def dec_pi(prec):
    getcontext().prec = prec + 10
    # Machin: pi = 16 atan(1/5) - 4 atan(1/239)
    def atan_inv(x):
        x = Decimal(x)
        s, t, n, sign = Decimal(0), 1 / x, 1, 1
        x2 = x * x
        while True:
            term = t / n
            if term == 0 or abs(term) < Decimal(10) ** (-(prec + 8)):
                break
            s += sign * term
            t /= x2
            n += 2
            sign = -sign
        return s
    return 16 * atan_inv(5) - 4 * atan_inv(239)


def dec_cos(x, prec):
    getcontext().prec = prec + 10
    s, term, k = Decimal(1), Decimal(1), 0
    x2 = x * x
    while True:
        k += 2
        term = -term * x2 / (k * (k - 1))
        if abs(term) < Decimal(10) ** (-(prec + 8)):
            break
        s += term
    return s


def encode_exact(z, delta, N, prec=60):
    """m_i = floor(v_i + 1/2 + 2^-30), v_i = (2 delta / N) sum_j z_j cos(pi 5^j i / N),
    evaluated in `prec` decimal digits (tiny N only)."""
    getcontext().prec = prec + 10
    pi = dec_pi(prec)
    S = N // 2
    pw = [pow(5, j, 2 * N) for j in range(S)]
    cosv = [dec_cos(pi * e / N, prec) for e in range(2 * N)]
    eps = Decimal(2) ** -30
    out = []
    for i in range(N):
        acc = Decimal(0)
        for j in range(S):
            acc += Decimal(z[j % len(z)]) * cosv[(pw[j] * i) % (2 * N)]
        v = acc * 2 * Decimal(delta) / N
        out.append(int((v + Decimal("0.5") + eps).to_integral_value(rounding="ROUND_FLOOR")))
    return out
