"""Oracle of the homomorphic PowerMethod round and the eigen-shift (section
6.1: covariance transformation on replicated vectors, Aggregate, Lazy
Normalization with TaylorInit and Newton InvSRT, AxisFlipping and the
eigenvalue; Algorithms Aggregate, TaylorInit, IterativeInvSRTbyNewton,
AxisFlipping, HEigenShift, HPowerMethod), plus the plain FP64 definitions the
decrypted results are compared with.

TEST INFRASTRUCTURE ONLY (like the rest of oracle/): the steps below are
written over the oracle's CKKS primitives (ckks_oracle.c through
oracle.py), one operation at a time in the paper's order, with these readings
where the paper is silent, garbled or inconsistent:

  * Blocks.  cov[r*k + c] is block (row block r, column block c) of the
    t x t covariance, t = k n; the paper's Cov_i[j] is block (j, i).
  * Replicated vectors.  Axis 0: every row of block i holds segment i of
    the vector (a row vector); axis 1: every column does (a column vector).
  * Aggregate(A; 0) adds Rot(A; i) for i = n, 2n, .. < n^2 (column sums in
    every row); Aggregate(A; 1) adds Rot(A; i) for i = 1, 2, .. < n, keeps
    column 0 with a 0/1 mask (one level) and spreads it with Rot(A; i),
    i = -1, -2, .. > -n (row sums in every column).
  * In the transformation the j-loop multiplies V[j] (the algorithm prints
    V_t[i]); axis 0 uses block (i, j), axis 1 block (j, i).
  * Newton step y <- y (3 - x y^2) / 2 (the algorithm prints the opposite
    sign), evaluated as y * (1.5 + (-x/2) y^2): with -x/2 formed once per
    normalisation, each step costs three products and three levels.
  * TaylorInit of order 1 (the experiments' linear expansion) at x0:
    T(x) = 1.5 x0^-1/2 - 0.5 x0^-3/2 x.
  * Constants and masks multiplied into a ciphertext at level l are encoded
    at scale q_l and followed by a rescale; constants added are encoded at
    the ciphertext's own scale.  Two operands of a product are taken to the
    lower of their levels by dropping limbs.
  * Refresh (interactive, client side): decrypt, centre the residue mod
    q_0 (exact while |m| < q_0 / 2), re-scale the integer polynomial to the
    nominal scale Delta, m' = round(m * r) with r = Delta / scale as a double
    and the product taken exactly (halves away from zero), and encrypt m' at
    the top level with scale Delta; nonces count up from a base.  Resetting
    the scale matters: every Newton step multiplies the relative drift of
    the scale (from dividing by primes that are not exactly Delta) by three.
    It is applied greedily: an operand of a product, or of a mask/constant
    multiplication, that sits at level 0 is refreshed right before it.
  * The last round (t = l_P) computes lambda = <Cov v, v> instead of
    normalising: v flipped by AxisFlipping, multiplied with Cov v, summed by
    Aggregate.
  * EigenShift subtracts lambda (v v^T) block by block; Cov is first brought
    to the level and scale of the subtrahend (drop, multiply by the constant
    1 encoded at the scale ratio, rescale, take the target scale).

Pins: the decrypted rounds, eigenvalue and shifted blocks against the FP64
replay below, lambda <= lambda_1 (Appendix B), the Lazy Normalization
averages printed in section 7, Newton's monotonicity.  Parity unpinned: the
placement of refreshes (the paper's flowchart for it is missing; the greedy
rule above is this reading, and the GPU path is held to it residue for
residue).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


# ---------------------------------------------------------------------------
# host schedule and plain FP64 definitions
# ---------------------------------------------------------------------------
def taylor1(x, x0):
    """order-1 Taylor expansion of x^-1/2 at x0 (TaylorInit)"""
    return 1.5 * x0 ** -0.5 - 0.5 * x0 ** -1.5 * x


def newton(y, x, tau):
    """tau Newton steps for x^-1/2 (Algorithm Newton's Method, sign as in
    the InvSRT recurrence y <- y (3 - x y^2) / 2)"""
    for _ in range(tau):
        y = y * (1.5 + (-0.5 * x) * (y * y))
    return y


def lazy_schedule(l_p, S=0.5, e=1e-5, precision=1e-3, B2=2.0 ** 16, max_tau=200):
    """Lazy Normalization (section 6.1.2): simulate l_p PowerMethod rounds on
    a unit vector shrunk by S per round; per round the smallest Newton count
    tau whose output S' keeps (l S' S)^2 >= precision, and in the last round
    also 1 - l S' < e.  Returns the list of tau."""
    x0 = B2 / 2 + 1
    l = 1.0
    taus = []
    for t in range(l_p):
        l *= S
        last = t == l_p - 1
        for tau in range(max_tau + 1):
            sp = newton(taylor1(l * l, x0), l * l, tau)
            ok = (l * sp * S) ** 2 >= precision and (not last or 1 - l * sp < e)
            if ok:
                break
        else:
            raise ValueError("no Newton count satisfies the bounds")
        taus.append(tau)
        l *= sp
    return taus


def goldschmidt(y, x, tau):
    """tau steps of Goldschmidt's iteration for x^-1/2 from y (the form the
    paper proves equal to Newton's): h = y/2, g = x y; r = 1/2 - g h,
    h <- h + h r, g <- g + g r; returns 2 h"""
    h, g = 0.5 * y, x * y
    for _ in range(tau):
        r = 0.5 - g * h
        h, g = h + h * r, g + g * r
    return 2.0 * h


def fp64_round(cov, v, tau, x0, last):
    """One PowerMethod round in FP64 with the same steps as the circuit:
    y = Cov v; not last: y * Newton_tau(T(<y,y>), <y,y>); last: lambda = <y, v>."""
    y = cov @ v
    if last:
        return v, float(y @ v)
    x = float(y @ y)
    return y * newton(taylor1(x, x0), x, tau), None


def _round_half_away(x: Fraction) -> int:
    f = (abs(x.numerator) * 2 + x.denominator) // (2 * x.denominator)
    return f if x >= 0 else -f


def replicate(v, k, n, axis):
    """the k n x n blocks of a replicated vector (axis 0: rows, 1: columns)"""
    out = []
    for i in range(k):
        seg = v[i * n:(i + 1) * n]
        out.append(np.tile(seg, (n, 1)) if axis == 0 else np.tile(seg[:, None], (1, n)))
    return out


def unreplicate(blocks, axis):
    return np.concatenate([b[0, :] if axis == 0 else b[:, 0] for b in blocks])


# ---------------------------------------------------------------------------
# the homomorphic circuit over the oracle's primitives
# ---------------------------------------------------------------------------
class Box:
    """a ciphertext slot that a refresh may replace"""

    def __init__(self, ct):
        self.ct = ct


class HePower:
    def __init__(self, o, n, nonce0=1 << 40):
        self.o = o
        self.n = n
        self.nonce = nonce0
        self.refreshes = 0
        self.packs = 0

    # -- plaintexts --------------------------------------------------------
    def _const(self, c, scale):
        return self.o.encode(np.full(self.n * self.n, float(c)), delta=scale)

    def _mask(self, kind, scale):
        n = self.n
        M = np.zeros((n, n))
        if kind == "col0":
            M[:, 0] = 1.0
        else:
            M[np.arange(n), np.arange(n)] = 1.0
        return self.o.encode(M.ravel(), delta=scale)

    def _line(self, col, idx, scale):
        """0/1 mask keeping column idx (col) or row idx"""
        n = self.n
        M = np.zeros((n, n))
        if col:
            M[:, idx] = 1.0
        else:
            M[idx, :] = 1.0
        return self.o.encode(M.ravel(), delta=scale)

    # -- refresh -------------------------------------------------------------
    def refresh(self, ct):
        o = self.o
        res = o.decrypt_residues(ct)[0].astype(np.int64)
        q0 = int(o.q[0])
        m = np.where(res > q0 // 2, res - q0, res)
        r = Fraction(o.delta / ct.scale)        # the double ratio, taken exactly
        m2 = np.array([_round_half_away(int(c) * r) for c in m], dtype=np.int64)
        out = o.encrypt_poly(m2, o.L, o.delta, nonce=self.nonce)
        self.nonce += 1
        self.refreshes += 1
        return out

    def _ready(self, *boxes):
        for b in boxes:
            if b.ct.level < 1:
                b.ct = self.refresh(b.ct)

    # -- operations ------------------------------------------------------------
    def _align(self, a, b):
        lv = min(a.level, b.level)
        return (a if a.level == lv else self.o.drop(a, lv)), (b if b.level == lv else self.o.drop(b, lv))

    def mul(self, A, B):
        """Mult with relinearisation, then Rescale"""
        self._ready(A, B)
        a, b = self._align(A.ct, B.ct)
        return self.o.rescale(self.o.mult(a, b))

    def pmul_pt(self, A, make_pt):
        self._ready(A)
        a = A.ct
        ql = float(self.o.q[a.level])
        return self.o.rescale(self.o.pmult(a, make_pt(ql), ql))

    def pmul_const(self, A, c):
        return self.pmul_pt(A, lambda s: self._const(c, s))

    def pmul_mask(self, A, kind):
        return self.pmul_pt(A, lambda s: self._mask(kind, s))

    def padd_const(self, a, c):
        return self.o.padd(a, self._const(c, a.scale))

    def add(self, a, b):
        a, b = self._align(a, b)
        if a.scale != b.scale:
            raise ValueError("addition of ciphertexts with different scales")
        return self.o.add(a, b)

    def aggregate(self, A, axis):
        o, n = self.o, self.n
        a = A.ct
        if axis == 0:
            i = n
            while i < n * n:
                a = o.add(a, o.rotate(a, i))
                i <<= 1
            return a
        i = 1
        while i < n:
            a = o.add(a, o.rotate(a, i))
            i <<= 1
        a = self.pmul_mask(Box(a), "col0")
        i = -1
        while i > -n:
            a = o.add(a, o.rotate(a, i))
            i <<= 1
        return a

    def axis_flip(self, V, axis):
        """AxisFlipping: identity mask, then Aggregate on the other axis"""
        return self.aggregate(Box(self.pmul_mask(V, "eye")), 1 - axis)

    def taylor(self, X, x0):
        c1 = -0.5 * x0 ** -1.5
        c0 = 1.5 * x0 ** -0.5
        return self.padd_const(self.pmul_const(X, c1), c0)

    def newton(self, X, Y, tau):
        if tau == 0:
            return Y
        Xh = Box(self.pmul_const(X, -0.5))
        for _ in range(tau):
            Y2 = Box(self.mul(Y, Y))
            P = self.mul(Y2, Xh)
            W = Box(self.padd_const(P, 1.5))
            Y = Box(self.mul(Y, W))
        return Y

    def goldschmidt_half(self, X, x0, tau):
        """Goldschmidt's iteration for x^-1/2 (section 3.5, equivalent to
        Newton's): h_0 = T(x)/2, g_0 = x T(x); c = 1/2 - g h;
        h <- h + h c, g <- g + g c; y_tau = 2 h_tau.  Here g is carried negated
        (gn = -g) and h + h c, g + g c are formed as h (1.5 + gn h) and
        gn (1.5 + gn h), plaintext additions and products only.  Returns
        h_tau.  Before each step, h or gn whose scale left
        [Delta/2, 2 Delta] is brought back to Delta (match, one level): the
        deviation of the scales triples with every step."""
        c1 = -0.5 * x0 ** -1.5
        c0 = 1.5 * x0 ** -0.5
        H = Box(self.padd_const(self.pmul_const(X, 0.5 * c1), 0.5 * c0))
        if tau == 0:
            return H
        Yn = Box(self.padd_const(self.pmul_const(X, -c1), -c0))
        Gn = Box(self.mul(X, Yn))
        d = self.o.delta

        def renorm(A):
            a = A.ct
            if a.level >= 1 and (a.scale > 2.0 * d or a.scale < 0.5 * d):
                A.ct = self.match(a, a.level - 1, d)

        for it in range(tau):
            renorm(H)
            renorm(Gn)
            W = Box(self.padd_const(self.mul(Gn, H), 1.5))
            H2 = Box(self.mul(H, W))
            if it + 1 < tau:
                Gn = Box(self.mul(Gn, W))
            H = H2
        return H

    def pack(self, V, axis):
        """Appendix C, the single-ciphertext refresh of a replicated vector:
        block i keeps its segment in column i (axis 1) or row i (axis 0)
        under a 0/1 mask, and the masked blocks are summed"""
        o = self.o
        P = None
        for i, A in enumerate(V):
            self._ready(A)
            a = A.ct
            ql = float(o.q[a.level])
            t = o.rescale(o.pmult(a, self._line(axis == 1, i, ql), ql))
            P = t if P is None else self.add(P, t)
        return P

    def unpack(self, P, axis, k):
        """block i from the packed ciphertext: rotated so that column / row i
        comes to position 0 (power-of-two steps), masked, and spread by
        Aggregate's rotations"""
        o, n = self.o, self.n
        unit = 1 if axis == 1 else n
        out = []
        for i in range(k):
            R = P
            b = 0
            while (1 << b) <= i:
                if (i >> b) & 1:
                    R = o.rotate(R, unit << b)
                b += 1
            ql = float(o.q[R.level])
            M = o.rescale(o.pmult(R, self._line(axis == 1, 0, ql), ql))
            if axis == 1:
                st = -1
                while st > -n:
                    M = o.add(M, o.rotate(M, st))
                    st *= 2
            else:
                M = self.aggregate(Box(M), 0)
            out.append(Box(M))
        return out

    def step(self, cov, k, V, axis, tau, x0, last, goldschmidt=False, pack=False):
        """One round of HPowerMethod.  cov: k*k Boxes (block (r, c) at r*k+c),
        V: k Boxes of the replicated vector in `axis` form.  Returns
        (V', axis') or, for the last round, (V, axis, lambda, V^T).
        goldschmidt: the inverse square root by goldschmidt_half, the vector
        scaled by 2 h as (v h) + (v h).  pack: an output vector that would
        have fewer than 3 levels is formed packed (masks on the blocks of
        Cov v, then the product with the factor), refreshed once and
        unpacked, when the blocks sit above the factor."""
        newV = []
        for i in range(k):
            S = None
            for j in range(k):
                C = cov[i * k + j] if axis == 0 else cov[j * k + i]
                P = self.mul(C, V[j])
                S = P if S is None else self.add(S, P)
            newV.append(Box(self.aggregate(Box(S), 1 - axis)))
        ax2 = 1 - axis
        S = None
        for i in range(k):
            P = self.mul(newV[i], newV[i])
            S = P if S is None else self.add(S, P)
        X = Box(self.aggregate(Box(S), 1 - ax2))
        if not last:
            Y = self.goldschmidt_half(X, x0, tau) if goldschmidt else self.newton(X, Box(self.taylor(X, x0)), tau)
            if pack and 1 < k <= self.n:
                yl = self.o.L if Y.ct.level < 1 else Y.ct.level
                ok = all(b.ct.level >= yl + 1 and b.ct.level == newV[0].ct.level and b.ct.scale == newV[0].ct.scale
                         for b in newV)
                if ok and yl - 1 < 3:
                    self.packs += 1
                    Q = Box(self.pack(newV, ax2))
                    P = self.mul(Q, Y)
                    if goldschmidt:
                        P = self.o.add(P, P)
                    return self.unpack(self.refresh(P), ax2, k), ax2
            out = []
            for i in range(k):
                P = self.mul(newV[i], Y)
                out.append(Box(self.o.add(P, P) if goldschmidt else P))
            return out, ax2
        VT = [Box(self.axis_flip(V[i], axis)) for i in range(k)]
        S = None
        for i in range(k):
            P = self.mul(newV[i], VT[i])
            S = P if S is None else self.add(S, P)
        lam = self.aggregate(Box(S), 1 - ax2)
        return V, axis, Box(lam), VT

    def match(self, x, level, scale):
        """x at a higher level brought to (level, scale)"""
        o = self.o
        if x.level <= level:
            raise ValueError("match needs a higher level")
        if x.level > level + 1:
            x = o.drop(x, level + 1)
        q = float(o.q[level + 1])
        p = scale * q / x.scale
        r = o.rescale(o.pmult(x, self._const(1.0, p), p))
        return o.ct_import(r.data(), r.level, False, scale)

    def sub_matched(self, A, b):
        """A.ct - b with A brought to b's level and scale when they differ"""
        o = self.o
        a = A.ct
        if a.scale == b.scale:
            a2, b2 = self._align(a, b)
            return o.sub(a2, b2)
        if a.level <= b.level:
            A.ct = self.refresh(a)
            a = A.ct
        return o.sub(self.match(a, b.level, b.scale), b)

    def eigen_shift(self, cov, k, lam, V, VT, axis):
        """HEigenShift: block (r, c) minus lambda (v v^T)_(r, c)"""
        out = []
        for r in range(k):
            for c in range(k):
                O = Box(self.mul(VT[r], V[c]) if axis == 0 else self.mul(V[r], VT[c]))
                T = self.mul(lam, O)
                out.append(Box(self.sub_matched(cov[r * k + c], T)))
        return out
