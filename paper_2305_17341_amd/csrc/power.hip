// The homomorphic PowerMethod round and the eigen-shift (section 6.1:
// covariance transformation on replicated vectors, Aggregate, Lazy
// Normalization with TaylorInit and Newton InvSRT, AxisFlipping and the
// eigenvalue; Algorithms Aggregate, TaylorInit, IterativeInvSRTbyNewton,
// AxisFlipping, HEigenShift, HPowerMethod) and the interactive refresh.
//
// Conventions (readings of the paper):
//   * cov[r*k + c] is block (row block r, column block c); the paper's
//     Cov_i[j] is block (j, i).  Axis 0: every row of a block holds the
//     vector segment (row vector); axis 1: every column does.
//   * Aggregate(A; 0) adds Rot(A; i), i = n, 2n, .. < n^2 (column sums);
//     Aggregate(A; 1) adds Rot(A; i), i = 1, 2, .. < n, keeps column 0 with
//     a 0/1 mask (one level), then adds Rot(A; i), i = -1, -2, .. > -n.
//   * The transformation's j-loop multiplies V[j]; axis 0 takes block (i, j),
//     axis 1 block (j, i).
//   * Newton: y <- y (1.5 + (-x/2) y^2), -x/2 formed once per normalisation;
//     three products and three levels per step.  Goldschmidt's form of the
//     same iterates (a variant): three products and two levels per step.  TaylorInit of order 1:
//     T(x) = 1.5 x0^-1/2 - 0.5 x0^-3/2 x.
//   * Constants and masks multiplied in at level l are encoded at scale q_l
//     and rescaled; constants added are encoded at the ciphertext's scale.
//     Product operands meet at the lower level by dropping limbs.
//   * An operand of a product or of a plaintext multiplication that sits at
//     level 0 is refreshed (through the caller's callback) right before it.
//     A refresh re-encrypts at the top level at the nominal scale Delta
//     (integer polynomial re-scaled exactly): every Newton step would
//     otherwise triple the relative drift of the scale.
#include <cmath>

#include "runtime.h"

// ---------------------------------------------------------------------------
// refresh (client side): decrypt to the centred integer polynomial (residue
// mod q_0, exact while |m| < q_0 / 2), m' = round(m Delta / scale) exactly,
// encrypt m' at the top level with scale Delta
// ---------------------------------------------------------------------------
DevBuf HeCtxImpl::decrypt_int(const HeCt& c) {
  if (!have_sk) fail(HE_EKEY, "keys not generated");
  if (c.qp || c.B != 1) fail(HE_EINVAL, "decrypt takes one ciphertext over Q");
  DevBuf t(&pool, N);
  LimbMap m0 = one(0);
  launch_mul(T, t.p, c.limb(1, 0), s_ntt.p, 1, m0, stream);
  launch_add(T, t.p, t.p, c.limb(0, 0), 1, m0, stream);
  launch_ntt(T, t.p, 1, m0, true, stream);
  DevBuf mi(&pool, N);
  launch_centre_to_int(T, (i64*)mi.p, t.p, 0, stream);
  return mi;
}

HeCt HeCtxImpl::refresh(const HeCt& c, u64 nonce) {
  DevBuf m = decrypt_int(c);
  const double r = delta / c.scale;
  int e = 0;
  const double f = std::frexp(r, &e);            // r = f 2^e, f in [1/2, 1)
  const u64 mant = (u64)std::ldexp(f, 53);       // exact: r = mant 2^(e - 53)
  const int shift = 53 - e;
  if (shift < 1 || shift > 120) fail(HE_ESCALE, "scale too far from the nominal one to refresh");
  launch_scale_int((i64*)m.p, mant, shift, N, stream);
  return encrypt_int((const i64*)m.p, L, delta, nonce);
}

HeCt HeCtxImpl::padd_int(const HeCt& a, const i64* m_dev) {
  if (a.qp || a.B != 1) fail(HE_EINVAL, "plaintext addition takes one ciphertext over Q");
  LimbMap m = qmap(a.level + 1);
  DevBuf pt(&pool, (size_t)a.nlimbs * N);
  int_to_ntt(pt.p, m_dev, m);
  HeCt c = ct_copy(a);
  launch_add(T, c.poly(0), a.poly(0), pt.p, a.nlimbs, m, stream);
  return c;
}

namespace {
struct Circuit {
  HeCtxImpl& c;
  int n;
  const RefreshFn& refresh;

  DevBuf const_pt(double v, double scale) {
    std::vector<double> z((size_t)n * n, v);
    return c.encode_batch(z.data(), n * n, 1, scale);
  }
  DevBuf mask_pt(bool col0, double scale) {
    std::vector<double> z((size_t)n * n, 0.0);
    for (int i = 0; i < n; i++) z[(size_t)i * n + (col0 ? 0 : i)] = 1.0;
    return c.encode_batch(z.data(), n * n, 1, scale);
  }
  // 0/1 mask keeping column idx (col) or row idx of an n x n block
  DevBuf line_pt(bool col, int idx, double scale) {
    std::vector<double> z((size_t)n * n, 0.0);
    for (int i = 0; i < n; i++) z[col ? (size_t)i * n + idx : (size_t)idx * n + i] = 1.0;
    return c.encode_batch(z.data(), n * n, 1, scale);
  }
  void ready(HeCt& x) {
    if (x.level < 1) refresh(x);
  }
  // Mult with relinearisation, then Rescale
  HeCt mul(HeCt& A, HeCt& B) {
    ready(A);
    if (&A != &B) ready(B);
    const int lv = std::min(A.level, B.level);
    HeCt a2, b2;
    const HeCt* pa = &A;
    const HeCt* pb = &B;
    if (A.level != lv) { a2 = c.drop(A, lv); pa = &a2; }
    if (B.level != lv) { b2 = c.drop(B, lv); pb = &b2; }
    HeCt t = c.mult(*pa, *pb);
    return c.rescale(t);
  }
  HeCt pmul_pt(HeCt& A, bool is_mask, bool col0, double v) {
    ready(A);
    const double ql = (double)c.mods[A.level];
    DevBuf pt = is_mask ? mask_pt(col0, ql) : const_pt(v, ql);
    HeCt t = c.pmult_int(A, (const i64*)pt.p, ql);
    return c.rescale(t);
  }
  HeCt pmul_const(HeCt& A, double v) { return pmul_pt(A, false, false, v); }
  HeCt pmul_mask(HeCt& A, bool col0) { return pmul_pt(A, true, col0, 0.0); }
  HeCt padd_const(const HeCt& a, double v) {
    DevBuf pt = const_pt(v, a.scale);
    return c.padd_int(a, (const i64*)pt.p);
  }
  HeCt add(const HeCt& a, const HeCt& b) {
    const int lv = std::min(a.level, b.level);
    HeCt a2, b2;
    const HeCt* pa = &a;
    const HeCt* pb = &b;
    if (a.level != lv) { a2 = c.drop(a, lv); pa = &a2; }
    if (b.level != lv) { b2 = c.drop(b, lv); pb = &b2; }
    return c.add(*pa, *pb, false);
  }
  HeCt aggregate(HeCt A, int axis) {
    if (axis == 0) {
      for (long i = n; i < (long)n * n; i <<= 1) A = c.add(A, c.rotate(A, i), false);
      return A;
    }
    for (long i = 1; i < n; i <<= 1) A = c.add(A, c.rotate(A, i), false);
    A = pmul_mask(A, true);
    for (long i = -1; i > -n; i *= 2) A = c.add(A, c.rotate(A, i), false);
    return A;
  }
  HeCt axis_flip(HeCt& V, int axis) { return aggregate(pmul_mask(V, false), 1 - axis); }
  HeCt taylor(HeCt& X, double x0) {
    const double c1 = -0.5 * std::pow(x0, -1.5), c0 = 1.5 * std::pow(x0, -0.5);
    return padd_const(pmul_const(X, c1), c0);
  }
  HeCt newton(HeCt& X, HeCt Y, int tau) {
    if (tau == 0) return Y;
    HeCt Xh = pmul_const(X, -0.5);
    for (int it = 0; it < tau; it++) {
      HeCt Y2 = mul(Y, Y);
      HeCt P = mul(Y2, Xh);
      HeCt W = padd_const(P, 1.5);
      Y = mul(Y, W);
    }
    return Y;
  }
  // Goldschmidt's iteration for x^-1/2, equal to Newton's step for step
  // (section 3.5): with h = y / 2 and g = x y, y_i = 2 h_i.  g is kept
  // negated so that c = 1.5 - g h is a plaintext addition; the updates
  // h + h (0.5 - g h) and g + g (0.5 - g h) are taken as h c and g c, so no
  // two ciphertexts of different scales are added.  Two levels per step
  // (Newton's form above takes three).  Returns h_tau = y_tau / 2.
  // The scales' deviation from Delta (primes that are not exactly Delta)
  // triples with every step, as in Newton's form; a pair of steps between
  // refreshes that would let it grow past a factor 2 is prevented by taking
  // any of h, g whose scale left [Delta/2, 2 Delta] back to Delta (match:
  // one level) before the step.
  HeCt goldschmidt_half(HeCt& X, double x0, int tau) {
    const double c1 = -0.5 * std::pow(x0, -1.5), c0 = 1.5 * std::pow(x0, -0.5);
    HeCt H = padd_const(pmul_const(X, 0.5 * c1), 0.5 * c0);  // T(x) / 2
    if (tau == 0) return H;
    HeCt Yn = padd_const(pmul_const(X, -c1), -c0);           // -T(x)
    HeCt Gn = mul(X, Yn);                                    // -x T(x)
    auto renorm = [&](HeCt& A) {
      if (A.level >= 1 && (A.scale > 2.0 * c.delta || A.scale < 0.5 * c.delta)) A = match(A, A.level - 1, c.delta);
    };
    for (int it = 0; it < tau; it++) {
      renorm(H);
      renorm(Gn);
      HeCt P = mul(Gn, H);
      HeCt W = padd_const(P, 1.5);
      HeCt H2 = mul(H, W);
      if (it + 1 < tau) Gn = mul(Gn, W);
      H = std::move(H2);
    }
    return H;
  }
  // A replicated vector refreshed through one ciphertext (Appendix C).
  // pack: the segment of block i kept in column i (axis 1: every column of a
  // block holds its segment) or row i (axis 0) by a 0/1 mask, the k masked
  // blocks summed (one level).  unpack: block i recovered from the one
  // ciphertext as the rotation bringing column / row i to position 0
  // (power-of-two steps), a mask keeping it (one level), and the spreading
  // rotations of Aggregate.
  HeCt pack(std::vector<HeCt>& V, int axis) {
    HeCt P;
    for (size_t i = 0; i < V.size(); i++) {
      HeCt& A = V[i];
      ready(A);
      const double ql = (double)c.mods[A.level];
      DevBuf m = line_pt(axis == 1, (int)i, ql);
      HeCt t = c.rescale(c.pmult_int(A, (const i64*)m.p, ql));
      P = i == 0 ? std::move(t) : add(P, t);
    }
    return P;
  }
  std::vector<HeCt> unpack(const HeCt& P, int axis, int k) {
    std::vector<HeCt> out;
    const long unit = axis == 1 ? 1 : n;
    for (int i = 0; i < k; i++) {
      HeCt R = c.ct_copy(P);
      for (int b = 0; (1 << b) <= i; b++)
        if ((i >> b) & 1) R = c.rotate(R, unit << b);
      const double ql = (double)c.mods[R.level];
      DevBuf m = line_pt(axis == 1, 0, ql);
      HeCt M = c.rescale(c.pmult_int(R, (const i64*)m.p, ql));
      if (axis == 1) {
        for (long st = -1; st > -n; st *= 2) M = c.add(M, c.rotate(M, st), false);
      } else {
        M = aggregate(std::move(M), 0);
      }
      out.push_back(std::move(M));
    }
    return out;
  }
  // x at a higher level brought to (level, scale)
  HeCt match(const HeCt& x, int level, double scale) {
    if (x.level <= level) fail(HE_ELEVEL, "scale matching needs a higher level");
    HeCt d;
    const HeCt* px = &x;
    if (x.level > level + 1) { d = c.drop(x, level + 1); px = &d; }
    const double q = (double)c.mods[level + 1];
    const double p = scale * q / px->scale;
    DevBuf one = const_pt(1.0, p);
    HeCt t = c.pmult_int(*px, (const i64*)one.p, p);
    HeCt r = c.rescale(t);
    r.scale = scale;
    return r;
  }
  HeCt sub_matched(HeCt& A, const HeCt& b) {
    if (A.scale == b.scale) {
      const int lv = std::min(A.level, b.level);
      HeCt a2, b2;
      const HeCt* pa = &A;
      const HeCt* pb = &b;
      if (A.level != lv) { a2 = c.drop(A, lv); pa = &a2; }
      if (b.level != lv) { b2 = c.drop(b, lv); pb = &b2; }
      return c.add(*pa, *pb, true);
    }
    if (A.level <= b.level) refresh(A);
    return c.add(match(A, b.level, b.scale), b, true);
  }
};
}  // namespace

void HeCtxImpl::power_step(std::vector<HeCt*>& cov, int k, int n, std::vector<HeCt*>& V, int axis, int tau,
                           double x0, bool last, bool goldschmidt, bool pack, const RefreshFn& refresh_fn,
                           std::vector<HeCt>& v_out, int& axis_out, HeCt& lambda_out, std::vector<HeCt>& vt_out) {
  if ((int)cov.size() != k * k || (int)V.size() != k || k < 1) fail(HE_EINVAL, "block counts");
  if ((u64)n * n > N / 2 || n < 2 || (n & (n - 1))) fail(HE_EINVAL, "block size must be a power of two, n^2 <= N/2");
  if (axis != 0 && axis != 1) fail(HE_EINVAL, "axis must be 0 or 1");
  Circuit C{*this, n, refresh_fn};
  std::vector<HeCt> nv(k);
  for (int i = 0; i < k; i++) {
    HeCt S;
    for (int j = 0; j < k; j++) {
      HeCt& blk = axis == 0 ? *cov[i * k + j] : *cov[j * k + i];
      HeCt P = C.mul(blk, *V[j]);
      S = j == 0 ? std::move(P) : C.add(S, P);
    }
    nv[i] = C.aggregate(std::move(S), 1 - axis);
  }
  const int ax2 = 1 - axis;
  HeCt S;
  for (int i = 0; i < k; i++) {
    HeCt P = C.mul(nv[i], nv[i]);
    S = i == 0 ? std::move(P) : C.add(S, P);
  }
  HeCt X = C.aggregate(std::move(S), 1 - ax2);
  if (!last) {
    v_out.clear();
    // the factor: y (Newton) or h = y / 2 (Goldschmidt, the product doubled
    // by an addition to itself)
    HeCt Y = goldschmidt ? C.goldschmidt_half(X, x0, tau) : C.newton(X, C.taylor(X, x0), tau);
    bool packed = false;
    if (pack && k > 1 && k <= n) {
      // a vector that would come out with fewer than the three levels the
      // next round's covariance transformation and inner product take is
      // formed packed instead (the mask on the blocks, whose level is higher
      // than the factor's, then one product), refreshed once and unpacked
      const int yl = Y.level < 1 ? L : Y.level;  // the factor's level in the product
      bool ok = true;
      for (int i = 0; i < k; i++)
        ok = ok && nv[i].level >= yl + 1 && nv[i].level == nv[0].level && nv[i].scale == nv[0].scale;
      if (ok && yl - 1 < 3) {
        HeCt Q = C.pack(nv, ax2);
        HeCt P = C.mul(Q, Y);
        if (goldschmidt) P = add(P, P, false);
        refresh_fn(P);
        v_out = C.unpack(P, ax2, k);
        packed = true;
      }
    }
    if (!packed)
      for (int i = 0; i < k; i++) {
        HeCt P = C.mul(nv[i], Y);
        v_out.push_back(goldschmidt ? add(P, P, false) : std::move(P));
      }
    axis_out = ax2;
    return;
  }
  vt_out.clear();
  for (int i = 0; i < k; i++) vt_out.push_back(C.axis_flip(*V[i], axis));
  HeCt S2;
  for (int i = 0; i < k; i++) {
    HeCt P = C.mul(nv[i], vt_out[i]);
    S2 = i == 0 ? std::move(P) : C.add(S2, P);
  }
  lambda_out = C.aggregate(std::move(S2), 1 - ax2);
  axis_out = axis;
}

void HeCtxImpl::eigen_shift(std::vector<HeCt*>& cov, int k, int n, HeCt& lambda, std::vector<HeCt*>& V,
                            std::vector<HeCt*>& VT, int axis, const RefreshFn& refresh_fn,
                            std::vector<HeCt>& out) {
  if ((int)cov.size() != k * k || (int)V.size() != k || (int)VT.size() != k) fail(HE_EINVAL, "block counts");
  Circuit C{*this, n, refresh_fn};
  out.clear();
  for (int r = 0; r < k; r++)
    for (int cc = 0; cc < k; cc++) {
      HeCt O = axis == 0 ? C.mul(*VT[r], *V[cc]) : C.mul(*V[r], *VT[cc]);
      HeCt Tm = C.mul(lambda, O);
      out.push_back(C.sub_matched(*cov[r * k + cc], Tm));
    }
}

// Covariance of a dataset that is not centred (section 5.2, Algorithm
// HCovMtrx): mu[j] = Aggregate(sum_r x[r k + j]; 0) times 1/s (the row-block
// sums, the column sums spread to every row, the true sample count), mu[a]^T
// by the transposition G, block (a, b) of mu^T mu = mu[a]^T (.) mu[b]
// (relinearised, rescaled), brought to the level and scale of the X^T X / s
// blocks and subtracted.  No operand reaches level 0 on this path: a refresh
// request is an error.
std::vector<HeCt> HeCtxImpl::covariance_uncentred(const std::vector<const HeCt*>& x, int rb, int k, int n,
                                                  u64 n_samples, int n1z, int n1t, int n1g, int npz, int npt,
                                                  bool lazy, bool fused_rs) {
  if ((int)x.size() != rb * k || rb < 1 || k < 1) fail(HE_EINVAL, "block count mismatch");
  std::vector<HeCt> xtx = covariance(x, rb, k, n, n_samples, n1z, n1t, n1g, npz, npt, lazy, fused_rs);
  RefreshFn no_refresh = [](HeCt&) { fail(HE_ELEVEL, "not enough levels for the mean path"); };
  Circuit C{*this, n, no_refresh};
  std::vector<HeCt> mu(k), mut(k);
  for (int j = 0; j < k; j++) {
    HeCt S = ct_copy(*x[j]);
    for (int r = 1; r < rb; r++) S = add(S, *x[r * k + j], false);
    HeCt A = C.aggregate(std::move(S), 0);
    mu[j] = C.pmul_const(A, 1.0 / (double)n_samples);
    mut[j] = lintrans(mu[j], LT_TRANSPOSE, n, n1g, 1.0);
  }
  std::vector<HeCt> out;
  for (int a = 0; a < k; a++)
    for (int b = 0; b < k; b++) {
      const HeCt& c = xtx[a * k + b];
      HeCt mm = C.mul(mut[a], mu[b]);
      out.push_back(add(c, C.match(mm, c.level, c.scale), true));
    }
  return out;
}
