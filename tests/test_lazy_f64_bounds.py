"""The lazy FP64 modular product used by the kernels for moduli below 2^46:
h = a w, l = fma(a, w, -h), k = rint(h * (1/q)), r = fma(-k, q, h) + l must
equal a w - k q exactly, with |r| < q, for |a| <= 16 q and 0 <= w < q; the
centred reduction fma(-rint(s / q), q, s) must stay within q/2 + 1; and the
2^52 mantissa conversions must be exact below 2^52 and equal the plain
conversion (double) x, the form in which the switching keys' limbs below 2^46
are stored (so a key read as a double multiplies exactly as a converted word
in [0, q) did).  Checked with the same IEEE operations on the host (C with
fma, 128-bit integers as reference)."""
import os
import shutil
import subprocess

import pytest

SRC = r"""
#include <stdio.h>
#include <math.h>
#include <string.h>
typedef unsigned long long u64;
typedef __int128 i128;
static u64 s = 88172645463325252ull;
static u64 xr(void) { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return s; }
static double mms(double a, double w, double q, double qi) {
  double h = a * w, l = fma(a, w, -h), k = rint(h * qi);
  return fma(-k, q, h) + l;
}
static double centre(double x, double q, double qi) { return fma(-rint(x * qi), q, x); }
static double u2d(u64 x) { u64 b = x | 0x4330000000000000ull; double d; memcpy(&d, &b, 8); return d - 0x1p52; }
static u64 d2u(double x) { double y = x + 0x1p52; u64 b; memcpy(&b, &y, 8); return b & 0x000FFFFFFFFFFFFFull; }
int main(void) {
  long bad = 0;
  double worst = 0;
  for (int t = 0; t < 80; t++) {
    int bits = 33 + (int)(xr() % 14);
    u64 q = ((1ull << (bits - 1)) + (xr() % (1ull << (bits - 1)))) | 1;
    if (t < 8) q = (1ull << 46) - 1 - 2 * (xr() % 1000);
    double qd = (double)q, qi = 1.0 / qd;
    for (int i = 0; i < 50000; i++) {
      long long a = (long long)(xr() % (32 * q + 1)) - (long long)(16 * q);
      if (i < 4) a = (i & 1) ? 16 * (long long)q : -16 * (long long)q;
      u64 w = xr() % q;
      if (i == 2) w = q - 1;
      double r = mms((double)a, (double)w, qd, qi);
      long long rr = (long long)r;
      if ((double)rr != r || (((i128)a * w - rr) % (i128)q) != 0 || fabs(r) >= qd) bad++;
      if (fabs(r) / qd > worst) worst = fabs(r) / qd;
      double c = centre((double)a, qd, qi);
      long long cc = (long long)c;
      if ((((i128)a - cc) % (i128)q) != 0 || fabs(c) > qd / 2 + 1) bad++;
      u64 x = xr() & ((1ull << 52) - 1);
      if (u2d(x) != (double)x || d2u((double)x) != x) bad++;
    }
  }
  printf("%ld %.6f\n", bad, worst);
  return 0;
}
"""


def test_lazy_f64_product_exact_and_bounded(tmp_path):
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "lazy.c"
    src.write_text(SRC)
    exe = tmp_path / "lazy"
    subprocess.run([cc, "-O2", "-mfma", "-ffp-contract=off", "-o", str(exe), str(src), "-lm"], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    bad, worst = int(out[0]), float(out[1])
    assert bad == 0
    assert worst < 0.875


SRC_PIECES = r"""
#include <stdio.h>
#include <math.h>
#include <string.h>
typedef unsigned long long u64;
typedef unsigned __int128 u128;
static u64 s = 0x9E3779B97F4A7C15ull;
static u64 xr(void) { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return s; }
static double u2d(u64 x) { u64 b = x | 0x4330000000000000ull; double d; memcpy(&d, &b, 8); return d - 0x1p52; }
static u64 d2u(double x) { double y = x + 0x1p52; u64 b; memcpy(&b, &y, 8); return b & 0x000FFFFFFFFFFFFFull; }
static void split(u64 x, double p[3]) { p[0] = u2d(x & 0xFFFFF); p[1] = u2d((x >> 20) & 0xFFFFF); p[2] = u2d(x >> 40); }
/* the 128-bit reduction of the 60-bit limbs' fold: 2^64 and 2^96 mod q fold
   the high word, the quotient is estimated in FP64 and corrected once */
static u64 red(u64 lo, u64 hi, u64 q, u64 r64, u64 r96, double qinvf) {
  u64 y0 = lo, y1 = 0, a[2] = {hi >> 32, hi & 0xffffffffull}, r[2] = {r96, r64};
  for (int t = 0; t < 2; t++) {
    u64 l = a[t] * (r[t] & 0xffffffffull), h = a[t] * (r[t] >> 32), hl = h << 32, sm = y0 + l;
    y1 += (sm < l) + (h >> 32);
    y0 = sm + hl;
    y1 += y0 < hl;
  }
  double yd = fma((double)y1, 0x1p64, (double)y0);
  u64 k = (u64)floor(yd * qinvf);
  long long rr = (long long)(y0 - k * q);
  if (rr < 0) rr += (long long)q; else if ((u64)rr >= q) rr -= (long long)q;
  return (u64)rr;
}
int main(void) {
  long bad = 0, n = 0;
  for (int t = 0; t < 40; t++) {
    int bits = 47 + (int)(xr() % 15);                     /* 47 .. 61 bits */
    u64 q = ((1ull << (bits - 1)) + (xr() % (1ull << (bits - 1)))) | 1;
    u64 r64 = (u64)(((u128)1 << 64) % q), r96 = (u64)(((u128)r64 << 32) % q);
    double qinvf = 1.0 / (double)q;
    for (int i = 0; i < 20000; i++) {
      int beta = 1 + (int)(xr() % 64);
      double S[5] = {0, 0, 0, 0, 0};
      u128 X = 0;
      for (int j = 0; j < beta; j++) {
        u64 d = xr() % q, k = xr() % q;
        if (i < 8) { d = q - 1; k = q - 1; }
        double dp[3], kp[3];
        split(d, dp); split(k, kp);
        for (int a = 0; a < 3; a++)
          for (int b = 0; b < 3; b++) S[a + b] = fma(dp[a], kp[b], S[a + b]);
        X += (u128)d * k;
      }
      u128 Y = 0;
      for (int w = 0; w < 5; w++) {
        double v = S[w];
        if (v != floor(v) || v >= 0x1p52) bad++;         /* exact integers below 2^52 */
        Y += (u128)d2u(v) << (20 * w);
      }
      if (Y != X) bad++;                                  /* the 128-bit sum of the products */
      u64 got = red((u64)X, (u64)(X >> 64), q, r64, r96, qinvf);
      if (got != (u64)(X % q)) bad++;
      /* values next to a multiple of q, where the estimate is off by one */
      u128 m = ((((u128)xr()) << 64 | xr()) % (((u128)1 << 125) / q)) * q;
      for (int e = -2; e <= 2; e++) {
        u128 Z = m + (u128)(long long)e;
        if (red((u64)Z, (u64)(Z >> 64), q, r64, r96, qinvf) != (u64)(Z % q)) bad++;
      }
      n++;
    }
  }
  printf("%ld %ld\n", bad, n);
  return 0;
}
"""


def test_piece_products_and_reduction_exact(tmp_path):
    """The key inner products of the 60-bit limbs: residues split into 20-bit
    pieces, the nine piece products summed by weight with FMAs are exact
    integers below 2^52 that recombine to the 128-bit sum of the products
    (up to 64 terms), and the FP64-estimated reduction of that sum equals
    its residue mod q, also next to multiples of q (47- to 61-bit moduli)."""
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "pieces.c"
    src.write_text(SRC_PIECES)
    exe = tmp_path / "pieces"
    subprocess.run([cc, "-O2", "-mfma", "-ffp-contract=off", "-o", str(exe), str(src), "-lm"], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    assert int(out[0]) == 0 and int(out[1]) == 800000
