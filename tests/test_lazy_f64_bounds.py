"""The lazy FP64 modular product used by the kernels for moduli below 2^46:
h = a w, l = fma(a, w, -h), k = rint(h * (1/q)), r = fma(-k, q, h) + l must
equal a w - k q exactly, with |r| < q, for |a| <= 16 q and 0 <= w < q; the
centred reduction fma(-rint(s / q), q, s) must stay within q/2 + 1; and the
2^52 mantissa conversions must be exact below 2^52.  Checked with the same
IEEE operations on the host (C with fma, 128-bit integers as reference)."""
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
