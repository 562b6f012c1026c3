"""ModDown's basis conversion as a dot product of 7-bit digits (the int8
matrix-product form of the fused ModDown): each source value v_a < p_a is cut
into nine 7-bit digits, the quotient r is one more byte, and each constant
hat_(a,t) 2^(7 i) mod q_t (and -D mod q_t for r) into seven 7-bit digits.
The digit sums S_j stay below 2^19.2 (37 bytes of at most 127 times 127),
S_2m + 2^7 S_(2m+1) below 2^26.3 fits 32 bits, P_hi = sum_{j>=3} S_j
2^(7(j-3)) stays below q, and one signed FP64 product by 2^21 plus one
centring give a representative of sum_a v_a hat_(a,t) - r D mod q_t of
absolute value at most q_t / 2 + 1.  Checked on the host with the same IEEE
operations against 128-bit integer arithmetic, for 1 to 4 sources of up to 63
bits and targets of 33 to 46 bits, random and extreme digits."""
import shutil
import subprocess

import pytest

SRC = r"""
#include <stdio.h>
#include <math.h>
typedef unsigned long long u64;
typedef unsigned __int128 u128;
static u64 s = 0x2545F4914F6CDD1Dull;
static u64 xr(void) { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return s; }
static double mms(double a, double w, double q, double qi) {
  double h = a * w, l = fma(a, w, -h), k = rint(h * qi);
  return fma(-k, q, h) + l;
}
static double centre(double x, double q, double qi) { return fma(-rint(x * qi), q, x); }
static u64 mulm(u64 a, u64 b, u64 q) { return (u64)((u128)a * b % q); }
int main(void) {
  long bad = 0, n = 0, bound = 0;
  for (int t = 0; t < 400; t++) {
    int ns = 1 + (int)(xr() % 4);
    u64 src[4];
    for (int a = 0; a < ns; a++) {
      int b = 30 + (int)(xr() % 34);                  /* 30 .. 63 bits */
      src[a] = ((1ull << (b - 1)) + (xr() % (1ull << (b - 1)))) | 1;
    }
    int qb = 33 + (int)(xr() % 14);                   /* 33 .. 46 bits */
    u64 q = ((1ull << (qb - 1)) + (xr() % (1ull << (qb - 1)))) | 1;
    if (t % 50 == 0) q = (1ull << qb) - 1;
    double qf = (double)q, qi = 1.0 / qf;
    u64 hat[4], D = 1, C[40] = {0};
    for (int a = 0; a < ns; a++) D = mulm(D, src[a] % q, q);
    for (int a = 0; a < ns; a++) {
      hat[a] = 1;
      for (int b = 0; b < ns; b++) if (b != a) hat[a] = mulm(hat[a], src[b] % q, q);
      for (int i = 0; i < 9; i++) C[9 * a + i] = mulm(hat[a], (u64)(((u128)1 << (7 * i)) % q), q);
    }
    C[9 * ns] = D == 0 ? 0 : q - D;
    for (int c = 0; c < 2000; c++) {
      u64 v[4], r = xr() % (u64)(ns + 1);
      for (int a = 0; a < ns; a++) {
        v[a] = xr() % src[a];
        if (c < 4) v[a] = c & 1 ? src[a] - 1 : 0;
      }
      if (c < 4) r = c & 2 ? (u64)ns : 0;
      int x[40] = {0};
      for (int a = 0; a < ns; a++)
        for (int i = 0; i < 9; i++) x[9 * a + i] = (int)((v[a] >> (7 * i)) & 127);
      x[9 * ns] = (int)r;
      int S[7];
      for (int j = 0; j < 7; j++) {
        long acc = 0;
        for (int k = 0; k <= 9 * ns; k++) acc += (long)x[k] * (long)((C[k] >> (7 * j)) & 127);
        if (acc >= 596774) bound++;
        S[j] = (int)acc;
      }
      int s01 = S[0] + (S[1] << 7), s34 = S[3] + (S[4] << 7), s56 = S[5] + (S[6] << 7);
      double ph = (double)s56 * 0x1p14 + (double)s34, pl = (double)S[2] * 0x1p14 + (double)s01;
      if (ph >= qf) bound++;
      double out = centre(mms(ph, 0x1p21, qf, qi) + pl, qf, qi);
      u128 want = 0;
      for (int a = 0; a < ns; a++) want += (u128)mulm(v[a] % q, hat[a], q);
      want = (want + (u128)q * ns - (u128)mulm(r, D, q)) % q;
      long long got = (long long)out;
      u64 gm = (u64)(((got % (long long)q) + (long long)q) % (long long)q);
      if ((double)got != out || gm != (u64)want || fabs(out) > qf / 2 + 1) bad++;
      n++;
    }
  }
  /* extreme digit sums: 37 bytes of 127 against constant digits of 127 */
  {
    long acc = 0;
    for (int k = 0; k < 37; k++) acc += 127L * 127L;
    if (acc >= 596774 || acc * 128 + acc >= (1L << 31)) bound++;
  }
  printf("%ld %ld %ld\n", bad, bound, n);
  return 0;
}
"""


def test_digit_lift_exact(tmp_path):
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "lift.c"
    src.write_text(SRC)
    exe = tmp_path / "lift"
    subprocess.run([cc, "-O2", "-mfma", "-ffp-contract=off", "-o", str(exe), str(src), "-lm"], check=True)
    bad, bound, n = map(int, subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split())
    assert bad == 0 and bound == 0 and n == 800000
