// Host-only table generation that needs quad precision (built with g++).
#include <quadmath.h>

namespace {
void split(__float128 x, double* out) {
  double hi = (double)x;
  out[0] = hi;
  out[1] = (double)(x - (__float128)hi);
}
}  // namespace

// fft_tw[k] = exp(-2 pi i k / N) for k < N/2, zeta[i] = (cos(pi i/N), sin(pi i/N))
// for i < N; each complex number stored as double-double (re_hi, re_lo, im_hi, im_lo).
extern "C" void he_host_dd_tables(int logN, double* fft_tw, double* zeta) {
  const long N = 1L << logN;
  for (long k = 0; k < N / 2; k++) {
    __float128 ang = 2 * M_PIq * (__float128)k / (__float128)N;
    split(cosq(ang), fft_tw + 4 * k);
    split(-sinq(ang), fft_tw + 4 * k + 2);
  }
  for (long i = 0; i < N; i++) {
    __float128 ang = M_PIq * (__float128)i / (__float128)N;
    split(cosq(ang), zeta + 4 * i);
    split(sinq(ang), zeta + 4 * i + 2);
  }
}
