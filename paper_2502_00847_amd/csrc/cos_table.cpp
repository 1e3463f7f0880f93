// Host table of cos(pi t / N), t < 2N, as double-double pairs (hi, lo) for the
// canonical-embedding encoder.  Evaluated in binary128 (libquadmath) and split.
#include <quadmath.h>
#include <stddef.h>

extern "C" void secpe_cos_table_dd(int log_n, double* hi, double* lo) {
  const long n = 1L << log_n;
  for (long t = 0; t < 2 * n; ++t) {
    const __float128 c = cosq(M_PIq * (__float128)t / (__float128)n);
    const double h = (double)c;
    hi[t] = h;
    lo[t] = (double)(c - (__float128)h);
  }
}
