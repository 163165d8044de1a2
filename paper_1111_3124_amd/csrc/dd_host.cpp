// Host build of dd.h for the CPU test-suite: element-wise double-double operations
// on arrays, so the error-free transforms can be checked against high precision.
#include "dd.h"

extern "C" {

// op: 0 add, 1 sub, 2 mul, 3 div, 4 sqrt(a), 5 two_prod(a.hi, b.hi), 6 two_sum(a.hi, b.hi)
// a, b, out: n pairs (hi, lo)
int dd_host_op(int op, long n, const double* a, const double* b, double* out) {
  for (long i = 0; i < n; ++i) {
    const dd::ddr x = {a[2 * i], a[2 * i + 1]}, y = {b[2 * i], b[2 * i + 1]};
    dd::ddr r;
    switch (op) {
      case 0: r = dd::add(x, y); break;
      case 1: r = dd::sub(x, y); break;
      case 2: r = dd::mul(x, y); break;
      case 3: r = dd::div(x, y); break;
      case 4: r = dd::sqrt(x); break;
      case 5: r = dd::two_prod(x.hi, y.hi); break;
      case 6: r = dd::two_sum(x.hi, y.hi); break;
      default: return -1;
    }
    out[2 * i] = r.hi;
    out[2 * i + 1] = r.lo;
  }
  return 0;
}

// complex multiply-accumulate of n terms: sum_i a_i * b_i, (re_hi, re_lo, im_hi, im_lo) each
int dd_host_cdot(long n, const double* a, const double* b, double* out) {
  dd::cacc s = {{0.0, 0.0}, {0.0, 0.0}};
  for (long i = 0; i < n; ++i) {
    const dd::cdd x = {{a[4 * i], a[4 * i + 1]}, {a[4 * i + 2], a[4 * i + 3]}};
    const dd::cdd y = {{b[4 * i], b[4 * i + 1]}, {b[4 * i + 2], b[4 * i + 3]}};
    dd::cacc_fma(s, x, y);
  }
  const dd::cdd r = dd::cnorm(s);
  out[0] = r.re.hi; out[1] = r.re.lo; out[2] = r.im.hi; out[3] = r.im.lo;
  return 0;
}
}
