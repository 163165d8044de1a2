// Double-double arithmetic (value = hi + lo, |lo| <= ulp(hi)/2, ~106-bit significand)
// for the refinement stage, usable on the host (tests) and on the device.
//
// Building blocks, written from their published definitions:
//   two_sum        Knuth, TAOCP vol. 2, 4.2.2 (error-free sum, any operand order)
//   quick_two_sum  Dekker 1971 "Fast2Sum" (requires |a| >= |b| or a == 0)
//   two_prod       exact product via one fused multiply-add: p = a*b, e = fma(a, b, -p)
//   add/mul/div/sqrt  as in Hida, Li, Bailey, "Algorithms for quad-double precision
//                  floating point arithmetic" (ARITH 15, 2001), double-double case.
// The error-free transforms must not be contracted or reassociated, so every
// function that relies on exact cancellation turns FP contraction off.
#pragma once
#include <cmath>

#if defined(__HIPCC__) || defined(__HIP__)
#include <hip/hip_runtime.h>
#define DD_FN __host__ __device__ inline
#else
#define DD_FN inline
#endif

namespace dd {

struct ddr {
  double hi, lo;
};

DD_FN ddr two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b;
  const double bb = s - a;
  const double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}

DD_FN ddr quick_two_sum(double a, double b) {
#pragma clang fp contract(off)
  const double s = a + b;
  const double e = b - (s - a);
  return {s, e};
}

DD_FN ddr two_prod(double a, double b) {
#pragma clang fp contract(off)
  const double p = a * b;
  const double e = std::fma(a, b, -p);
  return {p, e};
}

DD_FN ddr from(double a) { return {a, 0.0}; }

DD_FN ddr neg(ddr a) { return {-a.hi, -a.lo}; }

// accurate ("IEEE") double-double addition
DD_FN ddr add(ddr a, ddr b) {
#pragma clang fp contract(off)
  ddr s = two_sum(a.hi, b.hi);
  ddr t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = quick_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return quick_two_sum(s.hi, s.lo);
}

DD_FN ddr sub(ddr a, ddr b) { return add(a, neg(b)); }

DD_FN ddr add_d(ddr a, double b) {
#pragma clang fp contract(off)
  ddr s = two_sum(a.hi, b);
  s.lo += a.lo;
  return quick_two_sum(s.hi, s.lo);
}

DD_FN ddr mul(ddr a, ddr b) {
  ddr p = two_prod(a.hi, b.hi);
  p.lo += a.hi * b.lo + a.lo * b.hi;
  return quick_two_sum(p.hi, p.lo);
}

DD_FN ddr mul_d(ddr a, double b) {
  ddr p = two_prod(a.hi, b);
  p.lo += a.lo * b;
  return quick_two_sum(p.hi, p.lo);
}

DD_FN ddr div(ddr a, ddr b) {
  const double q1 = a.hi / b.hi;
  ddr r = sub(a, mul_d(b, q1));
  const double q2 = r.hi / b.hi;
  r = sub(r, mul_d(b, q2));
  const double q3 = r.hi / b.hi;
  ddr q = quick_two_sum(q1, q2);
  return add_d(q, q3);
}

// sqrt by one Newton correction of the binary64 root: q + (a - q^2) / (2q)
DD_FN ddr sqrt(ddr a) {
  if (a.hi <= 0.0) return {0.0, 0.0};
  const double q = std::sqrt(a.hi);
  ddr r = sub(a, two_prod(q, q));
  return quick_two_sum(q, r.hi / (2.0 * q));
}

DD_FN bool lt(ddr a, ddr b) { return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo); }

// ------------------------------------------------------------------ complex dd
struct cdd {
  ddr re, im;
};

DD_FN cdd cfrom(double re, double im, double re_lo, double im_lo) { return {{re, re_lo}, {im, im_lo}}; }
DD_FN cdd cadd(cdd a, cdd b) { return {add(a.re, b.re), add(a.im, b.im)}; }
DD_FN cdd csub(cdd a, cdd b) { return {sub(a.re, b.re), sub(a.im, b.im)}; }
DD_FN cdd cconj(cdd a) { return {a.re, neg(a.im)}; }
DD_FN cdd cmul(cdd a, cdd b) {
  return {sub(mul(a.re, b.re), mul(a.im, b.im)), add(mul(a.re, b.im), mul(a.im, b.re))};
}
DD_FN cdd cscale(cdd a, ddr s) { return {mul(a.re, s), mul(a.im, s)}; }

// Multiply-accumulate with exact high products and binary64 cross terms:
// acc += a * b where the hi*hi products enter through two_prod / two_sum and the
// hi*lo + lo*hi terms (relatively 2^-53 smaller) in binary64.  acc.lo gathers the
// small parts and is folded in by norm() at the end of a sum.
struct acc {
  double hi, lo;
};

DD_FN void acc_add_prod(acc& s, double a, double b) {
#pragma clang fp contract(off)
  const ddr p = two_prod(a, b);
  const ddr t = two_sum(s.hi, p.hi);
  s.hi = t.hi;
  s.lo += t.lo + p.lo;
}

DD_FN void acc_add(acc& s, double x) {
#pragma clang fp contract(off)
  const ddr t = two_sum(s.hi, x);
  s.hi = t.hi;
  s.lo += t.lo;
}

DD_FN ddr norm(acc s) { return quick_two_sum(s.hi, s.lo); }

struct cacc {
  acc re, im;
};

// s += a * b (complex), a and b double-double
DD_FN void cacc_fma(cacc& s, cdd a, cdd b) {
  acc_add_prod(s.re, a.re.hi, b.re.hi);
  acc_add_prod(s.re, -a.im.hi, b.im.hi);
  acc_add_prod(s.im, a.re.hi, b.im.hi);
  acc_add_prod(s.im, a.im.hi, b.re.hi);
  // cross terms hi*lo + lo*hi in binary64, each pair as one rounded product and one
  // fused multiply-add, written out so that no compiler contraction choice changes them
  const double rr = std::fma(a.re.lo, b.re.hi, a.re.hi * b.re.lo);
  const double ii = std::fma(a.im.lo, b.im.hi, a.im.hi * b.im.lo);
  const double ri = std::fma(a.re.lo, b.im.hi, a.re.hi * b.im.lo);
  const double ir = std::fma(a.im.lo, b.re.hi, a.im.hi * b.re.lo);
  s.re.lo += rr - ii;
  s.im.lo += ri + ir;
}

// s += conj(a) * b
DD_FN void cacc_fmac(cacc& s, cdd a, cdd b) { cacc_fma(s, cconj(a), b); }

DD_FN cdd cnorm(cacc s) { return {norm(s.re), norm(s.im)}; }

}  // namespace dd
