// Scalar matrix functions f(z) in FP64, shared by the host helper and the device
// f-grid kernel so that both evaluate exactly the same code.
//   kind 0: 1/(1 - z)        (linearly implicit steps)
//   kind 1: e^z              (phi_0)
//   kind 1 + l: phi_l(z)     (Section 4, eq. phi: phi_l = (phi_{l-1} - 1/(l-1)!)/z, phi_l(0) = 1/l!)
// phi_l cancels badly for small |z| when taken from the recurrence, so for |z| < 1
// it is summed from its Taylor series sum_{k>=0} z^k/(k+l)! (26 terms: the first
// neglected term is below 1e-26 there); elsewhere the recurrence is used.
#pragma once

#include <cmath>

#if defined(__HIPCC__)
#define FCGLE_HD __host__ __device__
#else
#define FCGLE_HD
#endif

namespace fcgle {

struct zc {
  double re, im;
};

FCGLE_HD inline zc zadd(zc a, zc b) { return {a.re + b.re, a.im + b.im}; }
FCGLE_HD inline zc zsub(zc a, zc b) { return {a.re - b.re, a.im - b.im}; }
FCGLE_HD inline zc zmul(zc a, zc b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
FCGLE_HD inline zc zscale(zc a, double s) { return {a.re * s, a.im * s}; }

// a / b by Smith's scaling (avoids overflow of |b|^2).
FCGLE_HD inline zc zdiv(zc a, zc b) {
  if (fabs(b.re) >= fabs(b.im)) {
    const double r = b.im / b.re, den = b.re + b.im * r;
    return {(a.re + a.im * r) / den, (a.im - a.re * r) / den};
  }
  const double r = b.re / b.im, den = b.re * r + b.im;
  return {(a.re * r + a.im) / den, (a.im * r - a.re) / den};
}

FCGLE_HD inline zc zexp(zc z) {
  const double e = exp(z.re);
  return {e * cos(z.im), e * sin(z.im)};
}

FCGLE_HD inline zc fz_eval(int kind, zc z) {
  if (kind == 0) return zdiv(zc{1.0, 0.0}, zc{1.0 - z.re, -z.im});
  if (kind == 1) return zexp(z);
  const int l = kind - 1;
  if (z.re * z.re + z.im * z.im < 1.0) {
    constexpr int kTerms = 26;
    double c[kTerms];
    double c0 = 1.0;  // 1/l!
    for (int m = 2; m <= l; ++m) c0 /= (double)m;
    c[0] = c0;
#pragma unroll
    for (int k = 1; k < kTerms; ++k) c[k] = c[k - 1] / (double)(k + l);
    zc acc{c[kTerms - 1], 0.0};
#pragma unroll
    for (int k = kTerms - 2; k >= 0; --k) {
      acc = zmul(acc, z);
      acc.re += c[k];
    }
    return acc;
  }
  zc p = zexp(z);
  double inv_fact = 1.0;  // 1/(j-1)!
  for (int j = 1; j <= l; ++j) {
    if (j > 1) inv_fact /= (double)(j - 1);
    p = zdiv(zc{p.re - inv_fact, p.im}, z);
  }
  return p;
}

}  // namespace fcgle
