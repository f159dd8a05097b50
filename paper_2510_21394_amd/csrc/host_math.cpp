// Host-side FP64 numerics of the plan set-up (see host_math.h).
#include "host_math.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <numeric>

namespace fcgle {

// Section 2: g_0 = Gamma(alpha+1)/Gamma(alpha/2+1)^2, g_k = (1 - (alpha+1)/(alpha/2+k)) g_{k-1}.
// Order 4 (eq. FD4): 4/3 g_k, minus g_{k/2}/(3 * 2^alpha) for even k.
std::vector<double> fd_weights(double alpha, int64_t n, int fd_order) {
  std::vector<double> g(n);
  g[0] = std::tgamma(alpha + 1.0) / (std::tgamma(alpha / 2.0 + 1.0) * std::tgamma(alpha / 2.0 + 1.0));
  for (int64_t k = 1; k < n; ++k) g[k] = (1.0 - (alpha + 1.0) / (alpha / 2.0 + (double)k)) * g[k - 1];
  if (fd_order == 4) {
    std::vector<double> c(n);
    const double s = 1.0 / (3.0 * std::pow(2.0, alpha));
    for (int64_t k = 0; k < n; ++k) c[k] = (4.0 / 3.0) * g[k] - ((k % 2 == 0) ? s * g[k / 2] : 0.0);
    return c;
  }
  return g;
}

// --- symmetric eigensolver ----------------------------------------------------------------
//
// Stage 1: Householder reduction A = P T P^T with T tridiagonal.  For column k the
// reflector H = I - beta v v^T maps A[k+1:, k] onto a multiple of e_1; the trailing block
// is updated as A22 <- A22 - v w^T - w v^T with p = beta A22 v, w = p - (beta/2)(p^T v) v.
// P = H_0 H_1 ... H_{n-3} is formed afterwards by applying the reflectors in reverse.
//
// Stage 2: implicit symmetric QR with the Wilkinson shift on the unreduced trailing
// block [l, m]: a rotation in plane (k, k+1) chosen from the shifted first column starts a
// bulge that successive rotations chase down the band.  Rotations are accumulated into
// Z = P^T (rows = eigenvectors), so each update touches two contiguous rows.

namespace {

void tridiagonalize(int64_t n, std::vector<double>& A, std::vector<double>& d, std::vector<double>& e,
                    std::vector<double>& P) {
  d.assign(n, 0.0);
  e.assign(n > 1 ? n - 1 : 0, 0.0);
  std::vector<double> betas(n, 0.0);
  std::vector<double> p(n), w(n);
  auto a = [&](int64_t i, int64_t j) -> double& { return A[i * n + j]; };
  for (int64_t k = 0; k + 2 < n; ++k) {
    const int64_t m = n - k - 1;
    double* v = &A[(k + 1) * n + k];  // strided column; copy for clarity
    std::vector<double> x(m);
    for (int64_t i = 0; i < m; ++i) x[i] = a(k + 1 + i, k);
    double sigma = 0.0;
    for (int64_t i = 1; i < m; ++i) sigma += x[i] * x[i];
    if (sigma == 0.0) {  // already reduced in this column
      betas[k] = 0.0;
      e[k] = x[0];
      for (int64_t i = 0; i < m; ++i) a(k + 1 + i, k) = 0.0;
      continue;
    }
    const double norm = std::sqrt(x[0] * x[0] + sigma);
    const double alpha_h = (x[0] >= 0.0) ? -norm : norm;
    x[0] -= alpha_h;
    const double vtv = x[0] * x[0] + sigma;
    const double beta = 2.0 / vtv;
    // p = beta * A22 x  (A22 symmetric; use full storage)
    for (int64_t i = 0; i < m; ++i) {
      const double* row = &A[(k + 1 + i) * n + (k + 1)];
      double s = 0.0;
      for (int64_t j = 0; j < m; ++j) s += row[j] * x[j];
      p[i] = beta * s;
    }
    double ptv = 0.0;
    for (int64_t i = 0; i < m; ++i) ptv += p[i] * x[i];
    const double K = 0.5 * beta * ptv;
    for (int64_t i = 0; i < m; ++i) w[i] = p[i] - K * x[i];
    for (int64_t i = 0; i < m; ++i) {
      double* row = &A[(k + 1 + i) * n + (k + 1)];
      const double xi = x[i], wi = w[i];
      for (int64_t j = 0; j < m; ++j) row[j] -= xi * w[j] + wi * x[j];
    }
    e[k] = alpha_h;
    betas[k] = beta;
    // keep the reflector in the (now eliminated) column below the diagonal
    for (int64_t i = 0; i < m; ++i) a(k + 1 + i, k) = x[i];
    (void)v;
  }
  if (n >= 2) e[n - 2] = a(n - 1, n - 2);
  for (int64_t i = 0; i < n; ++i) d[i] = a(i, i);
  // P = H_0 H_1 ... H_{n-3}: apply in reverse to the identity, each touching rows/cols > k.
  P.assign(n * n, 0.0);
  for (int64_t i = 0; i < n; ++i) P[i * n + i] = 1.0;
  std::vector<double> t(n);
  for (int64_t k = n - 3; k >= 0; --k) {
    const double beta = betas[k];
    if (beta == 0.0) continue;
    const int64_t m = n - k - 1;
    // t^T = v^T P22   (P22 = P[k+1:, k+1:])
    std::fill(t.begin(), t.begin() + m, 0.0);
    for (int64_t i = 0; i < m; ++i) {
      const double vi = a(k + 1 + i, k);
      if (vi == 0.0) continue;
      const double* row = &P[(k + 1 + i) * n + (k + 1)];
      for (int64_t j = 0; j < m; ++j) t[j] += vi * row[j];
    }
    for (int64_t i = 0; i < m; ++i) {
      const double f = beta * a(k + 1 + i, k);
      if (f == 0.0) continue;
      double* row = &P[(k + 1 + i) * n + (k + 1)];
      for (int64_t j = 0; j < m; ++j) row[j] -= f * t[j];
    }
  }
}

inline void rotate_rows(double* zi, double* zj, int64_t n, double c, double s) {
  // zi' = c zi - s zj ; zj' = s zi + c zj
  for (int64_t q = 0; q < n; ++q) {
    const double a = zi[q], b = zj[q];
    zi[q] = c * a - s * b;
    zj[q] = s * a + c * b;
  }
}

bool tridiag_qr(int64_t n, std::vector<double>& d, std::vector<double>& e, std::vector<double>& Z) {
  const double eps = std::numeric_limits<double>::epsilon();
  int64_t m = n - 1;
  int64_t iters = 0;
  const int64_t max_iters = 60 * n + 100;
  while (m > 0) {
    // deflate negligible off-diagonals
    for (int64_t i = 0; i < m; ++i)
      if (std::fabs(e[i]) <= eps * (std::fabs(d[i]) + std::fabs(d[i + 1]))) e[i] = 0.0;
    if (e[m - 1] == 0.0) {
      --m;
      continue;
    }
    int64_t l = m - 1;
    while (l > 0 && e[l - 1] != 0.0) --l;
    if (++iters > max_iters) return false;
    // Wilkinson shift from the trailing 2x2 [[d_{m-1}, e_{m-1}], [e_{m-1}, d_m]]
    const double dd = 0.5 * (d[m - 1] - d[m]);
    const double b = e[m - 1];
    const double r = std::hypot(dd, b);
    const double mu = d[m] - b * b / (dd + (dd >= 0.0 ? r : -r));
    double x = d[l] - mu;
    double z = e[l];
    for (int64_t k = l; k < m; ++k) {
      // rotation G with G^T [x; z] = [r; 0]:  c = x/r, s = -z/r
      double rr = std::hypot(x, z);
      double c, s;
      if (rr == 0.0) {
        c = 1.0;
        s = 0.0;
      } else {
        c = x / rr;
        s = -z / rr;
      }
      if (k > l) e[k - 1] = rr;  // T'[k-1][k]; the bulge at [k-1][k+1] becomes 0
      const double dk = d[k], dk1 = d[k + 1], ek = e[k];
      d[k] = c * c * dk - 2.0 * c * s * ek + s * s * dk1;
      d[k + 1] = s * s * dk + 2.0 * c * s * ek + c * c * dk1;
      e[k] = c * s * (dk - dk1) + (c * c - s * s) * ek;
      if (k + 1 < m) {
        const double ek1 = e[k + 1];
        z = -s * ek1;      // new bulge at [k][k+2]
        e[k + 1] = c * ek1;
        x = e[k];
      }
      rotate_rows(&Z[k * n], &Z[(k + 1) * n], n, c, s);
    }
  }
  return true;
}

}  // namespace

bool sym_eig(int64_t n, std::vector<double>& A, std::vector<double>& Q, std::vector<double>& lambda) {
  if (n == 1) {
    lambda.assign(1, A[0]);
    Q.assign(1, 1.0);
    return true;
  }
  std::vector<double> d, e, P;
  tridiagonalize(n, A, d, e, P);
  // Z = P^T
  std::vector<double> Z(n * n);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) Z[i * n + j] = P[j * n + i];
  if (!tridiag_qr(n, d, e, Z)) return false;
  std::vector<int64_t> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return d[a] < d[b]; });
  lambda.resize(n);
  Q.assign(n * n, 0.0);
  for (int64_t k = 0; k < n; ++k) {
    const int64_t src = order[k];
    lambda[k] = d[src];
    for (int64_t i = 0; i < n; ++i) Q[i * n + k] = Z[src * n + i];
  }
  return true;
}

// Stateless steps apply Q f(theta Lambda) Q^T every step, so a loss of orthogonality of Q
// (a few 1e-15 from the FP64 solver) would add up over the steps.  One Newton-Schulz sweep
// towards the orthogonal polar factor, X <- X + X (I - X^T X) / 2, carried out in x87 long
// double, brings Q^T Q = I to the rounding of the final FP64 entries; the eigenvalues are
// then taken as Rayleigh quotients lambda_c = x_c^T D x_c in the same precision.
void orthogonalize_extended(int64_t n, const std::vector<double>& D, std::vector<double>& Q,
                            std::vector<double>& lambda) {
  using ld = long double;
  std::vector<ld> X(Q.begin(), Q.end());  // row-major n x n
  std::vector<ld> XT(n * n);
  for (int64_t r = 0; r < n; ++r)
    for (int64_t c = 0; c < n; ++c) XT[c * n + r] = X[r * n + c];
  // H = I - X^T X  (symmetric; rows of XT are the columns of X)
  std::vector<ld> H(n * n);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = i; j < n; ++j) {
      const ld* a = &XT[i * n];
      const ld* b = &XT[j * n];
      ld s = 0;
      for (int64_t k = 0; k < n; ++k) s += a[k] * b[k];
      const ld v = (i == j ? (ld)1 : (ld)0) - s;
      H[i * n + j] = v;
      H[j * n + i] = v;
    }
  // Xn = X + X H / 2
  std::vector<ld> Xn(X);
  for (int64_t r = 0; r < n; ++r) {
    ld* out = &Xn[r * n];
    for (int64_t k = 0; k < n; ++k) {
      const ld f = X[r * n + k] / 2;
      const ld* hr = &H[k * n];
      for (int64_t c = 0; c < n; ++c) out[c] += f * hr[c];
    }
  }
  // Y = D Xn, lambda_c = sum_r Xn[r][c] Y[r][c]
  std::vector<ld> Y(n * n, 0);
  for (int64_t r = 0; r < n; ++r) {
    ld* y = &Y[r * n];
    for (int64_t k = 0; k < n; ++k) {
      const ld f = (ld)D[r * n + k];
      const ld* xr = &Xn[k * n];
      for (int64_t c = 0; c < n; ++c) y[c] += f * xr[c];
    }
  }
  std::vector<ld> lam(n, 0);
  for (int64_t r = 0; r < n; ++r)
    for (int64_t c = 0; c < n; ++c) lam[c] += Xn[r * n + c] * Y[r * n + c];
  for (int64_t i = 0; i < n * n; ++i) Q[i] = (double)Xn[i];
  for (int64_t c = 0; c < n; ++c) lambda[c] = (double)lam[c];
}

bool toeplitz_eig(int64_t n, double alpha, double h, int fd_order, std::vector<double>& Q,
                  std::vector<double>& lambda) {
  const std::vector<double> g = fd_weights(alpha, n, fd_order);
  const double scale = -std::pow(h, -alpha);
  std::vector<double> A(n * n);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < n; ++j) A[i * n + j] = scale * g[i > j ? i - j : j - i];
  const std::vector<double> D(A);
  if (!sym_eig(n, A, Q, lambda)) return false;
  orthogonalize_extended(n, D, Q, lambda);
  return true;
}

namespace {

// One Newton-Schulz sweep X <- X + X (I - X^T X) / 2 of the m x m block eigenvector matrix
// V (row-major, columns = eigenvectors) in long double, and Rayleigh quotients
// lam_c = x_c^T A x_c with the block A given in long double.
void sweep_block(int64_t m, const std::vector<double>& V, const std::vector<long double>& A,
                 std::vector<long double>& X, std::vector<long double>& lam) {
  using ld = long double;
  X.assign(V.begin(), V.end());
  std::vector<ld> H(m * m);
  for (int64_t i = 0; i < m; ++i)
    for (int64_t j = i; j < m; ++j) {
      ld acc = 0;
      for (int64_t k = 0; k < m; ++k) acc += X[k * m + i] * X[k * m + j];
      const ld v = (i == j ? (ld)1 : (ld)0) - acc;
      H[i * m + j] = v;
      H[j * m + i] = v;
    }
  std::vector<ld> Xn(X);
  for (int64_t r = 0; r < m; ++r)
    for (int64_t k = 0; k < m; ++k) {
      const ld f = X[r * m + k] / 2;
      for (int64_t c = 0; c < m; ++c) Xn[r * m + c] += f * H[k * m + c];
    }
  lam.assign(m, 0);
  for (int64_t r = 0; r < m; ++r)
    for (int64_t k = 0; k < m; ++k) {
      const ld a = A[r * m + k];
      for (int64_t c = 0; c < m; ++c) lam[c] += Xn[r * m + c] * a * Xn[k * m + c];
    }
  X.swap(Xn);
}

}  // namespace

bool toeplitz_eig_split(int64_t n, double alpha, double h, int fd_order, SplitEig& s) {
  using ld = long double;
  const std::vector<double> g = fd_weights(alpha, n, fd_order);
  const double scale = -std::pow(h, -alpha);
  std::vector<double> t(n);
  for (int64_t k = 0; k < n; ++k) t[k] = scale * g[k];
  const int64_t m = n / 2, me = n - m, mo = m;
  s.n = n;
  s.me = me;
  s.mo = mo;
  // the blocks in long double (the sums of two doubles are exact there) and in double
  const ld sq2 = std::sqrt((ld)2);
  std::vector<ld> Ae(me * me), Ao(mo * mo);
  for (int64_t i = 0; i < m; ++i)
    for (int64_t k = 0; k < m; ++k) {
      const ld a = t[i > k ? i - k : k - i], b = t[n - 1 - i - k];
      Ae[i * me + k] = a + b;
      Ao[i * mo + k] = a - b;
    }
  if (me > m) {  // odd n: the middle point belongs to the even block
    for (int64_t i = 0; i < m; ++i) Ae[i * me + m] = Ae[m * me + i] = sq2 * (ld)t[m - i];
    Ae[m * me + m] = t[0];
  }
  std::vector<double> De(Ae.begin(), Ae.end()), Do(Ao.begin(), Ao.end());
  std::vector<double> Ve, le, Vo, lo;
  if (!sym_eig(me, De, Ve, le)) return false;
  if (mo > 0 && !sym_eig(mo, Do, Vo, lo)) return false;
  std::vector<ld> Xe, Xo, lame, lamo;
  sweep_block(me, Ve, Ae, Xe, lame);
  if (mo > 0) sweep_block(mo, Vo, Ao, Xo, lamo);
  // Q = Z diag(Xe, Xo), rounded once from long double, with the mirror entries copied so the
  // even/odd structure holds exactly in FP64
  const ld r2 = 1 / sq2;
  s.Q.assign(n * n, 0.0);
  s.lam.resize(n);
  for (int64_t k = 0; k < me; ++k) {
    s.lam[k] = (double)lame[k];
    for (int64_t i = 0; i < m; ++i) s.Q[i * n + k] = s.Q[(n - 1 - i) * n + k] = (double)(r2 * Xe[i * me + k]);
    if (me > m) s.Q[m * n + k] = (double)Xe[m * me + k];
  }
  for (int64_t k = 0; k < mo; ++k) {
    s.lam[me + k] = (double)lamo[k];
    for (int64_t i = 0; i < m; ++i) {
      const double v = (double)(r2 * Xo[i * mo + k]);
      s.Q[i * n + me + k] = v;
      s.Q[(n - 1 - i) * n + me + k] = -v;
    }
  }
  return true;
}

void split_block_matrices(int64_t n, int64_t me, int64_t mo, const std::vector<double>& Q, int64_t ld,
                          std::vector<double>& F, std::vector<double>& B) {
  const int64_t m = n / 2;
  F.assign(2 * ld * ld, 0.0);
  B.assign(2 * ld * ld, 0.0);
  for (int64_t i = 0; i < me; ++i)
    for (int64_t k = 0; k < me; ++k) {
      F[i * ld + k] = (k < m) ? Q[k * n + i] : 0.5 * Q[m * n + i];
      B[i * ld + k] = Q[i * n + k];
    }
  for (int64_t i = 0; i < mo; ++i)
    for (int64_t k = 0; k < mo; ++k) {
      F[ld * ld + i * ld + k] = Q[k * n + me + i];
      B[ld * ld + i * ld + k] = Q[i * n + me + k];
    }
}

// --- bfloat16 ----------------------------------------------------------------------------

uint16_t bf16_round(double x) {
  if (x == 0.0 || !std::isfinite(x)) {
    float f = (float)x;
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return (uint16_t)(u >> 16);
  }
  int ex;
  std::frexp(x, &ex);  // x = m 2^ex, 0.5 <= |m| < 1
  // bf16 keeps 8 significant bits: round x * 2^(8 - ex) to an integer, ties to even
  const double scaled = std::ldexp(x, 8 - ex);
  const double r = std::nearbyint(scaled);  // default rounding mode: to nearest even
  const double y = std::ldexp(r, ex - 8);
  const float f = (float)y;  // exact: y has <= 8 significant bits in float range
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return (uint16_t)(u >> 16);
}

double bf16_value(uint16_t b) {
  uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return (double)f;
}

}  // namespace fcgle
