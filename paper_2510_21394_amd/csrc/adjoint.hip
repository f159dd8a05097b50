// Pointwise passes of the discrete adjoint of exponential Euler.
//
// Forward step (eigenspace form, Q = Q_1 x ... x Q_d real orthogonal, z = tau (nu + i eta) ell):
//     u_{n+1} = Q (E o Q^T u_n + tau P1 o Q^T g(t_n, u_n)),   E = e^z, P1 = phi_1(z).
// For a real loss and the cotangent convention ubar = dL/dRe u + i dL/dIm u, with the adjoint
// state kept in eigenspace (ahat_n = Q^T ubar_n), one adjoint step is
//     w       = Q (tau conj(P1) o ahat_{n+1})                          (backward Tucker)
//     q       = (gamma - 2 conj(c)|u_n|^2) w - c u_n^2 conj(w)          (adjoint of the
//               R-linear derivative of g(u) = gamma u - c |u|^2 u, c = kappa + i zeta)
//     ahat_n  = conj(E) o ahat_{n+1} + Q^T q                           (forward Tucker)
// and the parameter cotangents are
//     gamma: Re sum conj(w) u_n,  kappa: Re sum conj(w)(-|u_n|^2 u_n),
//     zeta:  Re sum conj(w)(-i |u_n|^2 u_n),
//     nu:    Re S,  eta: -Im S,  S = sum conj(ahat_{n+1}) tau ell X_n,
// where X_n = e^z uhat_n + tau phi_1'(z) ghat_n is recorded by the forward recompute.
//
// Sums are formed in FP64 per tensor row (the tensor viewed as (rows, nlast)) by one
// workgroup and added to that row's slot of `partial`; a single reduction over rows at the
// end keeps the result independent of scheduling.
#include "dispatch.hpp"

namespace fcgle {

namespace {

constexpr int kAdjThreads = 256;
constexpr int kAdjWaves = kAdjThreads / 64;
constexpr int kMaxRowBlocks = 65536;

inline unsigned row_blocks(int64_t rows) { return (unsigned)(rows < kMaxRowBlocks ? rows : kMaxRowBlocks); }

// Separable factor and eigenvalue sum over the axes slower than the last one, for row r.
struct RowCtx {
  zc E;
  double ell;
};

__device__ __forceinline__ RowCtx row_ctx(const SepParams& s, int64_t r) {
  RowCtx c{{1.0, 0.0}, 0.0};
  for (int nu = s.d - 2; nu >= 0; --nu) {
    const int64_t jn = r % s.n[nu];
    r /= s.n[nu];
    c.E = zmul(c.E, ((const zc*)s.fac[nu])[jn]);
    c.ell += s.lam[nu][jn];
  }
  return c;
}

// Sums W values over the workgroup and adds the totals to dst[0..W-1] (thread 0).
template <int W>
__device__ __forceinline__ void block_add(double (&v)[W], double (*sh)[W], double* dst) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < W; ++k)
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_down(v[k], off, 64);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < W; ++k) sh[wave][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < W; ++k) {
      double t = 0.0;
      for (int w = 0; w < kAdjWaves; ++w) t += sh[w][k];
      dst[k] += t;
    }
  __syncthreads();
}

__global__ void __launch_bounds__(kAdjThreads) fill_zero_kernel(double* x, int64_t count) {
  for (int64_t j = blockIdx.x * (int64_t)kAdjThreads + threadIdx.x; j < count; j += (int64_t)gridDim.x * kAdjThreads)
    x[j] = 0.0;
}

template <class C>
__global__ void __launch_bounds__(kAdjThreads)
    adj_init_kernel(int64_t N, const C* __restrict__ ahat, const C* __restrict__ P1, double tau, C* __restrict__ p) {
  for (int64_t j = blockIdx.x * (int64_t)kAdjThreads + threadIdx.x; j < N; j += (int64_t)gridDim.x * kAdjThreads) {
    const zc a = to_zc(ahat[j]), f = to_zc(P1[j]);
    p[j] = from_zc<C>(zscale(zmul(zc{f.re, -f.im}, a), tau));
  }
}

template <class C>
__global__ void __launch_bounds__(kAdjThreads)
    adj_phys_kernel(int64_t rows, int nlast, C* __restrict__ wq, const C* __restrict__ u, double gamma, double kre,
                    double kim, double* __restrict__ partial) {
  __shared__ double sh[kAdjWaves][3];
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
    double acc[3] = {0.0, 0.0, 0.0};
    const int64_t base = r * nlast;
    for (int i = threadIdx.x; i < nlast; i += kAdjThreads) {
      const zc w = to_zc(wq[base + i]), x = to_zc(u[base + i]);
      const double m = x.re * x.re + x.im * x.im;
      // (gamma - 2 conj(c) m) w
      const zc a{gamma - 2.0 * m * kre, 2.0 * m * kim};
      // c u^2 conj(w)
      const zc cu2 = zmul(zc{kre, kim}, zmul(x, x));
      const zc q = zsub(zmul(a, w), zmul(cu2, zc{w.re, -w.im}));
      wq[base + i] = from_zc<C>(q);
      const double rw = w.re * x.re + w.im * x.im;  // Re conj(w) u
      acc[0] += rw;
      acc[1] -= m * rw;
      acc[2] += m * (w.re * x.im - w.im * x.re);  // Re conj(w) (-i m u)
    }
    block_add<3>(acc, sh, partial + r * 5 + 2);
  }
}

template <class C>
__global__ void __launch_bounds__(kAdjThreads)
    adj_hat_kernel(int64_t rows, int nlast, const C* __restrict__ v, C* __restrict__ ahat, C* __restrict__ p,
                   const C* __restrict__ X, const C* __restrict__ P1, SepParams s, double tau,
                   double* __restrict__ partial) {
  __shared__ double sh[kAdjWaves][2];
  const zc* fl = (const zc*)s.fac[s.d - 1];
  const double* ll = s.lam[s.d - 1];
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
    const RowCtx c = row_ctx(s, r);
    double acc[2] = {0.0, 0.0};
    const int64_t base = r * nlast;
    for (int i = threadIdx.x; i < nlast; i += kAdjThreads) {
      const int64_t j = base + i;
      const zc a = to_zc(ahat[j]), x = to_zc(X[j]), vv = to_zc(v[j]), f = to_zc(P1[j]);
      const zc E = zmul(c.E, fl[i]);
      const double te = tau * (c.ell + ll[i]);
      const zc sx = zmul(zc{a.re, -a.im}, x);  // conj(a) X
      acc[0] += te * sx.re;
      acc[1] -= te * sx.im;
      const zc an = zadd(zmul(zc{E.re, -E.im}, a), vv);
      ahat[j] = from_zc<C>(an);
      p[j] = from_zc<C>(zscale(zmul(zc{f.re, -f.im}, an), tau));
    }
    block_add<2>(acc, sh, partial + r * 5);
  }
}

inline unsigned flat_blocks(int64_t N) {
  int64_t b = (N + kAdjThreads - 1) / kAdjThreads;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

hipError_t launch_fill_zero(double* x, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(fill_zero_kernel, dim3(flat_blocks(count)), dim3(kAdjThreads), 0, s, x, count);
  return hipGetLastError();
}

hipError_t launch_adj_init(int prec, int64_t N, const void* ahat, const void* P1, double tau, void* p,
                           hipStream_t s) {
  if (prec == P_F64)
    hipLaunchKernelGGL((adj_init_kernel<double2>), dim3(flat_blocks(N)), dim3(kAdjThreads), 0, s, N,
                       (const double2*)ahat, (const double2*)P1, tau, (double2*)p);
  else
    hipLaunchKernelGGL((adj_init_kernel<float2>), dim3(flat_blocks(N)), dim3(kAdjThreads), 0, s, N,
                       (const float2*)ahat, (const float2*)P1, tau, (float2*)p);
  return hipGetLastError();
}

hipError_t launch_adj_phys(int prec, int64_t N, int nlast, void* wq, const void* u, double gamma, double kappa,
                           double zeta, double* partial, hipStream_t s) {
  const int64_t rows = N / nlast;
  if (prec == P_F64)
    hipLaunchKernelGGL((adj_phys_kernel<double2>), dim3(row_blocks(rows)), dim3(kAdjThreads), 0, s, rows, nlast,
                       (double2*)wq, (const double2*)u, gamma, kappa, zeta, partial);
  else
    hipLaunchKernelGGL((adj_phys_kernel<float2>), dim3(row_blocks(rows)), dim3(kAdjThreads), 0, s, rows, nlast,
                       (float2*)wq, (const float2*)u, gamma, kappa, zeta, partial);
  return hipGetLastError();
}

hipError_t launch_adj_hat(int prec, int64_t N, int nlast, const void* v, void* ahat, void* p, const void* X,
                          const void* P1, const SepParams& sep, double tau, double* partial, hipStream_t s) {
  const int64_t rows = N / nlast;
  if (prec == P_F64)
    hipLaunchKernelGGL((adj_hat_kernel<double2>), dim3(row_blocks(rows)), dim3(kAdjThreads), 0, s, rows, nlast,
                       (const double2*)v, (double2*)ahat, (double2*)p, (const double2*)X, (const double2*)P1, sep,
                       tau, partial);
  else
    hipLaunchKernelGGL((adj_hat_kernel<float2>), dim3(row_blocks(rows)), dim3(kAdjThreads), 0, s, rows, nlast,
                       (const float2*)v, (float2*)ahat, (float2*)p, (const float2*)X, (const float2*)P1, sep, tau,
                       partial);
  return hipGetLastError();
}

}  // namespace fcgle
