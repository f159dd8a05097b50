// Eigenspace stage combinations of Krogstad's fourth-order exponential integrator (Section 4,
// eq. krogstad-v): one streaming pass per stage,
//   out[j] = E_j uh[j] + sum_{t < nt} F_t[j] (sum_{m < 5} c[t][m] v_m[j]),
// in FP64 arithmetic on operands stored in the state precision.  E is the separable
// exponential (per-axis FP64 factors, never stored as a grid); F_t are phi-function grids.
#include "kernels.hpp"

namespace fcgle {

namespace {

constexpr int kCombThreads = 256;

template <class C>
struct CombArgs {
  const C* uh;
  const C* F[3];
  const C* v[5];
  double c[3][5];
  int nt;
  SepParams sep;
  C* out;
};

template <class C>
__global__ void __launch_bounds__(kCombThreads) comb_kernel(int64_t N, int nlast, CombArgs<C> a) {
  for (int64_t j = blockIdx.x * (int64_t)kCombThreads + threadIdx.x; j < N; j += (int64_t)gridDim.x * kCombThreads) {
    zc acc{0.0, 0.0};
    if (a.uh) {
      const uint32_t row = (uint32_t)(j / nlast);
      const int i = (int)(j - (int64_t)row * nlast);
      const zc E = zmul(sep_other(a.sep, row, 0), ((const zc*)a.sep.fac[a.sep.mu])[i]);
      acc = zmul(E, to_zc(a.uh[j]));
    }
    zc v[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) v[m] = a.v[m] ? to_zc(a.v[m][j]) : zc{0.0, 0.0};
    for (int t = 0; t < a.nt; ++t) {
      zc s{0.0, 0.0};
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        s.re += a.c[t][m] * v[m].re;
        s.im += a.c[t][m] * v[m].im;
      }
      if (a.F[t]) s = zmul(to_zc(a.F[t][j]), s);
      acc = zadd(acc, s);
    }
    a.out[j] = from_zc<C>(acc);
  }
}

template <class C>
hipError_t comb_impl(int64_t N, int nlast, const CombParams& p, hipStream_t s) {
  CombArgs<C> a;
  a.uh = (const C*)p.uh;
  for (int t = 0; t < 3; ++t) {
    a.F[t] = (const C*)p.F[t];
    for (int m = 0; m < 5; ++m) a.c[t][m] = p.c[t][m];
  }
  for (int m = 0; m < 5; ++m) a.v[m] = (const C*)p.v[m];
  a.nt = p.nt;
  a.sep = p.sep;
  a.out = (C*)p.out;
  int64_t b = (N + kCombThreads - 1) / kCombThreads;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  hipLaunchKernelGGL((comb_kernel<C>), dim3((unsigned)b), dim3(kCombThreads), 0, s, N, nlast, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_comb(int prec, int64_t N, int nlast, const CombParams& p, hipStream_t s) {
  if (p.nt < 0 || p.nt > 3 || !p.out) return hipErrorInvalidValue;
  return prec == P_F64 ? comb_impl<double2>(N, nlast, p, s) : comb_impl<float2>(N, nlast, p, s);
}

}  // namespace fcgle
