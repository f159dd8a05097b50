// Pointwise passes: FP64 f-grids, unfused prologue/epilogue fallbacks, the
// non-finite scan and the reduction of per-block partial sums.
#include "dispatch.hpp"

namespace fcgle {

namespace {

constexpr int kPwThreads = 256;

inline unsigned pw_blocks(int64_t N) {
  int64_t b = (N + kPwThreads - 1) / kPwThreads;
  if (b > 65536) b = 65536;  // grid-stride beyond this
  if (b < 1) b = 1;
  return (unsigned)b;
}

template <class R, class Pro>
__global__ void __launch_bounds__(kPwThreads)
    pw_pro_kernel(int64_t N, const typename Cx<R>::T* __restrict__ in, typename Cx<R>::T* __restrict__ out,
                  Pro pro) {
  for (int64_t j = blockIdx.x * (int64_t)kPwThreads + threadIdx.x; j < N; j += (int64_t)gridDim.x * kPwThreads)
    out[j] = pro(j, in[j]);
}

// The tensor viewed as (rows, nlast); each workgroup pass takes kPwRows consecutive rows,
// a thread one element of each (loads of all of them before any store); the per-row
// context of the epilogue (the separable factor of the slower axes) is one table load.
constexpr int kPwRows = 8;

template <class R, class Epi>
__global__ void __launch_bounds__(kPwThreads)
    pw_epi_kernel(uint32_t rows, int nlast, const typename Cx<R>::T* __restrict__ v, Epi epi) {
  for (uint32_t r0 = blockIdx.x * kPwRows; r0 < rows; r0 += gridDim.x * kPwRows) {
    for (int i0 = threadIdx.x; i0 < nlast; i0 += kPwThreads) {
      int ii[kPwRows];
      int64_t jj[kPwRows];
      bool ok[kPwRows];
      R re[kPwRows], im[kPwRows];
      typename Epi::Pre pre[kPwRows];
#pragma unroll
      for (int u = 0; u < kPwRows; ++u) {
        ok[u] = r0 + u < rows;
        ii[u] = i0;
        jj[u] = (int64_t)(ok[u] ? r0 + u : r0) * nlast + i0;
        const auto x = ok[u] ? v[jj[u]] : typename Cx<R>::T{0, 0};
        re[u] = x.x;
        im[u] = x.y;
      }
      epi.template load<kPwRows>(ii, jj, ok, pre);
#pragma unroll
      for (int u = 0; u < kPwRows; ++u) {
        if (!ok[u]) continue;
        const auto ctx = epi.col(r0 + u, 0);
        epi.template store<1>(ctx, ii + u, jj + u, ok + u, re + u, im + u, pre + u);
      }
    }
  }
}

// F[j] = f(theta_c * ell_j), ell_j = sum_mu lambda_mu[j_mu], all in FP64.
template <class C>
__global__ void __launch_bounds__(kPwThreads)
    fgrid_kernel(int kind, double tr, double ti, SepParams s, int64_t N, C* __restrict__ F) {
  for (int64_t j = blockIdx.x * (int64_t)kPwThreads + threadIdx.x; j < N; j += (int64_t)gridDim.x * kPwThreads) {
    int64_t r = j;
    double ell = 0.0;
    for (int mu = s.d - 1; mu >= 0; --mu) {
      const int64_t jm = r % s.n[mu];
      r /= s.n[mu];
      ell += s.lam[mu][jm];
    }
    const zc z{tr * ell, ti * ell};
    F[j] = from_zc<C>(fz_eval(kind, z));
  }
}

__global__ void __launch_bounds__(kPwThreads)
    sep_table_kernel(SepParams s, int mu, int64_t count, zc* __restrict__ out) {
  s.mu = mu;
  for (int64_t j = blockIdx.x * (int64_t)kPwThreads + threadIdx.x; j < count; j += (int64_t)gridDim.x * kPwThreads)
    out[j] = (mu == 0) ? sep_other_direct(s, 0, (uint32_t)j) : sep_other_direct(s, (uint32_t)j, 0);
}

__global__ void __launch_bounds__(kPwThreads)
    sep_table_m1_kernel(SepParams s, int64_t count, zc* __restrict__ m1, double* __restrict__ lam) {
  for (int64_t j = blockIdx.x * (int64_t)kPwThreads + threadIdx.x; j < count; j += (int64_t)gridDim.x * kPwThreads) {
    uint32_t b = (uint32_t)j;
    zc a{0.0, 0.0};  // prod (1 + x_mu) - 1 over the axes done so far
    double l = 0.0;
    for (int nu = s.d - 1; nu > 0; --nu) {
      const uint32_t jn = b % (uint32_t)s.n[nu];
      b /= (uint32_t)s.n[nu];
      const zc x = ((const zc*)s.facm1[nu])[jn];
      a = zadd(zadd(a, x), zmul(a, x));
      l += s.lam[nu][jn];
    }
    m1[j] = a;
    lam[j] = l;
  }
}

template <class C>
__global__ void __launch_bounds__(kPwThreads) finite_kernel(int64_t N, const C* __restrict__ u, int* flag) {
  bool bad = false;
  for (int64_t j = blockIdx.x * (int64_t)kPwThreads + threadIdx.x; j < N; j += (int64_t)gridDim.x * kPwThreads) {
    const C x = u[j];
    bad |= !(isfinite(x.x) && isfinite(x.y));
  }
  if (bad) atomicOr(flag, 1);
}

__global__ void __launch_bounds__(kPwThreads)
    reduce_partials_kernel(const double* __restrict__ partial, int64_t count, int width, double* acc) {
  __shared__ double sh[kPwThreads];
  for (int c = 0; c < width; ++c) {
    double s = 0.0;
    for (int64_t r = threadIdx.x; r < count; r += kPwThreads) s += partial[r * width + c];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int st = kPwThreads / 2; st > 0; st >>= 1) {
      if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) acc[c] += sh[0];
    __syncthreads();
  }
}

template <class R>
hipError_t pro_impl(int64_t N, const void* in, void* out, ProKind pk, const ProParams& p, hipStream_t s) {
  using C = typename Cx<R>::T;
  if (pk == ProKind::Nonlin)
    hipLaunchKernelGGL((pw_pro_kernel<R, ProNonlinF<R>>), dim3(pw_blocks(N)), dim3(kPwThreads), 0, s, N,
                       (const C*)in, (C*)out, ProNonlinF<R>(p));
  else if (pk == ProKind::Flow)
    hipLaunchKernelGGL((pw_pro_kernel<R, ProFlowF<R>>), dim3(pw_blocks(N)), dim3(kPwThreads), 0, s, N,
                       (const C*)in, (C*)out, ProFlowF<R>(p));
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <class R, class Epi>
hipError_t epi_launch(int64_t N, int nlast, const void* v, const EpiParams& p, hipStream_t s) {
  using C = typename Cx<R>::T;
  const int64_t rows = N / nlast;
  const int64_t groups = (rows + kPwRows - 1) / kPwRows;
  hipLaunchKernelGGL((pw_epi_kernel<R, Epi>), dim3((unsigned)(groups < 65536 ? groups : 65536)), dim3(kPwThreads),
                     0, s, (uint32_t)rows, nlast, (const C*)v, Epi(p));
  return hipGetLastError();
}

template <class R>
hipError_t epi_impl(int64_t N, int nlast, const void* v, EpiKind ek, const EpiParams& p, hipStream_t s) {
  switch (ek) {
    case EpiKind::Store: return epi_launch<R, EpiStoreF<R>>(N, nlast, v, p, s);
    case EpiKind::Grid: return epi_launch<R, EpiGridF<R>>(N, nlast, v, p, s);
    case EpiKind::Sep: return epi_launch<R, EpiSepF<R>>(N, nlast, v, p, s);
    case EpiKind::ExpEuler: return epi_launch<R, EpiExpEulerF<R>>(N, nlast, v, p, s);
    case EpiKind::KeepOld: return epi_launch<R, EpiKeepOldF<R>>(N, nlast, v, p, s);
    case EpiKind::ExpEulerRec: return epi_launch<R, EpiExpEulerRecF<R>>(N, nlast, v, p, s);
    case EpiKind::Flow: return epi_launch<R, EpiFlowF<R>>(N, nlast, v, p, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool mp_supported(bool tloader, ProKind pk, EpiKind ek) {
  if (pk == ProKind::Update || pk == ProKind::UpdateOtf) return !tloader && ek == EpiKind::Store;
  if (pk != ProKind::Id) return ek == EpiKind::Store;
  if (!tloader)
    return ek == EpiKind::Store || ek == EpiKind::Grid || ek == EpiKind::Sep || ek == EpiKind::ExpEuler ||
           ek == EpiKind::Flow;
  return ek == EpiKind::Store || ek == EpiKind::Grid || ek == EpiKind::Sep || ek == EpiKind::ExpEuler ||
         ek == EpiKind::KeepOld || ek == EpiKind::Flow;
}

hipError_t launch_pointwise_pro(int prec, int64_t N, const void* in, void* out, ProKind pk, const ProParams& p,
                                hipStream_t s) {
  return prec == P_F64 ? pro_impl<double>(N, in, out, pk, p, s) : pro_impl<float>(N, in, out, pk, p, s);
}

hipError_t launch_pointwise_epi(int prec, int64_t N, int n_last, const void* v, EpiKind ek,
                                const EpiParams& p, hipStream_t s) {
  return prec == P_F64 ? epi_impl<double>(N, n_last, v, ek, p, s) : epi_impl<float>(N, n_last, v, ek, p, s);
}

hipError_t launch_sep_table(const SepParams& sep, int mu, int64_t count, void* other, hipStream_t s) {
  hipLaunchKernelGGL(sep_table_kernel, dim3(pw_blocks(count)), dim3(kPwThreads), 0, s, sep, mu, count, (zc*)other);
  return hipGetLastError();
}

hipError_t launch_sep_table_m1(const SepParams& sep, int64_t count, void* first_m1, double* first_lam,
                               hipStream_t s) {
  hipLaunchKernelGGL(sep_table_m1_kernel, dim3(pw_blocks(count)), dim3(kPwThreads), 0, s, sep, count, (zc*)first_m1,
                     first_lam);
  return hipGetLastError();
}

hipError_t launch_check_finite(int prec, int64_t N, const void* u, int* flag, hipStream_t s) {
  if (prec == P_F64)
    hipLaunchKernelGGL((finite_kernel<double2>), dim3(pw_blocks(N)), dim3(kPwThreads), 0, s, N,
                       (const double2*)u, flag);
  else
    hipLaunchKernelGGL((finite_kernel<float2>), dim3(pw_blocks(N)), dim3(kPwThreads), 0, s, N,
                       (const float2*)u, flag);
  return hipGetLastError();
}

hipError_t launch_reduce_partials(const double* partial, int64_t count, int width, double* acc,
                                  hipStream_t s) {
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(kPwThreads), 0, s, partial, count, width, acc);
  return hipGetLastError();
}

hipError_t launch_fgrid(int prec, int kind, double theta_re, double theta_im, const SepParams& sep,
                        int64_t N, void* F, hipStream_t s) {
  if (prec == P_F64)
    hipLaunchKernelGGL((fgrid_kernel<double2>), dim3(pw_blocks(N)), dim3(kPwThreads), 0, s, kind, theta_re,
                       theta_im, sep, N, (double2*)F);
  else
    hipLaunchKernelGGL((fgrid_kernel<float2>), dim3(pw_blocks(N)), dim3(kPwThreads), 0, s, kind, theta_re,
                       theta_im, sep, N, (float2*)F);
  return hipGetLastError();
}

int cfg_rows(int prec, int cfg, int split) { return kCfgRows[split ? 1 : 0][prec][cfg]; }
int cfg_cols(int prec, int cfg, int split) { return kCfgCols[split ? 1 : 0][prec][cfg]; }
int cfg_bufs(int prec, int cfg, int split) { return kCfgBufs[split ? 1 : 0][prec][cfg]; }
int cfg_tk_split(int prec, int cfg) { return kCfgTkSplit[prec][cfg]; }
int cfg_update_tile(int prec, int cfg, bool otf) { return kCfgUpdTile[prec][otf ? 1 : 0][cfg]; }
bool split_supported(int prec) { return prec >= P_F64 && prec <= P_BF16X6; }

}  // namespace fcgle
