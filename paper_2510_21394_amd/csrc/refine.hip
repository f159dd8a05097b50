// Pointwise passes of the refinement sweep of the inverse: differences, casts to and from
// the state type, and the FP64 squared norm (wavefront reductions, then one fixed-order sum
// of the per-workgroup partials, so the result does not depend on scheduling).
#include "kernels.hpp"

namespace fcgle {

namespace {

constexpr int kRfThreads = 256;
constexpr int kRfParts = 1024;  // workgroups of the norm pass = partial sums

inline unsigned rf_blocks(int64_t N) {
  int64_t b = (N + kRfThreads - 1) / kRfThreads;
  if (b > 65536) b = 65536;  // grid-stride beyond this
  if (b < 1) b = 1;
  return (unsigned)b;
}

#define RF_LOOP(j) \
  for (int64_t j = blockIdx.x * (int64_t)kRfThreads + threadIdx.x; j < N; j += (int64_t)gridDim.x * kRfThreads)

__global__ void __launch_bounds__(kRfThreads)
    rf_sub_kernel(int64_t N, const double2* __restrict__ v, const double2* __restrict__ x, double2* __restrict__ r) {
  RF_LOOP(j) {
    const double2 a = v[j], b = x[j];
    r[j] = make_double2(a.x - b.x, a.y - b.y);
  }
}

template <class C>
__global__ void __launch_bounds__(kRfThreads)
    rf_to_state_kernel(int64_t N, const double2* __restrict__ r, C* __restrict__ y) {
  RF_LOOP(j) y[j] = from_zc<C>(zc{r[j].x, r[j].y});
}

template <class C, bool Add>
__global__ void __launch_bounds__(kRfThreads) rf_acc_kernel(int64_t N, double2* __restrict__ x, const C* __restrict__ y) {
  RF_LOOP(j) {
    const zc t = to_zc(y[j]);
    if (Add) {
      const double2 a = x[j];
      x[j] = make_double2(a.x + t.re, a.y + t.im);
    } else {
      x[j] = make_double2(t.re, t.im);
    }
  }
}

__device__ __forceinline__ double wave_sum(double s) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  return s;
}

// partial[b] = sum over the elements of workgroup b of |r_j|^2
__global__ void __launch_bounds__(kRfThreads)
    rf_norm_partial_kernel(int64_t N, const double2* __restrict__ r, double* __restrict__ partial) {
  __shared__ double sh[kRfThreads / 64];
  double s = 0.0;
  RF_LOOP(j) {
    const double2 a = r[j];
    s += a.x * a.x + a.y * a.y;
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kRfThreads / 64; ++w) t += sh[w];
    partial[blockIdx.x] = t;
  }
}

// out[0] = sum of the kRfParts partials (one workgroup, fixed order)
__global__ void __launch_bounds__(kRfThreads) rf_norm_final_kernel(const double* __restrict__ partial, double* out) {
  __shared__ double sh[kRfThreads / 64];
  double s = 0.0;
  for (int k = threadIdx.x; k < kRfParts; k += kRfThreads) s += partial[k];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kRfThreads / 64; ++w) t += sh[w];
    out[0] = t;
  }
}

}  // namespace

hipError_t launch_rf_sub(int64_t N, const void* v, const void* x, void* r, hipStream_t s) {
  hipLaunchKernelGGL(rf_sub_kernel, dim3(rf_blocks(N)), dim3(kRfThreads), 0, s, N, (const double2*)v,
                     (const double2*)x, (double2*)r);
  return hipGetLastError();
}

hipError_t launch_rf_to_state(int prec, int64_t N, const void* r, void* y, hipStream_t s) {
  if (prec == P_F64)
    hipLaunchKernelGGL((rf_to_state_kernel<double2>), dim3(rf_blocks(N)), dim3(kRfThreads), 0, s, N,
                       (const double2*)r, (double2*)y);
  else
    hipLaunchKernelGGL((rf_to_state_kernel<float2>), dim3(rf_blocks(N)), dim3(kRfThreads), 0, s, N,
                       (const double2*)r, (float2*)y);
  return hipGetLastError();
}

hipError_t launch_rf_set(int prec, int64_t N, void* x, const void* y, hipStream_t s) {
  if (prec == P_F64)
    hipLaunchKernelGGL((rf_acc_kernel<double2, false>), dim3(rf_blocks(N)), dim3(kRfThreads), 0, s, N,
                       (double2*)x, (const double2*)y);
  else
    hipLaunchKernelGGL((rf_acc_kernel<float2, false>), dim3(rf_blocks(N)), dim3(kRfThreads), 0, s, N,
                       (double2*)x, (const float2*)y);
  return hipGetLastError();
}

hipError_t launch_rf_add(int prec, int64_t N, void* x, const void* y, hipStream_t s) {
  if (prec == P_F64)
    hipLaunchKernelGGL((rf_acc_kernel<double2, true>), dim3(rf_blocks(N)), dim3(kRfThreads), 0, s, N,
                       (double2*)x, (const double2*)y);
  else
    hipLaunchKernelGGL((rf_acc_kernel<float2, true>), dim3(rf_blocks(N)), dim3(kRfThreads), 0, s, N,
                       (double2*)x, (const float2*)y);
  return hipGetLastError();
}

int rf_norm_parts() { return kRfParts; }

hipError_t launch_rf_norm2(int64_t N, const void* r, double* partial, double* out, hipStream_t s) {
  hipLaunchKernelGGL(rf_norm_partial_kernel, dim3(kRfParts), dim3(kRfThreads), 0, s, N, (const double2*)r, partial);
  hipLaunchKernelGGL(rf_norm_final_kernel, dim3(1), dim3(kRfThreads), 0, s, (const double*)partial, out);
  return hipGetLastError();
}

}  // namespace fcgle
