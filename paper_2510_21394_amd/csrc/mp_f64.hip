// FP64 MFMA (v_mfma_f64_16x16x4f64) mode products, complex128 tensors.
#include "dispatch.hpp"

namespace fcgle {

struct F64K {
  static constexpr bool kUpdate = true;  // ProUpdateF instantiated
  static constexpr bool kFwd2 = true;    // fused even/odd forward tiles instantiated
  template <class T, int SP>
  static constexpr size_t operand_lds() {
    return mp_operand_lds<double, T, SP>();
  }
  using R = double;
  template <class T, bool TL, int SP, class Pro, class Epi>
  static hipError_t go(const MPLaunch& L, hipStream_t s) {
    const Geo g = make_geo<T>(L, TL, MfmaT<double>::G);
    hipLaunchKernelGGL((mp_mfma_kernel<double, T, TL, SP, Pro, Epi>), dim3(g.nblocks), dim3(T::THREADS), 0, s, g,
                       (const double*)L.M, (const double2*)L.in, Pro(L.pp), Epi(L.ep));
    return hipGetLastError();
  }
};

hipError_t launch_mp_f64(const MPLaunch& L, hipStream_t s) {
  if (mp_wide(L))
    return L.split ? dispatch_split<F64K, TileCfg<128, 32, 16, 2, 2, 2, true>>(L, s)
                   : dispatch_cfg<F64K, TileCfg<128, 32, 8, 2, 2, 2, true>>(L, s);
  if (L.split) {
    switch (L.cfg) {
      case 0: return dispatch_split<F64K, TileCfg<128, 32, 16, 2, 2>>(L, s);
      case 1: return dispatch_split<F64K, TileCfg<64, 32, 16, 1, 2, 1>>(L, s);
      case 2: return dispatch_split<F64K, TileCfg<128, 64, 16, 4, 4>>(L, s);
      case 3: return dispatch_split<F64K, TileCfg<128, 32, 16, 4, 2>>(L, s);
      case 4: return dispatch_split<F64K, TileCfg<128, 64, 16, 2, 4>>(L, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (L.cfg) {
    case 0: return dispatch_cfg<F64K, TileCfg<256, 32, 8, 2, 2>>(L, s);
    case 1: return dispatch_cfg<F64K, TileCfg<128, 32, 8, 2, 2>>(L, s);
    case 2: return dispatch_cfg<F64K, TileCfg<64, 32, 8, 1, 2>>(L, s);
    case 3: return dispatch_cfg<F64K, TileCfg<128, 32, 8, 4, 2>>(L, s);
    case 4: return dispatch_cfg<F64K, TileCfg<256, 32, 8, 4, 2>>(L, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fcgle
