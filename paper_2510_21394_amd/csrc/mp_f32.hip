// FP32 MFMA (v_mfma_f32_16x16x4f32) mode products, complex64 tensors.
#include "dispatch.hpp"

namespace fcgle {

struct F32K {
  static constexpr bool kUpdate = true;  // ProUpdateF instantiated
  static constexpr bool kFwd2 = true;    // fused even/odd forward tiles instantiated
  template <class T, int SP>
  static constexpr size_t operand_lds() {
    return mp_operand_lds<float, T, SP>();
  }
  using R = float;
  template <class T, bool TL, int SP, class Pro, class Epi>
  static hipError_t go(const MPLaunch& L, hipStream_t s) {
    const Geo g = make_geo<T>(L, TL, MfmaT<float>::G);
    hipLaunchKernelGGL((mp_mfma_kernel<float, T, TL, SP, Pro, Epi>), dim3(g.nblocks), dim3(T::THREADS), 0, s, g,
                       (const float*)L.M, (const float2*)L.in, Pro(L.pp), Epi(L.ep));
    return hipGetLastError();
  }
};

hipError_t launch_mp_f32(const MPLaunch& L, hipStream_t s) {
  if (mp_wide(L))
    return L.split ? dispatch_split<F32K, TileCfg<128, 64, 16, 2, 2, 2, true>>(L, s)
                   : dispatch_cfg<F32K, TileCfg<128, 64, 16, 2, 2, 2, true>>(L, s);
  if (L.split) {
    switch (L.cfg) {
      case 0: return dispatch_split<F32K, TileCfg<128, 64, 16, 2, 2>>(L, s);
      case 1: return dispatch_split<F32K, TileCfg<128, 128, 32, 2, 4, 1>>(L, s);
      case 2: return dispatch_split<F32K, TileCfg<128, 128, 16, 4, 4>>(L, s);
      case 3: return dispatch_split<F32K, TileCfg<128, 64, 16, 4, 2>>(L, s);
      case 4: return dispatch_split<F32K, TileCfg<128, 128, 16, 2, 4>>(L, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (L.cfg) {
    case 0: return dispatch_cfg<F32K, TileCfg<256, 64, 16, 2, 2>>(L, s);
    case 1: return dispatch_cfg<F32K, TileCfg<128, 64, 16, 2, 2>>(L, s);
    case 2: return dispatch_cfg<F32K, TileCfg<64, 64, 16, 1, 2>>(L, s);
    case 3: return dispatch_cfg<F32K, TileCfg<128, 64, 16, 4, 2>>(L, s);
    case 4: return dispatch_cfg<F32K, TileCfg<256, 64, 16, 4, 2>>(L, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fcgle
