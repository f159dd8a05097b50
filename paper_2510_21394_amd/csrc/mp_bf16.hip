// Split-BF16 MFMA (v_mfma_f32_16x16x32_bf16) mode products, complex64 tensors, FP32 accumulation.
#include "dispatch.hpp"

namespace fcgle {

template <int NP>
struct BFK {
  static constexpr bool kUpdate = true;  // ProUpdateF / ProUpdateOtfF instantiated
  static constexpr bool kFwd2 = true;    // fused even/odd forward tiles instantiated
  // LDS of the operand tiles of mp_bf16_kernel: NBUF buffers of NP pieces, k-tiles of TK
  // padded by 8
  template <class T, int SP>
  static constexpr size_t operand_lds() {
    constexpr size_t NB = (SP == kSplitBwd || SP == kSplitFwd2) ? 2 : 1, LDK = T::TK + 8;
    return T::NBUF * NB * NP * T::TM * LDK * 2 + T::NBUF * NB * NP * 2 * T::TNC * LDK * 2;
  }
  using R = float;
  template <class T, bool TL, int SP, class Pro, class Epi>
  static hipError_t go(const MPLaunch& L, hipStream_t s) {
    const Geo g = make_geo<T>(L, TL, 4);
    hipLaunchKernelGGL((mp_bf16_kernel<T, NP, TL, SP, Pro, Epi>), dim3(g.nblocks), dim3(T::THREADS), 0, s, g,
                       (const __bf16*)L.M, (const float2*)L.in, Pro(L.pp), Epi(L.ep));
    return hipGetLastError();
  }
};

hipError_t launch_mp_bf16(const MPLaunch& L, hipStream_t s) {
  // Split tiles stay within the 160 KB of LDS with two operand blocks of NP pieces each; the
  // single-buffered configurations (last template argument 1) let two workgroups share a CU.
  if (mp_wide(L)) {
    if (L.prec == P_BF16X3)
      return L.split ? dispatch_split<BFK<2>, TileCfg<128, 32, 32, 2, 2, 1, true>>(L, s)
                     : dispatch_cfg<BFK<2>, TileCfg<128, 64, 32, 2, 2, 2, true>>(L, s);
    return L.split ? dispatch_split<BFK<3>, TileCfg<64, 32, 32, 1, 2, 1, true>>(L, s)
                   : dispatch_cfg<BFK<3>, TileCfg<64, 64, 32, 1, 2, 2, true>>(L, s);
  }
  if (L.prec == P_BF16X3) {
    if (L.split) {
      switch (L.cfg) {
        case 0: return dispatch_split<BFK<2>, TileCfg<64, 32, 32, 1, 2, 1>>(L, s);
        case 1: return dispatch_split<BFK<2>, TileCfg<128, 32, 32, 2, 2>>(L, s);
        case 2: return dispatch_split<BFK<2>, TileCfg<128, 32, 64, 2, 2, 1>>(L, s);
        case 3: return dispatch_split<BFK<2>, TileCfg<128, 32, 32, 2, 2, 1>>(L, s);
        case 4: return dispatch_split<BFK<2>, TileCfg<64, 64, 32, 1, 2, 1>>(L, s);
        default: return hipErrorInvalidValue;
      }
    }
    switch (L.cfg) {
      case 0: return dispatch_cfg<BFK<2>, TileCfg<256, 64, 32, 2, 2>>(L, s);
      case 1: return dispatch_cfg<BFK<2>, TileCfg<128, 64, 32, 2, 2>>(L, s);
      case 2: return dispatch_cfg<BFK<2>, TileCfg<64, 64, 32, 1, 2>>(L, s);
      case 3: return dispatch_cfg<BFK<2>, TileCfg<128, 64, 32, 4, 2>>(L, s);
      case 4: return dispatch_cfg<BFK<2>, TileCfg<256, 64, 32, 4, 2>>(L, s);
      default: return hipErrorInvalidValue;
    }
  }
  if (L.split) {
    switch (L.cfg) {
      case 0: return dispatch_split<BFK<3>, TileCfg<64, 32, 32, 1, 2>>(L, s);
      case 1: return dispatch_split<BFK<3>, TileCfg<64, 16, 32, 1, 1, 1>>(L, s);
      case 2: return dispatch_split<BFK<3>, TileCfg<128, 16, 32, 2, 1>>(L, s);
      case 3: return dispatch_split<BFK<3>, TileCfg<64, 32, 32, 1, 2, 1>>(L, s);
      case 4: return dispatch_split<BFK<3>, TileCfg<128, 16, 32, 2, 1, 1>>(L, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (L.cfg) {
    case 0: return dispatch_cfg<BFK<3>, TileCfg<128, 64, 32, 2, 2>>(L, s);
    case 1: return dispatch_cfg<BFK<3>, TileCfg<64, 64, 32, 1, 2>>(L, s);
    case 2: return dispatch_cfg<BFK<3>, TileCfg<64, 32, 32, 1, 2>>(L, s);
    case 3: return dispatch_cfg<BFK<3>, TileCfg<64, 64, 32, 2, 2>>(L, s);
    case 4: return dispatch_cfg<BFK<3>, TileCfg<128, 64, 32, 4, 2>>(L, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fcgle
