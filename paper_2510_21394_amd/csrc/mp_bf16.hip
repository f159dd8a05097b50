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

// The Q-stationary BF16x3 even/odd products (mp_qres_bf16_kernel): both pieces of both blocks
// of 49..128 rows in LDS, N loader, no prologue or the plain nonlinearity on forward products,
// plain store, offsets of one batch index below 2 GiB; hipErrorNotSupported otherwise.
template <int SP, int MT, class Pro>
static hipError_t go_qres_bf16(const MPLaunch& L, hipStream_t s) {
  Geo g{};
  g.A = (uint32_t)L.A;
  g.B = (uint32_t)L.B;
  g.n = L.n;
  g.npad = L.npad;
  g.me = L.me;
  g.mo = L.mo;
  const uint64_t tiles = (uint64_t)L.A * (uint64_t)((L.B + 15) / 16);
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return hipErrorNotSupported;
  const uint64_t want = (tiles + kQresWaves - 1) / kQresWaves;
  const uint32_t grid = (uint32_t)(want < (uint64_t)cus ? want : (uint64_t)cus);
  hipLaunchKernelGGL((mp_qres_bf16_kernel<SP, MT, Pro>), dim3(grid), dim3(64 * kQresWaves), 0, s, g,
                     (const __bf16*)L.M, (const float2*)L.in, (float2*)L.ep.out, Pro(L.pp));
  return hipGetLastError();
}

template <int SP, class Pro>
static hipError_t go_qres_bf16_rows(const MPLaunch& L, hipStream_t s) {
  switch ((L.me + 15) / 16) {
    case 4: return go_qres_bf16<SP, 4, Pro>(L, s);
    case 5: return go_qres_bf16<SP, 5, Pro>(L, s);
    case 6: return go_qres_bf16<SP, 6, Pro>(L, s);
    case 7: return go_qres_bf16<SP, 7, Pro>(L, s);
    case 8: return go_qres_bf16<SP, 8, Pro>(L, s);
    default: return hipErrorNotSupported;
  }
}

static hipError_t launch_qres_bf16x3(const MPLaunch& L, hipStream_t s) {
  if (L.ek != EpiKind::Store || L.wide || L.B <= 1) return hipErrorNotSupported;
  if ((uint64_t)L.n * (uint64_t)L.B * sizeof(float2) >= 0x80000000ull) return hipErrorNotSupported;
  if (L.split == kSplitBwd)
    return L.pk == ProKind::Id ? go_qres_bf16_rows<kSplitBwd, ProIdF>(L, s) : hipErrorNotSupported;
  if (L.split != kSplitFwd2) return hipErrorNotSupported;
  if (L.pk == ProKind::Id) return go_qres_bf16_rows<kSplitFwd2, ProIdF>(L, s);
  if (L.pk == ProKind::Nonlin && L.pp.ns == 0 && !L.pp.up)
    return go_qres_bf16_rows<kSplitFwd2, ProNonlinF<float, true>>(L, s);
  return hipErrorNotSupported;
}

hipError_t launch_mp_bf16(const MPLaunch& L, hipStream_t s) {
  // BF16x3 split configuration 2: the Q-stationary kernel where it applies, else the
  // single-buffered 128 x 32 tile (configuration 3)
  if (L.prec == P_BF16X3 && L.split && L.cfg == 2 && !mp_wide(L)) {
    const hipError_t e = launch_qres_bf16x3(L, s);
    if (e != hipErrorNotSupported) return e;
    return dispatch_split<BFK<2>, TileCfg<128, 32, 32, 2, 2, 1>>(L, s);
  }
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
        case 2: return dispatch_split<BFK<2>, TileCfg<128, 32, 32, 2, 2, 1>>(L, s);  // handled above
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
