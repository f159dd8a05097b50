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

// The Q-stationary even/odd products (mp_qres_kernel): both blocks of 49..128 rows in LDS,
// either loader, no prologue (or the plain nonlinearity on forward products), plain store,
// offsets of one tile below 2 GiB; hipErrorNotSupported for every other case.
template <int SP, int MT, bool TL, class Pro>
static hipError_t go_qres(const MPLaunch& L, hipStream_t s) {
  Geo g{};
  g.A = (uint32_t)L.A;
  g.B = (uint32_t)L.B;
  g.n = L.n;
  g.npad = L.npad;
  g.me = L.me;
  g.mo = L.mo;
  const uint64_t tiles = TL ? (uint64_t)((L.A + 15) / 16) : (uint64_t)L.A * (uint64_t)((L.B + 15) / 16);
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return hipErrorNotSupported;
  const uint64_t want = (tiles + kQresWaves - 1) / kQresWaves;
  const uint32_t grid = (uint32_t)(want < (uint64_t)cus ? want : (uint64_t)cus);
  hipLaunchKernelGGL((mp_qres_kernel<SP, MT, TL, Pro>), dim3(grid), dim3(64 * kQresWaves), 0, s, g,
                     (const float*)L.M, (const float2*)L.in, (float2*)L.ep.out, Pro(L.pp));
  return hipGetLastError();
}

template <int SP, bool TL, class Pro>
static hipError_t go_qres_rows(const MPLaunch& L, hipStream_t s) {
  switch ((L.me + 15) / 16) {
    case 4: return go_qres<SP, 4, TL, Pro>(L, s);
    case 5: return go_qres<SP, 5, TL, Pro>(L, s);
    case 6: return go_qres<SP, 6, TL, Pro>(L, s);
    case 7: return go_qres<SP, 7, TL, Pro>(L, s);
    case 8: return go_qres<SP, 8, TL, Pro>(L, s);
    default: return hipErrorNotSupported;
  }
}

template <bool TL>
static hipError_t launch_qres_loader(const MPLaunch& L, hipStream_t s) {
  if (L.split == kSplitBwd) {
    if (L.pk == ProKind::Id) return go_qres_rows<kSplitBwd, TL, ProIdF>(L, s);
    if constexpr (!TL)
      if (L.pk == ProKind::UpdateOtf && L.n <= kOtfMaxRows &&
          (uint64_t)L.A * (uint64_t)L.n * (uint64_t)L.B * sizeof(float2) < 0x80000000ull)
        return go_qres_rows<kSplitBwd, TL, ProUpdateOtfF<float>>(L, s);
    return hipErrorNotSupported;
  }
  if (L.split != kSplitFwd2) return hipErrorNotSupported;
  if (L.pk == ProKind::Id) return go_qres_rows<kSplitFwd2, TL, ProIdF>(L, s);
  if (L.pk == ProKind::Nonlin && L.pp.ns == 0 && !L.pp.up)
    return go_qres_rows<kSplitFwd2, TL, ProNonlinF<float, true>>(L, s);
  return hipErrorNotSupported;
}

static hipError_t launch_qres_f32(const MPLaunch& L, hipStream_t s) {
  if (L.ek != EpiKind::Store || L.wide) return hipErrorNotSupported;
  if (L.B > 1) {
    if ((uint64_t)L.n * (uint64_t)L.B * sizeof(float2) >= 0x80000000ull) return hipErrorNotSupported;
    return launch_qres_loader<false>(L, s);
  }
  if ((uint64_t)16 * (uint64_t)L.n * sizeof(float2) >= 0x80000000ull) return hipErrorNotSupported;
  return launch_qres_loader<true>(L, s);
}

hipError_t launch_mp_f32(const MPLaunch& L, hipStream_t s) {
  // split configuration 1: the Q-stationary kernel where it applies, else the 128 x 128 tile
  if (L.split && L.cfg == 1 && !mp_wide(L)) {
    const hipError_t e = launch_qres_f32(L, s);
    if (e != hipErrorNotSupported) return e;
    return dispatch_split<F32K, TileCfg<128, 128, 16, 2, 4>>(L, s);
  }
  if (mp_wide(L))
    return L.split ? dispatch_split<F32K, TileCfg<128, 64, 16, 2, 2, 2, true>>(L, s)
                   : dispatch_cfg<F32K, TileCfg<128, 64, 16, 2, 2, 2, true>>(L, s);
  if (L.split) {
    switch (L.cfg) {
      case 0: return dispatch_split<F32K, TileCfg<128, 64, 16, 2, 2>>(L, s);
      case 1: return dispatch_split<F32K, TileCfg<128, 128, 16, 2, 4>>(L, s);  // handled above
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
