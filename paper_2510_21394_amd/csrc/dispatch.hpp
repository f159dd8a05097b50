// Maps a host-side MPLaunch onto one instantiation of the mode-product kernels.
#pragma once

#include "kernels.hpp"

namespace fcgle {

// Rows (M tile) and complex columns per workgroup of the three configurations of each
// precision; index [prec][cfg].
constexpr int kCfgRows[4][kNumCfg] = {{256, 128, 64}, {256, 128, 64}, {256, 128, 64}, {128, 64, 64}};
constexpr int kCfgCols[4][kNumCfg] = {{32, 32, 32}, {64, 64, 64}, {64, 64, 64}, {64, 64, 32}};

template <class K, class T>
hipError_t dispatch_cfg(const MPLaunch& L, hipStream_t s) {
  using R = typename K::R;
  const bool tl = (L.B == 1);
  if (!tl) {
    if (L.ek != EpiKind::Store) return hipErrorInvalidValue;
    if (L.pk == ProKind::Id) return K::template go<T, false, ProIdF, EpiStoreF<R>>(L, s);
    return K::template go<T, false, ProNonlinF<R>, EpiStoreF<R>>(L, s);
  }
  if (L.pk != ProKind::Id) return hipErrorInvalidValue;
  switch (L.ek) {
    case EpiKind::Store:
      return K::template go<T, true, ProIdF, EpiStoreF<R>>(L, s);
    case EpiKind::Grid:
      return K::template go<T, true, ProIdF, EpiGridF<R>>(L, s);
    case EpiKind::Sep:
      return K::template go<T, true, ProIdF, EpiSepF<R>>(L, s);
    case EpiKind::ExpEuler:
      return K::template go<T, true, ProIdF, EpiExpEulerF<R>>(L, s);
    case EpiKind::KeepOld:
      return K::template go<T, true, ProIdF, EpiKeepOldF<R>>(L, s);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace fcgle
