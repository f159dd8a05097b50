// Maps a host-side MPLaunch onto one instantiation of the mode-product kernels.
#pragma once

#include "kernels.hpp"

namespace fcgle {

// Rows (M tile) and complex columns per workgroup of the three configurations of each
// precision; index [split ? 1 : 0][prec][cfg].  The even/odd split kernels contract half-size
// blocks (at most n/2 + 1 rows each) and the backward form carries two accumulator sets, so
// their tiles are smaller.
constexpr int kCfgRows[2][4][kNumCfg] = {
    {{256, 128, 64, 128, 256}, {256, 128, 64, 128, 256}, {256, 128, 64, 128, 256}, {128, 64, 64, 64, 128}},
    {{128, 64, 128, 128, 128}, {128, 128, 128, 128, 128}, {64, 128, 128, 128, 64}, {64, 64, 128, 64, 128}}};
constexpr int kCfgCols[2][4][kNumCfg] = {
    {{32, 32, 32, 32, 32}, {64, 64, 64, 64, 64}, {64, 64, 64, 64, 64}, {64, 64, 32, 64, 64}},
    {{32, 32, 64, 32, 64}, {64, 128, 128, 64, 128}, {32, 32, 32, 32, 64}, {32, 16, 16, 32, 16}}};
// k-tile length of the split configurations (the dense ones use 16 for FP32, 8 for FP64 and
// 32 for split BF16); index [prec][cfg].
constexpr int kCfgTkSplit[4][kNumCfg] = {
    {16, 16, 16, 16, 16}, {16, 16, 16, 16, 16}, {32, 32, 32, 32, 32}, {32, 32, 32, 32, 32}};
// LDS buffers of the operand tiles (1: single-buffered configurations).
constexpr int kCfgBufs[2][4][kNumCfg] = {
    {{2, 2, 2, 2, 2}, {2, 2, 2, 2, 2}, {2, 2, 2, 2, 2}, {2, 2, 2, 2, 2}},
    {{2, 1, 2, 2, 2}, {2, 2, 2, 2, 2}, {1, 2, 1, 1, 1}, {2, 1, 2, 1, 1}}};

// Even/odd configuration whose tile runs the update prologue of configuration c; index
// [prec][otf][c] (otf: the on-the-fly form, else the P1-grid form).  The 16-wave tiles (FP64
// and FP32 configuration 2) leave 128 VGPRs per lane, which the update prologue overflows into
// scratch, and so does FP32 configuration 3 with the P1-grid form; each hands the update to the
// tile of the same shape with fewer waves (same rows, columns and LDS, so the same results).
constexpr int kCfgUpdTile[4][2][kNumCfg] = {
    {{0, 1, 4, 3, 4}, {0, 1, 4, 3, 4}},
    {{0, 1, 4, 0, 4}, {0, 1, 4, 3, 4}},
    {{0, 1, 2, 3, 4}, {0, 1, 2, 3, 4}},
    {{0, 1, 2, 3, 4}, {0, 1, 2, 3, 4}}};

// Instantiates the (loader, prologue, epilogue) combination of L for structure SP; the
// combinations a structure never needs are not instantiated.
template <class K, class T, int SP>
hipError_t dispatch_combo(const MPLaunch& L, hipStream_t s) {
  using R = typename K::R;
  const bool tl = (L.B == 1);
  if (L.pk == ProKind::Update || L.pk == ProKind::UpdateOtf) {
    if constexpr (SP == kSplitBwd && K::kUpdate) {
      if (!tl && L.ek == EpiKind::Store) {
        if (L.pk == ProKind::Update) return K::template go<T, false, SP, ProUpdateF<R>, EpiStoreF<R>>(L, s);
        if constexpr (K::template operand_lds<T, SP>() + kOtfMaxRows * sizeof(typename ProUpdateOtfF<R>::RowEnt) <=
                      kLdsBytes)
          if (L.n <= kOtfMaxRows) return K::template go<T, false, SP, ProUpdateOtfF<R>, EpiStoreF<R>>(L, s);
      }
    }
    return hipErrorInvalidValue;
  }
  if (!tl) {
    if (L.pk != ProKind::Id) {
      if constexpr (SP != kSplitBwd)
        if (L.ek == EpiKind::Store) {
          if (L.pk == ProKind::Flow) return K::template go<T, false, SP, ProFlowF<R>, EpiStoreF<R>>(L, s);
          if (L.pp.ns == 0 && !L.pp.up) return K::template go<T, false, SP, ProNonlinF<R, true>, EpiStoreF<R>>(L, s);
          return K::template go<T, false, SP, ProNonlinF<R>, EpiStoreF<R>>(L, s);
        }
      return hipErrorInvalidValue;
    }
    switch (L.ek) {
      case EpiKind::Store:
        return K::template go<T, false, SP, ProIdF, EpiStoreF<R>>(L, s);
      case EpiKind::Grid:
        if constexpr (SP != kSplitBwd) return K::template go<T, false, SP, ProIdF, EpiGridF<R>>(L, s);
        return hipErrorInvalidValue;
      case EpiKind::Sep:
        if constexpr (SP != kSplitBwd) return K::template go<T, false, SP, ProIdF, EpiSepF<R>>(L, s);
        return hipErrorInvalidValue;
      case EpiKind::ExpEuler:
        if constexpr (SP != kSplitBwd) return K::template go<T, false, SP, ProIdF, EpiExpEulerF<R>>(L, s);
        return hipErrorInvalidValue;
      case EpiKind::Axpy:
        if constexpr (SP == kDense && std::is_same<R, double>::value)
          return K::template go<T, false, SP, ProIdF, EpiAxpyF<R>>(L, s);
        return hipErrorInvalidValue;
      case EpiKind::Flow:
        if constexpr (SP == kDense || SP == kSplitBwd) return K::template go<T, false, SP, ProIdF, EpiFlowF<R>>(L, s);
        return hipErrorInvalidValue;
      default:
        return hipErrorInvalidValue;
    }
  }
  if constexpr (T::WIDE) {
    return hipErrorInvalidValue;  // T-loader offsets always fit the buffer views
  } else {
  if (L.pk != ProKind::Id) {
    if constexpr (SP != kSplitBwd)
      if (L.ek == EpiKind::Store) {
        if (L.pk == ProKind::Flow) return K::template go<T, true, SP, ProFlowF<R>, EpiStoreF<R>>(L, s);
        if (L.pp.ns == 0 && !L.pp.up) return K::template go<T, true, SP, ProNonlinF<R, true>, EpiStoreF<R>>(L, s);
        return K::template go<T, true, SP, ProNonlinF<R>, EpiStoreF<R>>(L, s);
      }
    return hipErrorInvalidValue;
  }
  switch (L.ek) {
    case EpiKind::Store:
      return K::template go<T, true, SP, ProIdF, EpiStoreF<R>>(L, s);
    case EpiKind::Grid:
      if constexpr (SP != kSplitBwd) return K::template go<T, true, SP, ProIdF, EpiGridF<R>>(L, s);
      return hipErrorInvalidValue;
    case EpiKind::Sep:
      if constexpr (SP != kSplitBwd) return K::template go<T, true, SP, ProIdF, EpiSepF<R>>(L, s);
      return hipErrorInvalidValue;
    case EpiKind::ExpEuler:
      if constexpr (SP != kSplitBwd) return K::template go<T, true, SP, ProIdF, EpiExpEulerF<R>>(L, s);
      return hipErrorInvalidValue;
    case EpiKind::KeepOld:
      if constexpr (SP != kSplitFwd && SP != kSplitFwd2) return K::template go<T, true, SP, ProIdF, EpiKeepOldF<R>>(L, s);
      return hipErrorInvalidValue;
    case EpiKind::Axpy:
      if constexpr (SP == kDense && std::is_same<R, double>::value)
        return K::template go<T, true, SP, ProIdF, EpiAxpyF<R>>(L, s);
      return hipErrorInvalidValue;
    case EpiKind::Flow:
      if constexpr (SP == kDense || SP == kSplitBwd) return K::template go<T, true, SP, ProIdF, EpiFlowF<R>>(L, s);
      return hipErrorInvalidValue;
    default:
      return hipErrorInvalidValue;
  }
  }
}

template <class K, class T>
hipError_t dispatch_cfg(const MPLaunch& L, hipStream_t s) {
  return dispatch_combo<K, T, kDense>(L, s);
}

template <class K, class T>
hipError_t dispatch_split(const MPLaunch& L, hipStream_t s) {
  if (L.split == kSplitFwd) return dispatch_combo<K, T, kSplitFwd>(L, s);
  if (L.split == kSplitBwd) return dispatch_combo<K, T, kSplitBwd>(L, s);
  if constexpr (K::kFwd2)
    if (L.split == kSplitFwd2) return dispatch_combo<K, T, kSplitFwd2>(L, s);
  return hipErrorInvalidValue;
}

}  // namespace fcgle
