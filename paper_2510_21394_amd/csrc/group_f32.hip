// Grouped FP32 MFMA mode products and grouped streaming epilogues: one launch per phase
// of a time step over many independent problems of uneven sizes (batched instances).
#include <cstring>

#include "dispatch.hpp"

namespace fcgle {

namespace {

template <bool TL, int SP, class Pro, class Epi>
struct Combo {
  static constexpr bool tl = TL;
  static constexpr int sp = SP;
  using P = Pro;
  using E = Epi;
};

// Forward (Q^T) combinations of the even/odd form SP (kSplitFwd or kSplitFwd2).
template <int SP, class F>
bool with_fwd_combo(bool tl, ProKind pk, EpiKind ek, F&& f) {
  using R = float;
  if (!tl && pk == ProKind::Nonlin && ek == EpiKind::Store) {
    // batched instances carry no source terms and no extrapolated state (group_build_f32
    // refuses items that do): the plain form of the nonlinearity
    f(Combo<false, SP, ProNonlinF<R, true>, EpiStoreF<R>>{});
    return true;
  }
  if (!tl && pk == ProKind::Id && ek == EpiKind::Store) {
    f(Combo<false, SP, ProIdF, EpiStoreF<R>>{});
    return true;
  }
  if (tl && pk == ProKind::Id && ek == EpiKind::Store) {
    f(Combo<true, SP, ProIdF, EpiStoreF<R>>{});
    return true;
  }
  if (tl && pk == ProKind::Id && ek == EpiKind::ExpEuler) {
    f(Combo<true, SP, ProIdF, EpiExpEulerF<R>>{});
    return true;
  }
  return false;
}

// Calls f(Combo<...>{}) for the supported (loader, prologue, epilogue) combination of the
// even/odd form sp: kSplitFwd or kSplitFwd2 (Q^T), kSplitBwd (Q).
template <class F>
bool with_combo(bool tl, ProKind pk, EpiKind ek, int sp, F&& f) {
  using R = float;
  if (sp == kSplitFwd) return with_fwd_combo<kSplitFwd>(tl, pk, ek, f);
  if (sp == kSplitFwd2) return with_fwd_combo<kSplitFwd2>(tl, pk, ek, f);
  if (sp != kSplitBwd || pk != ProKind::Id || ek != EpiKind::Store) return false;
  if (tl)
    f(Combo<true, kSplitBwd, ProIdF, EpiStoreF<R>>{});
  else
    f(Combo<false, kSplitBwd, ProIdF, EpiStoreF<R>>{});
  return true;
}

// The FP32 tile configurations of the grouped even/odd kernels (rows x complex columns x k,
// waves): the 64-row tiles waste fewer padded rows on the half-block lengths 48..256 of
// the batched instances.
template <class F>
bool with_cfg(int cfg, F&& f) {
  switch (cfg) {
    case 0: f(TileCfg<128, 64, 16, 2, 2>{}); return true;
    case 1: f(TileCfg<64, 64, 16, 1, 2>{}); return true;
    case 2: f(TileCfg<128, 32, 16, 2, 2>{}); return true;
    case 3: f(TileCfg<64, 64, 16, 2, 2>{}); return true;
    case 4: f(TileCfg<64, 128, 16, 1, 4>{}); return true;
    default: return false;
  }
}

template <class Epi>
struct PwItem {
  uint32_t first;  // first row of this item in the launch
  int nlast;
  const void* v;
  Epi epi;
};

template <class R, class Epi>
__global__ void __launch_bounds__(256)
    pw_group_kernel(const PwItem<Epi>* __restrict__ items, int count, uint32_t total_rows) {
  using C = typename Cx<R>::T;
  for (uint32_t r = blockIdx.x; r < total_rows; r += gridDim.x) {
    const int k = find_item(items, count, r);
    const PwItem<Epi>& it = items[k];
    const uint32_t a = r - it.first;
    const auto ctx = it.epi.col(a, 0);
    const int64_t base = (int64_t)a * it.nlast;
    const C* v = (const C*)it.v;
    for (int i = threadIdx.x; i < it.nlast; i += 256) {
      const C x = v[base + i];
      const int ii[1] = {i};
      const int64_t jj[1] = {base + i};
      const bool ok[1] = {true};
      const R re[1] = {x.x}, im[1] = {x.y};
      it.epi.template apply<1>(ctx, ii, jj, ok, re, im);
    }
  }
}

}  // namespace

int group_cfg_rows(int cfg) {
  int r = 0;
  with_cfg(cfg, [&](auto t) { r = decltype(t)::TM; });
  return r;
}

bool group_supported(bool tloader, ProKind pk, EpiKind ek, bool fwd) {
  return with_combo(tloader, pk, ek, fwd ? kSplitFwd : kSplitBwd, [](auto) {});
}

size_t group_item_bytes(ProKind pk, EpiKind ek) {
  size_t b = 0;
  for (int tl = 0; tl < 2; ++tl)
    for (int sp = kSplitFwd; sp <= kSplitFwd2; ++sp)
      with_combo(tl != 0, pk, ek, sp, [&](auto c) {
        using Cb = decltype(c);
        b = sizeof(GroupItem<typename Cb::P, typename Cb::E>);
      });
  return b;
}

uint32_t group_build_f32(int cfg, bool tloader, ProKind pk, EpiKind ek, const MPLaunch* L, int count,
                         void* items_host) {
  uint32_t total = 0;
  if (pk == ProKind::Nonlin)
    for (int k = 0; k < count; ++k)
      if (L[k].pp.ns != 0 || L[k].pp.up != nullptr) return 0;  // only the plain nonlinearity is grouped
  const int sp = count > 0 ? L[0].split : 0;
  with_cfg(cfg, [&](auto t) {
    using T = decltype(t);
    with_combo(tloader, pk, ek, sp, [&](auto c) {
      using Cb = decltype(c);
      using Item = GroupItem<typename Cb::P, typename Cb::E>;
      unsigned char* dst = (unsigned char*)items_host;
      for (int k = 0; k < count; ++k) {
        Item it;
        it.g = make_geo<T>(L[k], Cb::tl, 4);
        it.M = L[k].M;
        it.U = L[k].in;
        it.first = total;
        it.pro = typename Cb::P(L[k].pp);
        it.epi = typename Cb::E(L[k].ep);
        std::memcpy(dst + k * sizeof(Item), &it, sizeof(Item));
        total += it.g.nblocks;
      }
    });
  });
  return total;
}

hipError_t launch_group_f32(int cfg, bool tloader, ProKind pk, EpiKind ek, int sp, const void* items_dev,
                            int count, uint32_t nblocks, hipStream_t s) {
  hipError_t err = hipErrorInvalidValue;
  if (count < 1 || nblocks == 0) return err;
  with_cfg(cfg, [&](auto t) {
    using T = decltype(t);
    with_combo(tloader, pk, ek, sp, [&](auto c) {
      using Cb = decltype(c);
      using Item = GroupItem<typename Cb::P, typename Cb::E>;
      hipLaunchKernelGGL((mp_group_kernel<float, T, Cb::tl, Cb::sp, typename Cb::P, typename Cb::E>),
                         dim3(nblocks), dim3(T::THREADS), 0, s, (const Item*)items_dev, count, nblocks);
      err = hipGetLastError();
    });
  });
  return err;
}

// ---------------------------------------------------------------------------------------
// Persistent batched exponential Euler (batch_persist_kernel): tile configurations with an
// instantiation, item arrays of its four phases, grid and launch.
// ---------------------------------------------------------------------------------------

namespace {

template <class F>
bool with_persist_cfg(int cfg, F&& f) {
  switch (cfg) {
    case 0: f(TileCfg<128, 64, 16, 2, 2>{}); return true;
    case 1: f(TileCfg<64, 64, 16, 1, 2>{}); return true;
    case 3: f(TileCfg<64, 64, 16, 2, 2>{}); return true;
    default: return false;
  }
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

}  // namespace

bool persist_supported(int cfg) {
  return with_persist_cfg(cfg, [](auto) {});
}

size_t persist_item_bytes(int phase) {
  if (phase == 0) return sizeof(GroupItem<ProNonlinF<float>, EpiStoreF<float>>);
  if (phase == 1) return sizeof(GroupItem<ProIdF, EpiExpEulerF<float>>);
  return sizeof(GroupItem<ProIdF, EpiStoreF<float>>);
}

uint32_t persist_build_f32(int cfg, int phase, const MPLaunch* L, int count, void* items_host, uint32_t* tiles) {
  uint32_t total = 0;
  with_persist_cfg(cfg, [&](auto t) {
    using T = decltype(t);
    auto build = [&](auto item_tag, bool tl) {
      using Item = decltype(item_tag);
      unsigned char* dst = (unsigned char*)items_host;
      for (int k = 0; k < count; ++k) {
        Item it;
        it.g = make_geo<T>(L[k], tl, 4);
        it.M = L[k].M;
        it.U = L[k].in;
        it.first = total;
        it.pro = decltype(it.pro)(L[k].pp);
        it.epi = decltype(it.epi)(L[k].ep);
        std::memcpy(dst + k * sizeof(Item), &it, sizeof(Item));
        tiles[k] = it.g.nblocks;
        total += it.g.nblocks;
      }
    };
    if (phase == 0) build(GroupItem<ProNonlinF<float>, EpiStoreF<float>>{}, false);
    else if (phase == 1) build(GroupItem<ProIdF, EpiExpEulerF<float>>{}, true);
    else build(GroupItem<ProIdF, EpiStoreF<float>>{}, phase == 3);
  });
  return total;
}

int persist_grid(int cfg) {
  int grid = 0;
  with_persist_cfg(cfg, [&](auto t) {
    using T = decltype(t);
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batch_persist_kernel<T, kSplitFwd2>, T::THREADS, 0) !=
            hipSuccess)
      return;
    grid = cus * (per > 0 ? per : 1);
  });
  return grid;
}

hipError_t launch_persist_f32(int cfg, const PersistArgs& a, uint32_t grid, hipStream_t s) {
  hipError_t err = hipErrorInvalidValue;
  with_persist_cfg(cfg, [&](auto t) {
    using T = decltype(t);
    hipLaunchKernelGGL((batch_persist_kernel<T, kSplitFwd2>), dim3(grid), dim3(T::THREADS), 0, s, a);
    err = hipGetLastError();
  });
  return err;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t n, hipStream_t s) {
  const uint32_t blocks = (n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

size_t pw_group_item_bytes(EpiKind ek) {
  return ek == EpiKind::ExpEuler ? sizeof(PwItem<EpiExpEulerF<float>>) : 0;
}

uint32_t pw_group_build_f32(EpiKind ek, const int64_t* rows, const int* nlast, const void* const* v,
                            const EpiParams* ep, int count, void* items_host) {
  if (ek != EpiKind::ExpEuler) return 0;
  using Item = PwItem<EpiExpEulerF<float>>;
  unsigned char* dst = (unsigned char*)items_host;
  uint32_t total = 0;
  for (int k = 0; k < count; ++k) {
    Item it;
    it.first = total;
    it.nlast = nlast[k];
    it.v = v[k];
    it.epi = EpiExpEulerF<float>(ep[k]);
    std::memcpy(dst + k * sizeof(Item), &it, sizeof(Item));
    total += (uint32_t)rows[k];
  }
  return total;
}

hipError_t launch_pw_group_f32(EpiKind ek, const void* items_dev, int count, uint32_t total_rows, hipStream_t s) {
  if (ek != EpiKind::ExpEuler || count < 1 || total_rows == 0) return hipErrorInvalidValue;
  using Item = PwItem<EpiExpEulerF<float>>;
  const uint32_t blocks = total_rows < 65536 ? total_rows : 65536;
  hipLaunchKernelGGL((pw_group_kernel<float, EpiExpEulerF<float>>), dim3(blocks), dim3(256), 0, s,
                     (const Item*)items_dev, count, total_rows);
  return hipGetLastError();
}

}  // namespace fcgle
