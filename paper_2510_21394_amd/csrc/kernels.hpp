// Device code of the library: complex helpers, the prologue/epilogue functors
// and the MFMA mode-product kernels for gfx950.
//
// A mode product (Section 3) multiplies a real n x n matrix M (Q_mu or Q_mu^T) onto
// the mode-mu fibres of a complex tensor.  With the tensor viewed as (A, n, B)
// (A = product of the slower extents, B = product of the faster ones):
//     out[a, i, b] = sum_k M[i, k] in[a, k, b].
// Each workgroup computes a TM x TNC block of (rows i) x (complex columns) with M as
// the MFMA A operand and the tensor as the B operand.  Two loaders fill the B tile:
//   N loader (B > 1): columns are b = fixed a, contiguous b; coalesced along b.
//   T loader (B == 1, the fastest axis): columns are a; each column is a contiguous
//     run of k in memory, so rows of the tile are read contiguously and transposed
//     for free by the LDS layout.
// In LDS both operands are stored k-contiguous ([row][k]) and the real and imaginary
// parts of the tensor are de-interleaved into two halves of the B tile, so that a
// lane ends up holding the real and imaginary part of the same output element in the
// same accumulator slot of two MFMA tiles.  That lets the epilogue apply complex
// pointwise maps (f-grid scaling, the exponential-Euler update, ...) directly.
//
// The order of the contraction inside a group of 4*G k-values is permuted so that a
// lane reads G consecutive k-values of both operands with one 16-byte LDS load; the
// same permutation is used for both operands, so the sum is unchanged.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <utility>

#include "fz.hpp"
#include "launch.h"

namespace fcgle {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef __bf16 v4bf __attribute__((ext_vector_type(4)));

template <class R>
struct Cx;
template <>
struct Cx<float> {
  using T = float2;
};
template <>
struct Cx<double> {
  using T = double2;
};

__device__ __forceinline__ zc to_zc(float2 v) { return {(double)v.x, (double)v.y}; }
__device__ __forceinline__ zc to_zc(double2 v) { return {v.x, v.y}; }
template <class C>
__device__ __forceinline__ C from_zc(zc z);
template <>
__device__ __forceinline__ float2 from_zc<float2>(zc z) {
  return make_float2((float)z.re, (float)z.im);
}
template <>
__device__ __forceinline__ double2 from_zc<double2>(zc z) {
  return make_double2(z.re, z.im);
}

// Hardware dispatches workgroup w to XCD (w mod 8).  Renumber so that consecutive
// logical blocks (the M tiles of one column tile, then neighbouring column tiles)
// land on the same XCD and share its L2.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t w, uint32_t nblocks) {
  const uint32_t per = nblocks >> 3, rem = nblocks & 7;
  const uint32_t x = w & 7, slot = w >> 3;
  return x * per + (x < rem ? x : rem) + slot;
}

// ---------------------------------------------------------------------------------------
// Prologue functors: map one loaded input element (flat index j) before the contraction.
// ---------------------------------------------------------------------------------------

struct ProIdF {
  static constexpr bool kId = true;
  static constexpr bool kUpdate = false;  // see ProUpdateF
  static constexpr bool kRowLds = false;  // see ProUpdateOtfF
  struct Pre {};
  ProIdF() = default;
  explicit ProIdF(const ProParams&) {}
  template <class C>
  __device__ __forceinline__ C operator()(int64_t, C u) const {
    return u;
  }
};

// out = cu u + cp up + cg g(t, e),  e = eu u + ep up,
// g(t, e) = gamma e - (kappa + i zeta)|e|^2 e + sum_k sc_k S_k[j]   (Section 2, the map g;
// sc_k = exp(c_k t) complex)
// Plain: no previous state and no source terms (up == nullptr, ns == 0), so no per-element
// index arithmetic or extra loads.
template <class R, bool Plain = false>
struct ProNonlinF {
  static constexpr bool kId = false;
  static constexpr bool kUpdate = false;
  static constexpr bool kRowLds = false;  // see ProUpdateOtfF
  struct Pre {};
  using C = typename Cx<R>::T;
  const C* up;
  const C* S[4];
  R sc[4], sci[4];
  int ns;
  R gamma, kre, kim, eu, ep, cu, cp, cg;
  ProNonlinF() = default;
  explicit ProNonlinF(const ProParams& p) {
    up = (const C*)p.up;
    for (int k = 0; k < 4; ++k) {
      S[k] = (const C*)p.S[k];
      sc[k] = (R)p.sc[k];
      sci[k] = (R)p.sci[k];
    }
    ns = p.ns;
    gamma = (R)p.gamma;
    kre = (R)p.kappa;
    kim = (R)p.zeta;
    eu = (R)p.eu;
    ep = (R)p.ep;
    cu = (R)p.cu;
    cp = (R)p.cp;
    cg = (R)p.cg;
  }
  __device__ __forceinline__ C operator()(int64_t j, C u) const {
    if constexpr (Plain) {
      const R er = eu * u.x, ei = eu * u.y;
      const R m = er * er + ei * ei;
      const R gr = gamma * er - m * (kre * er - kim * ei);
      const R gi = gamma * ei - m * (kre * ei + kim * er);
      C o;
      o.x = cu * u.x + cg * gr;
      o.y = cu * u.y + cg * gi;
      return o;
    } else {
      C p = {0, 0};
      if (up) p = up[j];
      const R er = eu * u.x + ep * p.x, ei = eu * u.y + ep * p.y;
      const R m = er * er + ei * ei;
      R gr = gamma * er - m * (kre * er - kim * ei);
      R gi = gamma * ei - m * (kre * ei + kim * er);
      for (int k = 0; k < ns; ++k) {
        const C s = S[k][j];
        gr += sc[k] * s.x - sci[k] * s.y;
        gi += sc[k] * s.y + sci[k] * s.x;
      }
      C o;
      o.x = cu * u.x + cp * p.x + cg * gr;
      o.y = cu * u.y + cp * p.y + cg * gi;
      return o;
    }
  }
};

// Exact flow of the nonlinear subproblem of Strang splitting (Section 4, eq. Strang) over a
// time t, in the state precision:  w -> w e^{gamma t} (1 + 2 kappa a)^{-1/2} e^{-i zeta L},
// a = t phi_1(2 gamma t) |w|^2, L = log(1 + 2 kappa a) / (2 kappa), and L = a for kappa = 0
// (the limit).  Rewritten from the printed exponent t gamma - (kappa + i zeta)/(2 kappa) log(...):
// its real part gives the modulus factor, its imaginary part the phase.  The scalars t phi_1,
// e^{gamma t} and 2 kappa are formed on the host in FP64.
template <class R>
struct FlowF {
  using C = typename Cx<R>::T;
  R tp1, eg, k2, zeta;
  FlowF() = default;
  explicit FlowF(const FlowParams& f) : tp1((R)f.tp1), eg((R)f.eg), k2((R)f.k2), zeta((R)f.zeta) {}
  __device__ __forceinline__ C operator()(C w) const {
    const R a = tp1 * (w.x * w.x + w.y * w.y);
    R L = a, s = eg;
    if (k2 > (R)0) {
      const R x = k2 * a;
      if constexpr (std::is_same<R, float>::value) {
        L = log1pf(x) / k2;
        s = eg * rsqrtf(1.0f + x);
      } else {
        L = log1p(x) / k2;
        s = eg * rsqrt(1.0 + x);
      }
    }
    R sn, cs;
    if constexpr (std::is_same<R, float>::value)
      sincosf(-zeta * L, &sn, &cs);
    else
      sincos(-zeta * L, &sn, &cs);
    C o;
    o.x = s * (w.x * cs - w.y * sn);
    o.y = s * (w.x * sn + w.y * cs);
    return o;
  }
};

template <class R>
struct ProFlowF {
  static constexpr bool kId = false;
  static constexpr bool kUpdate = false;
  static constexpr bool kRowLds = false;
  struct Pre {};
  FlowF<R> f;
  ProFlowF() = default;
  explicit ProFlowF(const ProParams& p) : f(p.flow) {}
  template <class C>
  __device__ __forceinline__ C operator()(int64_t, C u) const {
    return f(u);
  }
};

// ---------------------------------------------------------------------------------------
// Epilogue functors.  col(a, b) is evaluated once per output column (a: flat index over the
// axes slower than mu, b: over the faster ones).  Each functor works in two phases over V
// output elements (i: mode-mu index, j: flat index, ok: inside the tensor):
//   load<V>(i, j, ok, pre)                     issues every global load it needs,
//   store<V>(ctx, i, j, ok, re, im, pre)       computes and stores.
// Callers run the loads of several columns before their stores, so loads are not
// serialised behind stores the compiler cannot prove independent (the exponential-Euler
// update reads and writes the same array).  apply<V> is load followed by store.
// ---------------------------------------------------------------------------------------

struct NoCtx {};
struct NoPre {};

// Product over the axes other than mu of the separable per-axis factors (a: flat index over
// the slower axes, b: over the faster ones).
__device__ __forceinline__ zc sep_other_direct(const SepParams& s, uint32_t a, uint32_t b) {
  zc E{1.0, 0.0};
  for (int nu = s.d - 1; nu > s.mu; --nu) {
    const uint32_t jn = b % (uint32_t)s.n[nu];
    b /= (uint32_t)s.n[nu];
    E = zmul(E, ((const zc*)s.fac[nu])[jn]);
  }
  for (int nu = s.mu - 1; nu >= 0; --nu) {
    const uint32_t jn = a % (uint32_t)s.n[nu];
    a /= (uint32_t)s.n[nu];
    E = zmul(E, ((const zc*)s.fac[nu])[jn]);
  }
  return E;
}

__device__ __forceinline__ zc sep_other(const SepParams& s, uint32_t a, uint32_t b) {
  if (s.mu == s.d - 1 && s.other_last) return ((const zc*)s.other_last)[a];
  if (s.mu == 0 && s.other_first) return ((const zc*)s.other_first)[b];
  return sep_other_direct(s, a, b);
}

template <class C, class R>
__device__ __forceinline__ C mkc(R re, R im) {
  C v;
  v.x = re;
  v.y = im;
  return v;
}

// Complex arithmetic in the state precision (float2 / double2).
template <class C>
__device__ __forceinline__ C cmul(C a, C b) {
  C o;
  o.x = a.x * b.x - a.y * b.y;
  o.y = a.x * b.y + a.y * b.x;
  return o;
}

#define FCGLE_EPI_APPLY                                                                              \
  template <int V>                                                                                   \
  __device__ __forceinline__ void apply(const Ctx& ctx, const int* i, const int64_t* j, const bool* ok, \
                                        const R* re, const R* im) const {                           \
    Pre pre[V];                                                                                      \
    this->template load<V>(i, j, ok, pre);                                                           \
    this->template store<V>(ctx, i, j, ok, re, im, pre);                                             \
  }

template <class R>
struct EpiStoreF {
  using C = typename Cx<R>::T;
  using Ctx = NoCtx;
  using Pre = NoPre;
  C* out;
  EpiStoreF() = default;
  explicit EpiStoreF(const EpiParams& p) : out((C*)p.out) {}
  __device__ __forceinline__ Ctx col(uint32_t, uint32_t) const { return {}; }
  template <int V>
  __device__ __forceinline__ void load(const int*, const int64_t*, const bool*, Pre*) const {}
  template <int V>
  __device__ __forceinline__ void store(const Ctx&, const int*, const int64_t* j, const bool* ok, const R* re,
                                        const R* im, const Pre*) const {
#pragma unroll
    for (int v = 0; v < V; ++v)
      if (ok[v]) out[j[v]] = mkc<C>(re[v], im[v]);
  }
  FCGLE_EPI_APPLY
};

// out[j] = phi_t(v): the trailing half step of Strang splitting on the backward product.
template <class R>
struct EpiFlowF {
  using C = typename Cx<R>::T;
  using Ctx = NoCtx;
  using Pre = NoPre;
  C* out;
  FlowF<R> f;
  EpiFlowF() = default;
  explicit EpiFlowF(const EpiParams& p) : out((C*)p.out), f(p.flow) {}
  __device__ __forceinline__ Ctx col(uint32_t, uint32_t) const { return {}; }
  template <int V>
  __device__ __forceinline__ void load(const int*, const int64_t*, const bool*, Pre*) const {}
  template <int V>
  __device__ __forceinline__ void store(const Ctx&, const int*, const int64_t* j, const bool* ok, const R* re,
                                        const R* im, const Pre*) const {
#pragma unroll
    for (int v = 0; v < V; ++v)
      if (ok[v]) out[j[v]] = f(mkc<C>(re[v], im[v]));
  }
  FCGLE_EPI_APPLY
};

template <class R>
struct EpiGridF {
  using C = typename Cx<R>::T;
  using Ctx = NoCtx;
  using Pre = C;
  C* out;
  const C* F;
  EpiGridF() = default;
  explicit EpiGridF(const EpiParams& p) : out((C*)p.out), F((const C*)p.F) {}
  __device__ __forceinline__ Ctx col(uint32_t, uint32_t) const { return {}; }
  template <int V>
  __device__ __forceinline__ void load(const int*, const int64_t* j, const bool* ok, Pre* f) const {
#pragma unroll
    for (int v = 0; v < V; ++v) f[v] = ok[v] ? F[j[v]] : C{0, 0};
  }
  template <int V>
  __device__ __forceinline__ void store(const Ctx&, const int*, const int64_t* j, const bool* ok, const R* re,
                                        const R* im, const Pre* f) const {
#pragma unroll
    for (int v = 0; v < V; ++v)
      if (ok[v]) out[j[v]] = mkc<C>(f[v].x * re[v] - f[v].y * im[v], f[v].x * im[v] + f[v].y * re[v]);
  }
  FCGLE_EPI_APPLY
};

// out[j] = E_j v with E the separable exponential (product of the per-axis FP64 factors),
// formed and applied in FP64: E is the same every step, so a rounding of E in the state
// precision would act as a fixed per-element bias that grows linearly over a trajectory.
template <class R>
struct EpiSepF {
  using C = typename Cx<R>::T;
  using Ctx = zc;
  using Pre = zc;
  C* out;
  SepParams s;
  EpiSepF() = default;
  explicit EpiSepF(const EpiParams& p) : out((C*)p.out), s(p.sep) {}
  __device__ __forceinline__ Ctx col(uint32_t a, uint32_t b) const { return sep_other(s, a, b); }
  template <int V>
  __device__ __forceinline__ void load(const int* i, const int64_t*, const bool* ok, Pre* f) const {
#pragma unroll
    for (int v = 0; v < V; ++v) f[v] = ok[v] ? ((const zc*)s.fac[s.mu])[i[v]] : zc{0, 0};
  }
  template <int V>
  __device__ __forceinline__ void store(const Ctx& Eo, const int*, const int64_t* j, const bool* ok,
                                        const R* re, const R* im, const Pre* f) const {
#pragma unroll
    for (int v = 0; v < V; ++v)
      if (ok[v]) out[j[v]] = from_zc<C>(zmul(zmul(Eo, f[v]), zc{(double)re[v], (double)im[v]}));
  }
  FCGLE_EPI_APPLY
};

// uhat[j] <- E_j uhat[j] + tau P1[j] v   (v = transformed nonlinearity).  E uhat is formed in
// FP64 (see EpiSepF); the small correction tau P1 v in the state precision.
template <class R>
struct EpiExpEulerF {
  using C = typename Cx<R>::T;
  using Ctx = zc;
  struct Pre {
    C u, P;
    zc f;
  };
  C* uhat;
  const C* P1;
  C* ghat_out;
  SepParams s;
  double tau;
  EpiExpEulerF() = default;
  explicit EpiExpEulerF(const EpiParams& p)
      : uhat((C*)p.out), P1((const C*)p.F), ghat_out((C*)p.ghat_out), s(p.sep), tau(p.tau) {}
  __device__ __forceinline__ Ctx col(uint32_t a, uint32_t b) const { return sep_other(s, a, b); }
  template <int V>
  __device__ __forceinline__ void load(const int* i, const int64_t* j, const bool* ok, Pre* pre) const {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      pre[v].u = ok[v] ? uhat[j[v]] : C{0, 0};
      pre[v].P = ok[v] ? P1[j[v]] : C{0, 0};
      pre[v].f = ok[v] ? ((const zc*)s.fac[s.mu])[i[v]] : zc{0, 0};
    }
  }
  template <int V>
  __device__ __forceinline__ void store(const Ctx& Eo, const int*, const int64_t* j, const bool* ok,
                                        const R* re, const R* im, const Pre* pre) const {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      if (!ok[v]) continue;
      const zc eu = zmul(zmul(Eo, pre[v].f), to_zc(pre[v].u));
      const C pg = cmul(pre[v].P, mkc<C>(re[v], im[v]));
      uhat[j[v]] = from_zc<C>(zc{eu.re + tau * (double)pg.x, eu.im + tau * (double)pg.y});
      if (ghat_out) ghat_out[j[v]] = mkc<C>(re[v], im[v]);
    }
  }
  FCGLE_EPI_APPLY
};

// Exponential-Euler update that also records what the adjoint needs for the derivatives
// with respect to nu and eta (d u_{n+1} / dz = Q (e^z uhat_n + tau phi_1'(z) ghat_n), with
// phi_1' = phi_1 - phi_2):
//   uhat[j] <- E_j uhat[j] + tau P1[j] v,   X[j] = uhat_new[j] - tau P2[j] v,  in FP64.
template <class R>
struct EpiExpEulerRecF {
  using C = typename Cx<R>::T;
  using Ctx = zc;
  struct Pre {
    C u, p1, p2;
    zc f;
  };
  C* uhat;
  const C* P1;
  const C* P2;
  C* X;
  SepParams s;
  double tau;
  EpiExpEulerRecF() = default;
  explicit EpiExpEulerRecF(const EpiParams& p)
      : uhat((C*)p.out), P1((const C*)p.F), P2((const C*)p.F2), X((C*)p.out2), s(p.sep), tau(p.tau) {}
  __device__ __forceinline__ Ctx col(uint32_t a, uint32_t b) const { return sep_other(s, a, b); }
  template <int V>
  __device__ __forceinline__ void load(const int* i, const int64_t* j, const bool* ok, Pre* pre) const {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      pre[v].u = ok[v] ? uhat[j[v]] : C{0, 0};
      pre[v].p1 = ok[v] ? P1[j[v]] : C{0, 0};
      pre[v].p2 = ok[v] ? P2[j[v]] : C{0, 0};
      pre[v].f = ok[v] ? ((const zc*)s.fac[s.mu])[i[v]] : zc{0, 0};
    }
  }
  template <int V>
  __device__ __forceinline__ void store(const Ctx& Eo, const int*, const int64_t* j, const bool* ok,
                                        const R* re, const R* im, const Pre* pre) const {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      if (!ok[v]) continue;
      const zc E = zmul(Eo, pre[v].f);
      const zc g{(double)re[v], (double)im[v]};
      const zc r = zadd(zmul(E, to_zc(pre[v].u)), zscale(zmul(to_zc(pre[v].p1), g), tau));
      uhat[j[v]] = from_zc<C>(r);
      X[j[v]] = from_zc<C>(zsub(r, zscale(zmul(to_zc(pre[v].p2), g), tau)));
    }
  }
  FCGLE_EPI_APPLY
};

template <class R>
struct EpiKeepOldF {
  using C = typename Cx<R>::T;
  using Ctx = NoCtx;
  using Pre = C;
  C* out;
  C* save;
  EpiKeepOldF() = default;
  explicit EpiKeepOldF(const EpiParams& p) : out((C*)p.out), save((C*)p.save) {}
  __device__ __forceinline__ Ctx col(uint32_t, uint32_t) const { return {}; }
  template <int V>
  __device__ __forceinline__ void load(const int*, const int64_t* j, const bool* ok, Pre* old) const {
#pragma unroll
    for (int v = 0; v < V; ++v) old[v] = ok[v] ? out[j[v]] : C{0, 0};
  }
  template <int V>
  __device__ __forceinline__ void store(const Ctx&, const int*, const int64_t* j, const bool* ok, const R* re,
                                        const R* im, const Pre* old) const {
#pragma unroll
    for (int v = 0; v < V; ++v)
      if (ok[v]) {
        save[j[v]] = old[v];
        out[j[v]] = mkc<C>(re[v], im[v]);
      }
  }
  FCGLE_EPI_APPLY
};

// out[j] += c v with a complex coefficient c (the FP64 residual r += theta (nu + i eta) D_mu x_mu
// of the refinement sweep): each output element is read and written by the one thread that
// computes it.
template <class R>
struct EpiAxpyF {
  using C = typename Cx<R>::T;
  using Ctx = NoCtx;
  using Pre = C;
  C* out;
  R cre, cim;
  EpiAxpyF() = default;
  explicit EpiAxpyF(const EpiParams& p) : out((C*)p.out), cre((R)p.cre), cim((R)p.cim) {}
  __device__ __forceinline__ Ctx col(uint32_t, uint32_t) const { return {}; }
  template <int V>
  __device__ __forceinline__ void load(const int*, const int64_t* j, const bool* ok, Pre* old) const {
#pragma unroll
    for (int v = 0; v < V; ++v) old[v] = ok[v] ? out[j[v]] : C{0, 0};
  }
  template <int V>
  __device__ __forceinline__ void store(const Ctx&, const int*, const int64_t* j, const bool* ok, const R* re,
                                        const R* im, const Pre* old) const {
#pragma unroll
    for (int v = 0; v < V; ++v)
      if (ok[v]) out[j[v]] = mkc<C>(old[v].x + (cre * re[v] - cim * im[v]), old[v].y + (cre * im[v] + cim * re[v]));
  }
  FCGLE_EPI_APPLY
};

#undef FCGLE_EPI_APPLY

// Complex elements through a buffer resource of `bytes` bytes: the hardware bounds check reads
// an offset at or beyond the extent as zero and drops a store there, so masked element accesses
// need neither clamped indices nor branches.  Offsets are 32-bit byte offsets (the update
// prologue is only used for tensors below kBufMaxBytes); kOob is the offset of a masked access.
constexpr uint32_t kBufMaxBytes = 0x80000000u;
constexpr uint32_t kOob = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float2 buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off, float2*) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ double2 buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off, double2*) {
  return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}
template <class C>
__device__ __forceinline__ C buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return buf_load(r, off, (C*)nullptr);
}
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, uint32_t off, float2 v) {
  typedef unsigned int u2 __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, off, 0, 0);
}
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, uint32_t off, double2 v) {
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), r, off, 0, 0);
}

// Exponential-Euler update applied while the first backward product loads its input
// (instead of in the epilogue of the last forward product):
//   uhat_out[j] = E_j uhat[j] + tau P1[j] ghat[j],
// where ghat (the transformed nonlinearity) is the tensor the product reads; the product
// then contracts uhat_out.  Same arithmetic as EpiExpEulerF: E uhat in FP64 from the
// separable factors, tau P1 ghat in the state precision.  The operands uhat[j] and P1[j]
// are loaded together with the tile (load), the update is applied when the tile is
// written to LDS (update); the per-column factor of the axes other than mu comes from
// col() once per loader unit.  uhat_out must not alias uhat: with several row tiles per
// column the other row tiles still read uhat after the first has written uhat_out.
template <class R>
struct ProUpdateF {
  static constexpr bool kId = false;
  static constexpr bool kUpdate = true;
  static constexpr bool kRowLds = false;
  struct RowEnt {};
  using C = typename Cx<R>::T;
  struct Pre {
    C u, P;
    zc f;  // factor of axis mu for the element's row
  };
  const C* uhat;
  const C* P1;
  C* uhat_out;
  const zc* fac;  // factors of axis mu
  SepParams s;
  double tau;
  ProUpdateF() = default;
  explicit ProUpdateF(const ProParams& p)
      : uhat((const C*)p.uhat), P1((const C*)p.F), uhat_out((C*)p.uhat_out), fac((const zc*)p.sep.fac[p.sep.mu]),
        s(p.sep), tau(p.tau) {}
  __device__ __forceinline__ zc col(uint32_t a, uint32_t b) const { return sep_other(s, a, b); }
  // operands of the element at byte offset off (kOob: reads zero) of row i (a valid row)
  __device__ __forceinline__ Pre load(uint32_t off, int i, uint32_t bytes) const {
    return Pre{buf_load<C>(buf_rsrc(uhat, bytes), off), buf_load<C>(buf_rsrc(P1, bytes), off), fac[i]};
  }
  __device__ __forceinline__ C update(const zc& Eo, C g, const Pre& pre) const {
    const zc eu = zmul(zmul(Eo, pre.f), to_zc(pre.u));
    const C pg = cmul(pre.P, g);
    return from_zc<C>(zc{eu.re + tau * (double)pg.x, eu.im + tau * (double)pg.y});
  }
  __device__ __forceinline__ void save(uint32_t off, C v, uint32_t bytes) const {
    buf_store(buf_rsrc(uhat_out, bytes), off, v);
  }
};

// Reciprocal in the arithmetic precision: the hardware approximation (1 ulp) for FP32, the
// correctly rounded quotient for FP64.
__device__ __forceinline__ float rcp_r(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_r(double x) { return 1.0 / x; }
__device__ __forceinline__ float fma_r(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_r(double a, double b, double c) { return __builtin_fma(a, b, c); }

// The same update with P1 = phi_1(z) = (e^z - 1) / z formed on the fly instead of read from the
// P1 grid (one HBM stream less), in the arithmetic precision R throughout.  All exponents of a
// plan share one complex direction: z = zs (lam_row + lam_col) with zs = (zre + i zim) and a real
// eigenvalue sum l < 0.  With m = e^z - 1 = a + b + a b, a = E_col - 1 and b = E_row - 1 from
// separable expm1 tables (both with Re <= 0 on every axis, so the sum does not cancel and keeps
// full relative accuracy however small z is):
//   uhat_new = E uhat + tau P1 ghat = uhat + m uhat + ((tau / zs) m / l) ghat,
// one real reciprocal per element, tau / zs formed once on the host in FP64.  E itself is never
// rounded: the only per-element constant that is rounded every step is m, whose rounding is
// about |z| times smaller than one of E would be for the slowly decaying modes (for which a
// rounded E would act as a bias growing over a trajectory).  When zs = 0 every m is exactly 0
// and P1 = 1: tau / zs is then set to 0 and the constant tau used instead.  The row entries
// (E_row - 1 and lam_row) of all n rows are staged in LDS once per workgroup (n <= kOtfMaxRows);
// the column context once per loader unit.
template <class R>
struct ProUpdateOtfF {
  static constexpr bool kId = false;
  static constexpr bool kUpdate = true;
  static constexpr bool kRowLds = true;
  using C = typename Cx<R>::T;
  struct Pre {
    C u;
  };
  struct __attribute__((aligned(4 * sizeof(R)))) RowEnt {
    R m1re, m1im, lam, pad_;
  };
  struct Col {
    R m1re, m1im, lam;
  };
  const C* uhat;
  C* uhat_out;
  SepParams s;
  double c1re = 0, c1im = 0;  // tau / zs (0 when zs = 0)
  double t0 = 0;              // tau when zs = 0, else 0
  ProUpdateOtfF() = default;
  explicit ProUpdateOtfF(const ProParams& p) : uhat((const C*)p.uhat), uhat_out((C*)p.uhat_out), s(p.sep) {
    const double zq = p.sep.zre * p.sep.zre + p.sep.zim * p.sep.zim;
    if (zq > 0.0) {
      c1re = p.tau * p.sep.zre / zq;
      c1im = -p.tau * p.sep.zim / zq;
    } else {
      t0 = p.tau;
    }
  }
  __device__ __forceinline__ RowEnt row_entry(int i) const {
    const zc m1 = ((const zc*)s.facm1[s.mu])[i];
    return RowEnt{(R)m1.re, (R)m1.im, (R)s.lam[s.mu][i], (R)0};
  }
  __device__ __forceinline__ Col col(uint32_t, uint32_t b) const {
    const zc m1 = ((const zc*)s.first_m1)[b];
    return Col{(R)m1.re, (R)m1.im, (R)s.first_lam[b]};
  }
  __device__ __forceinline__ Pre load(uint32_t off, int, uint32_t bytes) const {
    return Pre{buf_load<C>(buf_rsrc(uhat, bytes), off)};
  }
  __device__ __forceinline__ C update(const Col& c, const RowEnt& r, C g, const Pre& pre) const {
    const R ar = c.m1re, ai = c.m1im, br = r.m1re, bi = r.m1im;
    const R mr = (ar + br) + (ar * br - ai * bi), mi = (ai + bi) + (ar * bi + ai * br);
    const R rl = rcp_r(c.lam + r.lam);  // every eigenvalue is negative, so the sum is too
    const R q1r = (R)c1re, q1i = (R)c1im;
    const R pr = (mr * q1r - mi * q1i) * rl + (R)t0, pi = (mr * q1i + mi * q1r) * rl;
    // the two small terms are summed first, so the state is rounded once at its own magnitude
    const R ur = pre.u.x, ui = pre.u.y;
    C out;
    out.x = ur + fma_r(mr, ur, fma_r(-mi, ui, fma_r(pr, g.x, -pi * g.y)));
    out.y = ui + fma_r(mr, ui, fma_r(mi, ur, fma_r(pr, g.y, pi * g.x)));
    return out;
  }
  __device__ __forceinline__ void save(uint32_t off, C v, uint32_t bytes) const {
    buf_store(buf_rsrc(uhat_out, bytes), off, v);
  }
};

// ---------------------------------------------------------------------------------------
// Tile configurations and geometry
// ---------------------------------------------------------------------------------------

// NBUF_: operand tiles in LDS double-buffered (2: one barrier per k-tile) or single-buffered (1:
// half the LDS, so more workgroups can share a CU, for a second barrier per k-tile).
// WIDE_: the B operand is read with 64-bit element indices (load_b_unit_wide) instead of
// per-k-tile buffer views, for products whose k-tile rows span more than the views' 2 GiB.
template <int TM_, int TNC_, int TK_, int WM_, int WN_, int NBUF_ = 2, bool WIDE_ = false>
struct TileCfg {
  static constexpr int TM = TM_, TNC = TNC_, TK = TK_, WM = WM_, WN = WN_, NBUF = NBUF_;
  static constexpr bool WIDE = WIDE_;
  static_assert(NBUF == 1 || NBUF == 2, "operand buffers");
  static constexpr int THREADS = 64 * WM * WN;
  static constexpr int NW = WM * WN;
  static constexpr int WTM = TM / WM, WTNC = TNC / WN;
  static constexpr int FM = WTM / 16, FNC = WTNC / 16;
  static_assert(FM >= 1 && FNC >= 1 && WTM % 16 == 0 && WTNC % 16 == 0, "wave tile");
  static_assert(TM % 64 == 0, "rows per tile");
};

// Structure of a mode product.
//  kDense:    out[a, i, b] = sum_{k<n} M[i, k] in[a, k, b]                    (M = Q^T or Q)
//  kSplitFwd: Q^T with Q = Z diag(Ve, Vo) (the even/odd block form of a persymmetric D):
//             a row tile lies in the even block (eigen rows [0, me)) or the odd block
//             (rows [me, n)) and contracts only the half-length combination
//             out[a, base + i, b] = sum_{k<K} Mblk[i, k] (in[a, k, b] +- in[a, n-1-k, b]),
//             K = me or mo, with the 1/sqrt(2) (1/2 for the odd-n middle) folded into Mblk.
//  kSplitBwd: Q: two half-length contractions per physical row i < me,
//             p_i = sum_{k<me} Me[i, k] in[a, k, b], q_i = sum_{k<mo} Mo[i, k] in[a, me+k, b],
//             then out[a, i, b] = p_i + q_i and, for i < mo, out[a, n-1-i, b] = p_i - q_i.
// Both split forms do half the multiply-adds of kDense for the same bytes moved.
//  kSplitFwd2: Q^T as kSplitFwd, with both blocks in one tile: each workgroup loads the pair
//             in[a, k, b], in[a, n-1-k, b] once (k < me), forms the sum and the difference,
//             contracts the sum with Fe and the difference with Fo (two accumulator sets) and
//             writes rows base 0 and base me; half the loads and prologue work of kSplitFwd
//             for the same multiply-adds (the odd-n middle difference is exactly zero).
// (the values kDense, kSplitFwd, kSplitBwd, kSplitFwd2 are declared in launch.h: MPLaunch::split)

struct Geo {
  uint32_t A, B;      // batch (slower) and inner (faster) extents, complex elements
  int n, npad;        // axis length; leading dimension of M (of each block matrix when split)
  int ntm;            // number of row tiles
  uint32_t bt;        // N loader: column tiles per batch index
  uint32_t nblocks;   // total workgroups
  int me, mo;         // split: even and odd block sizes
  int te;             // kSplitFwd: row tiles of the even block
  int pad_;
};

template <class R>
struct MfmaT;
template <>
struct MfmaT<float> {
  static constexpr int G = 4;
  typedef float fragT __attribute__((ext_vector_type(4)));
  using acc_t = v4f;
  __device__ __forceinline__ static acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // accumulator slot r of lane l holds row 4*(l/16) + r, column l % 16
  __device__ __forceinline__ static int row(int lane, int r) { return (lane >> 4) * 4 + r; }
};
template <>
struct MfmaT<double> {
  static constexpr int G = 2;
  typedef double fragT __attribute__((ext_vector_type(2)));
  using acc_t = v4d;
  __device__ __forceinline__ static acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // accumulator slot r of lane l holds row (l/16) + 4*r, column l % 16
  __device__ __forceinline__ static int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

// The B loaders move units of G consecutive k-values of one tile column.
// N loader: column b of batch a (element stride B along k).  T loader: row a (k contiguous).
// Loads are raw; the prologue is applied when the unit is written to LDS, so that the
// global loads of the next k-tile stay in flight during the MFMA work of the current one.
// Element k (kb <= k < kb + G) of a B unit is tensor row koff + k, or n - 1 - k when rev;
// rows with k >= klim read as zero.
//
// Each load set of a k-tile (rows koff + k, or n - 1 - k, for k0 <= k < k0 + TK) is read
// through a buffer resource of its own (BView): for the N loader it is based at the set's
// lowest row of batch a0, so that an element's byte offset ((row - rb) B + b) sizeof(C) stays
// below TK B sizeof(C); for the T loader it is based at the tile's first column a0, and the
// offset ((a - a0) n + row) sizeof(C) stays below TNC n sizeof(C).  Both must stay below 2^31
// (kOob): the host launches the WIDE configurations (load_b_unit_wide) for N-loader products
// with 32 B sizeof(C) above that.  Masked elements take offset kOob and read as zero, so that
// every load of a k-tile is issued unconditionally: no branch, no wait inside the loader, and
// 32-bit offsets.
template <class C>
struct BView {
  __amdgpu_buffer_rsrc_t r;
  int rb;  // N loader: tensor row at the base
};

template <class C, int TK, bool TL>
__device__ __forceinline__ BView<C> b_view(const Geo& g, const C* U, uint64_t tbytes, uint32_t a0, int k0, int koff,
                                           bool rev) {
  int rb = 0;
  uint64_t e0;
  if (TL) {
    e0 = (uint64_t)a0 * (uint32_t)g.n;
  } else {
    rb = rev ? max(g.n - k0 - TK, 0) : koff + k0;
    e0 = ((uint64_t)a0 * (uint32_t)g.n + (uint32_t)rb) * g.B;
  }
  const uint64_t left = tbytes - e0 * sizeof(C);
  const uint32_t nrec = left < kBufMaxBytes ? (uint32_t)left : kBufMaxBytes;
  return {buf_rsrc(U + e0, nrec), rb};
}

// The same unit through 64-bit element indices, each element loaded under its own condition:
// for products whose k-tile rows span more than 2 GiB (T::WIDE configurations only).
template <class C, int G, bool TL>
__device__ __forceinline__ void load_b_unit_wide(const Geo& g, const C* __restrict__ U, uint32_t a, uint32_t b,
                                                 int kb, int klim, int koff, bool rev, C (&v)[G]) {
#pragma unroll
  for (int e = 0; e < G; ++e) {
    const int k = kb + e;
    const int row = rev ? g.n - 1 - k : koff + k;
    const bool ok = (TL ? a < g.A : b < g.B) && k < klim;
    const int64_t j = TL ? (int64_t)a * g.n + row : ((int64_t)a * g.n + row) * g.B + b;
    v[e] = ok ? U[j] : C{0, 0};
  }
}

template <class C, int G, bool TL>
__device__ __forceinline__ void load_b_unit(const Geo& g, const BView<C>& vw, uint32_t a0, uint32_t a, uint32_t b,
                                            int kb, int klim, int koff, bool rev, C (&v)[G]) {
  const bool colok = TL ? a < g.A : b < g.B;
  const int row0 = rev ? g.n - 1 - kb : koff + kb;
  const uint32_t st = TL ? (uint32_t)sizeof(C) : g.B * (uint32_t)sizeof(C);
  const uint32_t o0 = TL ? ((a - a0) * (uint32_t)g.n + (uint32_t)row0) * (uint32_t)sizeof(C)
                         : ((uint32_t)(row0 - vw.rb) * g.B + b) * (uint32_t)sizeof(C);
#pragma unroll
  for (int e = 0; e < G; ++e) {
    const uint32_t o = rev ? o0 - (uint32_t)e * st : o0 + (uint32_t)e * st;
    v[e] = buf_load<C>(vw.r, (colok && kb + e < klim) ? o : kOob);
  }
}

template <class C, int G, bool TL, class Pro>
__device__ __forceinline__ void pro_b_unit(const Geo& g, uint32_t a, uint32_t b, int kb, int klim, int koff,
                                           bool rev, const Pro& pro, C (&v)[G]) {
  if constexpr (!Pro::kId && !Pro::kUpdate) {  // the update prologue has its own path
#pragma unroll
    for (int e = 0; e < G; ++e) {
      const int k = kb + e;
      const int row = rev ? g.n - 1 - k : koff + k;
      const bool ok = (TL ? a < g.A : b < g.B) && k < klim;
      const int64_t j = TL ? (int64_t)a * g.n + row : ((int64_t)a * g.n + row) * g.B + b;
      if (ok) v[e] = pro(j, v[e]);
    }
  }
}

// Column context type of an update prologue (zc for the other prologues).
template <class Pro, bool U>
struct UpdColOf {
  using type = zc;
};
template <class Pro>
struct UpdColOf<Pro, true> {
  using type = decltype(std::declval<const Pro&>().col(0u, 0u));
};

// Element accesses of the update-prologue kernels (N loader only: column b of batch a, element
// stride B along k).  Element e of a B unit is tensor row koff + kb + e; upd_offsets gives its
// byte offset, or kOob where the column lies outside the tensor or kb + e >= klim, so that the
// tensor element (ghat), the update's operands and the store of the new state all go through
// bounds-checked buffer accesses at one offset per element: every load of a k-tile is issued
// unconditionally (elements outside read as zero and the update of zeros is zero), and no store
// needs a branch.
template <int G>
__device__ __forceinline__ void upd_offsets(const Geo& g, uint32_t a, uint32_t b, int kb, int klim, int koff,
                                            uint32_t esize, uint32_t (&off)[G]) {
  const bool colok = b < g.B;
  const uint32_t o0 = (((uint32_t)a * (uint32_t)g.n + (uint32_t)(koff + kb)) * g.B + b) * esize;
  const uint32_t st = g.B * esize;
#pragma unroll
  for (int e = 0; e < G; ++e) off[e] = (colok && kb + e < klim) ? o0 + (uint32_t)e * st : kOob;
}

// Bytes of the update prologue's tensors (below kBufMaxBytes, checked by the host).
template <class C>
__device__ __forceinline__ uint32_t upd_bytes(const Geo& g) {
  return g.A * (uint32_t)g.n * g.B * (uint32_t)sizeof(C);
}

template <class C, int G>
__device__ __forceinline__ void load_b_unit_buf(__amdgpu_buffer_rsrc_t rU, const uint32_t (&off)[G], C (&v)[G]) {
#pragma unroll
  for (int e = 0; e < G; ++e) v[e] = buf_load<C>(rU, off[e]);
}

template <class C, int G, class Pro>
__device__ __forceinline__ void pre_b_unit(const Pro& pro, int kb, int klim, int koff, const uint32_t (&off)[G],
                                           uint32_t bytes, typename Pro::Pre (&p)[G]) {
#pragma unroll
  for (int e = 0; e < G; ++e) p[e] = pro.load(off[e], kb + e < klim ? koff + kb + e : 0, bytes);
}

template <class C, int G, class Pro, class Ctx, class RowT>
__device__ __forceinline__ void upd_b_unit(const Pro& pro, int kb, int klim, int koff, const uint32_t (&off)[G],
                                           uint32_t bytes, const Ctx& Eo, const typename Pro::Pre (&p)[G], bool write,
                                           const RowT* rows, C (&v)[G]) {
#pragma unroll
  for (int e = 0; e < G; ++e) {
    // outside the tensor the operands read as zero, so the update gives zero there
    if constexpr (Pro::kRowLds)
      v[e] = pro.update(Eo, rows[(kb + e < klim) ? koff + kb + e : 0], v[e], p[e]);
    else
      v[e] = pro.update(Eo, v[e], p[e]);
    pro.save(write ? off[e] : kOob, v[e], bytes);
  }
}

// ---------------------------------------------------------------------------------------
// Shared epilogue.  get(fm, fn, p, r) returns accumulator slot r (p = 0 real, 1 imaginary)
// of MFMA tile (fm, fn); rowmap(lane, r) its row inside the 16x16 tile.
//  N loader: rows of one column are B elements apart; handled directly, 4 slots at a time.
//  T loader: rows of one column are contiguous in memory, so the tile is passed through LDS
//    in chunks of 16 columns and each wave then walks one column with 64 consecutive rows per
//    instruction (dense 512-byte runs for complex64).
// ---------------------------------------------------------------------------------------

// The T-loader epilogue passes the tile through LDS so that each wave stores dense
// 512-byte runs of one column; building with FCGLE_TL_EPI_DIRECT stores straight from the
// accumulators instead (64-128 byte runs, fewer LDS round trips).  Measured on the 256^3
// workload the LDS form is as fast or faster for every precision.
#ifdef FCGLE_TL_EPI_DIRECT
constexpr bool kTlDirectEpilogue = true;
#else
constexpr bool kTlDirectEpilogue = false;
#endif

// Columns whose epilogue loads are issued together in the T-loader epilogue: at most
// kEpiGroupBytes of loaded operands per lane, and none for functors without loads (their
// stores need no grouping and the extra live values would cost occupancy).  Measured on the
// 256^3 workload, grouping did not speed up the exponential-Euler epilogue, so the budget
// keeps one column at a time for it.
constexpr size_t kEpiGroupBytes = 64;
template <class Pre>
constexpr int epi_column_group(int V, int cpw) {
  if (std::is_same<Pre, NoPre>::value) return 1;
  int cg = (int)(kEpiGroupBytes / (sizeof(Pre) * (size_t)V));
  if (cg < 1) cg = 1;
  if (cg > cpw) cg = cpw;
  while (cpw % cg) --cg;
  return cg;
}

// Rows m0 + r of the tile (r < TM) are valid below row_end; phys(i) maps a valid row to the
// index along the mode axis that the output element has (identity except for the mirrored
// half of kSplitBwd).
template <class R, class T, bool TL, class Epi, class Get, class RowMap, class Phys>
__device__ __forceinline__ void run_epilogue(const Geo& g, uint32_t a_fix, uint32_t c0, int m0, int row_end,
                                             const Epi& epi, Get get, RowMap rowmap, Phys phys, void* smem) {
  using C = typename Cx<R>::T;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / T::WN, wn = wave % T::WN;
  const int lr = lane & 15;
  if (!TL) {
#pragma unroll
    for (int fn = 0; fn < T::FNC; ++fn) {
      const uint32_t col = c0 + wn * T::WTNC + fn * 16 + lr;
      if (col >= g.B) continue;
      const auto ctx = epi.col(a_fix, col);
#pragma unroll
      for (int fm = 0; fm < T::FM; ++fm) {
        int i[4];
        int64_t j[4];
        bool ok[4];
        R re[4], im[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + wm * T::WTM + fm * 16 + rowmap(lane, r);
          ok[r] = row < row_end;
          i[r] = phys(row);
          j[r] = ((int64_t)a_fix * g.n + i[r]) * g.B + col;
          re[r] = get(fm, fn, 0, r);
          im[r] = get(fm, fn, 1, r);
        }
        epi.template apply<4>(ctx, i, j, ok, re, im);
      }
    }
  } else if (kTlDirectEpilogue) {
    // A lane's accumulator slots of one column cover consecutive rows (4 for FP32, 1 per
    // 16-lane group for FP64), so each store instruction writes 64-128 byte runs of 16
    // columns; no LDS round trip and no accumulator copies are needed.
#pragma unroll
    for (int fn = 0; fn < T::FNC; ++fn) {
      const uint32_t col = c0 + wn * T::WTNC + fn * 16 + lr;
      if (col >= g.A) continue;
      const auto ctx = epi.col(col, 0);
#pragma unroll
      for (int fm = 0; fm < T::FM; ++fm) {
        int i[4];
        int64_t j[4];
        bool ok[4];
        R re[4], im[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + wm * T::WTM + fm * 16 + rowmap(lane, r);
          ok[r] = row < row_end;
          i[r] = phys(row);
          j[r] = (int64_t)col * g.n + i[r];
          re[r] = get(fm, fn, 0, r);
          im[r] = get(fm, fn, 1, r);
        }
        epi.template apply<4>(ctx, i, j, ok, re, im);
      }
    }
  } else {
    constexpr int CW = 16;         // columns per LDS chunk
    constexpr int LDC = T::TM + 1; // padded column length in complex elements
    constexpr int V = T::TM / 64;  // rows per lane per column
    C* Cs = reinterpret_cast<C*>(smem);
#pragma unroll
    for (int q = 0; q < T::TNC / CW; ++q) {
#pragma unroll
      for (int fn = 0; fn < T::FNC; ++fn) {
        const int colt = wn * T::WTNC + fn * 16;  // first tile column of this fragment
        if (colt / CW != q) continue;
#pragma unroll
        for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = wm * T::WTM + fm * 16 + rowmap(lane, r);
            Cs[(colt - q * CW + lr) * LDC + row] = mkc<C>(get(fm, fn, 0, r), get(fm, fn, 1, r));
          }
      }
      __syncthreads();
      // each wave owns columns wave, wave + NW, ...; the loads of CG columns are issued
      // together before their stores
      constexpr int CPW = CW / T::NW;
      constexpr int CG = epi_column_group<typename Epi::Pre>(V, CPW);
#pragma unroll
      for (int c1 = 0; c1 < CPW; c1 += CG) {
        int i[CG * V];
        int64_t j[CG * V];
        bool ok[CG * V];
        R re[CG * V], im[CG * V];
        typename Epi::Pre pre[CG * V];
#pragma unroll
        for (int cg = 0; cg < CG; ++cg) {
          const int cc = wave + (c1 + cg) * T::NW;
          const uint32_t col = c0 + q * CW + cc;
          const bool colok = (c1 + cg < CPW) && col < g.A;
#pragma unroll
          for (int v = 0; v < V; ++v) {
            const int row = lane + 64 * v, e = cg * V + v;
            ok[e] = colok && m0 + row < row_end;
            i[e] = phys(m0 + row);
            j[e] = (int64_t)col * g.n + i[e];
            const C x = colok ? Cs[cc * LDC + row] : C{0, 0};
            re[e] = x.x;
            im[e] = x.y;
          }
        }
        epi.template load<CG * V>(i, j, ok, pre);
#pragma unroll
        for (int cg = 0; cg < CG; ++cg) {
          const int cc = wave + (c1 + cg) * T::NW;
          const uint32_t col = c0 + q * CW + cc;
          if (!((c1 + cg < CPW) && col < g.A)) continue;
          const auto ctx = epi.col(col, 0);
          epi.template store<V>(ctx, i + cg * V, j + cg * V, ok + cg * V, re + cg * V, im + cg * V, pre + cg * V);
        }
      }
      __syncthreads();
    }
  }
}

// LDS of the operand tiles of mp_mfma_tile (N loader; the T-loader epilogue may need more),
// and whether the rows of the on-the-fly update fit beside them.
template <class R, class T, int SP>
constexpr size_t mp_operand_lds() {
  constexpr int NB = (SP == kSplitBwd || SP == kSplitFwd2) ? 2 : 1;
  constexpr int LDK = T::TK + (sizeof(R) == 8 ? 2 : 4);
  return (size_t)T::NBUF * NB * T::TM * LDK * sizeof(R) + (size_t)T::NBUF * NB * 2 * T::TNC * LDK * sizeof(R);
}
constexpr size_t kLdsBytes = 163840;  // 160 KB per workgroup on gfx950

template <class C, class T>
constexpr size_t epi_lds_bytes() {
  return (size_t)16 * (T::TM + 1) * sizeof(C);
}

constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }

// ---------------------------------------------------------------------------------------
// FP64 / FP32 MFMA mode product
// ---------------------------------------------------------------------------------------

// One workgroup's tile (logical block index bid) of the mode product described by g, with
// structure SP (kDense / kSplitFwd / kSplitBwd, see Geo).
// LDS bytes of one mp_mfma_tile (operand tiles, or the T-loader epilogue's column chunks).
template <class R, class T, bool TL, int SP>
constexpr size_t mp_tile_lds() {
  constexpr int NB = (SP == kSplitBwd || SP == kSplitFwd2) ? 2 : 1;
  constexpr int LDK = T::TK + MfmaT<R>::G;
  constexpr size_t ab = (size_t)T::NBUF * NB * T::TM * LDK * sizeof(R) + (size_t)T::NBUF * NB * 2 * T::TNC * LDK * sizeof(R);
  return cmax(ab, (TL && !kTlDirectEpilogue) ? (size_t)16 * (T::TM + 1) * sizeof(typename Cx<R>::T) : 0);
}

// smem: mp_tile_lds<R, T, TL, SP>() bytes of LDS owned by the caller (16-byte aligned), so that
// a kernel running tiles of several products in turn gives them one shared block.
template <class R, class T, bool TL, int SP, class Pro, class Epi>
__device__ __forceinline__ void mp_mfma_tile(const Geo& g, const R* __restrict__ M,
                                             const typename Cx<R>::T* __restrict__ U, const Pro& pro,
                                             const Epi& epi, uint32_t bid, unsigned char* smem) {
  using C = typename Cx<R>::T;
  using MT = MfmaT<R>;
  using fragT = typename MT::fragT;
  using acc_t = typename MT::acc_t;
  constexpr int G = MT::G;
  constexpr int TM = T::TM, TNC = T::TNC, TK = T::TK;
  constexpr int NB = (SP == kSplitBwd || SP == kSplitFwd2) ? 2 : 1;  // operand pairs (even / odd block)
  constexpr int LDK = TK + G;  // padded row keeps 16-byte alignment and spreads LDS banks
  static_assert(TK % (4 * G) == 0, "k tile");
  constexpr size_t kAsBytes = (size_t)T::NBUF * NB * TM * LDK * sizeof(R);
  R (*As)[NB][TM * LDK] = reinterpret_cast<R (*)[NB][TM * LDK]>(smem);
  R (*Bs)[NB][2 * TNC * LDK] = reinterpret_cast<R (*)[NB][2 * TNC * LDK]>(smem + kAsBytes);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / T::WN, wn = wave % T::WN;
  const int mt = (int)(bid % (uint32_t)g.ntm);
  const uint32_t ct = bid / (uint32_t)g.ntm;
  // row tile -> block, first row, contraction length, valid rows
  int m0, K, row_end, base = 0;
  bool odd = false;
  const R* Ma = M;
  if (SP == kDense) {
    m0 = mt * TM;
    K = g.n;
    row_end = g.n;
  } else if (SP == kSplitFwd) {
    odd = mt >= g.te;
    m0 = (odd ? mt - g.te : mt) * TM;
    K = odd ? g.mo : g.me;
    row_end = K;
    base = odd ? g.me : 0;
    Ma = M + (odd ? (int64_t)g.npad * g.npad : 0);
  } else {  // kSplitBwd, kSplitFwd2: both blocks, contraction over the even length
    m0 = mt * TM;
    K = g.me;
    row_end = g.me;
  }
  uint32_t a_fix = 0, c0;
  if (TL) {
    c0 = ct * TNC;
  } else {
    a_fix = ct / g.bt;
    c0 = (ct % g.bt) * TNC;
  }

  constexpr int KU = TK / G;  // units per tile row
  constexpr int AU = TM * KU;
  constexpr int AIT = (AU + T::THREADS - 1) / T::THREADS;
  constexpr int BU = TNC * KU;
  constexpr int BIT = (BU + T::THREADS - 1) / T::THREADS;
  constexpr int NR = (SP == kDense) ? 1 : 2;  // B values per unit element (pair or block)

  fragT ra[NB][AIT];
  C rb[NR][BIT][G];
  // update prologue (ProUpdateF, backward split products only): operands loaded with the
  // tile, and the per-unit factor of the other axes (a unit keeps its column for all k)
  constexpr bool UPD = Pro::kUpdate;
  static_assert(!UPD || SP == kSplitBwd, "the update prologue runs on backward even/odd products");
  typename Pro::Pre rp[UPD ? NR : 1][UPD ? BIT : 1][G];
  using ColT = typename UpdColOf<Pro, UPD>::type;
  ColT eo[UPD ? BIT : 1];
  // row entries of the on-the-fly update, staged in LDS for all n rows of the axis
  using RowT = typename std::conditional_t<UPD, Pro, ProUpdateF<R>>::RowEnt;
  constexpr int kRows = Pro::kRowLds ? kOtfMaxRows : 1;
  __shared__ RowT rowtab[kRows];
  if constexpr (Pro::kRowLds) {
    for (int k = tid; k < g.n; k += T::THREADS) rowtab[k] = pro.row_entry(k);
    __syncthreads();
  }

  auto unit_b = [&](int u, int& row, int& kq) {
    if (TL) {
      row = u / KU;
      kq = u % KU;
    } else {
      row = u % TNC;
      kq = u / TNC;
    }
  };
  const uint64_t tbytes = (uint64_t)g.A * (uint32_t)g.n * g.B * sizeof(C);
  const uint32_t a0 = TL ? c0 : a_fix;
  auto gload = [&](int kt) {
    const int k0 = kt * TK;
#pragma unroll
    for (int h = 0; h < NB; ++h) {
      const R* Mh = Ma + (int64_t)h * g.npad * g.npad;
#pragma unroll
      for (int it = 0; it < AIT; ++it) {
        const int u = tid + it * T::THREADS;
        if (AU % T::THREADS == 0 || u < AU) {
          const int row = u / KU, kq = u % KU;
          ra[h][it] = *(const fragT*)&Mh[(int64_t)(m0 + row) * g.npad + k0 + kq * G];
        }
      }
    }
    // the k-tile's B views: set 0 is rows k (koff 0); set 1 is rows n - 1 - k (forward
    // even/odd products) or rows me + k (backward even/odd products)
    const BView<C> v0 = b_view<C, TK, TL>(g, U, tbytes, a0, k0, 0, false);
    const BView<C> v1 = b_view<C, TK, TL>(g, U, tbytes, a0, k0, SP == kSplitBwd ? g.me : 0,
                                          SP == kSplitFwd || SP == kSplitFwd2);
    auto ldb = [&](int set, uint32_t a, uint32_t b, int kb, int klim, int koff, bool rev, C (&dst)[G]) {
      if constexpr (T::WIDE)
        load_b_unit_wide<C, G, TL>(g, U, a, b, kb, klim, koff, rev, dst);
      else
        load_b_unit<C, G, TL>(g, set ? v1 : v0, a0, a, b, kb, klim, koff, rev, dst);
    };
#pragma unroll
    for (int it = 0; it < BIT; ++it) {
      const int u = tid + it * T::THREADS;
      if (BU % T::THREADS == 0 || u < BU) {
        int row, kq;
        unit_b(u, row, kq);
        const uint32_t a = TL ? c0 + row : a_fix, b = TL ? 0 : c0 + row;
        const int kb = k0 + kq * G;
        if (SP == kDense) {
          ldb(0, a, b, kb, g.n, 0, false, rb[0][it]);
        } else if (SP == kSplitFwd) {
          ldb(0, a, b, kb, K, 0, false, rb[0][it]);
          ldb(1, a, b, kb, K, 0, true, rb[NR - 1][it]);
        } else if (SP == kSplitFwd2) {
          ldb(0, a, b, kb, g.me, 0, false, rb[0][it]);
          ldb(1, a, b, kb, g.me, 0, true, rb[NR - 1][it]);
        } else if constexpr (UPD) {
          static_assert(!TL, "the update prologue runs on N-loader products");
          const uint32_t bytes = upd_bytes<C>(g);
          uint32_t o[G];
          upd_offsets<G>(g, a, b, kb, g.me, 0, sizeof(C), o);
          load_b_unit_buf<C, G>(buf_rsrc(U, bytes), o, rb[0][it]);
          pre_b_unit<C, G>(pro, kb, g.me, 0, o, bytes, rp[0][it]);
          upd_offsets<G>(g, a, b, kb, g.mo, g.me, sizeof(C), o);
          load_b_unit_buf<C, G>(buf_rsrc(U, bytes), o, rb[NR - 1][it]);
          pre_b_unit<C, G>(pro, kb, g.mo, g.me, o, bytes, rp[NR - 1][it]);
        } else {
          ldb(0, a, b, kb, g.me, 0, false, rb[0][it]);
          ldb(1, a, b, kb, g.mo, g.me, false, rb[NR - 1][it]);
        }
      }
    }
  };
  auto put_b = [&](R (*dst)[2 * TNC * LDK], int buf, int row, int kq, const C (&v)[G]) {
    fragT re, im;
#pragma unroll
    for (int e = 0; e < G; ++e) {
      re[e] = v[e].x;
      im[e] = v[e].y;
    }
    *(fragT*)&dst[buf][row * LDK + kq * G] = re;
    *(fragT*)&dst[buf][(TNC + row) * LDK + kq * G] = im;
  };
  auto sstore = [&](int buf, int kt) {
    const int k0 = kt * TK;
#pragma unroll
    for (int h = 0; h < NB; ++h)
#pragma unroll
      for (int it = 0; it < AIT; ++it) {
        const int u = tid + it * T::THREADS;
        if (AU % T::THREADS == 0 || u < AU) {
          const int row = u / KU, kq = u % KU;
          *(fragT*)&As[buf][h][row * LDK + kq * G] = ra[h][it];
        }
      }
#pragma unroll
    for (int it = 0; it < BIT; ++it) {
      const int u = tid + it * T::THREADS;
      if (BU % T::THREADS == 0 || u < BU) {
        int row, kq;
        unit_b(u, row, kq);
        const uint32_t a = TL ? c0 + row : a_fix, b = TL ? 0 : c0 + row;
        const int kb = k0 + kq * G;
        if (SP == kDense) {
          pro_b_unit<C, G, TL, Pro>(g, a, b, kb, g.n, 0, false, pro, rb[0][it]);
          put_b(reinterpret_cast<R (*)[2 * TNC * LDK]>(&Bs[0][0]), buf * NB, row, kq, rb[0][it]);
        } else if (SP == kSplitFwd) {
          pro_b_unit<C, G, TL, Pro>(g, a, b, kb, K, 0, false, pro, rb[0][it]);
          pro_b_unit<C, G, TL, Pro>(g, a, b, kb, K, 0, true, pro, rb[NR - 1][it]);
          C v[G];
          const R sg = odd ? (R)-1 : (R)1;
#pragma unroll
          for (int e = 0; e < G; ++e) {
            v[e].x = rb[0][it][e].x + sg * rb[NR - 1][it][e].x;
            v[e].y = rb[0][it][e].y + sg * rb[NR - 1][it][e].y;
          }
          put_b(reinterpret_cast<R (*)[2 * TNC * LDK]>(&Bs[0][0]), buf * NB, row, kq, v);
        } else if (SP == kSplitFwd2) {
          pro_b_unit<C, G, TL, Pro>(g, a, b, kb, g.me, 0, false, pro, rb[0][it]);
          pro_b_unit<C, G, TL, Pro>(g, a, b, kb, g.me, 0, true, pro, rb[NR - 1][it]);
          C sv[G], dv[G];
#pragma unroll
          for (int e = 0; e < G; ++e) {
            sv[e].x = rb[0][it][e].x + rb[NR - 1][it][e].x;
            sv[e].y = rb[0][it][e].y + rb[NR - 1][it][e].y;
            dv[e].x = rb[0][it][e].x - rb[NR - 1][it][e].x;
            dv[e].y = rb[0][it][e].y - rb[NR - 1][it][e].y;
          }
          put_b(reinterpret_cast<R (*)[2 * TNC * LDK]>(&Bs[0][0]), buf * NB, row, kq, sv);
          put_b(reinterpret_cast<R (*)[2 * TNC * LDK]>(&Bs[0][0]), buf * NB + 1, row, kq, dv);
        } else {
          if constexpr (UPD) {
            // the first row tile writes the updated state; every row tile contracts it
            const uint32_t bytes = upd_bytes<C>(g);
            uint32_t o[G];
            upd_offsets<G>(g, a, b, kb, g.me, 0, sizeof(C), o);
            upd_b_unit<C, G>(pro, kb, g.me, 0, o, bytes, eo[it], rp[0][it], mt == 0, rowtab, rb[0][it]);
            upd_offsets<G>(g, a, b, kb, g.mo, g.me, sizeof(C), o);
            upd_b_unit<C, G>(pro, kb, g.mo, g.me, o, bytes, eo[it], rp[NR - 1][it], mt == 0, rowtab,
                                rb[NR - 1][it]);
          }
          put_b(reinterpret_cast<R (*)[2 * TNC * LDK]>(&Bs[0][0]), buf * NB, row, kq, rb[0][it]);
          put_b(reinterpret_cast<R (*)[2 * TNC * LDK]>(&Bs[0][0]), buf * NB + 1, row, kq, rb[NR - 1][it]);
        }
      }
    }
  };

  acc_t acc[NB][T::FM][T::FNC][2];
#pragma unroll
  for (int h = 0; h < NB; ++h)
#pragma unroll
    for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < T::FNC; ++fn)
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int r = 0; r < 4; ++r) acc[h][fm][fn][p][r] = 0;

  const int lr = lane & 15, lk = (lane >> 4) * G;
  // part `part` of `parts` of the tile's MFMA work, split over its (block, row fragment) pairs
  auto compute = [&](int buf, int part, int parts) {
#pragma unroll
    for (int h = 0; h < NB; ++h) {
      const R* as = As[buf][h];
      const R* bs = Bs[buf][h];
      bool any = false;
#pragma unroll
      for (int fm = 0; fm < T::FM; ++fm) any |= (h * T::FM + fm) * parts / (NB * T::FM) == part;
      if (!any) continue;
#pragma unroll
      for (int kg = 0; kg < TK; kg += 4 * G) {
        fragT bf[T::FNC][2];
#pragma unroll
        for (int fn = 0; fn < T::FNC; ++fn)
#pragma unroll
          for (int p = 0; p < 2; ++p)
            bf[fn][p] = *(const fragT*)&bs[(p * TNC + wn * T::WTNC + fn * 16 + lr) * LDK + kg + lk];
#pragma unroll
        for (int fm = 0; fm < T::FM; ++fm) {
          if ((h * T::FM + fm) * parts / (NB * T::FM) != part) continue;
          const fragT af = *(const fragT*)&as[(wm * T::WTM + fm * 16 + lr) * LDK + kg + lk];
#pragma unroll
          for (int s = 0; s < G; ++s)
#pragma unroll
            for (int fn = 0; fn < T::FNC; ++fn)
#pragma unroll
              for (int p = 0; p < 2; ++p)
                acc[h][fm][fn][p] = MT::mma(af[s], bf[fn][p][s], acc[h][fm][fn][p]);
        }
      }
    }
  };

  if constexpr (UPD) {
#pragma unroll
    for (int it = 0; it < BIT; ++it) {
      const int u = tid + it * T::THREADS;
      eo[it] = ColT{};
      if (BU % T::THREADS == 0 || u < BU) {
        int row, kq;
        unit_b(u, row, kq);
        const uint32_t a = TL ? c0 + row : a_fix, b = TL ? 0 : c0 + row;
        if (TL ? a < g.A : b < g.B) eo[it] = pro.col(a, b);
      }
    }
  }
  const int KT = (K + TK - 1) / TK;
  gload(0);
  sstore(0, 0);
  __syncthreads();
  // steady state without conditions; the last tile is contracted after the loop.  The
  // scheduling barriers fix the order of each iteration: the next tile's global loads are all
  // issued first (left to itself the scheduler sinks them towards their use, into the last few
  // MFMAs, where their latency is exposed), then the first part of this tile's MFMA work, the
  // waits for the loads with the prologue and the LDS stores into the other buffer, and the
  // rest of the MFMA work, so that the stores overlap MFMAs and the barrier ends the iteration
  // right after the last of them.  With one buffer the stores wait for every wave's reads; the
  // update prologue (a long VALU block per element) goes after the whole MFMA block, which
  // measured faster for it (122 against 129 us on the 256^3 FP32 product).
  for (int kt = 0; kt + 1 < KT; ++kt) {
    const int cur = (T::NBUF == 2) ? (kt & 1) : 0;
    gload(kt + 1);
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (T::NBUF == 2 && UPD) {
      compute(cur, 0, 1);
      __builtin_amdgcn_sched_barrier(0);
      sstore(cur ^ 1, kt + 1);
    } else if constexpr (T::NBUF == 2) {
      compute(cur, 0, 2);
      __builtin_amdgcn_sched_barrier(0);
      sstore(cur ^ 1, kt + 1);
      __builtin_amdgcn_sched_barrier(0);
      compute(cur, 1, 2);
    } else {
      compute(cur, 0, 1);
      __syncthreads();  // every wave is done reading the one buffer
      sstore(0, kt + 1);
    }
    __syncthreads();
  }
  compute((T::NBUF == 2) ? ((KT - 1) & 1) : 0, 0, 1);
  __syncthreads();

  auto rowmap = [](int l, int r) { return MT::row(l, r); };
  if (SP == kSplitFwd2) {
    run_epilogue<R, T, TL>(
        g, a_fix, c0, m0, g.me, epi, [&](int fm, int fn, int p, int r) { return (R)acc[0][fm][fn][p][r]; },
        rowmap, [](int i) { return i; }, smem);
    run_epilogue<R, T, TL>(
        g, a_fix, c0, g.me + m0, g.me + g.mo, epi,
        [&](int fm, int fn, int p, int r) { return (R)acc[NB - 1][fm][fn][p][r]; }, rowmap,
        [](int i) { return i; }, smem);
  } else if (SP != kSplitBwd) {
    run_epilogue<R, T, TL>(
        g, a_fix, c0, base + m0, base + row_end, epi,
        [&](int fm, int fn, int p, int r) { return (R)acc[0][fm][fn][p][r]; }, rowmap, [](int i) { return i; },
        smem);
  } else {
    const int n1 = g.n - 1;
    run_epilogue<R, T, TL>(
        g, a_fix, c0, m0, g.me, epi,
        [&](int fm, int fn, int p, int r) { return (R)(acc[0][fm][fn][p][r] + acc[NB - 1][fm][fn][p][r]); },
        rowmap, [](int i) { return i; }, smem);
    run_epilogue<R, T, TL>(
        g, a_fix, c0, m0, g.mo, epi,
        [&](int fm, int fn, int p, int r) { return (R)(acc[0][fm][fn][p][r] - acc[NB - 1][fm][fn][p][r]); },
        rowmap, [n1](int i) { return n1 - i; }, smem);
  }
}

// Waves per SIMD asked of the register allocator for a workgroup of T::THREADS threads using
// `lds` bytes of LDS: an 8-wave workgroup whose LDS leaves room for a second one is held to
// 128 VGPRs (4 waves per SIMD), so that two workgroups share a CU and one's prologue and
// epilogue overlap the other's MFMA loop; no request otherwise (1).
template <class T>
constexpr int mp_waves_per_eu(size_t lds) {
  return (T::THREADS == 512 && 2 * lds <= kLdsBytes) ? 4 : 1;
}
template <class R, class Pro>
constexpr size_t pro_row_lds() {
  using RowT = typename std::conditional_t<Pro::kUpdate, Pro, ProUpdateF<R>>::RowEnt;
  return Pro::kRowLds ? (size_t)kOtfMaxRows * sizeof(RowT) : 0;
}

template <class R, class T, bool TL, int SP, class Pro, class Epi>
__global__ void __launch_bounds__(T::THREADS)
    __attribute__((amdgpu_waves_per_eu(mp_waves_per_eu<T>(mp_tile_lds<R, T, TL, SP>() + pro_row_lds<R, Pro>()))))
    mp_mfma_kernel(Geo g, const R* __restrict__ M, const typename Cx<R>::T* __restrict__ U, Pro pro,
                   Epi epi) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[mp_tile_lds<R, T, TL, SP>()];
  mp_mfma_tile<R, T, TL, SP, Pro, Epi>(g, M, U, pro, epi, xcd_remap(blockIdx.x, g.nblocks), smem);
}

// ---------------------------------------------------------------------------------------
// Grouped mode products: one launch covers the same mode product of many independent
// problems (items).  Item k owns logical blocks [first, first + g.nblocks); a workgroup
// finds its item by binary search over `first` (items sorted by it).
// ---------------------------------------------------------------------------------------

template <class Pro, class Epi>
struct GroupItem {
  Geo g;
  const void* M;
  const void* U;
  uint32_t first;
  Pro pro;
  Epi epi;
};

template <class Item>
__device__ __forceinline__ int find_item(const Item* __restrict__ items, int count, uint32_t b) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].first <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <class R, class T, bool TL, int SP, class Pro, class Epi>
__global__ void __launch_bounds__(T::THREADS)
    mp_group_kernel(const GroupItem<Pro, Epi>* __restrict__ items, int count, uint32_t nblocks) {
  const uint32_t b = xcd_remap(blockIdx.x, nblocks);
  const int k = find_item(items, count, b);
  const GroupItem<Pro, Epi>& it = items[k];
  __shared__ __attribute__((aligned(16))) unsigned char smem[mp_tile_lds<R, T, TL, SP>()];
  mp_mfma_tile<R, T, TL, SP, Pro, Epi>(it.g, (const R*)it.M, (const typename Cx<R>::T*)it.U, it.pro, it.epi,
                                       b - it.first, smem);
}

// ---------------------------------------------------------------------------------------
// Persistent batched exponential Euler: one launch runs `steps` steps of every instance.
// The tiles of a launch are numbered in the order (step, phase, instance, tile) with the
// phases F0 (axis-0 forward product, nonlinearity in its loads), F1 (axis-1 forward product
// with the eigenspace update in its stores), B0, B1 (backward products); workgroups take them
// in that order from an atomic ticket.  Each phase of an instance needs the whole result of the
// instance's previous phase, so before a tile the workgroup waits until the instance's count
// of completed tiles reaches the number of tiles that precede its phase; those tiles have
// smaller tickets, were taken by running workgroups and wait only on still smaller ones, so the
// wait always ends, for any grid size.  It is bounded all the same: after `spin_limit` polls
// (about 1 us each) the workgroup raises the error flag and every workgroup leaves.  Completion is published with an
// agent-scope release (stores written back past the workgroup's L2) and observed with an acquire
// (stale lines of the other XCDs' writes invalidated), since consecutive phases of an instance
// may run on different XCDs.  Instances of different sizes overlap across phases instead of
// meeting at a barrier after every phase.
// ---------------------------------------------------------------------------------------

template <class T, int SPF>
__global__ void __launch_bounds__(T::THREADS) batch_persist_kernel(PersistArgs a) {
  using R = float;
  using C = float2;
  using I0 = GroupItem<ProNonlinF<R>, EpiStoreF<R>>;
  using I1 = GroupItem<ProIdF, EpiExpEulerF<R>>;
  using IB = GroupItem<ProIdF, EpiStoreF<R>>;
  constexpr size_t kLds = cmax(cmax(mp_tile_lds<R, T, false, SPF>(), mp_tile_lds<R, T, true, SPF>()),
                               cmax(mp_tile_lds<R, T, false, kSplitBwd>(), mp_tile_lds<R, T, true, kSplitBwd>()));
  __shared__ __attribute__((aligned(16))) unsigned char smem[kLds];
  __shared__ uint32_t s_ticket, s_stop;
  for (;;) {
    if (threadIdx.x == 0) {
      s_ticket = __hip_atomic_fetch_add(&a.ctl->next, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_stop = __hip_atomic_load(&a.ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    const uint32_t tk = s_ticket;
    if (tk >= a.total || s_stop) break;
    const uint32_t step = tk / a.phase0[4], r = tk - step * a.phase0[4];
    const int p = r < a.phase0[1] ? 0 : r < a.phase0[2] ? 1 : r < a.phase0[3] ? 2 : 3;
    const uint32_t b = r - a.phase0[p];
    int i;
    if (p == 0)
      i = find_item((const I0*)a.items[0], a.count, b);
    else if (p == 1)
      i = find_item((const I1*)a.items[1], a.count, b);
    else
      i = find_item((const IB*)a.items[p], a.count, b);
    // wait for the instance's previous phase (its tiles precede this phase within the step).
    // The polls are relaxed loads: an acquire per poll would invalidate the L2 of the XCD on
    // every poll of every waiting workgroup and starve the workgroups doing the work.  The
    // acquire comes once, after the count is reached.
    if (threadIdx.x == 0) {
      const uint32_t need = step * a.pre[5 * i + 4] + a.pre[5 * i + p];
      uint32_t polls = 0;
      while (__hip_atomic_load(&a.done[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
        if (++polls > a.spin_limit || __hip_atomic_load(&a.ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          __hip_atomic_store(&a.ctl->error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          s_stop = 1;
          break;
        }
        __builtin_amdgcn_s_sleep(32);
      }
    }
    __syncthreads();
    if (s_stop) break;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (p == 0) {
      const I0& it = ((const I0*)a.items[0])[i];
      mp_mfma_tile<R, T, false, SPF>(it.g, (const R*)it.M, (const C*)it.U, it.pro, it.epi, b - it.first, smem);
    } else if (p == 1) {
      const I1& it = ((const I1*)a.items[1])[i];
      mp_mfma_tile<R, T, true, SPF>(it.g, (const R*)it.M, (const C*)it.U, it.pro, it.epi, b - it.first, smem);
    } else if (p == 2) {
      const IB& it = ((const IB*)a.items[2])[i];
      mp_mfma_tile<R, T, false, kSplitBwd>(it.g, (const R*)it.M, (const C*)it.U, it.pro, it.epi, b - it.first,
                                           smem);
    } else {
      const IB& it = ((const IB*)a.items[3])[i];
      mp_mfma_tile<R, T, true, kSplitBwd>(it.g, (const R*)it.M, (const C*)it.U, it.pro, it.epi, b - it.first,
                                          smem);
    }
    // publish the tile: every thread's stores, then one count per tile
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(&a.done[i], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---------------------------------------------------------------------------------------
// Split-BF16 MFMA mode product (FP32 data, NP BF16 pieces, FP32 accumulation)
//
// Q is split on the host (in FP64) into NP pieces q = q0 + q1 (+ q2); each loaded FP32
// tensor value is split on the fly, u0 = bf16(u), u1 = bf16(u - u0), u2 = bf16(u - u0 - u1)
// (remainders exact in FP32).  NP = 2 takes q0u0 + q0u1 + q1u0; NP = 3 adds q0u2 + q1u1 + q2u0.
// ---------------------------------------------------------------------------------------

template <int NP>
__device__ __forceinline__ void split_bf16(float x, __bf16 (&p)[NP]) {
  float r = x;
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    p[q] = (__bf16)r;
    r = r - (float)p[q];
  }
}

// Structure SP as for the FP32/FP64 kernels (see Geo).  Block matrices of the split forms
// are stored block-major: block h, piece q at Mp + (h * NP + q) * npad^2.
template <class T, int NP, bool TL, int SP, class Pro, class Epi>
__global__ void __launch_bounds__(T::THREADS)
    mp_bf16_kernel(Geo g, const __bf16* __restrict__ Mp, const float2* __restrict__ U, Pro pro, Epi epi) {
  using C = float2;
  constexpr int TM = T::TM, TNC = T::TNC, TK = T::TK;
  static_assert(TK % 32 == 0, "k tile");
  constexpr int NB = (SP == kSplitBwd || SP == kSplitFwd2) ? 2 : 1;
  constexpr int NR = (SP == kDense) ? 1 : 2;
  constexpr int LDK = TK + 8;  // 16-byte pad
  constexpr int LG = 4;        // B loader unit: 4 consecutive k of one column
  constexpr size_t kAsBytes = (size_t)T::NBUF * NB * NP * TM * LDK * sizeof(__bf16);
  constexpr size_t kBsBytes = (size_t)T::NBUF * NB * NP * 2 * TNC * LDK * sizeof(__bf16);
  constexpr size_t kSmem = cmax(kAsBytes + kBsBytes, (TL && !kTlDirectEpilogue) ? epi_lds_bytes<C, T>() : 0);
  __shared__ __attribute__((aligned(16))) unsigned char smem[kSmem];
  // [buffer][block][piece][...]
  __bf16 (*As)[NB][NP][TM * LDK] = reinterpret_cast<__bf16 (*)[NB][NP][TM * LDK]>(smem);
  __bf16 (*Bs)[NB][NP][2 * TNC * LDK] = reinterpret_cast<__bf16 (*)[NB][NP][2 * TNC * LDK]>(smem + kAsBytes);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / T::WN, wn = wave % T::WN;
  const uint32_t bid = xcd_remap(blockIdx.x, g.nblocks);
  const int mt = (int)(bid % (uint32_t)g.ntm);
  const uint32_t ct = bid / (uint32_t)g.ntm;
  const int64_t piece = (int64_t)g.npad * g.npad;
  int m0, K, row_end, base = 0;
  bool odd = false;
  const __bf16* Ma = Mp;
  if (SP == kDense) {
    m0 = mt * TM;
    K = g.n;
    row_end = g.n;
  } else if (SP == kSplitFwd) {
    odd = mt >= g.te;
    m0 = (odd ? mt - g.te : mt) * TM;
    K = odd ? g.mo : g.me;
    row_end = K;
    base = odd ? g.me : 0;
    Ma = Mp + (odd ? NP * piece : 0);
  } else {
    m0 = mt * TM;
    K = g.me;
    row_end = g.me;
  }
  uint32_t a_fix = 0, c0;
  if (TL) {
    c0 = ct * TNC;
  } else {
    a_fix = ct / g.bt;
    c0 = (ct % g.bt) * TNC;
  }

  constexpr int KUA = TK / 8;  // A units: 8 bf16 (16 bytes)
  constexpr int AU = TM * KUA * NP;
  constexpr int AIT = (AU + T::THREADS - 1) / T::THREADS;
  constexpr int KUB = TK / LG;
  constexpr int BU = TNC * KUB;
  constexpr int BIT = (BU + T::THREADS - 1) / T::THREADS;

  v8bf ra[NB][AIT];
  C rb[NR][BIT][LG];
  // update prologue (ProUpdateF / ProUpdateOtfF, backward split products), as in mp_mfma_tile
  constexpr bool UPD = Pro::kUpdate;
  static_assert(!UPD || SP == kSplitBwd, "the update prologue runs on backward even/odd products");
  typename Pro::Pre rp[UPD ? NR : 1][UPD ? BIT : 1][LG];
  using ColT = typename UpdColOf<Pro, UPD>::type;
  ColT eo[UPD ? BIT : 1];
  using RowT = typename std::conditional_t<UPD, Pro, ProUpdateF<float>>::RowEnt;
  constexpr int kRows = Pro::kRowLds ? kOtfMaxRows : 1;
  __shared__ RowT rowtab[kRows];
  if constexpr (Pro::kRowLds) {
    for (int k = tid; k < g.n; k += T::THREADS) rowtab[k] = pro.row_entry(k);
    __syncthreads();
  }

  auto unit_b = [&](int u, int& row, int& kq) {
    if (TL) {
      row = u / KUB;
      kq = u % KUB;
    } else {
      row = u % TNC;
      kq = u / TNC;
    }
  };
  const uint64_t tbytes = (uint64_t)g.A * (uint32_t)g.n * g.B * sizeof(C);
  const uint32_t a0 = TL ? c0 : a_fix;
  auto gload = [&](int kt) {
    const int k0 = kt * TK;
#pragma unroll
    for (int h = 0; h < NB; ++h)
#pragma unroll
      for (int it = 0; it < AIT; ++it) {
        const int u = tid + it * T::THREADS;
        if (AU % T::THREADS == 0 || u < AU) {
          const int q = u / (TM * KUA), rem = u % (TM * KUA);
          const int row = rem / KUA, kq = rem % KUA;
          ra[h][it] = *(const v8bf*)&Ma[(h * NP + q) * piece + (int64_t)(m0 + row) * g.npad + k0 + kq * 8];
        }
      }
    // the k-tile's B views: set 0 is rows k (koff 0); set 1 is rows n - 1 - k (forward
    // even/odd products) or rows me + k (backward even/odd products)
    const BView<C> v0 = b_view<C, TK, TL>(g, U, tbytes, a0, k0, 0, false);
    const BView<C> v1 = b_view<C, TK, TL>(g, U, tbytes, a0, k0, SP == kSplitBwd ? g.me : 0,
                                          SP == kSplitFwd || SP == kSplitFwd2);
    auto ldb = [&](int set, uint32_t a, uint32_t b, int kb, int klim, int koff, bool rev, C (&dst)[LG]) {
      if constexpr (T::WIDE)
        load_b_unit_wide<C, LG, TL>(g, U, a, b, kb, klim, koff, rev, dst);
      else
        load_b_unit<C, LG, TL>(g, set ? v1 : v0, a0, a, b, kb, klim, koff, rev, dst);
    };
#pragma unroll
    for (int it = 0; it < BIT; ++it) {
      const int u = tid + it * T::THREADS;
      if (BU % T::THREADS == 0 || u < BU) {
        int row, kq;
        unit_b(u, row, kq);
        const uint32_t a = TL ? c0 + row : a_fix, b = TL ? 0 : c0 + row;
        const int kb = k0 + kq * LG;
        if (SP == kDense) {
          ldb(0, a, b, kb, g.n, 0, false, rb[0][it]);
        } else if (SP == kSplitFwd) {
          ldb(0, a, b, kb, K, 0, false, rb[0][it]);
          ldb(1, a, b, kb, K, 0, true, rb[NR - 1][it]);
        } else if (SP == kSplitFwd2) {
          ldb(0, a, b, kb, g.me, 0, false, rb[0][it]);
          ldb(1, a, b, kb, g.me, 0, true, rb[NR - 1][it]);
        } else if constexpr (UPD) {
          static_assert(!TL, "the update prologue runs on N-loader products");
          const uint32_t bytes = upd_bytes<C>(g);
          uint32_t o[LG];
          upd_offsets<LG>(g, a, b, kb, g.me, 0, sizeof(C), o);
          load_b_unit_buf<C, LG>(buf_rsrc(U, bytes), o, rb[0][it]);
          pre_b_unit<C, LG>(pro, kb, g.me, 0, o, bytes, rp[0][it]);
          upd_offsets<LG>(g, a, b, kb, g.mo, g.me, sizeof(C), o);
          load_b_unit_buf<C, LG>(buf_rsrc(U, bytes), o, rb[NR - 1][it]);
          pre_b_unit<C, LG>(pro, kb, g.mo, g.me, o, bytes, rp[NR - 1][it]);
        } else {
          ldb(0, a, b, kb, g.me, 0, false, rb[0][it]);
          ldb(1, a, b, kb, g.mo, g.me, false, rb[NR - 1][it]);
        }
      }
    }
  };
  auto put_b = [&](int buf, int h, int row, int kq, const C (&v)[LG]) {
    v4bf re[NP], im[NP];
#pragma unroll
    for (int e = 0; e < LG; ++e) {
      __bf16 pr[NP], pi[NP];
      split_bf16<NP>(v[e].x, pr);
      split_bf16<NP>(v[e].y, pi);
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        re[q][e] = pr[q];
        im[q][e] = pi[q];
      }
    }
#pragma unroll
    for (int q = 0; q < NP; ++q) {
      *(v4bf*)&Bs[buf][h][q][row * LDK + kq * LG] = re[q];
      *(v4bf*)&Bs[buf][h][q][(TNC + row) * LDK + kq * LG] = im[q];
    }
  };
  auto sstore = [&](int buf, int kt) {
    const int k0 = kt * TK;
#pragma unroll
    for (int h = 0; h < NB; ++h)
#pragma unroll
      for (int it = 0; it < AIT; ++it) {
        const int u = tid + it * T::THREADS;
        if (AU % T::THREADS == 0 || u < AU) {
          const int q = u / (TM * KUA), rem = u % (TM * KUA);
          const int row = rem / KUA, kq = rem % KUA;
          *(v8bf*)&As[buf][h][q][row * LDK + kq * 8] = ra[h][it];
        }
      }
#pragma unroll
    for (int it = 0; it < BIT; ++it) {
      const int u = tid + it * T::THREADS;
      if (BU % T::THREADS == 0 || u < BU) {
        int row, kq;
        unit_b(u, row, kq);
        const uint32_t a = TL ? c0 + row : a_fix, b = TL ? 0 : c0 + row;
        const int kb = k0 + kq * LG;
        if (SP == kDense) {
          pro_b_unit<C, LG, TL, Pro>(g, a, b, kb, g.n, 0, false, pro, rb[0][it]);
          put_b(buf, 0, row, kq, rb[0][it]);
        } else if (SP == kSplitFwd) {
          pro_b_unit<C, LG, TL, Pro>(g, a, b, kb, K, 0, false, pro, rb[0][it]);
          pro_b_unit<C, LG, TL, Pro>(g, a, b, kb, K, 0, true, pro, rb[NR - 1][it]);
          C v[LG];
          const float sg = odd ? -1.0f : 1.0f;
#pragma unroll
          for (int e = 0; e < LG; ++e) {
            v[e].x = rb[0][it][e].x + sg * rb[NR - 1][it][e].x;
            v[e].y = rb[0][it][e].y + sg * rb[NR - 1][it][e].y;
          }
          put_b(buf, 0, row, kq, v);
        } else if (SP == kSplitFwd2) {
          pro_b_unit<C, LG, TL, Pro>(g, a, b, kb, g.me, 0, false, pro, rb[0][it]);
          pro_b_unit<C, LG, TL, Pro>(g, a, b, kb, g.me, 0, true, pro, rb[NR - 1][it]);
          C sv[LG], dv[LG];
#pragma unroll
          for (int e = 0; e < LG; ++e) {
            sv[e].x = rb[0][it][e].x + rb[NR - 1][it][e].x;
            sv[e].y = rb[0][it][e].y + rb[NR - 1][it][e].y;
            dv[e].x = rb[0][it][e].x - rb[NR - 1][it][e].x;
            dv[e].y = rb[0][it][e].y - rb[NR - 1][it][e].y;
          }
          put_b(buf, 0, row, kq, sv);
          put_b(buf, NB - 1, row, kq, dv);
        } else {
          if constexpr (UPD) {
            // the first row tile writes the updated state; every row tile contracts it
            const uint32_t bytes = upd_bytes<C>(g);
            uint32_t o[LG];
            upd_offsets<LG>(g, a, b, kb, g.me, 0, sizeof(C), o);
            upd_b_unit<C, LG>(pro, kb, g.me, 0, o, bytes, eo[it], rp[0][it], mt == 0, rowtab, rb[0][it]);
            upd_offsets<LG>(g, a, b, kb, g.mo, g.me, sizeof(C), o);
            upd_b_unit<C, LG>(pro, kb, g.mo, g.me, o, bytes, eo[it], rp[NR - 1][it], mt == 0, rowtab,
                                rb[NR - 1][it]);
          }
          put_b(buf, 0, row, kq, rb[0][it]);
          put_b(buf, NB - 1, row, kq, rb[NR - 1][it]);
        }
      }
    }
  };

  v4f acc[NB][T::FM][T::FNC][2];
#pragma unroll
  for (int h = 0; h < NB; ++h)
#pragma unroll
    for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < T::FNC; ++fn)
#pragma unroll
        for (int p = 0; p < 2; ++p) acc[h][fm][fn][p] = v4f{0, 0, 0, 0};

  const int lr = lane & 15, lk = (lane >> 4) * 8;
  auto compute = [&](int buf) {
#pragma unroll
    for (int h = 0; h < NB; ++h)
#pragma unroll
      for (int kg = 0; kg < TK; kg += 32) {
        v8bf bf[T::FNC][2][NP];
#pragma unroll
        for (int fn = 0; fn < T::FNC; ++fn)
#pragma unroll
          for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q < NP; ++q)
              bf[fn][p][q] = *(const v8bf*)&Bs[buf][h][q][(p * TNC + wn * T::WTNC + fn * 16 + lr) * LDK + kg + lk];
#pragma unroll
        for (int fm = 0; fm < T::FM; ++fm) {
          v8bf af[NP];
#pragma unroll
          for (int q = 0; q < NP; ++q) af[q] = *(const v8bf*)&As[buf][h][q][(wm * T::WTM + fm * 16 + lr) * LDK + kg + lk];
#pragma unroll
          for (int fn = 0; fn < T::FNC; ++fn)
#pragma unroll
            for (int p = 0; p < 2; ++p) {
              v4f c = acc[h][fm][fn][p];
              // smallest terms first
              if (NP == 3) {
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0], bf[fn][p][NP - 1], c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1], bf[fn][p][1], c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[NP - 1], bf[fn][p][0], c, 0, 0, 0);
              }
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0], bf[fn][p][1], c, 0, 0, 0);
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1], bf[fn][p][0], c, 0, 0, 0);
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0], bf[fn][p][0], c, 0, 0, 0);
              acc[h][fm][fn][p] = c;
            }
        }
      }
  };

  if constexpr (UPD) {
#pragma unroll
    for (int it = 0; it < BIT; ++it) {
      const int u = tid + it * T::THREADS;
      eo[it] = ColT{};
      if (BU % T::THREADS == 0 || u < BU) {
        int row, kq;
        unit_b(u, row, kq);
        const uint32_t a = TL ? c0 + row : a_fix, b = TL ? 0 : c0 + row;
        if (TL ? a < g.A : b < g.B) eo[it] = pro.col(a, b);
      }
    }
  }
  const int KT = (K + TK - 1) / TK;
  gload(0);
  sstore(0, 0);
  __syncthreads();
  // steady state without conditions; the last tile is contracted after the loop.  The
  // scheduling barriers keep each iteration in three phases: the next tile's global loads are
  // all issued first, so that their latency is covered by this tile's whole MFMA block (left to
  // itself the scheduler sinks them towards their use, into the last few MFMAs), and the waits
  // for them, the prologue and the LDS stores follow the block instead of splitting it.
  for (int kt = 0; kt + 1 < KT; ++kt) {
    const int cur = (T::NBUF == 2) ? (kt & 1) : 0;
    gload(kt + 1);
    __builtin_amdgcn_sched_barrier(0);
    compute(cur);
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (T::NBUF == 1) __syncthreads();  // every wave is done reading the one buffer
    sstore(T::NBUF == 2 ? cur ^ 1 : 0, kt + 1);
    __syncthreads();
  }
  compute((T::NBUF == 2) ? ((KT - 1) & 1) : 0);
  __syncthreads();

  auto rowmap = [](int l, int r) { return MfmaT<float>::row(l, r); };
  if (SP == kSplitFwd2) {
    run_epilogue<float, T, TL>(
        g, a_fix, c0, m0, g.me, epi, [&](int fm, int fn, int p, int r) { return acc[0][fm][fn][p][r]; }, rowmap,
        [](int i) { return i; }, smem);
    run_epilogue<float, T, TL>(
        g, a_fix, c0, g.me + m0, g.me + g.mo, epi,
        [&](int fm, int fn, int p, int r) { return acc[NB - 1][fm][fn][p][r]; }, rowmap, [](int i) { return i; },
        smem);
  } else if (SP != kSplitBwd) {
    run_epilogue<float, T, TL>(
        g, a_fix, c0, base + m0, base + row_end, epi,
        [&](int fm, int fn, int p, int r) { return acc[0][fm][fn][p][r]; }, rowmap, [](int i) { return i; }, smem);
  } else {
    const int n1 = g.n - 1;
    run_epilogue<float, T, TL>(
        g, a_fix, c0, m0, g.me, epi,
        [&](int fm, int fn, int p, int r) { return acc[0][fm][fn][p][r] + acc[NB - 1][fm][fn][p][r]; }, rowmap,
        [](int i) { return i; }, smem);
    run_epilogue<float, T, TL>(
        g, a_fix, c0, m0, g.mo, epi,
        [&](int fm, int fn, int p, int r) { return acc[0][fm][fn][p][r] - acc[NB - 1][fm][fn][p][r]; }, rowmap,
        [n1](int i) { return n1 - i; }, smem);
  }
}

// ---------------------------------------------------------------------------------------
// Q-stationary even/odd FP32 mode product (no prologue or the plain nonlinearity, plain
// store).  The two half-size blocks of the operator stay in LDS for the workgroup's lifetime
// (rows and k below KP = 16 MT, k contiguous, rows padded to LDQ floats), and each of the 8
// waves streams column tiles of 16 tensor columns on its own: its B fragments go from global
// memory straight into registers one 16-deep k-chunk ahead of the MFMAs that use them, so
// after the set-up there is no barrier and no LDS store.  (Loading the wave's next tile during
// the last chunk instead of nothing measured slower: its second tile context costs registers.)  SP = kSplitFwd2: the forward fold (pro(x[k]) +
// pro(x[n-1-k]) for the even block, the difference for the odd one, k < m_e), outputs to rows i
// and m_e + i; SP = kSplitBwd: inputs rows k and m_e + k, outputs p + q to rows i and p - q to
// rows n-1-i.  N loader (TL false): a tile is 16 consecutive columns b of one batch index a,
// element (a, row, b) at (a n + row) B + b; T loader (TL true, B = 1): a tile is 16 consecutive
// fibres a, element (a, row) at a n + row.  The MFMA sequence per output element is that of
// mp_mfma_tile (k in steps of 4 per lane group, 16 per chunk, chunks in order), so results are
// the same.  Wave w of workgroup b takes tiles t = 8 b + w, 8 (b + grid) + w, ...; the host keeps
// a tile's offsets below 2^31 (N loader: n B sizeof(float2) < 2^31).
constexpr int kQresWaves = 8;

template <int MT>
constexpr size_t qres_lds_bytes() {
  return (size_t)2 * (16 * MT) * (16 * MT + 4) * sizeof(float);
}

// Where one wave's tile lives: a buffer view of its input and of its output (based at the
// batch index for the N loader, at the tile's first fibre for the T loader), the lane's
// column (N: b; T: fibre offset within the tile) and whether that column exists.
struct QresTile {
  __amdgpu_buffer_rsrc_t rin, rout;
  uint32_t col;
  bool colok;
};

template <bool TL>
__device__ __forceinline__ QresTile qres_tile(const Geo& g, const float2* U, float2* out, uint32_t t, int lr) {
  QresTile q;
  if constexpr (TL) {
    const uint32_t a0 = t * 16;
    const uint64_t left = ((uint64_t)g.A - a0) * (uint32_t)g.n * sizeof(float2);
    const uint32_t nrec = left < kBufMaxBytes ? (uint32_t)left : kBufMaxBytes;
    q.rin = buf_rsrc(U + (uint64_t)a0 * (uint32_t)g.n, nrec);
    q.rout = buf_rsrc(out + (uint64_t)a0 * (uint32_t)g.n, nrec);
    q.col = (uint32_t)lr;
    q.colok = a0 + (uint32_t)lr < g.A;
  } else {
    const uint32_t tilesB = (g.B + 15) / 16, nB = (uint32_t)g.n * g.B;
    const uint32_t a = t / tilesB;
    q.rin = buf_rsrc(U + (uint64_t)a * nB, nB * (uint32_t)sizeof(float2));
    q.rout = buf_rsrc(out + (uint64_t)a * nB, nB * (uint32_t)sizeof(float2));
    q.col = (t % tilesB) * 16 + (uint32_t)lr;
    q.colok = q.col < g.B;
  }
  return q;
}

// Byte offset (from `base`) of row `row` of the lane's column; a masked element gets the top
// bit set (an offset of at least 2^31 = kOob, which the bounds check of a view below 2 GiB
// reads as zero and drops on store): no select the compiler could turn into a branch around
// the access.  The bit is set after the base is added, so no sum wraps into the view.
template <bool TL>
__device__ __forceinline__ uint32_t qres_off(const Geo& g, const QresTile& q, int row, bool ok, uint32_t base = 0) {
  const uint32_t e = TL ? q.col * (uint32_t)g.n + (uint32_t)row : (uint32_t)row * g.B + q.col;
  return (base + e * (uint32_t)sizeof(float2)) | ((uint32_t)(!(ok && q.colok)) << 31);
}

template <int SP, int MT, bool TL, class Pro>
__global__ void __launch_bounds__(64 * kQresWaves)
    mp_qres_kernel(Geo g, const float* __restrict__ M, const float2* __restrict__ U, float2* __restrict__ out, Pro pro) {
  static_assert(SP == kSplitFwd2 || SP == kSplitBwd, "even/odd forms with both blocks");
  constexpr bool UPD = Pro::kUpdate;
  static_assert(Pro::kId || (UPD ? (SP == kSplitBwd && !TL) : SP == kSplitFwd2),
                "the nonlinearity belongs to forward products, the update to N-loader backward ones");
  constexpr int KP = 16 * MT, LDQ = KP + 4;
  constexpr int kRows = UPD ? kOtfMaxRows : 1;
  using RowT = typename std::conditional_t<UPD, Pro, ProUpdateOtfF<float>>::RowEnt;
  static_assert(qres_lds_bytes<MT>() + (UPD ? kRows * sizeof(RowT) : 0) <= kLdsBytes, "both blocks in LDS");
  __shared__ __attribute__((aligned(16))) float qs[2 * KP * LDQ];
  __shared__ RowT rowtab[kRows];
  const int tid = threadIdx.x;
  if constexpr (UPD)
    for (int k = tid; k < g.n; k += 64 * kQresWaves) rowtab[k] = pro.row_entry(k);
  for (int q = tid; q < 2 * KP * (KP / 4); q += 64 * kQresWaves) {
    const int h = q / (KP * (KP / 4)), rem = q % (KP * (KP / 4));
    const int row = rem / (KP / 4), k4 = rem % (KP / 4);
    *(float4*)&qs[(h * KP + row) * LDQ + 4 * k4] =
        *(const float4*)&M[(int64_t)h * g.npad * g.npad + (int64_t)row * g.npad + 4 * k4];
  }
  __syncthreads();
  const int lane = tid & 63, lr = lane & 15, lg = lane >> 4;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t ntiles = TL ? (g.A + 15) / 16 : g.A * ((g.B + 15) / 16);
  const uint32_t stride = gridDim.x * kQresWaves;
  uint32_t t = blockIdx.x * kQresWaves + wave;
  // update prologue: the operands and the new state are addressed over the whole tensor (the
  // host keeps it below 2 GiB), batch index a at byte a n B sizeof(float2)
  const uint32_t ubytes = UPD ? g.A * (uint32_t)g.n * g.B * (uint32_t)sizeof(float2) : 0;
  // the input values of rows k = 16 kc + 4 lg + s (s < 4) of the two sets of tile q (and with
  // the update prologue the state's values at the same elements)
  using PreT = typename std::conditional_t<UPD, Pro, ProUpdateOtfF<float>>::Pre;
  auto load = [&](const QresTile& q, uint32_t gbase, int kc, float2 (&l0)[4], float2 (&l1)[4], PreT (&p0)[4],
                  PreT (&p1)[4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = 16 * kc + 4 * lg + s;
      if constexpr (SP == kSplitFwd2) {
        l0[s] = buf_load<float2>(q.rin, qres_off<TL>(g, q, k, k < g.me));
        l1[s] = buf_load<float2>(q.rin, qres_off<TL>(g, q, g.n - 1 - k, k < g.me));
      } else {
        const uint32_t o0 = qres_off<TL>(g, q, k, k < g.me), o1 = qres_off<TL>(g, q, g.me + k, k < g.mo);
        l0[s] = buf_load<float2>(q.rin, o0);
        l1[s] = buf_load<float2>(q.rin, o1);
        if constexpr (UPD) {
          p0[s] = pro.load(qres_off<TL>(g, q, k, k < g.me, gbase), 0, ubytes);
          p1[s] = pro.load(qres_off<TL>(g, q, g.me + k, k < g.mo, gbase), 0, ubytes);
        }
      }
    }
  };
  for (; t < ntiles; t += stride) {
    const QresTile cur = qres_tile<TL>(g, U, out, t, lr);
    const uint32_t gbase = TL ? 0u : (t / ((g.B + 15) / 16)) * ((uint32_t)g.n * g.B * (uint32_t)sizeof(float2));
    using ColT = typename UpdColOf<Pro, UPD>::type;
    ColT eo{};
    if constexpr (UPD)
      if (cur.colok) eo = pro.col(0u, cur.col);
    float2 x0[4], x1[4];
    PreT p0[4], p1[4];
    load(cur, gbase, 0, x0, x1, p0, p1);
    v4f acc[2][MT][2];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[h][mt][0] = acc[h][mt][1] = v4f{0.f, 0.f, 0.f, 0.f};
    // one chunk per iteration, not unrolled: the chunk's B values are formed from the loads in
    // flight, then the next chunk's loads are issued into the same registers (the scheduling
    // barrier keeps them ahead of the MFMAs), and the MFMAs run row tile by row tile with both
    // blocks' A fragments of that tile from LDS (four independent accumulators per k step)
#pragma unroll 1
    for (int kc = 0; kc < MT; ++kc) {
      float2 bv[2][4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        if constexpr (SP == kSplitFwd2) {
          const float2 p0 = pro(0, x0[s]), p1 = pro(0, x1[s]);
          bv[0][s] = float2{p0.x + p1.x, p0.y + p1.y};
          bv[1][s] = float2{p0.x - p1.x, p0.y - p1.y};
        } else if constexpr (UPD) {
          // the new state of both elements, stored, then contracted
          const int k = 16 * kc + 4 * lg + s;
          const bool ok0 = k < g.me, ok1 = k < g.mo;
          bv[0][s] = pro.update(eo, rowtab[ok0 ? k : 0], x0[s], p0[s]);
          bv[1][s] = pro.update(eo, rowtab[ok1 ? g.me + k : 0], x1[s], p1[s]);
          pro.save(qres_off<TL>(g, cur, k, ok0, gbase), bv[0][s], ubytes);
          pro.save(qres_off<TL>(g, cur, g.me + k, ok1, gbase), bv[1][s], ubytes);
        } else {
          bv[0][s] = x0[s];
          bv[1][s] = x1[s];
        }
      }
      load(cur, gbase, kc + 1 < MT ? kc + 1 : kc, x0, x1, p0, p1);  // the last chunk's reload goes unused
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        float4 af[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) af[h] = *(const float4*)&qs[(h * KP + mt * 16 + lr) * LDQ + 16 * kc + 4 * lg];
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const float av = s == 0 ? af[h].x : s == 1 ? af[h].y : s == 2 ? af[h].z : af[h].w;
            acc[h][mt][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[h][s].x, acc[h][mt][0], 0, 0, 0);
            acc[h][mt][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv[h][s].y, acc[h][mt][1], 0, 0, 0);
          }
      }
    }
    // accumulator slot r of lane l holds row 4 (l / 16) + r of its 16-row tile, column l % 16
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = mt * 16 + 4 * lg + r;
        if constexpr (SP == kSplitFwd2) {
          buf_store(cur.rout, qres_off<TL>(g, cur, i, i < g.me), float2{acc[0][mt][0][r], acc[0][mt][1][r]});
          buf_store(cur.rout, qres_off<TL>(g, cur, g.me + i, i < g.mo), float2{acc[1][mt][0][r], acc[1][mt][1][r]});
        } else {
          buf_store(cur.rout, qres_off<TL>(g, cur, i, i < g.me),
                    float2{acc[0][mt][0][r] + acc[1][mt][0][r], acc[0][mt][1][r] + acc[1][mt][1][r]});
          buf_store(cur.rout, qres_off<TL>(g, cur, g.n - 1 - i, i < g.mo),
                    float2{acc[0][mt][0][r] - acc[1][mt][0][r], acc[0][mt][1][r] - acc[1][mt][1][r]});
        }
      }
  }
}

// Q-stationary even/odd product in split BF16 with two pieces (BF16x3: hi*lo + lo*hi + hi*hi,
// FP32 accumulation), N loader, no prologue or the plain nonlinearity, plain store: the FP32
// kernel above with 32-deep k-chunks (v_mfma_f32_16x16x32_bf16) and both pieces of both blocks
// in LDS (rows below 16 MT, k below 32 KC, KC = ceil(MT / 2), rows padded to LDQ halves).  A
// lane holds k = 32 kc + 8 lg + e, e < 8, of its column, folds (forward) and splits the values
// into pieces in registers; per accumulator the MFMA sequence is that of mp_bf16_kernel
// (chunks in order, hi*lo, lo*hi, hi*hi within a chunk), so results are the same.
template <int MT>
constexpr size_t qres_bf16_lds_bytes() {
  return (size_t)2 * 2 * (16 * MT) * (32 * ((MT + 1) / 2) + 8) * sizeof(__bf16);
}

template <int SP, int MT, class Pro>
__global__ void __launch_bounds__(64 * kQresWaves)
    mp_qres_bf16_kernel(Geo g, const __bf16* __restrict__ Mp, const float2* __restrict__ U, float2* __restrict__ out,
                        Pro pro) {
  static_assert(SP == kSplitFwd2 || SP == kSplitBwd, "even/odd forms with both blocks");
  static_assert(Pro::kId || SP == kSplitFwd2, "the nonlinearity belongs to forward products");
  constexpr int KC = (MT + 1) / 2, KP = 32 * KC, RP = 16 * MT, LDQ = KP + 8;
  static_assert(qres_bf16_lds_bytes<MT>() <= kLdsBytes, "both pieces of both blocks in LDS");
  __shared__ __attribute__((aligned(16))) __bf16 qs[2 * 2 * RP * LDQ];  // [h][piece][row][k]
  const int tid = threadIdx.x;
  const int64_t piece = (int64_t)g.npad * g.npad;
  for (int q = tid; q < 4 * RP * (KP / 8); q += 64 * kQresWaves) {
    const int hq = q / (RP * (KP / 8)), rem = q % (RP * (KP / 8));
    const int row = rem / (KP / 8), k8 = rem % (KP / 8);
    *(v8bf*)&qs[(hq * RP + row) * LDQ + 8 * k8] = *(const v8bf*)&Mp[hq * piece + (int64_t)row * g.npad + 8 * k8];
  }
  __syncthreads();
  const int lane = tid & 63, lr = lane & 15, lg = lane >> 4;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const uint32_t ntiles = g.A * ((g.B + 15) / 16);
  const uint32_t stride = gridDim.x * kQresWaves;
  auto load = [&](const QresTile& q, int kc, float2 (&l0)[8], float2 (&l1)[8]) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = 32 * kc + 8 * lg + e;
      if constexpr (SP == kSplitFwd2) {
        l0[e] = buf_load<float2>(q.rin, qres_off<false>(g, q, k, k < g.me));
        l1[e] = buf_load<float2>(q.rin, qres_off<false>(g, q, g.n - 1 - k, k < g.me));
      } else {
        l0[e] = buf_load<float2>(q.rin, qres_off<false>(g, q, k, k < g.me));
        l1[e] = buf_load<float2>(q.rin, qres_off<false>(g, q, g.me + k, k < g.mo));
      }
    }
  };
  for (uint32_t t = blockIdx.x * kQresWaves + wave; t < ntiles; t += stride) {
    const QresTile cur = qres_tile<false>(g, U, out, t, lr);
    float2 x0[8], x1[8];
    load(cur, 0, x0, x1);
    v4f acc[2][MT][2];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[h][mt][0] = acc[h][mt][1] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int kc = 0; kc < KC; ++kc) {
      // B pieces [block][re/im][piece] of this chunk, then the next chunk's loads
      v8bf bp[2][2][2];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        float2 v[2];
        if constexpr (SP == kSplitFwd2) {
          const float2 p0 = pro(0, x0[e]), p1 = pro(0, x1[e]);
          v[0] = float2{p0.x + p1.x, p0.y + p1.y};
          v[1] = float2{p0.x - p1.x, p0.y - p1.y};
        } else {
          v[0] = x0[e];
          v[1] = x1[e];
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          __bf16 pr[2], pi[2];
          split_bf16<2>(v[h].x, pr);
          split_bf16<2>(v[h].y, pi);
          bp[h][0][0][e] = pr[0];
          bp[h][0][1][e] = pr[1];
          bp[h][1][0][e] = pi[0];
          bp[h][1][1][e] = pi[1];
        }
      }
      load(cur, kc + 1 < KC ? kc + 1 : kc, x0, x1);  // the last chunk's reload goes unused
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        v8bf af[2][2];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int q = 0; q < 2; ++q)
            af[h][q] = *(const v8bf*)&qs[((h * 2 + q) * RP + mt * 16 + lr) * LDQ + 32 * kc + 8 * lg];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int p = 0; p < 2; ++p) {
            v4f c = acc[h][mt][p];
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[h][0], bp[h][p][1], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[h][1], bp[h][p][0], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[h][0], bp[h][p][0], c, 0, 0, 0);
            acc[h][mt][p] = c;
          }
      }
    }
    // accumulator slot r of lane l holds row 4 (l / 16) + r of its 16-row tile, column l % 16
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = mt * 16 + 4 * lg + r;
        if constexpr (SP == kSplitFwd2) {
          buf_store(cur.rout, qres_off<false>(g, cur, i, i < g.me), float2{acc[0][mt][0][r], acc[0][mt][1][r]});
          buf_store(cur.rout, qres_off<false>(g, cur, g.me + i, i < g.mo), float2{acc[1][mt][0][r], acc[1][mt][1][r]});
        } else {
          buf_store(cur.rout, qres_off<false>(g, cur, i, i < g.me),
                    float2{acc[0][mt][0][r] + acc[1][mt][0][r], acc[0][mt][1][r] + acc[1][mt][1][r]});
          buf_store(cur.rout, qres_off<false>(g, cur, g.n - 1 - i, i < g.mo),
                    float2{acc[0][mt][0][r] - acc[1][mt][0][r], acc[0][mt][1][r] - acc[1][mt][1][r]});
        }
      }
  }
}

// ---------------------------------------------------------------------------------------
// Host-side helpers shared by the per-precision dispatch units
// ---------------------------------------------------------------------------------------

template <class T>
inline Geo make_geo(const MPLaunch& L, bool tl, int /*vec_units*/) {
  Geo g;
  g.A = (uint32_t)L.A;
  g.B = (uint32_t)L.B;
  g.n = L.n;
  g.npad = L.npad;
  g.me = L.me;
  g.mo = L.mo;
  g.pad_ = 0;
  if (L.split == kSplitFwd) {
    g.te = (L.me + T::TM - 1) / T::TM;
    g.ntm = g.te + (L.mo + T::TM - 1) / T::TM;
  } else if (L.split == kSplitBwd || L.split == kSplitFwd2) {
    g.te = 0;
    g.ntm = (L.me + T::TM - 1) / T::TM;
  } else {
    g.te = 0;
    g.ntm = (L.n + T::TM - 1) / T::TM;
  }
  if (tl) {
    g.bt = 1;
    g.nblocks = (uint32_t)(((L.A + T::TNC - 1) / T::TNC) * g.ntm);
  } else {
    g.bt = (uint32_t)((L.B + T::TNC - 1) / T::TNC);
    g.nblocks = (uint32_t)(L.A * g.bt * g.ntm);
  }
  return g;
}

}  // namespace fcgle
