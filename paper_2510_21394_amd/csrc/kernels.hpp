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
  ProIdF() = default;
  explicit ProIdF(const ProParams&) {}
  template <class C>
  __device__ __forceinline__ C operator()(int64_t, C u) const {
    return u;
  }
};

// out = cu u + cp up + cg g(t, e),  e = eu u + ep up,
// g(t, e) = gamma e - (kappa + i zeta)|e|^2 e + sum_k sc_k S_k[j]   (Section 2, the map g)
template <class R>
struct ProNonlinF {
  static constexpr bool kId = false;
  using C = typename Cx<R>::T;
  const C* up;
  const C* S[4];
  R sc[4];
  int ns;
  R gamma, kre, kim, eu, ep, cu, cp, cg;
  ProNonlinF() = default;
  explicit ProNonlinF(const ProParams& p) {
    up = (const C*)p.up;
    for (int k = 0; k < 4; ++k) {
      S[k] = (const C*)p.S[k];
      sc[k] = (R)p.sc[k];
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
    C p = {0, 0};
    if (up) p = up[j];
    const R er = eu * u.x + ep * p.x, ei = eu * u.y + ep * p.y;
    const R m = er * er + ei * ei;
    R gr = gamma * er - m * (kre * er - kim * ei);
    R gi = gamma * ei - m * (kre * ei + kim * er);
    for (int k = 0; k < ns; ++k) {
      const C s = S[k][j];
      gr += sc[k] * s.x;
      gi += sc[k] * s.y;
    }
    C o;
    o.x = cu * u.x + cp * p.x + cg * gr;
    o.y = cu * u.y + cp * p.y + cg * gi;
    return o;
  }
};

// ---------------------------------------------------------------------------------------
// Epilogue functors.  col(a, b) is evaluated once per output column (a: flat index over the
// axes slower than mu, b: over the faster ones); op(ctx, i, j, re, im) once per element,
// i being the mode-mu index and j the flat index.
// ---------------------------------------------------------------------------------------

struct NoCtx {};

// Product over the axes other than mu of the separable per-axis factors.
__device__ __forceinline__ zc sep_other(const SepParams& s, uint32_t a, uint32_t b) {
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

template <class R>
struct EpiStoreF {
  using C = typename Cx<R>::T;
  using Ctx = NoCtx;
  C* out;
  EpiStoreF() = default;
  explicit EpiStoreF(const EpiParams& p) : out((C*)p.out) {}
  __device__ __forceinline__ Ctx col(uint32_t, uint32_t) const { return {}; }
  __device__ __forceinline__ void operator()(const Ctx&, int, int64_t j, R re, R im) const {
    C v;
    v.x = re;
    v.y = im;
    out[j] = v;
  }
};

template <class R>
struct EpiGridF {
  using C = typename Cx<R>::T;
  using Ctx = NoCtx;
  C* out;
  const C* F;
  EpiGridF() = default;
  explicit EpiGridF(const EpiParams& p) : out((C*)p.out), F((const C*)p.F) {}
  __device__ __forceinline__ Ctx col(uint32_t, uint32_t) const { return {}; }
  __device__ __forceinline__ void operator()(const Ctx&, int, int64_t j, R re, R im) const {
    const C f = F[j];
    C v;
    v.x = f.x * re - f.y * im;
    v.y = f.x * im + f.y * re;
    out[j] = v;
  }
};

template <class R>
struct EpiSepF {
  using C = typename Cx<R>::T;
  using Ctx = zc;
  C* out;
  SepParams s;
  EpiSepF() = default;
  explicit EpiSepF(const EpiParams& p) : out((C*)p.out), s(p.sep) {}
  __device__ __forceinline__ Ctx col(uint32_t a, uint32_t b) const { return sep_other(s, a, b); }
  __device__ __forceinline__ void operator()(const Ctx& Eo, int i, int64_t j, R re, R im) const {
    const zc E = zmul(Eo, ((const zc*)s.fac[s.mu])[i]);
    out[j] = from_zc<C>(zmul(E, zc{(double)re, (double)im}));
  }
};

// uhat[j] <- E_j uhat[j] + tau P1[j] v   (v = transformed nonlinearity), in FP64.
template <class R>
struct EpiExpEulerF {
  using C = typename Cx<R>::T;
  using Ctx = zc;
  C* uhat;
  const C* P1;
  C* ghat_out;
  SepParams s;
  double tau;
  EpiExpEulerF() = default;
  explicit EpiExpEulerF(const EpiParams& p)
      : uhat((C*)p.out), P1((const C*)p.F), ghat_out((C*)p.ghat_out), s(p.sep), tau(p.tau) {}
  __device__ __forceinline__ Ctx col(uint32_t a, uint32_t b) const { return sep_other(s, a, b); }
  __device__ __forceinline__ void operator()(const Ctx& Eo, int i, int64_t j, R re, R im) const {
    const zc E = zmul(Eo, ((const zc*)s.fac[s.mu])[i]);
    const zc u = to_zc(uhat[j]);
    const zc P = to_zc(P1[j]);
    const zc g{(double)re, (double)im};
    const zc r = zadd(zmul(E, u), zscale(zmul(P, g), tau));
    uhat[j] = from_zc<C>(r);
    if (ghat_out) {
      C gv;
      gv.x = re;
      gv.y = im;
      ghat_out[j] = gv;
    }
  }
};

template <class R>
struct EpiKeepOldF {
  using C = typename Cx<R>::T;
  using Ctx = NoCtx;
  C* out;
  C* save;
  EpiKeepOldF() = default;
  explicit EpiKeepOldF(const EpiParams& p) : out((C*)p.out), save((C*)p.save) {}
  __device__ __forceinline__ Ctx col(uint32_t, uint32_t) const { return {}; }
  __device__ __forceinline__ void operator()(const Ctx&, int, int64_t j, R re, R im) const {
    save[j] = out[j];
    C v;
    v.x = re;
    v.y = im;
    out[j] = v;
  }
};

// ---------------------------------------------------------------------------------------
// Tile configurations and geometry
// ---------------------------------------------------------------------------------------

template <int TM_, int TNC_, int TK_, int WM_, int WN_>
struct TileCfg {
  static constexpr int TM = TM_, TNC = TNC_, TK = TK_, WM = WM_, WN = WN_;
  static constexpr int THREADS = 64 * WM * WN;
  static constexpr int WTM = TM / WM, WTNC = TNC / WN;
  static constexpr int FM = WTM / 16, FNC = WTNC / 16;
  static_assert(FM >= 1 && FNC >= 1 && WTM % 16 == 0 && WTNC % 16 == 0, "wave tile");
};

struct Geo {
  uint32_t A, B;      // batch (slower) and inner (faster) extents, complex elements
  int n, npad;        // contraction length and padded leading dimension of M
  int ntm;            // number of M tiles
  uint32_t bt;        // N loader: column tiles per batch index
  uint32_t nblocks;   // total workgroups
  int vec_ok;         // T loader: rows are 16-byte aligned for vector loads
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

// Load G consecutive-k complex values of one tile column (the "unit" of the B loaders).
// N loader: column b of batch a, k = kb .. kb+G-1 (stride B).  T loader: row a, k contiguous.
template <class C, int G, bool TL, class Pro>
__device__ __forceinline__ void load_b_unit(const Geo& g, const C* __restrict__ U, uint32_t a, uint32_t b,
                                            int kb, const Pro& pro, C (&v)[G]) {
  if (!TL) {
#pragma unroll
    for (int e = 0; e < G; ++e) {
      const int k = kb + e;
      C x = {0, 0};
      if (b < g.B && k < g.n) {
        const int64_t j = ((int64_t)a * g.n + k) * g.B + b;
        x = U[j];
        if (!Pro::kId) x = pro(j, x);
      }
      v[e] = x;
    }
  } else {
    if (a < g.A) {
      const int64_t jb = (int64_t)a * g.n + kb;
      if (g.vec_ok && kb + G <= g.n) {
#pragma unroll
        for (int e = 0; e < G; ++e) v[e] = U[jb + e];
      } else {
#pragma unroll
        for (int e = 0; e < G; ++e) v[e] = (kb + e < g.n) ? U[jb + e] : C{0, 0};
      }
      if (!Pro::kId) {
#pragma unroll
        for (int e = 0; e < G; ++e)
          if (kb + e < g.n) v[e] = pro(jb + e, v[e]);
      }
    } else {
#pragma unroll
      for (int e = 0; e < G; ++e) v[e] = C{0, 0};
    }
  }
}

// ---------------------------------------------------------------------------------------
// FP64 / FP32 MFMA mode product
// ---------------------------------------------------------------------------------------

template <class R, class T, bool TL, class Pro, class Epi>
__global__ void __launch_bounds__(T::THREADS)
    mp_mfma_kernel(Geo g, const R* __restrict__ M, const typename Cx<R>::T* __restrict__ U, Pro pro,
                   Epi epi) {
  using C = typename Cx<R>::T;
  using MT = MfmaT<R>;
  using fragT = typename MT::fragT;
  using acc_t = typename MT::acc_t;
  constexpr int G = MT::G;
  constexpr int TM = T::TM, TNC = T::TNC, TK = T::TK;
  constexpr int LDK = TK + G;  // padded row keeps 16-byte alignment and spreads LDS banks
  static_assert(TK % (4 * G) == 0, "k tile");
  __shared__ __attribute__((aligned(16))) R As[2][TM * LDK];
  __shared__ __attribute__((aligned(16))) R Bs[2][2 * TNC * LDK];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / T::WN, wn = wave % T::WN;
  const uint32_t bid = xcd_remap(blockIdx.x, g.nblocks);
  const int mt = (int)(bid % (uint32_t)g.ntm);
  const uint32_t ct = bid / (uint32_t)g.ntm;
  const int m0 = mt * TM;
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

  fragT ra[AIT];
  C rb[BIT][G];

  auto gload = [&](int kt) {
    const int k0 = kt * TK;
#pragma unroll
    for (int it = 0; it < AIT; ++it) {
      const int u = tid + it * T::THREADS;
      if (AU % T::THREADS == 0 || u < AU) {
        const int row = u / KU, kq = u % KU;
        ra[it] = *(const fragT*)&M[(int64_t)(m0 + row) * g.npad + k0 + kq * G];
      }
    }
#pragma unroll
    for (int it = 0; it < BIT; ++it) {
      const int u = tid + it * T::THREADS;
      if (BU % T::THREADS == 0 || u < BU) {
        int row, kq;
        if (TL) {
          row = u / KU;
          kq = u % KU;
        } else {
          row = u % TNC;
          kq = u / TNC;
        }
        if (TL)
          load_b_unit<C, G, TL, Pro>(g, U, c0 + row, 0, k0 + kq * G, pro, rb[it]);
        else
          load_b_unit<C, G, TL, Pro>(g, U, a_fix, c0 + row, k0 + kq * G, pro, rb[it]);
      }
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int it = 0; it < AIT; ++it) {
      const int u = tid + it * T::THREADS;
      if (AU % T::THREADS == 0 || u < AU) {
        const int row = u / KU, kq = u % KU;
        *(fragT*)&As[buf][row * LDK + kq * G] = ra[it];
      }
    }
#pragma unroll
    for (int it = 0; it < BIT; ++it) {
      const int u = tid + it * T::THREADS;
      if (BU % T::THREADS == 0 || u < BU) {
        int row, kq;
        if (TL) {
          row = u / KU;
          kq = u % KU;
        } else {
          row = u % TNC;
          kq = u / TNC;
        }
        fragT re, im;
#pragma unroll
        for (int e = 0; e < G; ++e) {
          re[e] = rb[it][e].x;
          im[e] = rb[it][e].y;
        }
        *(fragT*)&Bs[buf][row * LDK + kq * G] = re;
        *(fragT*)&Bs[buf][(TNC + row) * LDK + kq * G] = im;
      }
    }
  };

  acc_t acc[T::FM][T::FNC][2];
#pragma unroll
  for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < T::FNC; ++fn)
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[fm][fn][p][r] = 0;

  const int lr = lane & 15, lk = (lane >> 4) * G;
  auto compute = [&](int buf) {
    const R* as = As[buf];
    const R* bs = Bs[buf];
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
        const fragT af = *(const fragT*)&as[(wm * T::WTM + fm * 16 + lr) * LDK + kg + lk];
#pragma unroll
        for (int s = 0; s < G; ++s)
#pragma unroll
          for (int fn = 0; fn < T::FNC; ++fn)
#pragma unroll
            for (int p = 0; p < 2; ++p) acc[fm][fn][p] = MT::mma(af[s], bf[fn][p][s], acc[fm][fn][p]);
      }
    }
  };

  const int KT = (g.n + TK - 1) / TK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < KT; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < KT) gload(kt + 1);
    compute(cur);
    if (kt + 1 < KT) sstore(cur ^ 1);
    __syncthreads();
  }

  // Epilogue: slot r of a lane holds row MT::row(lane, r), column lane % 16 of each 16x16 tile.
#pragma unroll
  for (int fn = 0; fn < T::FNC; ++fn) {
    const uint32_t col = c0 + wn * T::WTNC + fn * 16 + lr;
    const bool cvalid = TL ? (col < g.A) : (col < g.B);
    if (!cvalid) continue;
    const auto ctx = TL ? epi.col(col, 0) : epi.col(a_fix, col);
#pragma unroll
    for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = m0 + wm * T::WTM + fm * 16 + MT::row(lane, r);
        if (i < g.n) {
          const int64_t j = TL ? (int64_t)col * g.n + i : ((int64_t)a_fix * g.n + i) * g.B + col;
          epi(ctx, i, j, (R)acc[fm][fn][0][r], (R)acc[fm][fn][1][r]);
        }
      }
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

template <class T, int NP, bool TL, class Pro, class Epi>
__global__ void __launch_bounds__(T::THREADS)
    mp_bf16_kernel(Geo g, const __bf16* __restrict__ Mp, const float2* __restrict__ U, Pro pro, Epi epi) {
  using C = float2;
  constexpr int TM = T::TM, TNC = T::TNC, TK = T::TK;
  static_assert(TK % 32 == 0, "k tile");
  constexpr int LDK = TK + 8;  // 16-byte pad
  constexpr int LG = 4;        // B loader unit: 4 consecutive k of one column
  __shared__ __attribute__((aligned(16))) __bf16 As[2][NP][TM * LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[2][NP][2 * TNC * LDK];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / T::WN, wn = wave % T::WN;
  const uint32_t bid = xcd_remap(blockIdx.x, g.nblocks);
  const int mt = (int)(bid % (uint32_t)g.ntm);
  const uint32_t ct = bid / (uint32_t)g.ntm;
  const int m0 = mt * TM;
  uint32_t a_fix = 0, c0;
  if (TL) {
    c0 = ct * TNC;
  } else {
    a_fix = ct / g.bt;
    c0 = (ct % g.bt) * TNC;
  }
  const int64_t piece = (int64_t)g.npad * g.npad;

  constexpr int KUA = TK / 8;  // A units: 8 bf16 (16 bytes)
  constexpr int AU = TM * KUA * NP;
  constexpr int AIT = (AU + T::THREADS - 1) / T::THREADS;
  constexpr int KUB = TK / LG;
  constexpr int BU = TNC * KUB;
  constexpr int BIT = (BU + T::THREADS - 1) / T::THREADS;

  v8bf ra[AIT];
  C rb[BIT][LG];

  auto gload = [&](int kt) {
    const int k0 = kt * TK;
#pragma unroll
    for (int it = 0; it < AIT; ++it) {
      const int u = tid + it * T::THREADS;
      if (AU % T::THREADS == 0 || u < AU) {
        const int q = u / (TM * KUA), rem = u % (TM * KUA);
        const int row = rem / KUA, kq = rem % KUA;
        ra[it] = *(const v8bf*)&Mp[q * piece + (int64_t)(m0 + row) * g.npad + k0 + kq * 8];
      }
    }
#pragma unroll
    for (int it = 0; it < BIT; ++it) {
      const int u = tid + it * T::THREADS;
      if (BU % T::THREADS == 0 || u < BU) {
        int row, kq;
        if (TL) {
          row = u / KUB;
          kq = u % KUB;
          load_b_unit<C, LG, TL, Pro>(g, U, c0 + row, 0, k0 + kq * LG, pro, rb[it]);
        } else {
          row = u % TNC;
          kq = u / TNC;
          load_b_unit<C, LG, TL, Pro>(g, U, a_fix, c0 + row, k0 + kq * LG, pro, rb[it]);
        }
      }
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int it = 0; it < AIT; ++it) {
      const int u = tid + it * T::THREADS;
      if (AU % T::THREADS == 0 || u < AU) {
        const int q = u / (TM * KUA), rem = u % (TM * KUA);
        const int row = rem / KUA, kq = rem % KUA;
        *(v8bf*)&As[buf][q][row * LDK + kq * 8] = ra[it];
      }
    }
#pragma unroll
    for (int it = 0; it < BIT; ++it) {
      const int u = tid + it * T::THREADS;
      if (BU % T::THREADS == 0 || u < BU) {
        int row, kq;
        if (TL) {
          row = u / KUB;
          kq = u % KUB;
        } else {
          row = u % TNC;
          kq = u / TNC;
        }
        v4bf re[NP], im[NP];
#pragma unroll
        for (int e = 0; e < LG; ++e) {
          __bf16 pr[NP], pi[NP];
          split_bf16<NP>(rb[it][e].x, pr);
          split_bf16<NP>(rb[it][e].y, pi);
#pragma unroll
          for (int q = 0; q < NP; ++q) {
            re[q][e] = pr[q];
            im[q][e] = pi[q];
          }
        }
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          *(v4bf*)&Bs[buf][q][row * LDK + kq * LG] = re[q];
          *(v4bf*)&Bs[buf][q][(TNC + row) * LDK + kq * LG] = im[q];
        }
      }
    }
  };

  v4f acc[T::FM][T::FNC][2];
#pragma unroll
  for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < T::FNC; ++fn)
#pragma unroll
      for (int p = 0; p < 2; ++p) acc[fm][fn][p] = v4f{0, 0, 0, 0};

  const int lr = lane & 15, lk = (lane >> 4) * 8;
  auto compute = [&](int buf) {
#pragma unroll
    for (int kg = 0; kg < TK; kg += 32) {
      v8bf bf[T::FNC][2][NP];
#pragma unroll
      for (int fn = 0; fn < T::FNC; ++fn)
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int q = 0; q < NP; ++q)
            bf[fn][p][q] = *(const v8bf*)&Bs[buf][q][(p * TNC + wn * T::WTNC + fn * 16 + lr) * LDK + kg + lk];
#pragma unroll
      for (int fm = 0; fm < T::FM; ++fm) {
        v8bf af[NP];
#pragma unroll
        for (int q = 0; q < NP; ++q) af[q] = *(const v8bf*)&As[buf][q][(wm * T::WTM + fm * 16 + lr) * LDK + kg + lk];
#pragma unroll
        for (int fn = 0; fn < T::FNC; ++fn)
#pragma unroll
          for (int p = 0; p < 2; ++p) {
            v4f c = acc[fm][fn][p];
            // smallest terms first
            if (NP == 3) {
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0], bf[fn][p][NP - 1], c, 0, 0, 0);
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1], bf[fn][p][1], c, 0, 0, 0);
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[NP - 1], bf[fn][p][0], c, 0, 0, 0);
            }
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0], bf[fn][p][1], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[1], bf[fn][p][0], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[0], bf[fn][p][0], c, 0, 0, 0);
            acc[fm][fn][p] = c;
          }
      }
    }
  };

  const int KT = (g.n + TK - 1) / TK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < KT; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < KT) gload(kt + 1);
    compute(cur);
    if (kt + 1 < KT) sstore(cur ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int fn = 0; fn < T::FNC; ++fn) {
    const uint32_t col = c0 + wn * T::WTNC + fn * 16 + lr;
    const bool cvalid = TL ? (col < g.A) : (col < g.B);
    if (!cvalid) continue;
    const auto ctx = TL ? epi.col(col, 0) : epi.col(a_fix, col);
#pragma unroll
    for (int fm = 0; fm < T::FM; ++fm)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = m0 + wm * T::WTM + fm * 16 + (lane >> 4) * 4 + r;
        if (i < g.n) {
          const int64_t j = TL ? (int64_t)col * g.n + i : ((int64_t)a_fix * g.n + i) * g.B + col;
          epi(ctx, i, j, acc[fm][fn][0][r], acc[fm][fn][1][r]);
        }
      }
  }
}

// ---------------------------------------------------------------------------------------
// Host-side helpers shared by the per-precision dispatch units
// ---------------------------------------------------------------------------------------

template <class T>
inline Geo make_geo(const MPLaunch& L, bool tl, int vec_units) {
  Geo g;
  g.A = (uint32_t)L.A;
  g.B = (uint32_t)L.B;
  g.n = L.n;
  g.npad = L.npad;
  g.ntm = (L.n + T::TM - 1) / T::TM;
  if (tl) {
    g.bt = 1;
    g.nblocks = (uint32_t)(((L.A + T::TNC - 1) / T::TNC) * g.ntm);
  } else {
    g.bt = (uint32_t)((L.B + T::TNC - 1) / T::TNC);
    g.nblocks = (uint32_t)(L.A * g.bt * g.ntm);
  }
  g.vec_ok = (L.n % vec_units == 0) ? 1 : 0;
  return g;
}

}  // namespace fcgle
