// The plan and the C ABI declared in include/fcgle.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/fcgle.h"
#include "fz.hpp"
#include "host_math.h"
#include "launch.h"
#include "plan.h"

using namespace fcgle;
namespace {

thread_local std::string g_last_error;

}  // namespace

// Work space of the allocation-free entry point fcgle_apply_f_noalloc: three state-sized
// tensors of kNoAllocTensorBytes each in one file-scope device array, which every device the
// library runs on holds from the load of its code object until the process ends.  In host code
// the array's name is only a host-side stand-in: its device address on each device comes from
// hipGetSymbolAddress, resolved once per device when a plan is set up there (with that device
// current), and only that address is ever passed to kernels.
constexpr size_t kNoAllocTensorBytes = (size_t)FCGLE_NOALLOC_TENSOR_BYTES;
static __device__ __align__(256) unsigned char scratch[3 * kNoAllocTensorBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev, which must be current.  A failure leaves the
// entry point unusable on that device (it then reports it) but not the rest of the plan.
void resolve_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev]) return;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess && p)
    g_scratch_ptr[dev] = p;
  else
    (void)hipGetLastError();  // do not leave the failure for the caller's next HIP call
}

unsigned char* scratch_ptr(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return (unsigned char*)g_scratch_ptr[dev];
}

}  // namespace

int fcgle::fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int fcgle::plan_alloc(void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(FCGLE_ERR_NOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
  }
  return FCGLE_OK;
}

namespace {

int precision_of(const fcgle_plan* P) {
  switch (P->prec) {
    case FCGLE_FP64: return P_F64;
    case FCGLE_FP32: return P_F32;
    case FCGLE_BF16X3: return P_BF16X3;
    default: return P_BF16X6;
  }
}

// Upload M (n x n FP64, M[i][k]) in the plan's precision layout, zero padded to npad.
int upload_matrix(fcgle_plan* P, const std::vector<double>& M, int64_t n, int64_t npad, void** dst) {
  const int pr = precision_of(P);
  if (pr == P_F64) {
    std::vector<double> buf(npad * npad, 0.0);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t k = 0; k < n; ++k) buf[i * npad + k] = M[i * n + k];
    FC_TRY(plan_alloc(dst, buf.size() * sizeof(double)));
    HIP_TRY(hipMemcpy(*dst, buf.data(), buf.size() * sizeof(double), hipMemcpyHostToDevice));
  } else if (pr == P_F32) {
    std::vector<float> buf(npad * npad, 0.0f);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t k = 0; k < n; ++k) buf[i * npad + k] = (float)M[i * n + k];
    FC_TRY(plan_alloc(dst, buf.size() * sizeof(float)));
    HIP_TRY(hipMemcpy(*dst, buf.data(), buf.size() * sizeof(float), hipMemcpyHostToDevice));
  } else {
    const int np = (pr == P_BF16X3) ? 2 : 3;
    std::vector<uint16_t> buf(np * npad * npad, 0);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t k = 0; k < n; ++k) {
        double r = M[i * n + k];  // split in FP64: q0 = bf16(q), q1 = bf16(q - q0), ...
        for (int q = 0; q < np; ++q) {
          const uint16_t b = bf16_round(r);
          buf[q * npad * npad + i * npad + k] = b;
          r -= bf16_value(b);
        }
      }
    FC_TRY(plan_alloc(dst, buf.size() * sizeof(uint16_t)));
    HIP_TRY(hipMemcpy(*dst, buf.data(), buf.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
  }
  return FCGLE_OK;
}

// Upload the stacked split block matrices of one axis (split_block_matrices: forward
// [Fe; Fo], backward [Be; Bo], read off the plan's Q), each block ld x ld, in the plan's
// precision.
int upload_split(fcgle_plan* P, int mu) {
  const int64_t ld = P->ldsp[mu];
  std::vector<double> F, B;
  split_block_matrices(P->n[mu], P->me[mu], P->mo[mu], P->Q[mu], ld, F, B);
  const int pr = precision_of(P);
  // FP64 / FP32 as is; split-BF16 as NP pieces per block, block-major ([h][piece][ld x ld]),
  // each entry split in FP64: q0 = bf16(q), q1 = bf16(q - q0), ...
  auto up = [&](const std::vector<double>& M, void** dst) -> int {
    if (pr == P_F64) {
      FC_TRY(plan_alloc(dst, M.size() * sizeof(double)));
      HIP_TRY(hipMemcpy(*dst, M.data(), M.size() * sizeof(double), hipMemcpyHostToDevice));
    } else if (pr == P_F32) {
      std::vector<float> f(M.begin(), M.end());
      FC_TRY(plan_alloc(dst, f.size() * sizeof(float)));
      HIP_TRY(hipMemcpy(*dst, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
    } else {
      const int np = (pr == P_BF16X3) ? 2 : 3;
      const int64_t blk = ld * ld;
      std::vector<uint16_t> b(2 * np * blk, 0);
      for (int h = 0; h < 2; ++h)
        for (int64_t e = 0; e < blk; ++e) {
          double r = M[h * blk + e];
          for (int q = 0; q < np; ++q) {
            const uint16_t bits = bf16_round(r);
            b[(h * np + q) * blk + e] = bits;
            r -= bf16_value(bits);
          }
        }
      FC_TRY(plan_alloc(dst, b.size() * sizeof(uint16_t)));
      HIP_TRY(hipMemcpy(*dst, b.data(), b.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
    }
    return FCGLE_OK;
  };
  FC_TRY(up(F, &P->Mfs[mu]));
  FC_TRY(up(B, &P->Mbs[mu]));
  return FCGLE_OK;
}

SepParams sep_base(const fcgle_plan* P) {
  SepParams s;
  s.d = P->d;
  for (int m = 0; m < P->d; ++m) {
    s.n[m] = (int)P->n[m];
    s.lam[m] = P->dlam[m];
  }
  return s;
}

// Device f-grid for (kind, theta) if it was built, else nullptr.
const void* find_grid(const fcgle_plan* P, int kind, double theta) {
  for (auto& g : P->grids)
    if (g.kind == kind && g.theta == theta) return g.F;
  return nullptr;
}

// Device f-grid for (kind, theta), built on first use.
int get_grid(fcgle_plan* P, int kind, double theta, hipStream_t st, const void** out) {
  if ((*out = find_grid(P, kind, theta)) != nullptr) return FCGLE_OK;
  GridBuf g{kind, theta, nullptr};
  FC_TRY(plan_alloc(&g.F, (size_t)P->N * P->elem));
  SepParams s = sep_base(P);
  HIP_TRY(launch_fgrid(precision_of(P), kind, theta * P->p.nu, theta * P->p.eta, s, P->N, g.F, st));
  P->grids.push_back(g);
  *out = g.F;
  return FCGLE_OK;
}

// Separable exponential factors exp(theta (nu + i eta) lambda_mu[j]) per axis, FP64 on the host.
// e^z - 1 for z = x + i y without cancellation: (expm1(x) cos y - 2 sin^2(y/2)) + i e^x sin y.
zc expm1_c(double x, double y) {
  const double s = std::sin(0.5 * y);
  return zc{std::expm1(x) * std::cos(y) - 2.0 * s * s, std::exp(x) * std::sin(y)};
}

void fill_sep(const SepBuf& e, const fcgle_plan* P, SepParams* sp) {
  for (int m = 0; m < P->d; ++m) {
    sp->fac[m] = e.fac[m];
    sp->facm1[m] = e.facm1[m];
  }
  sp->other_last = e.other_last;
  sp->other_first = e.other_first;
  sp->first_m1 = e.first_m1;
  sp->first_lam = e.first_lam;
  sp->zre = e.theta * P->p.nu;
  sp->zim = e.theta * P->p.eta;
}

// Separable factors for theta into sp if they were built (true), else false.
bool find_sep(const fcgle_plan* P, double theta, SepParams* sp) {
  *sp = sep_base(P);
  for (auto& e : P->seps)
    if (e.theta == theta) {
      fill_sep(e, P, sp);
      return true;
    }
  return false;
}

int get_sep(fcgle_plan* P, double theta, SepParams* sp) {
  if (find_sep(P, theta, sp)) return FCGLE_OK;
  SepBuf e{};
  e.theta = theta;
  int rc = FCGLE_OK;
  for (int m = 0; m < P->d && rc == FCGLE_OK; ++m) {
    std::vector<double> buf(2 * P->n[m]), bm1(2 * P->n[m]);
    for (int64_t j = 0; j < P->n[m]; ++j) {
      const double x = theta * P->p.nu * P->lam[m][j], y = theta * P->p.eta * P->lam[m][j];
      const zc z = fz_eval(1, zc{x, y});
      buf[2 * j] = z.re;
      buf[2 * j + 1] = z.im;
      const zc w = expm1_c(x, y);
      bm1[2 * j] = w.re;
      bm1[2 * j + 1] = w.im;
    }
    rc = plan_alloc(&e.fac[m], buf.size() * sizeof(double));
    if (rc == FCGLE_OK) rc = plan_alloc(&e.facm1[m], bm1.size() * sizeof(double));
    if (rc == FCGLE_OK && (hipMemcpy(e.fac[m], buf.data(), buf.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
                           hipMemcpy(e.facm1[m], bm1.data(), bm1.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess))
      rc = fail(FCGLE_ERR_HIP, "separable factor upload failed");
  }
  // per-column tables for epilogues on the last and on the first axis, and for phi_1 on the
  // fly on the first axis
  const int64_t cl = P->N / P->n[P->d - 1], cf = P->N / P->n[0];
  if (rc == FCGLE_OK) rc = plan_alloc(&e.other_last, (size_t)cl * 2 * sizeof(double));
  if (rc == FCGLE_OK) rc = plan_alloc(&e.other_first, (size_t)cf * 2 * sizeof(double));
  if (rc == FCGLE_OK) rc = plan_alloc(&e.first_m1, (size_t)cf * 2 * sizeof(double));
  if (rc == FCGLE_OK) rc = plan_alloc((void**)&e.first_lam, (size_t)cf * sizeof(double));
  if (rc == FCGLE_OK) {
    fill_sep(e, P, sp);
    if (launch_sep_table(*sp, P->d - 1, cl, e.other_last, nullptr) != hipSuccess ||
        launch_sep_table(*sp, 0, cf, e.other_first, nullptr) != hipSuccess ||
        launch_sep_table_m1(*sp, cf, e.first_m1, e.first_lam, nullptr) != hipSuccess)
      rc = fail(FCGLE_ERR_HIP, "separable factor table: launch failed");
  }
  if (rc == FCGLE_OK && hipDeviceSynchronize() != hipSuccess) rc = fail(FCGLE_ERR_HIP, "separable factor table");
  if (rc != FCGLE_OK) {
    for (int m = 0; m < 4; ++m) {
      if (e.fac[m]) (void)hipFree(e.fac[m]);
      if (e.facm1[m]) (void)hipFree(e.facm1[m]);
    }
    if (e.other_last) (void)hipFree(e.other_last);
    if (e.other_first) (void)hipFree(e.other_first);
    if (e.first_m1) (void)hipFree(e.first_m1);
    if (e.first_lam) (void)hipFree(e.first_lam);
    return rc;
  }
  P->seps.push_back(e);
  return FCGLE_OK;
}

int launch_timed(fcgle_plan* P, const MPLaunch& L, int axis, hipStream_t st) {
  const bool timed = P->timing_cap > 0 && (int)P->timed.size() < P->timing_cap;
  TimedLaunch tl{};
  if (timed) {
    tl.e0 = P->ev_pool[2 * P->timed.size()];
    tl.e1 = P->ev_pool[2 * P->timed.size() + 1];
    tl.axis = axis;
    tl.fwd = L.split ? (L.split != 2 ? 1 : 0) : (L.M == P->Mf[axis] ? 1 : 0);
    tl.sig = L.split * 4096 + ((((L.prec * 8 + L.cfg) * 2 + (L.B == 1 ? 1 : 0)) * 8 + (int)L.pk) * 8) + (int)L.ek;
    HIP_TRY(hipEventRecord(tl.e0, st));
  }
  HIP_TRY(launch_mode_product(L, st));
  if (timed) {
    HIP_TRY(hipEventRecord(tl.e1, st));
    P->timed.push_back(tl);
  }
  return FCGLE_OK;
}

MPLaunch base_launch(const fcgle_plan* P, int mu, bool fwd) {
  MPLaunch L;
  L.prec = precision_of(P);
  L.cfg = P->cfg[mu][fwd ? 1 : 0];
  int64_t A = 1, B = 1;
  for (int m = 0; m < mu; ++m) A *= P->n[m];
  for (int m = mu + 1; m < P->d; ++m) B *= P->n[m];
  L.A = A;
  L.B = B;
  L.n = (int)P->n[mu];
  L.wide = P->wide_force;
  if (P->split) {
    L.split = fwd ? (P->fwd2[mu] ? 3 : 1) : 2;
    L.me = P->me[mu];
    L.mo = P->mo[mu];
    L.npad = P->ldsp[mu];
    L.M = fwd ? P->Mfs[mu] : P->Mbs[mu];
  } else {
    L.npad = P->npad[mu];
    L.M = fwd ? P->Mf[mu] : P->Mb[mu];
  }
  return L;
}

// Whether the backward even/odd tile configuration cfg leaves LDS for the staged rows of the
// on-the-fly update (the same budget the kernels are instantiated under: operand tiles with
// the configuration's k-tile, padded by one MFMA operand group, plus kOtfMaxRows rows of 4
// values of the arithmetic precision: 32 bytes for FP64, 16 bytes for FP32).
bool otf_fits(int pr, int cfg) {
  const size_t tm = (size_t)cfg_rows(pr, cfg, 1), tnc = (size_t)cfg_cols(pr, cfg, 1);
  const size_t nbuf = (size_t)cfg_bufs(pr, cfg, 1);
  size_t ops;
  const size_t tk = (size_t)cfg_tk_split(pr, cfg);
  if (pr == P_F64 || pr == P_F32) {
    const size_t r = (pr == P_F64) ? 8 : 4, ldk = tk + (pr == P_F64 ? 2 : 4);
    ops = nbuf * 2 * tm * ldk * r + nbuf * 2 * 2 * tnc * ldk * r;
  } else {  // split BF16: NP pieces of 2 bytes, k-tiles padded by 8
    const size_t np = (pr == P_BF16X3) ? 2 : 3, ldk = tk + 8;
    ops = nbuf * 2 * np * tm * ldk * 2 + nbuf * 2 * np * 2 * tnc * ldk * 2;
  }
  return ops + (size_t)kOtfMaxRows * (pr == P_F64 ? 32 : 16) <= 163840;
}

// One Tucker operator: out = epi( pro(in) x_1 M_1 ... x_d M_d ) with M = Q^T (fwd) or Q.
// tmp0/tmp1 are scratch tensors distinct from in and from the epilogue's buffers.
int tucker(fcgle_plan* P, bool fwd, const void* in, ProKind pk, const ProParams& pp, EpiKind ek,
           EpiParams ep, void* tmp0, void* tmp1, hipStream_t st) {
  const int pr = precision_of(P);
  void* tmps[2] = {tmp0, tmp1};
  int next_tmp = 0;
  auto pick = [&](const void* avoid) -> void* {
    void* t = tmps[next_tmp];
    if (t == avoid) {
      next_tmp ^= 1;
      t = tmps[next_tmp];
    }
    next_tmp ^= 1;
    return t;
  };
  const void* cur = in;
  // Forward operators may run their mode products from the fastest axis to the slowest, so
  // the epilogue (f-scale, update) lands on an N-loader product (the products commute).
  const bool rev = fwd && P->fwd_rev;
  for (int step = 0; step < P->d; ++step) {
    const int mu = rev ? P->d - 1 - step : step;
    const bool first = (step == 0), last = (step == P->d - 1);
    MPLaunch L = base_launch(P, mu, fwd);
    const bool tl = (L.B == 1);
    L.in = cur;
    if (first && pk != ProKind::Id) {
      if (pk == ProKind::Update || pk == ProKind::UpdateOtf) {
        // no streaming form: callers check update_prologue_ok first
        L.pk = pk;
        L.pp = pp;
        L.pp.sep.mu = mu;
        if (P->cfg_upd >= 0) L.cfg = P->cfg_upd;
        if (pk == ProKind::UpdateOtf && !otf_fits(L.prec, L.cfg)) L.pk = ProKind::Update;  // reads the P1 grid
        if (L.split) L.cfg = cfg_update_tile(L.prec, L.cfg, L.pk == ProKind::UpdateOtf);  // a tile that keeps its registers
      } else if ((pk == ProKind::Flow ? (P->fusion & 64) : (P->fusion & 1)) &&
                 mp_supported(tl, pk, last ? ek : EpiKind::Store)) {
        L.pk = pk;
        L.pp = pp;
      } else {
        void* t = pick(cur);
        HIP_TRY(launch_pointwise_pro(pr, P->N, cur, t, pk, pp, st));
        L.in = t;
      }
    }
    if (last) {
      ep.sep.mu = mu;
      const int epi_bit = (ek == EpiKind::Flow) ? 64 : 2;
      if ((ek == EpiKind::Store || (P->fusion & epi_bit)) && mp_supported(tl, L.pk, ek)) {
        L.ek = ek;
        L.ep = ep;
        FC_TRY(launch_timed(P, L, mu, st));
      } else {
        void* t = pick(L.in);
        L.ek = EpiKind::Store;
        L.ep = EpiParams();
        L.ep.out = t;
        FC_TRY(launch_timed(P, L, mu, st));
        // the streaming pass views the tensor as (rows, n_d) whatever the last product was
        ep.sep.mu = P->d - 1;
        HIP_TRY(launch_pointwise_epi(pr, P->N, (int)P->n[P->d - 1], t, ek, ep, st));
      }
    } else {
      void* t = pick(L.in);
      L.ek = EpiKind::Store;
      L.ep.out = t;
      FC_TRY(launch_timed(P, L, mu, st));
      cur = t;
    }
  }
  return FCGLE_OK;
}

ProParams nonlin_params(const fcgle_plan* P, double t_eval) {
  ProParams pp;
  pp.gamma = P->p.gamma;
  pp.kappa = P->p.kappa;
  pp.zeta = P->p.zeta;
  pp.ns = P->ns;
  for (int k = 0; k < P->ns; ++k) {
    pp.S[k] = P->S[k];
    const double m = std::exp(P->rate[k] * t_eval), ph = P->rate_im[k] * t_eval;
    pp.sc[k] = m * std::cos(ph);
    pp.sci[k] = m * std::sin(ph);
  }
  return pp;
}

int check_plan(const fcgle_plan* P) {
  if (!P) return fail(FCGLE_ERR_ARG, "plan is NULL");
  if (P->batch) return fail(FCGLE_ERR_ARG, "this entry point takes a single-problem plan, not a batch plan");
  return FCGLE_OK;
}

int ensure_state_buffers(fcgle_plan* P) {
  if (!P->uhat) FC_TRY(plan_alloc(&P->uhat, (size_t)P->N * P->elem));
  if (!P->uprev) FC_TRY(plan_alloc(&P->uprev, (size_t)P->N * P->elem));
  return FCGLE_OK;
}

int default_cfg(int pr, int64_t n, bool split) {
  // smallest row tile that covers the rows of one tile column (fewest padded MFMA rows),
  // else the largest; the split forms tile blocks of n - n/2 rows
  const int64_t rows = split ? n - n / 2 : n;
  const int sp = split ? 1 : 0;
  int best = 0;
  for (int c = 0; c < kNumCfg; ++c)
    if (cfg_rows(pr, c, sp) >= rows && cfg_rows(pr, c, sp) <= cfg_rows(pr, best, sp)) best = c;
  return best;
}

// The exponential-Euler update can run in the loads of the first backward product (axis 0,
// N loader) when that product is an even/odd one (any precision) and the state is below 2 GiB
// (its element accesses use 32-bit byte offsets into bounds-checked buffers).
bool update_prologue_ok(const fcgle_plan* P) {
  return P->split && P->d > 1 && (uint64_t)P->N * (uint64_t)P->elem < 0x80000000ull &&
         mp_supported(false, ProKind::Update, EpiKind::Store);
}

// ... and with phi_1 formed on the fly (rows of axis 0 staged in LDS)
bool update_otf_ok(const fcgle_plan* P) { return update_prologue_ok(P) && P->n[0] <= kOtfMaxRows; }


// One exponential-Euler step on the eigenspace state uhat (Section 4, eq. for the scheme):
// ghat = Q^T g(t, u_n), uhat <- E uhat + tau P1 ghat, u <- Q uhat.  With fusion bit 3 the
// update is applied by the first backward product while it loads ghat (the new state goes to
// the second buffer, which then becomes the state); otherwise by the epilogue of the last
// forward product (bit 1) or a streaming pass.
int expeuler_body(fcgle_plan* P, void* u, double t, hipStream_t st) {
  const double tau = P->tau;
  const void* P1;
  FC_TRY(get_grid(P, FCGLE_PHI1, tau, st, &P1));
  SepParams sep;
  FC_TRY(get_sep(P, tau, &sep));
  const ProParams pp = nonlin_params(P, t);  // g(t_n, u_n)
  EpiParams eb;
  eb.out = u;
  if ((P->fusion & 8) && update_prologue_ok(P)) {
    if (!P->uhat2) FC_TRY(plan_alloc(&P->uhat2, (size_t)P->N * P->elem));
    EpiParams eg;
    eg.out = P->s[2];
    FC_TRY(tucker(P, true, u, ProKind::Nonlin, pp, EpiKind::Store, eg, P->s[0], P->s[1], st));
    ProParams up;
    up.uhat = P->uhat;
    up.F = P1;
    up.uhat_out = P->uhat2;
    up.sep = sep;
    up.tau = tau;
    const ProKind pk = ((P->fusion & 32) && update_otf_ok(P)) ? ProKind::UpdateOtf : ProKind::Update;
    FC_TRY(tucker(P, false, P->s[2], pk, up, EpiKind::Store, eb, P->s[0], P->s[1], st));
    std::swap(P->uhat, P->uhat2);
    return FCGLE_OK;
  }
  EpiParams ep;
  ep.out = P->uhat;
  ep.F = P1;
  ep.tau = tau;
  ep.sep = sep;
  FC_TRY(tucker(P, true, u, ProKind::Nonlin, pp, EpiKind::ExpEuler, ep, P->s[0], P->s[1], st));
  FC_TRY(tucker(P, false, P->uhat, ProKind::Id, ProParams(), EpiKind::Store, eb, P->s[0], P->s[1], st));
  return FCGLE_OK;
}

// Scalars of the exact flow over a time t of w' = gamma w - (kappa + i zeta)|w|^2 w
// (Section 4, Strang splitting), in FP64: t phi_1(2 gamma t) = t (e^x - 1)/x with x = 2 gamma t
// (expm1 keeps it accurate for small x), e^{gamma t}, 2 kappa, zeta.
FlowParams flow_params(const fcgle_plan* P, double t) {
  FlowParams f;
  const double x = 2.0 * P->p.gamma * t;
  f.tp1 = (x == 0.0) ? t : t * std::expm1(x) / x;
  f.eg = std::exp(P->p.gamma * t);
  f.k2 = 2.0 * P->p.kappa;
  f.zeta = P->p.zeta;
  return f;
}

// nsteps Strang steps (Section 4, eq. Strang) on u in place.  The e^{tau K} substep runs as
// Q (E . (Q^T v)) with the separable E in the last forward epilogue.  The trailing flow over
// tau/2 of one step and the leading one of the next merge into a single flow over tau
// (phi_{tau/2} o phi_{tau/2} = phi_tau, the flow of an autonomous equation), so a call runs
// phi_{tau/2}, then per step the exponential substep followed by phi_tau, or phi_{tau/2} after
// its last step; only the state at the end of the call is observable.  The flows run as
// streaming passes unless fusion bit 6 puts them into the first forward / last backward product
// (measured at 256^3: the fused flow's log1p and sincos add more to the product than a
// streaming pass costs).
int strang_run(fcgle_plan* P, void* u, int64_t nsteps, hipStream_t st) {
  if (P->ns > 0) return fail(FCGLE_ERR_UNSUPPORTED, "Strang splitting: the exact nonlinear flow takes no source term");
  P->uhat_valid = false;
  P->hist_valid = false;
  const double tau = P->tau;
  ProParams pp;
  pp.flow = flow_params(P, 0.5 * tau);
  const FlowParams full = flow_params(P, tau);
  EpiParams ep;
  ep.out = P->s[2];
  FC_TRY(get_sep(P, tau, &ep.sep));
  // A fused separable exponential is cheapest in the epilogue of an N-loader product (no LDS
  // staging), so the forward products run from the last axis to the first and end on axis 0.
  struct RevGuard {
    fcgle_plan* P;
    bool saved;
    ~RevGuard() { P->fwd_rev = saved; }
  } rev_guard{P, P->fwd_rev};
  if (P->fusion & 2) P->fwd_rev = true;
  for (int64_t k = 0; k < nsteps; ++k) {
    FC_TRY(tucker(P, true, u, k == 0 ? ProKind::Flow : ProKind::Id, pp, EpiKind::Sep, ep, P->s[0], P->s[1], st));
    EpiParams eb;
    eb.out = u;
    eb.flow = (k + 1 == nsteps) ? pp.flow : full;
    FC_TRY(tucker(P, false, P->s[2], ProKind::Id, ProParams(), EpiKind::Flow, eb, P->s[0], P->s[1], st));
  }
  return FCGLE_OK;
}

// One step of Krogstad's fourth-order exponential integrator (Section 4, eq. krogstad-v) with
// the state kept in eigenspace (uhat = Q^T u, cached between steps like exponential Euler's).
// In eigenspace K is (nu + i eta) ell, so the stage values take the exponential form
// u_hat + theta phi_1(theta K) f_n = E_theta u_hat + theta phi_1(theta K) g_n (E_theta = e^{theta K},
// theta phi_1(theta z) z = e^{theta z} - 1), and with d_i = g_i - g_n:
//   A2 = E_{tau/2} uhat + tau/2 P1_{tau/2} g_n                    -> u_2 = Q A2, g_2 = Q^T g(t + tau/2, u_2)
//   A3 = A2 + tau P2_{tau/2} (g_2 - g_n)                          -> g_3 at t + tau/2
//   A4 = E_tau uhat + tau P1_tau g_n + 2 tau P2_tau (g_3 - g_n)    -> g_4 at t + tau
//   uhat' = E_tau uhat + tau P1_tau g_n + tau P2_tau (2 g_2 + 2 g_3 - g_4 - 3 g_n)
//           + tau P3_tau (-4 g_2 - 4 g_3 + 4 g_4 + 4 g_n),        u' = Q uhat'.
// Per step: four forward and four backward Tucker operators (the nonlinearity fused into the
// forward ones) and four streaming combination passes.
int krogstad_body(fcgle_plan* P, void* u, double t, hipStream_t st) {
  const double tau = P->tau;
  for (int k = 0; k < 5; ++k)
    if (!P->kg[k]) FC_TRY(plan_alloc(&P->kg[k], (size_t)P->N * P->elem));
  void* const G0 = P->kg[0];
  void* const G2 = P->kg[1];
  void* const G3 = P->kg[2];
  void* const G4 = P->kg[3];
  void* const A = P->kg[4];
  void* const phys = P->s[2];
  const void *P1h, *P2h, *P1f, *P2f, *P3f;
  FC_TRY(get_grid(P, FCGLE_PHI1, 0.5 * tau, st, &P1h));
  FC_TRY(get_grid(P, FCGLE_PHI2, 0.5 * tau, st, &P2h));
  FC_TRY(get_grid(P, FCGLE_PHI1, tau, st, &P1f));
  FC_TRY(get_grid(P, FCGLE_PHI2, tau, st, &P2f));
  FC_TRY(get_grid(P, FCGLE_PHI3, tau, st, &P3f));
  SepParams Eh, Ef;
  FC_TRY(get_sep(P, 0.5 * tau, &Eh));
  FC_TRY(get_sep(P, tau, &Ef));
  Eh.mu = Ef.mu = P->d - 1;
  const int pr = precision_of(P);
  const int nlast = (int)P->n[P->d - 1];
  // forward transform of g(t_c, v) into G
  auto gtrans = [&](const void* v, double tc, void* G) {
    EpiParams eg;
    eg.out = G;
    return tucker(P, true, v, ProKind::Nonlin, nonlin_params(P, tc), EpiKind::Store, eg, P->s[0], P->s[1], st);
  };
  auto back = [&](const void* vhat, void* out) {
    EpiParams eb;
    eb.out = out;
    return tucker(P, false, vhat, ProKind::Id, ProParams(), EpiKind::Store, eb, P->s[0], P->s[1], st);
  };
  FC_TRY(gtrans(u, t, G0));
  CombParams c;
  c.out = A;
  c.uh = P->uhat;
  c.sep = Eh;
  c.nt = 1;
  c.F[0] = P1h;
  c.v[0] = G0;
  c.c[0][0] = 0.5 * tau;
  HIP_TRY(launch_comb(pr, P->N, nlast, c, st));
  FC_TRY(back(A, phys));
  FC_TRY(gtrans(phys, t + 0.5 * tau, G2));
  c = CombParams();
  c.out = A;
  c.nt = 2;
  c.v[0] = G0;
  c.v[1] = G2;
  c.v[4] = A;
  c.c[0][4] = 1.0;  // A2 (F_0 = 1)
  c.F[1] = P2h;
  c.c[1][1] = tau;
  c.c[1][0] = -tau;
  HIP_TRY(launch_comb(pr, P->N, nlast, c, st));
  FC_TRY(back(A, phys));
  FC_TRY(gtrans(phys, t + 0.5 * tau, G3));
  c = CombParams();
  c.out = A;
  c.uh = P->uhat;
  c.sep = Ef;
  c.nt = 2;
  c.v[0] = G0;
  c.v[2] = G3;
  c.F[0] = P1f;
  c.c[0][0] = tau;
  c.F[1] = P2f;
  c.c[1][2] = 2.0 * tau;
  c.c[1][0] = -2.0 * tau;
  HIP_TRY(launch_comb(pr, P->N, nlast, c, st));
  FC_TRY(back(A, phys));
  FC_TRY(gtrans(phys, t + tau, G4));
  c = CombParams();
  c.out = A;
  c.uh = P->uhat;
  c.sep = Ef;
  c.nt = 3;
  c.v[0] = G0;
  c.v[1] = G2;
  c.v[2] = G3;
  c.v[3] = G4;
  c.F[0] = P1f;
  c.c[0][0] = tau;
  c.F[1] = P2f;
  c.c[1][0] = -3.0 * tau;
  c.c[1][1] = 2.0 * tau;
  c.c[1][2] = 2.0 * tau;
  c.c[1][3] = -tau;
  c.F[2] = P3f;
  c.c[2][0] = 4.0 * tau;
  c.c[2][1] = -4.0 * tau;
  c.c[2][2] = -4.0 * tau;
  c.c[2][3] = 4.0 * tau;
  HIP_TRY(launch_comb(pr, P->N, nlast, c, st));
  FC_TRY(back(A, u));
  std::swap(P->uhat, P->kg[4]);  // the new eigenspace state
  return FCGLE_OK;
}

int step_impl(fcgle_plan* P, int scheme, void* u, double t, hipStream_t st) {
  if (scheme == FCGLE_STRANG) return strang_run(P, u, 1, st);
  FC_TRY(ensure_state_buffers(P));
  const double tau = P->tau;
  if (scheme == FCGLE_EXP_EULER || scheme == FCGLE_KROGSTAD) {
    if (!(P->uhat_valid && P->uhat_src == u)) {
      EpiParams ep;
      ep.out = P->uhat;
      FC_TRY(tucker(P, true, u, ProKind::Id, ProParams(), EpiKind::Store, ep, P->s[0], P->s[1], st));
    }
    P->uhat_valid = false;  // until the step has written the new state
    if (scheme == FCGLE_EXP_EULER)
      FC_TRY(expeuler_body(P, u, t, st));
    else
      FC_TRY(krogstad_body(P, u, t, st));
    P->uhat_valid = true;
    P->uhat_src = u;
    P->hist_valid = false;
    return FCGLE_OK;
  }
  P->uhat_valid = false;
  if (scheme == FCGLE_LAWSON || scheme == FCGLE_LIE ||
      (scheme == FCGLE_LBDF2 && !(P->hist_valid && P->hist_src == u))) {
    // u + tau g(t_n, u_n), then e^{tau K} (Lawson) or (I - tau K)^{-1} (BFE)
    ProParams pp = nonlin_params(P, t);
    pp.cu = 1.0;
    pp.cg = tau;
    EpiParams ep;
    ep.out = P->s[2];
    EpiKind ek;
    if (scheme == FCGLE_LAWSON) {
      ek = EpiKind::Sep;
      FC_TRY(get_sep(P, tau, &ep.sep));
    } else {
      ek = EpiKind::Grid;
      FC_TRY(get_grid(P, FCGLE_INV, tau, st, &ep.F));
    }
    FC_TRY(tucker(P, true, u, ProKind::Nonlin, pp, ek, ep, P->s[0], P->s[1], st));
    EpiParams eb;
    eb.out = u;
    EpiKind ekb = EpiKind::Store;
    if (scheme == FCGLE_LBDF2) {
      eb.save = P->uprev;
      ekb = EpiKind::KeepOld;
    }
    FC_TRY(tucker(P, false, P->s[2], ProKind::Id, ProParams(), ekb, eb, P->s[0], P->s[1], st));
    if (scheme == FCGLE_LBDF2) {
      P->hist_valid = true;
      P->hist_src = u;
    } else {
      P->hist_valid = false;
    }
    return FCGLE_OK;
  }
  if (scheme == FCGLE_LBDF2) {
    // 4/3 u_n - 1/3 u_{n-1} + 2tau/3 g(t_{n+1}, 2u_n - u_{n-1}), then (I - 2tau/3 K)^{-1}
    ProParams pp = nonlin_params(P, t + tau);
    pp.up = P->uprev;
    pp.eu = 2.0;
    pp.ep = -1.0;
    pp.cu = 4.0 / 3.0;
    pp.cp = -1.0 / 3.0;
    pp.cg = 2.0 * tau / 3.0;
    EpiParams ep;
    ep.out = P->s[2];
    FC_TRY(get_grid(P, FCGLE_INV, 2.0 * tau / 3.0, st, &ep.F));
    FC_TRY(tucker(P, true, u, ProKind::Nonlin, pp, EpiKind::Grid, ep, P->s[0], P->s[1], st));
    EpiParams eb;
    eb.out = u;
    eb.save = P->uprev;
    FC_TRY(tucker(P, false, P->s[2], ProKind::Id, ProParams(), EpiKind::KeepOld, eb, P->s[0], P->s[1], st));
    P->hist_valid = true;
    P->hist_src = u;
    return FCGLE_OK;
  }
  return fail(FCGLE_ERR_ARG, "unknown scheme %d", scheme);
}

int ensure_adjoint_buffers(fcgle_plan* P, int64_t m) {
  const size_t bytes = (size_t)P->N * P->elem;
  FC_TRY(ensure_state_buffers(P));
  for (int k = 0; k < 3; ++k)
    if (!P->adj[k]) FC_TRY(plan_alloc(&P->adj[k], bytes));
  const int64_t rows = P->N / P->n[P->d - 1];
  if (!P->partial) {
    FC_TRY(plan_alloc((void**)&P->partial, (size_t)rows * 5 * sizeof(double)));
    P->partial_rows = rows;
  }
  while ((int64_t)P->traj_u.size() < m) {
    void *u = nullptr, *x = nullptr;
    FC_TRY(plan_alloc(&u, bytes));
    if (plan_alloc(&x, bytes) != FCGLE_OK) {
      (void)hipFree(u);
      return FCGLE_ERR_NOMEM;
    }
    P->traj_u.push_back(u);
    P->traj_x.push_back(x);
  }
  return FCGLE_OK;
}

// Adjoint of m exponential-Euler steps from u_start (time t0).  ubar: cotangent of u_m on
// entry, of u_start on exit.  pbar (device, 5 doubles) is added to.
//  1. Recompute u_0..u_{m-1} (physical) and X_0..X_{m-1} with the eigenspace forward step.
//  2. ahat = Q^T ubar; per step backwards: w = Q(tau conj(P1) ahat), pointwise adjoint of g,
//     ahat <- conj(E) ahat + Q^T q (with the nu/eta sums); finally ubar = Q ahat.
int vjp_run_impl(fcgle_plan* P, const void* u_start, int64_t m, void* ubar, double* pbar, double t0,
                 hipStream_t st) {
  if (m == 0) return FCGLE_OK;
  FC_TRY(ensure_adjoint_buffers(P, m));
  const int pr = precision_of(P);
  const double tau = P->tau;
  const size_t bytes = (size_t)P->N * P->elem;
  const int nlast = (int)P->n[P->d - 1];
  const void *P1, *P2;
  FC_TRY(get_grid(P, FCGLE_PHI1, tau, st, &P1));
  FC_TRY(get_grid(P, FCGLE_PHI2, tau, st, &P2));
  SepParams sep;
  FC_TRY(get_sep(P, tau, &sep));
  void *ahat = P->adj[0], *pbuf = P->adj[1], *vbuf = P->adj[2];
  void *s0 = P->s[0], *s1 = P->s[1], *s2 = P->s[2];
  P->uhat_valid = false;  // the recompute below uses the plan's eigenspace buffer
  P->hist_valid = false;

  // 1. forward recompute of the segment
  HIP_TRY(hipMemcpyAsync(P->traj_u[0], u_start, bytes, hipMemcpyDeviceToDevice, st));
  {
    EpiParams ep;
    ep.out = P->uhat;
    FC_TRY(tucker(P, true, P->traj_u[0], ProKind::Id, ProParams(), EpiKind::Store, ep, s0, s1, st));
  }
  for (int64_t k = 0; k < m; ++k) {
    EpiParams ep;
    ep.out = P->uhat;
    ep.F = P1;
    ep.F2 = P2;
    ep.out2 = P->traj_x[k];
    ep.tau = tau;
    ep.sep = sep;
    const ProParams pp = nonlin_params(P, t0 + (double)k * tau);
    FC_TRY(tucker(P, true, P->traj_u[k], ProKind::Nonlin, pp, EpiKind::ExpEulerRec, ep, s0, s1, st));
    if (k + 1 < m) {
      EpiParams eb;
      eb.out = P->traj_u[k + 1];
      FC_TRY(tucker(P, false, P->uhat, ProKind::Id, ProParams(), EpiKind::Store, eb, s0, s1, st));
    }
  }

  // 2. adjoint sweep in eigenspace
  HIP_TRY(launch_fill_zero(P->partial, P->partial_rows * 5, st));
  {
    EpiParams ea;
    ea.out = ahat;
    FC_TRY(tucker(P, true, ubar, ProKind::Id, ProParams(), EpiKind::Store, ea, s0, s1, st));
  }
  HIP_TRY(launch_adj_init(pr, P->N, ahat, P1, tau, pbuf, st));
  for (int64_t k = m - 1; k >= 0; --k) {
    EpiParams ew;
    ew.out = s2;
    FC_TRY(tucker(P, false, pbuf, ProKind::Id, ProParams(), EpiKind::Store, ew, s0, s1, st));
    HIP_TRY(launch_adj_phys(pr, P->N, nlast, s2, P->traj_u[k], P->p.gamma, P->p.kappa, P->p.zeta, P->partial, st));
    EpiParams ev;
    ev.out = vbuf;
    FC_TRY(tucker(P, true, s2, ProKind::Id, ProParams(), EpiKind::Store, ev, s0, s1, st));
    HIP_TRY(launch_adj_hat(pr, P->N, nlast, vbuf, ahat, pbuf, P->traj_x[k], P1, sep, tau, P->partial, st));
  }
  {
    EpiParams eu;
    eu.out = ubar;
    FC_TRY(tucker(P, false, ahat, ProKind::Id, ProParams(), EpiKind::Store, eu, s0, s1, st));
  }
  HIP_TRY(launch_reduce_partials(P->partial, P->partial_rows, 5, pbar, st));
  return FCGLE_OK;
}

// Eigenpairs (Q row-major, column k <-> l[k]) reordered by ascending eigenvalue.
void sorted_eigenpairs(int64_t n, const std::vector<double>& q, const std::vector<double>& l, double* Q,
                       double* lambda) {
  std::vector<int64_t> order(n);
  for (int64_t k = 0; k < n; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return l[a] < l[b]; });
  for (int64_t k = 0; k < n; ++k) {
    lambda[k] = l[order[k]];
    for (int64_t i = 0; i < n; ++i) Q[i * n + k] = q[i * n + order[k]];
  }
}

void free_plan(fcgle_plan* P) {
  auto f = [](void* q) {
    if (q) (void)hipFree(q);
  };
  if (P->batch) {
    batch_free(P->batch);
    P->batch = nullptr;
  }
  for (int m = 0; m < 4; ++m) {
    f(P->Mf[m]);
    f(P->Mb[m]);
    f(P->Mfs[m]);
    f(P->Mbs[m]);
    f(P->dlam[m]);
  }
  for (auto& g : P->grids) f(g.F);
  for (auto& e : P->seps) {
    for (int m = 0; m < 4; ++m) {
      f(e.fac[m]);
      f(e.facm1[m]);
    }
    f(e.other_last);
    f(e.other_first);
    f(e.first_m1);
    f(e.first_lam);
  }
  for (int k = 0; k < 3; ++k) f(P->s[k]);
  for (int m = 0; m < 4; ++m) f(P->Md[m]);
  f(P->rf_r);
  f(P->rf_y);
  f(P->rf_part);
  f(P->uhat);
  f(P->uhat2);
  for (int k = 0; k < 5; ++k) f(P->kg[k]);
  f(P->uprev);
  f(P->dflag);
  for (int k = 0; k < 3; ++k) f(P->adj[k]);
  for (void* q : P->traj_u) f(q);
  for (void* q : P->traj_x) f(q);
  f(P->partial);
  for (auto e : P->ev_pool) (void)hipEventDestroy(e);
  for (auto& g : P->run_graphs) (void)hipGraphExecDestroy(g.exec);
  P->run_graphs.clear();
  if (P->cap_stream) (void)hipStreamDestroy(P->cap_stream);
}

// --- refinement sweep of the inverse ------------------------------------------------

int ensure_refine(fcgle_plan* P) {
  if (!P->Md[0]) {
    for (int m = 0; m < P->d; ++m) {
      // D_mu = -h^{-alpha} Toep(g), g the fractional centred-difference weights
      const int64_t n = P->n[m], np = P->npad[m];
      const std::vector<double> g = fd_weights(P->alpha[m], n, P->fd_order);
      const double scale = -std::pow(P->h[m], -P->alpha[m]);
      std::vector<double> buf(np * np, 0.0);
      for (int64_t i = 0; i < n; ++i)
        for (int64_t k = 0; k < n; ++k) buf[i * np + k] = scale * g[i > k ? i - k : k - i];
      FC_TRY(plan_alloc(&P->Md[m], buf.size() * sizeof(double)));
      HIP_TRY(hipMemcpy(P->Md[m], buf.data(), buf.size() * sizeof(double), hipMemcpyHostToDevice));
    }
  }
  if (!P->rf_r) FC_TRY(plan_alloc(&P->rf_r, (size_t)P->N * 16));
  if (!P->rf_y) FC_TRY(plan_alloc(&P->rf_y, (size_t)P->N * P->elem));
  if (!P->rf_part) FC_TRY(plan_alloc((void**)&P->rf_part, (size_t)(rf_norm_parts() + 16) * sizeof(double)));
  return FCGLE_OK;
}

// rf_r = v - (I - theta (nu + i eta) K) x = v - x + theta (nu + i eta) sum_mu D_mu x_mu x, all in FP64
// (dense FP64 MFMA products with the Toeplitz D_mu accumulating into rf_r).
int refine_residual(fcgle_plan* P, double theta, const void* v, const void* x, hipStream_t st) {
  HIP_TRY(launch_rf_sub(P->N, v, x, P->rf_r, st));
  for (int mu = 0; mu < P->d; ++mu) {
    MPLaunch L;
    L.prec = P_F64;
    L.cfg = default_cfg(P_F64, P->n[mu], false);
    int64_t A = 1, B = 1;
    for (int m = 0; m < mu; ++m) A *= P->n[m];
    for (int m = mu + 1; m < P->d; ++m) B *= P->n[m];
    L.A = A;
    L.B = B;
    L.n = (int)P->n[mu];
    L.npad = P->npad[mu];
    L.M = P->Md[mu];
    L.in = x;
    L.ek = EpiKind::Axpy;
    L.ep.out = P->rf_r;
    L.ep.cre = theta * P->p.nu;
    L.ep.cim = theta * P->p.eta;
    HIP_TRY(launch_mode_product(L, st));
  }
  return FCGLE_OK;
}

// rf_y <- R o rf_y = (I - theta (nu + i eta) K)^{-1} rf_y with the plan's precision
// Steady-state exponential-Euler steps captured once into a HIP graph and replayed: without a
// source term a step launches the same kernels with the same arguments whatever t is, and with
// the update in the backward prologue the two eigenspace buffers trade places every step, so a
// capture of an even number of steps starts and ends in the same buffer assignment and can be
// replayed back to back.  Graphs are keyed by the state buffer, the eigenspace buffers and the
// configuration generation; no memset is captured.
// Steps per captured graph: a run is cut greedily into these (even) chunk lengths, so that runs
// of any length replay graphs, with at most one step left to run directly.
constexpr int64_t kGraphChunks[] = {64, 16, 4, 2};
constexpr size_t kMaxRunGraphs = 8;

int run_graph(fcgle_plan* P, void* u, int64_t steps, hipGraphExec_t* out) {
  for (auto& g : P->run_graphs)
    if (g.u == u && g.uhat == P->uhat && g.uhat2 == P->uhat2 && g.steps == steps && g.gen == P->gen) {
      *out = g.exec;
      return FCGLE_OK;
    }
  if (!P->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
  void* const uh = P->uhat;
  void* const uh2 = P->uhat2;
  HIP_TRY(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal));
  int rc = FCGLE_OK;
  for (int64_t k = 0; k < steps && rc == FCGLE_OK; ++k) rc = step_impl(P, FCGLE_EXP_EULER, u, 0.0, P->cap_stream);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(P->cap_stream, &graph);
  P->uhat = uh;  // nothing ran: the buffers keep their roles (an even count swaps them back anyway)
  P->uhat2 = uh2;
  if (rc != FCGLE_OK || e != hipSuccess || !graph) {
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    return rc != FCGLE_OK ? rc : fail(FCGLE_ERR_HIP, "run graph capture: %s", hipGetErrorString(e));
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) return fail(FCGLE_ERR_HIP, "run graph instantiate: %s", hipGetErrorString(ei));
  if (P->run_graphs.size() >= kMaxRunGraphs) {
    (void)hipGraphExecDestroy(P->run_graphs.front().exec);
    P->run_graphs.erase(P->run_graphs.begin());
  }
  P->run_graphs.push_back(RunGraph{u, uh, uh2, steps, P->gen, exec});
  *out = exec;
  return FCGLE_OK;
}

// nsteps exponential-Euler steps from t0 with the steady-state ones replayed from graphs (no
// source term, timing off).  The first step runs directly unless the state of u is cached and a
// step already ran directly under the plan's current configuration: that step forms the
// eigenspace state if needed and builds the grids, tables and buffers that the captured steps
// then only read.  An odd remainder is run directly at the end.
int expeuler_run(fcgle_plan* P, void* u, double t0, int64_t nsteps, hipStream_t st) {
  int64_t k = 0;
  const bool ready = P->uhat_valid && P->uhat_src == u && P->ready_gen == P->gen;
  if (nsteps > 0 && !ready) {
    FC_TRY(step_impl(P, FCGLE_EXP_EULER, u, t0, st));
    P->ready_gen = P->gen;
    k = 1;
  }
  for (const int64_t chunk : kGraphChunks) {
    static_assert(kGraphChunks[0] % 2 == 0 && kGraphChunks[3] % 2 == 0,
                  "a replayed run must keep the eigenspace buffer assignment");
    while (nsteps - k >= chunk) {
      hipGraphExec_t exec;
      FC_TRY(run_graph(P, u, chunk, &exec));
      HIP_TRY(hipGraphLaunch(exec, st));
      P->uhat_valid = true;
      P->uhat_src = u;
      P->hist_valid = false;
      k += chunk;
    }
  }
  for (; k < nsteps; ++k) FC_TRY(step_impl(P, FCGLE_EXP_EULER, u, t0 + (double)k * P->tau, st));
  return FCGLE_OK;
}

int refine_inverse(fcgle_plan* P, double theta, hipStream_t st) {
  EpiParams ep;
  ep.out = P->s[2];
  FC_TRY(get_grid(P, FCGLE_INV, theta, st, &ep.F));
  FC_TRY(tucker(P, true, P->rf_y, ProKind::Id, ProParams(), EpiKind::Grid, ep, P->s[0], P->s[1], st));
  EpiParams eb;
  eb.out = P->rf_y;
  FC_TRY(tucker(P, false, P->s[2], ProKind::Id, ProParams(), EpiKind::Store, eb, P->s[0], P->s[1], st));
  return FCGLE_OK;
}

}  // namespace

// ---------------------------------------------------------------------------------------
// Exported entry points
// ---------------------------------------------------------------------------------------

extern "C" {

const char* fcgle_last_error(void) { return g_last_error.c_str(); }

int fcgle_host_fd_weights(double alpha, int64_t n, int fd_order, double* g) {
  if (!g || n < 1 || !(alpha > 0.0 && alpha <= 2.0) || (fd_order != 2 && fd_order != 4))
    return fail(FCGLE_ERR_ARG, "fd_weights: bad argument");
  const std::vector<double> w = fd_weights(alpha, n, fd_order);
  std::memcpy(g, w.data(), n * sizeof(double));
  return FCGLE_OK;
}

int fcgle_host_eig(int64_t n, double alpha, double h, int fd_order, double* Q, double* lambda) {
  if (!Q || !lambda || n < 1 || n > 8192 || !(alpha > 0.0 && alpha <= 2.0) || !(h > 0.0) ||
      (fd_order != 2 && fd_order != 4))
    return fail(FCGLE_ERR_ARG, "host_eig: bad argument");
  SplitEig se;
  if (!toeplitz_eig_split(n, alpha, h, fd_order, se)) return fail(FCGLE_ERR_ARG, "host_eig: QR did not converge");
  sorted_eigenpairs(n, se.Q, se.lam, Q, lambda);
  return FCGLE_OK;
}

int fcgle_host_fz(int kind, int64_t count, const double* z, double* out) {
  if (kind < FCGLE_INV || kind > FCGLE_PHI3 || count < 0 || (count > 0 && (!z || !out)))
    return fail(FCGLE_ERR_ARG, "host_fz: bad argument");
  for (int64_t i = 0; i < count; ++i) {
    const zc r = fz_eval(kind, zc{z[2 * i], z[2 * i + 1]});
    out[2 * i] = r.re;
    out[2 * i + 1] = r.im;
  }
  return FCGLE_OK;
}

int fcgle_setup(int d, const int64_t* n, const double* alpha, const double* h, const fcgle_params* params,
                int fd_order, int precision, double tau, fcgle_plan** out) {
  if (!out) return fail(FCGLE_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (d < 1 || d > 4) return fail(FCGLE_ERR_ARG, "d = %d outside 1..4", d);
  if (!n || !alpha || !h || !params) return fail(FCGLE_ERR_ARG, "NULL argument");
  if (fd_order != 2 && fd_order != 4) return fail(FCGLE_ERR_ARG, "fd_order must be 2 or 4");
  if (precision < FCGLE_FP64 || precision > FCGLE_BF16X6) return fail(FCGLE_ERR_ARG, "bad precision");
  if (!(tau > 0.0) || !std::isfinite(tau)) return fail(FCGLE_ERR_ARG, "tau must be > 0");
  const fcgle_params& p = *params;
  if (!(std::isfinite(p.nu) && std::isfinite(p.eta) && std::isfinite(p.gamma) && std::isfinite(p.kappa) &&
        std::isfinite(p.zeta)))
    return fail(FCGLE_ERR_ARG, "non-finite parameter");
  if (p.nu < 0.0 || p.kappa < 0.0) return fail(FCGLE_ERR_ARG, "nu and kappa must be >= 0");
  int64_t N = 1;
  for (int m = 0; m < d; ++m) {
    if (n[m] < 2 || n[m] > 4096) return fail(FCGLE_ERR_ARG, "n[%d] = %lld outside 2..4096", m, (long long)n[m]);
    if (!(alpha[m] > 1.0 && alpha[m] <= 2.0)) return fail(FCGLE_ERR_ARG, "alpha[%d] outside (1, 2]", m);
    if (!(h[m] > 0.0) || !std::isfinite(h[m])) return fail(FCGLE_ERR_ARG, "h[%d] must be > 0", m);
    N *= n[m];
  }
  if (N > ((int64_t)1 << 31) - 1) return fail(FCGLE_ERR_ARG, "tensor too large (N = %lld)", (long long)N);

  auto* P = new (std::nothrow) fcgle_plan();
  if (!P) return fail(FCGLE_ERR_NOMEM, "host allocation failed");
  hipError_t e = hipGetDevice(&P->device);
  if (e != hipSuccess) {
    delete P;
    return fail(FCGLE_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
  }
  P->d = d;
  P->p = p;
  P->fd_order = fd_order;
  P->prec = precision;
  P->tau = tau;
  P->N = N;
  P->elem = (precision == FCGLE_FP64) ? 16 : 8;
  for (int m = 0; m < d; ++m) {
    P->n[m] = n[m];
    P->alpha[m] = alpha[m];
    P->h[m] = h[m];
    P->npad[m] = (int)round_up(n[m], 256);
  }
  // FP64 eigendecompositions on the host, axes in parallel, through the even/odd blocks of
  // the persymmetric D (eigenpairs in block order: even block, then odd block).
  std::vector<int> ok(d, 0);
  std::vector<SplitEig> se(d);
  {
    std::vector<std::thread> th;
    for (int m = 0; m < d; ++m)
      th.emplace_back([&, m] {
        ok[m] = toeplitz_eig_split(n[m], alpha[m], h[m], fd_order, se[m]);
        if (ok[m]) {
          P->Q[m].swap(se[m].Q);
          P->lam[m].swap(se[m].lam);
        }
      });
    for (auto& t : th) t.join();
  }
  P->split = split_supported(precision_of(P));
  for (int m = 0; m < d; ++m) {
    P->me[m] = (int)se[m].me;
    P->mo[m] = (int)se[m].mo;
    P->ldsp[m] = (int)round_up(se[m].me, 128);
  }
  int rc = FCGLE_OK;
  for (int m = 0; m < d && rc == FCGLE_OK; ++m)
    if (!ok[m]) rc = fail(FCGLE_ERR_ARG, "eigensolver did not converge on axis %d", m);
  const int pr = precision_of(P);
  for (int m = 0; m < d && rc == FCGLE_OK; ++m) {
    const int64_t nm = n[m];
    std::vector<double> QT(nm * nm);
    for (int64_t i = 0; i < nm; ++i)
      for (int64_t k = 0; k < nm; ++k) QT[i * nm + k] = P->Q[m][k * nm + i];
    rc = upload_matrix(P, QT, nm, P->npad[m], &P->Mf[m]);
    if (rc == FCGLE_OK) rc = upload_matrix(P, P->Q[m], nm, P->npad[m], &P->Mb[m]);
    if (rc == FCGLE_OK && split_supported(pr)) rc = upload_split(P, m);
    if (rc == FCGLE_OK) rc = plan_alloc((void**)&P->dlam[m], nm * sizeof(double));
    if (rc == FCGLE_OK) {
      e = hipMemcpy(P->dlam[m], P->lam[m].data(), nm * sizeof(double), hipMemcpyHostToDevice);
      if (e != hipSuccess) rc = fail(FCGLE_ERR_HIP, "hipMemcpy: %s", hipGetErrorString(e));
    }
    P->cfg[m][0] = P->cfg[m][1] = default_cfg(pr, nm, P->split);
  }
  for (int k = 0; k < 3 && rc == FCGLE_OK; ++k) rc = plan_alloc(&P->s[k], (size_t)N * P->elem);
  if (rc == FCGLE_OK) rc = plan_alloc((void**)&P->dflag, sizeof(int));
  if (rc != FCGLE_OK) {
    free_plan(P);
    delete P;
    return rc;
  }
  resolve_scratch(P->device);  // the plan's device is current here
  *out = P;
  return FCGLE_OK;
}

void fcgle_destroy(fcgle_plan* plan) {
  if (!plan) return;
  DeviceGuard g(plan->device);
  (void)hipDeviceSynchronize();
  free_plan(plan);
  delete plan;
}

int fcgle_get_eig(const fcgle_plan* plan, int mu, double* Q, double* lambda) {
  FC_TRY(check_plan(plan));
  if (mu < 0 || mu >= plan->d || !Q || !lambda) return fail(FCGLE_ERR_ARG, "get_eig: bad argument");
  sorted_eigenpairs(plan->n[mu], plan->Q[mu], plan->lam[mu], Q, lambda);
  return FCGLE_OK;
}

int fcgle_set_source(fcgle_plan* plan, int nterms, const double* rate, const double* rate_im,
                     const void* const* S_dev) {
  FC_TRY(check_plan(plan));
  plan->gen++;  // captured runs no longer match the plan's configuration
  if (nterms < 0 || nterms > 4) return fail(FCGLE_ERR_ARG, "nterms must be 0..4");
  if (nterms > 0 && (!rate || !S_dev)) return fail(FCGLE_ERR_ARG, "NULL source arrays");
  for (int k = 0; k < nterms; ++k) {
    if (!S_dev[k]) return fail(FCGLE_ERR_ARG, "source tensor %d is NULL", k);
    if (!std::isfinite(rate[k]) || (rate_im && !std::isfinite(rate_im[k])))
      return fail(FCGLE_ERR_ARG, "source rate %d not finite", k);
  }
  plan->ns = nterms;
  for (int k = 0; k < 4; ++k) {
    plan->S[k] = k < nterms ? S_dev[k] : nullptr;
    plan->rate[k] = k < nterms ? rate[k] : 0.0;
    plan->rate_im[k] = (k < nterms && rate_im) ? rate_im[k] : 0.0;
  }
  return FCGLE_OK;
}

int fcgle_apply_f(fcgle_plan* plan, int kind, double theta, const void* u_dev, void* out_dev, void* stream) {
  FC_TRY(check_plan(plan));
  if (!u_dev || !out_dev) return fail(FCGLE_ERR_ARG, "NULL tensor");
  if (kind < FCGLE_INV || kind > FCGLE_PHI3) return fail(FCGLE_ERR_ARG, "bad kind %d", kind);
  if (!std::isfinite(theta)) return fail(FCGLE_ERR_ARG, "theta not finite");
  DeviceGuard g(plan->device);
  hipStream_t st = as_stream(stream);
  EpiParams ep;
  ep.out = plan->s[2];
  EpiKind ek;
  if (kind == FCGLE_EXP) {
    ek = EpiKind::Sep;
    FC_TRY(get_sep(plan, theta, &ep.sep));
  } else {
    ek = EpiKind::Grid;
    FC_TRY(get_grid(plan, kind, theta, st, &ep.F));
  }
  FC_TRY(tucker(plan, true, u_dev, ProKind::Id, ProParams(), ek, ep, plan->s[0], plan->s[1], st));
  EpiParams eb;
  eb.out = out_dev;
  FC_TRY(tucker(plan, false, plan->s[2], ProKind::Id, ProParams(), EpiKind::Store, eb, plan->s[0], plan->s[1], st));
  if (out_dev == plan->uhat_src) plan->uhat_valid = false;
  return FCGLE_OK;
}

int fcgle_apply_f_noalloc(fcgle_plan* plan, int kind, double theta, const void* u_dev, void* out_dev,
                          void* stream) {
  FC_TRY(check_plan(plan));
  if (!u_dev || !out_dev) return fail(FCGLE_ERR_ARG, "NULL tensor");
  if (kind < FCGLE_INV || kind > FCGLE_PHI3) return fail(FCGLE_ERR_ARG, "bad kind %d", kind);
  if (!std::isfinite(theta)) return fail(FCGLE_ERR_ARG, "theta not finite");
  const size_t bytes = (size_t)plan->N * plan->elem;
  if (bytes > kNoAllocTensorBytes)
    return fail(FCGLE_ERR_ARG, "apply_f_noalloc: a state tensor of %zu bytes exceeds the work space limit of %zu "
                "bytes per tensor", bytes, kNoAllocTensorBytes);
  unsigned char* w = scratch_ptr(plan->device);
  if (!w) return fail(FCGLE_ERR_HIP, "apply_f_noalloc: no work space address on device %d", plan->device);
  EpiParams ep;
  ep.out = w + 2 * kNoAllocTensorBytes;
  EpiKind ek;
  if (kind == FCGLE_EXP) {
    ek = EpiKind::Sep;
    if (!find_sep(plan, theta, &ep.sep))
      return fail(FCGLE_ERR_STATE, "apply_f_noalloc: no separable exponential for theta %.17g yet (fcgle_apply_f "
                  "builds it on its first call with this theta)", theta);
  } else {
    ek = EpiKind::Grid;
    if (!(ep.F = find_grid(plan, kind, theta)))
      return fail(FCGLE_ERR_STATE, "apply_f_noalloc: no f-grid for (kind %d, theta %.17g) yet (fcgle_apply_f "
                  "builds it on its first call with this pair)", kind, theta);
  }
  DeviceGuard g(plan->device);
  hipStream_t st = as_stream(stream);
  void* w0 = w;
  void* w1 = w + kNoAllocTensorBytes;
  FC_TRY(tucker(plan, true, u_dev, ProKind::Id, ProParams(), ek, ep, w0, w1, st));
  EpiParams eb;
  eb.out = out_dev;
  FC_TRY(tucker(plan, false, ep.out, ProKind::Id, ProParams(), EpiKind::Store, eb, w0, w1, st));
  if (out_dev == plan->uhat_src) plan->uhat_valid = false;
  return FCGLE_OK;
}

int fcgle_apply_inv_refined(fcgle_plan* plan, double theta, const void* v_dev, void* x_dev, int sweeps,
                            double* rnorm, void* stream) {
  FC_TRY(check_plan(plan));
  if (!v_dev || !x_dev) return fail(FCGLE_ERR_ARG, "NULL tensor");
  if (v_dev == x_dev) return fail(FCGLE_ERR_ARG, "apply_inv_refined: x must not alias v");
  if (sweeps < 0 || sweeps > 8) return fail(FCGLE_ERR_ARG, "apply_inv_refined: sweeps must be 0..8");
  if (!std::isfinite(theta)) return fail(FCGLE_ERR_ARG, "theta not finite");
  DeviceGuard g(plan->device);
  hipStream_t st = as_stream(stream);
  FC_TRY(ensure_refine(plan));
  const int pr = precision_of(plan);
  const int parts = rf_norm_parts();
  double* nrm = plan->rf_part + parts;  // [0] = |v|^2, [1 + k] = |r_k|^2
  if (rnorm) HIP_TRY(launch_rf_norm2(plan->N, v_dev, plan->rf_part, nrm, st));
  // x_0 = R o v in the plan's precision
  HIP_TRY(launch_rf_to_state(pr, plan->N, v_dev, plan->rf_y, st));
  FC_TRY(refine_inverse(plan, theta, st));
  HIP_TRY(launch_rf_set(pr, plan->N, x_dev, plan->rf_y, st));
  for (int k = 0; k <= sweeps; ++k) {
    if (k == sweeps && !rnorm) break;
    FC_TRY(refine_residual(plan, theta, v_dev, x_dev, st));
    if (rnorm) HIP_TRY(launch_rf_norm2(plan->N, plan->rf_r, plan->rf_part, nrm + 1 + k, st));
    if (k == sweeps) break;
    HIP_TRY(launch_rf_to_state(pr, plan->N, plan->rf_r, plan->rf_y, st));
    FC_TRY(refine_inverse(plan, theta, st));
    HIP_TRY(launch_rf_add(pr, plan->N, x_dev, plan->rf_y, st));
  }
  if (rnorm) {
    double h[10];
    HIP_TRY(hipMemcpyAsync(h, nrm, (size_t)(sweeps + 2) * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const double vn = std::sqrt(h[0]);
    for (int k = 0; k <= sweeps; ++k) rnorm[k] = vn > 0.0 ? std::sqrt(h[1 + k]) / vn : std::sqrt(h[1 + k]);
  }
  if (x_dev == plan->uhat_src) plan->uhat_valid = false;
  return FCGLE_OK;
}

int fcgle_set_state(fcgle_plan* plan, const void* u_dev, const void* u_prev_dev, void* stream) {
  FC_TRY(check_plan(plan));
  if (!u_dev) return fail(FCGLE_ERR_ARG, "u_dev is NULL");
  DeviceGuard g(plan->device);
  plan->uhat_valid = false;
  plan->uhat_src = nullptr;
  plan->hist_valid = false;
  plan->hist_src = nullptr;
  if (u_prev_dev) {
    FC_TRY(ensure_state_buffers(plan));
    HIP_TRY(hipMemcpyAsync(plan->uprev, u_prev_dev, (size_t)plan->N * plan->elem, hipMemcpyDeviceToDevice,
                           as_stream(stream)));
    plan->hist_valid = true;
    plan->hist_src = u_dev;
  }
  return FCGLE_OK;
}

int fcgle_step(fcgle_plan* plan, int scheme, void* u_dev, double t, double tau, void* stream) {
  FC_TRY(check_plan(plan));
  if (!u_dev) return fail(FCGLE_ERR_ARG, "u_dev is NULL");
  if (tau != plan->tau) return fail(FCGLE_ERR_ARG, "tau %.17g differs from the plan's %.17g", tau, plan->tau);
  if (!std::isfinite(t)) return fail(FCGLE_ERR_ARG, "t not finite");
  if (scheme < FCGLE_EXP_EULER || scheme > FCGLE_KROGSTAD) return fail(FCGLE_ERR_ARG, "bad scheme %d", scheme);
  DeviceGuard g(plan->device);
  return step_impl(plan, scheme, u_dev, t, as_stream(stream));
}

int fcgle_run(fcgle_plan* plan, int scheme, void* u_dev, double t0, double tau, int64_t nsteps, void* stream) {
  FC_TRY(check_plan(plan));
  if (nsteps < 0) return fail(FCGLE_ERR_ARG, "nsteps < 0");
  if (scheme == FCGLE_STRANG && nsteps > 0) {
    if (!u_dev) return fail(FCGLE_ERR_ARG, "u_dev is NULL");
    if (tau != plan->tau) return fail(FCGLE_ERR_ARG, "tau %.17g differs from the plan's %.17g", tau, plan->tau);
    if (!std::isfinite(t0)) return fail(FCGLE_ERR_ARG, "t0 not finite");
    DeviceGuard g(plan->device);
    return strang_run(plan, u_dev, nsteps, as_stream(stream));
  }
  if (scheme == FCGLE_EXP_EULER && plan->ns == 0 && plan->timing_cap == 0 && nsteps >= 2) {
    if (!u_dev) return fail(FCGLE_ERR_ARG, "u_dev is NULL");
    if (tau != plan->tau) return fail(FCGLE_ERR_ARG, "tau %.17g differs from the plan's %.17g", tau, plan->tau);
    if (!std::isfinite(t0)) return fail(FCGLE_ERR_ARG, "t0 not finite");
    DeviceGuard g(plan->device);
    return expeuler_run(plan, u_dev, t0, nsteps, as_stream(stream));
  }
  for (int64_t k = 0; k < nsteps; ++k) FC_TRY(fcgle_step(plan, scheme, u_dev, t0 + (double)k * tau, tau, stream));
  return FCGLE_OK;
}

int fcgle_check_finite(fcgle_plan* plan, const void* u_dev, void* stream) {
  FC_TRY(check_plan(plan));
  if (!u_dev) return fail(FCGLE_ERR_ARG, "u_dev is NULL");
  DeviceGuard g(plan->device);
  hipStream_t st = as_stream(stream);
  int h = 0;
  HIP_TRY(hipMemsetAsync(plan->dflag, 0, sizeof(int), st));
  HIP_TRY(launch_check_finite(precision_of(plan), plan->N, u_dev, plan->dflag, st));
  HIP_TRY(hipMemcpyAsync(&h, plan->dflag, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (h) return fail(FCGLE_ERR_NONFINITE, "tensor holds NaN or Inf");
  return FCGLE_OK;
}

int fcgle_plan_shape(const fcgle_plan* plan, int64_t* N, int* elem_bytes) {
  FC_TRY(check_plan(plan));
  if (N) *N = plan->N;
  if (elem_bytes) *elem_bytes = plan->elem;
  return FCGLE_OK;
}

}  // extern "C"

namespace {

// Mean duration (ms) of `reps` runs of fn() on stream st after one warm-up run.
template <class Fn>
int time_ms(hipStream_t st, hipEvent_t e0, hipEvent_t e1, int reps, Fn fn, float* out) {
  if (fn() != hipSuccess) return fail(FCGLE_ERR_HIP, "autotune: launch failed");
  HIP_TRY(hipEventRecord(e0, st));
  for (int r = 0; r < reps; ++r)
    if (fn() != hipSuccess) return fail(FCGLE_ERR_HIP, "autotune: launch failed");
  HIP_TRY(hipEventRecord(e1, st));
  HIP_TRY(hipEventSynchronize(e1));
  float ms = 0;
  HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  *out = ms / reps;
  return FCGLE_OK;
}

int autotune_impl(fcgle_plan* plan, int reps, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  const int pr = precision_of(plan);
  const size_t bytes = (size_t)plan->N * plan->elem;
  HIP_TRY(hipMemsetAsync(plan->s[0], 0, bytes, st));
  HIP_TRY(hipMemsetAsync(plan->s[2], 0, bytes, st));
  // 1. tile configuration of every plain mode product (the runner-up is kept for step 3)
  int second_c[4][2], second_f2[4][2];  // [axis][fwd], like the plan's cfg
  for (int mu = 0; mu < plan->d; ++mu)
    for (int dir = 0; dir < 2; ++dir) {
      float best = 1e30f, second = 1e30f;
      int best_c = plan->cfg[mu][dir];
      second_c[mu][dir] = -1;
      second_f2[mu][dir] = 0;
      // forward even/odd products: also the form with both blocks in one tile
      const int nform = (dir == 1 && plan->split) ? 2 : 1;
      bool best_f2 = false;
      for (int form = 0; form < nform; ++form)
        for (int c = 0; c < kNumCfg; ++c) {
          plan->fwd2[mu] = (form == 1);
          MPLaunch L = base_launch(plan, mu, dir == 1);
          L.cfg = c;
          L.in = plan->s[0];
          L.ep.out = plan->s[1];
          float ms;
          FC_TRY(time_ms(st, e0, e1, reps * 3 > 10 ? reps * 3 : 10, [&] { return launch_mode_product(L, st); }, &ms));
          if (ms < best) {
            second = best;
            second_c[mu][dir] = best < 1e30f ? best_c : -1;
            second_f2[mu][dir] = best_f2;
            best = ms;
            best_c = c;
            best_f2 = (form == 1);
          } else if (ms < second) {
            second = ms;
            second_c[mu][dir] = c;
            second_f2[mu][dir] = (form == 1);
          }
        }
      plan->cfg[mu][dir] = best_c;
      if (dir == 1) plan->fwd2[mu] = best_f2;
    }
  // 2. order of the forward products and where the nonlinearity and the exponential-Euler
  //    update run (fused prologue / epilogue, streaming passes, or the update in the first
  //    backward product): time a whole exponential-Euler step for each choice, on zero data
  FC_TRY(ensure_state_buffers(plan));
  HIP_TRY(hipMemsetAsync(plan->uprev, 0, bytes, st));
  HIP_TRY(hipMemsetAsync(plan->uhat, 0, bytes, st));
  if (update_prologue_ok(plan)) {
    if (!plan->uhat2) FC_TRY(plan_alloc(&plan->uhat2, bytes));
    HIP_TRY(hipMemsetAsync(plan->uhat2, 0, bytes, st));
  }
  // with the update in the first backward product that product is timed in every tile
  // configuration again (its loads differ from the plain product's)
  static const int kFusions[] = {0, 1, 2, 3, 8, 9, 40, 41};
  const int nfus = update_otf_ok(plan) ? 8 : update_prologue_ok(plan) ? 6 : 4;
  // whole steps differ by a few percent between the best choices: time more of them, then
  // time the fastest few again in interleaved rounds and keep each one's best time, so that a
  // single slow or fast measurement does not decide
  const int reps2 = reps * 3 > 10 ? reps * 3 : 10;
  struct Cand {
    bool rev;
    int fusion, cfg_upd;
    float ms;
  };
  std::vector<Cand> cands;
  auto time_step = [&](const Cand& c, float* ms) {
    plan->fwd_rev = c.rev;
    plan->fusion = c.fusion;
    plan->cfg_upd = c.cfg_upd;
    return time_ms(st, e0, e1, reps2, [&] {
      const int rc = expeuler_body(plan, plan->uprev, 0.0, st);
      return rc == FCGLE_OK ? hipSuccess : hipErrorUnknown;
    }, ms);
  };
  for (int rev = 0; rev < (plan->d > 1 ? 2 : 1); ++rev)
    for (int fi = 0; fi < nfus; ++fi) {
      const int fusion = kFusions[fi];
      const bool upd = (fusion & 8) != 0;
      for (int c = upd ? 0 : -1; c < (upd ? kNumCfg : 0); ++c) {
        // a configuration that hands its update prologue to another tile would time that tile again
        if (upd && cfg_update_tile(pr, c, (fusion & 32) && otf_fits(pr, c)) != c) continue;
        Cand cd{rev != 0, fusion, c, 0.f};
        FC_TRY(time_step(cd, &cd.ms));
        cands.push_back(cd);
      }
    }
  std::stable_sort(cands.begin(), cands.end(), [](const Cand& a, const Cand& b) { return a.ms < b.ms; });
  const size_t top = cands.size() < 4 ? cands.size() : 4;
  for (int round = 0; round < 3; ++round)
    for (size_t i = 0; i < top; ++i) {
      float ms;
      FC_TRY(time_step(cands[i], &ms));
      if (ms < cands[i].ms) cands[i].ms = ms;
    }
  size_t bi = 0;
  for (size_t i = 1; i < top; ++i)
    if (cands[i].ms < cands[bi].ms) bi = i;
  const bool best_rev = cands[bi].rev;
  int best_fusion = cands[bi].fusion;
  const int best_cfg_upd = cands[bi].cfg_upd;
  (void)pr;
  plan->fwd_rev = best_rev;
  // with the update in the backward prologue the last forward product of an exponential-Euler
  // step only stores, so bit 1 has no effect there; set it for the separable-exponential
  // epilogue of the Lawson and Strang forward operators (fused is the faster form of it)
  if (best_fusion & 8) best_fusion |= 2;
  plan->fusion = best_fusion;
  plan->cfg_upd = best_cfg_upd;
  // 3. products timed alone can rank two tiles within noise, or otherwise than inside a step:
  //    compare each product's runner-up with its choice in whole steps (interleaved rounds,
  //    best time of each) and keep the faster
  for (int mu = 0; mu < plan->d; ++mu)
    for (int dir = 0; dir < 2; ++dir) {
      if (second_c[mu][dir] < 0) continue;
      const int cc[2] = {plan->cfg[mu][dir], second_c[mu][dir]};
      const bool ff[2] = {dir == 1 && plan->fwd2[mu], dir == 1 && second_f2[mu][dir] != 0};
      float t[2] = {1e30f, 1e30f};
      bool ok1 = true;  // the runner-up runs inside the step (else the choice stays)
      for (int round = 0; round < 3 && ok1; ++round)
        for (int k = 0; k < 2 && ok1; ++k) {
          plan->cfg[mu][dir] = cc[k];
          if (dir == 1) plan->fwd2[mu] = ff[k];
          float ms;
          auto body = [&] {
            const int rc = expeuler_body(plan, plan->uprev, 0.0, st);
            return rc == FCGLE_OK ? hipSuccess : hipErrorUnknown;
          };
          if (k == 0) {
            FC_TRY(time_ms(st, e0, e1, reps2, body, &ms));
          } else if (time_ms(st, e0, e1, reps2, body, &ms) != FCGLE_OK) {
            ok1 = false;
            break;
          }
          if (ms < t[k]) t[k] = ms;
        }
      const int k = (ok1 && t[1] < t[0]) ? 1 : 0;
      plan->cfg[mu][dir] = cc[k];
      if (dir == 1) plan->fwd2[mu] = ff[k];
    }
  return FCGLE_OK;
}

}  // namespace

extern "C" int fcgle_autotune(fcgle_plan* plan, int reps, void* stream) {
  if (reps < 1) reps = 3;
  if (plan && plan->batch) {
    DeviceGuard g(plan->device);
    return batch_autotune(plan, reps, as_stream(stream));
  }
  FC_TRY(check_plan(plan));
  plan->gen++;  // captured runs no longer match the plan's configuration
  DeviceGuard g(plan->device);
  hipStream_t st = as_stream(stream);
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  const int rc = autotune_impl(plan, reps, st, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  plan->tuned = (rc == FCGLE_OK);
  // the timed steps ran on the plan's own buffers: the eigenspace state and u_{n-1} of the
  // LBDF2 history were overwritten, so both caches are forgotten
  plan->uhat_valid = false;
  plan->uhat_src = nullptr;
  plan->hist_valid = false;
  plan->hist_src = nullptr;
  return rc;
}

extern "C" {

int fcgle_set_tiles(fcgle_plan* plan, int axis, int fwd, int cfg) {
  FC_TRY(check_plan(plan));
  plan->gen++;  // captured runs no longer match the plan's configuration
  const int pr = precision_of(plan);
  const bool f2 = fwd == 1 && cfg >= kNumCfg;
  if (axis < 0 || axis >= plan->d || (fwd != 0 && fwd != 1) || cfg < 0 || cfg >= (fwd ? 2 * kNumCfg : kNumCfg))
    return fail(FCGLE_ERR_ARG, "set_tiles: bad argument");
  (void)pr;
  if (f2 && !plan->split) return fail(FCGLE_ERR_UNSUPPORTED, "set_tiles: fused forward tiles need an even/odd plan");
  if (fwd == 1) plan->fwd2[axis] = f2;
  plan->cfg[axis][fwd] = f2 ? cfg - kNumCfg : cfg;
  if (axis == 0 && fwd == 0) plan->cfg_upd = -1;  // the update-prologue product follows it again
  return FCGLE_OK;
}

int fcgle_set_structure(fcgle_plan* plan, int split) {
  FC_TRY(check_plan(plan));
  plan->gen++;  // captured runs no longer match the plan's configuration
  if (split != 0 && split != 1) return fail(FCGLE_ERR_ARG, "set_structure: split must be 0 or 1");
  if (split && !split_supported(precision_of(plan)))
    return fail(FCGLE_ERR_UNSUPPORTED, "set_structure: no even/odd kernels for this precision");
  if ((bool)split != plan->split) {
    plan->split = (split != 0);
    for (int m = 0; m < plan->d; ++m) {
      plan->cfg[m][0] = plan->cfg[m][1] = default_cfg(precision_of(plan), plan->n[m], plan->split);
      plan->fwd2[m] = false;
    }
    plan->cfg_upd = -1;
    plan->tuned = false;
  }
  return FCGLE_OK;
}

int fcgle_set_wide_loads(fcgle_plan* plan, int force) {
  FC_TRY(check_plan(plan));
  if (force != 0 && force != 1) return fail(FCGLE_ERR_ARG, "set_wide_loads: force must be 0 or 1");
  plan->gen++;  // captured runs no longer match the plan's configuration
  plan->wide_force = (force != 0);
  return FCGLE_OK;
}

int fcgle_set_fusion(fcgle_plan* plan, int flags) {
  FC_TRY(check_plan(plan));
  plan->gen++;  // captured runs no longer match the plan's configuration
  if (flags < 0 || flags > 111 || (flags & 16))
    return fail(FCGLE_ERR_ARG, "set_fusion: flags must be 0..15, optionally with bits 5 (32) and 6 (64)");
  plan->fusion = flags & 107;
  plan->fwd_rev = (flags & 4) != 0;
  return FCGLE_OK;
}

int fcgle_describe(const fcgle_plan* plan, char* buf, size_t len) {
  if (!buf || len == 0) return fail(FCGLE_ERR_ARG, "bad buffer");
  if (plan && plan->batch) return batch_describe(plan, buf, len);
  FC_TRY(check_plan(plan));
  static const char* names[] = {"fp64", "fp32", "bf16x3", "bf16x6"};
  std::string s = "d=" + std::to_string(plan->d) + " n=(";
  for (int m = 0; m < plan->d; ++m) s += std::to_string(plan->n[m]) + (m + 1 < plan->d ? "," : ")");
  s += std::string(" precision=") + names[plan->prec] + " tiles[axis](bwd/fwd rows x cols)=";
  const int pr = precision_of(plan);
  const int sp = plan->split ? 1 : 0;
  for (int m = 0; m < plan->d; ++m) {
    // suffix s: single-buffered operand tiles; F: both even/odd blocks per forward tile
    auto tile = [&](int c) {
      return std::to_string(cfg_rows(pr, c, sp)) + "x" + std::to_string(cfg_cols(pr, c, sp)) +
             (cfg_bufs(pr, c, sp) == 1 ? "s" : "");
    };
    s += "[" + tile(plan->cfg[m][0]) + "/" + tile(plan->cfg[m][1]) + (plan->split && plan->fwd2[m] ? "F" : "") + "]";
  }
  s += plan->split ? " structure=even-odd" : " structure=dense";
  s += std::string(" fusion=") + ((plan->fusion & 1) ? "pro" : "-") + "/" + ((plan->fusion & 2) ? "epi" : "-") +
       ((plan->fusion & 64) ? "/flows" : "");
  if (plan->fusion & 8) {
    if (update_prologue_ok(plan)) {
      const int c = plan->cfg_upd >= 0 ? plan->cfg_upd : plan->cfg[0][0];
      s += " update=backward-prologue(" + std::to_string(cfg_rows(pr, c, 1)) + "x" + std::to_string(cfg_cols(pr, c, 1)) +
           ((plan->fusion & 32) && update_otf_ok(plan) ? ",phi1-on-the-fly" : "") + ")";
    } else {
      s += " update=backward-prologue(unsupported:epilogue)";
    }
  }
  s += plan->fwd_rev ? " forward-order=reversed" : " forward-order=natural";
  {
    std::string w;
    for (int m = 0; m < plan->d; ++m) {
      const MPLaunch L = base_launch(plan, m, false);
      if (mp_wide(L)) w += (w.empty() ? "" : ",") + std::to_string(m);
    }
    if (!w.empty()) s += " loads=64-bit-index(axes " + w + ")";
  }
  s += plan->tuned ? " tuned" : " default";
  std::snprintf(buf, len, "%s", s.c_str());
  return FCGLE_OK;
}

int fcgle_timing_enable(fcgle_plan* plan, int capacity) {
  FC_TRY(check_plan(plan));
  DeviceGuard g(plan->device);
  if (capacity < 0) return fail(FCGLE_ERR_ARG, "capacity < 0");
  plan->timed.clear();
  while ((int)plan->ev_pool.size() < 2 * capacity) {
    hipEvent_t e;
    HIP_TRY(hipEventCreate(&e));
    plan->ev_pool.push_back(e);
  }
  plan->timing_cap = capacity;
  return FCGLE_OK;
}

int fcgle_timing_read(fcgle_plan* plan, int cap, int* axis, int* fwd, int* sig, double* ms, int64_t* count) {
  FC_TRY(check_plan(plan));
  if (plan->timing_cap <= 0) return fail(FCGLE_ERR_STATE, "timing is not enabled");
  if (!count || (cap > 0 && (!axis || !fwd || !sig || !ms))) return fail(FCGLE_ERR_ARG, "NULL output");
  DeviceGuard g(plan->device);
  int64_t k = 0;
  for (auto& t : plan->timed) {
    HIP_TRY(hipEventSynchronize(t.e1));
    float e = 0;
    HIP_TRY(hipEventElapsedTime(&e, t.e0, t.e1));
    if (k < cap) {
      axis[k] = t.axis;
      fwd[k] = t.fwd;
      sig[k] = t.sig;
      ms[k] = e;
    }
    ++k;
  }
  *count = k < cap ? k : cap;
  plan->timed.clear();
  return FCGLE_OK;
}

int fcgle_vjp_run(fcgle_plan* plan, int scheme, const void* u_start_dev, int64_t m, void* ubar_dev,
                  double* pbar_dev, double t0, double tau, void* stream) {
  FC_TRY(check_plan(plan));
  if (!u_start_dev || !ubar_dev || !pbar_dev) return fail(FCGLE_ERR_ARG, "vjp: NULL argument");
  if (m < 0) return fail(FCGLE_ERR_ARG, "vjp: m < 0");
  if (tau != plan->tau) return fail(FCGLE_ERR_ARG, "tau %.17g differs from the plan's %.17g", tau, plan->tau);
  if (!std::isfinite(t0)) return fail(FCGLE_ERR_ARG, "t0 not finite");
  if (scheme < FCGLE_EXP_EULER || scheme > FCGLE_KROGSTAD) return fail(FCGLE_ERR_ARG, "bad scheme %d", scheme);
  if (scheme != FCGLE_EXP_EULER) return fail(FCGLE_ERR_UNSUPPORTED, "vjp: only FCGLE_EXP_EULER has an adjoint");
  if (u_start_dev == ubar_dev) return fail(FCGLE_ERR_ARG, "vjp: u_start and ubar must be distinct buffers");
  DeviceGuard g(plan->device);
  return vjp_run_impl(plan, u_start_dev, m, ubar_dev, pbar_dev, t0, as_stream(stream));
}

int fcgle_vjp(fcgle_plan* plan, int scheme, const void* u_n_dev, const void* ubar_next_dev, void* ubar_n_dev,
              double* pbar_dev, double t, double tau, void* stream) {
  FC_TRY(check_plan(plan));
  if (!u_n_dev || !ubar_next_dev || !ubar_n_dev || !pbar_dev) return fail(FCGLE_ERR_ARG, "vjp: NULL argument");
  if (u_n_dev == ubar_n_dev || u_n_dev == ubar_next_dev)
    return fail(FCGLE_ERR_ARG, "vjp: u_n must not alias a cotangent buffer");
  if (tau != plan->tau) return fail(FCGLE_ERR_ARG, "tau %.17g differs from the plan's %.17g", tau, plan->tau);
  if (scheme < FCGLE_EXP_EULER || scheme > FCGLE_KROGSTAD) return fail(FCGLE_ERR_ARG, "bad scheme %d", scheme);
  if (scheme != FCGLE_EXP_EULER) return fail(FCGLE_ERR_UNSUPPORTED, "vjp: only FCGLE_EXP_EULER has an adjoint");
  if (ubar_n_dev != ubar_next_dev) {
    DeviceGuard g(plan->device);
    HIP_TRY(hipMemcpyAsync(ubar_n_dev, ubar_next_dev, (size_t)plan->N * plan->elem, hipMemcpyDeviceToDevice,
                           as_stream(stream)));
  }
  return fcgle_vjp_run(plan, scheme, u_n_dev, 1, ubar_n_dev, pbar_dev, t, tau, stream);
}

}  // extern "C"
