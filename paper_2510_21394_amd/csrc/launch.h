// Host-side description of one kernel launch of the library.  Shared by the
// plan code (api.cpp) and the kernel translation units; contains no device code.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fcgle {

enum Prec : int { P_F64 = 0, P_F32 = 1, P_BF16X3 = 2, P_BF16X6 = 3 };

// Structure of a mode product (MPLaunch::split; the forms are described in kernels.hpp).
enum : int { kDense = 0, kSplitFwd = 1, kSplitBwd = 2, kSplitFwd2 = 3 };

// Pointwise map applied to the input of a mode product while its tile is loaded.
//  Update: the exponential-Euler update uhat_out = E uhat + tau P1 v of the input v (the
//  transformed nonlinearity), contracted and also stored (first backward even/odd product).
//  UpdateOtf: as Update with P1 = (E - 1) / z formed on the fly from separable tables (no
//  P1 grid read; axis lengths n_1 <= kOtfMaxRows).
//  Flow: the exact flow of the nonlinear subproblem of Strang splitting (FlowParams).
enum class ProKind : int { Id = 0, Nonlin = 1, Update = 2, UpdateOtf = 3, Flow = 4 };
constexpr int kOtfMaxRows = 512;
// What the last stage of a mode product does with each output element.
enum class EpiKind : int {
  Store = 0,     // out[j] = v
  Grid = 1,      // out[j] = F[j] v                      (stored f-grid)
  Sep = 2,       // out[j] = prod_mu f_mu[j_mu] v          (separable exponential)
  ExpEuler = 3,  // uhat[j] = E_j uhat[j] + tau P1[j] v     (eigenspace exponential Euler)
  KeepOld = 4,   // save[j] = out[j]; out[j] = v           (LBDF2 history)
  ExpEulerRec = 5,  // as ExpEuler, and X[j] = uhat_new[j] - tau P2[j] v  (adjoint recompute;
                    //   streaming pass only)
  Axpy = 6,         // out[j] += c v, c complex            (FP64 residual of the refinement sweep;
                    //   dense FP64 products only)
  Flow = 7,         // out[j] = phi_t(v), the exact nonlinear flow (FlowParams; backward products)
  Count = 8
};

// Separable per-axis complex factors (FP64): value(j) = prod_mu fac[mu][j_mu].
// other_last / other_first (optional) hold prod over the axes other than the last / the
// first, indexed by the flat index over the remaining axes, so an epilogue on the last
// (first) axis gets its per-column factor with one load.
struct SepParams {
  int d = 0;
  int mu = 0;  // axis of the mode product (its index comes from the output row)
  int n[4] = {1, 1, 1, 1};
  const void* fac[4] = {nullptr, nullptr, nullptr, nullptr};  // double2[n_mu]
  const double* lam[4] = {nullptr, nullptr, nullptr, nullptr}; // eigenvalues (adjoint)
  const void* other_last = nullptr;   // double2[N / n_{d-1}]
  const void* other_first = nullptr;  // double2[N / n_0]
  // for phi_1 on the fly: the exponent scale z = (zre + i zim) ell, expm1 of each axis factor,
  // and over the axes after the first prod e^{z_mu} - 1 (double2) and sum lambda_mu (double)
  double zre = 0, zim = 0;
  const void* facm1[4] = {nullptr, nullptr, nullptr, nullptr};
  const void* first_m1 = nullptr;
  const double* first_lam = nullptr;
};

// Exact flow over a time t of w' = gamma w - (kappa + i zeta)|w|^2 w (Section 4, Strang
// splitting): w e^{gamma t} (1 + 2 kappa a)^{-1/2} e^{-i zeta L} with a = t phi_1(2 gamma t)|w|^2
// and L = log(1 + 2 kappa a)/(2 kappa) (L = a when kappa = 0).  The scalars, in FP64:
struct FlowParams {
  double tp1 = 0;   // t phi_1(2 gamma t)
  double eg = 1;    // e^{gamma t}
  double k2 = 0;    // 2 kappa
  double zeta = 0;
};

// Nonlin: g(t, e) = gamma e - (kappa + i zeta)|e|^2 e + sum_k sc[k] S_k[j], with
// e = eu u + ep up; output = cu u + cp up + cg g.
// Update: uhat_out[j] = E_j uhat[j] + tau F[j] v[j] (E from sep, F = the phi_1 grid).
struct ProParams {
  const void* up = nullptr;
  const void* S[4] = {nullptr, nullptr, nullptr, nullptr};
  double sc[4] = {0, 0, 0, 0};   // exp(c_k t): real part
  double sci[4] = {0, 0, 0, 0};  //   and imaginary part
  int ns = 0;
  double gamma = 0, kappa = 0, zeta = 0;
  double eu = 1, ep = 0, cu = 0, cp = 0, cg = 1;
  const void* uhat = nullptr;
  const void* F = nullptr;
  void* uhat_out = nullptr;
  SepParams sep;
  double tau = 0;
  FlowParams flow;  // Flow
};

struct EpiParams {
  void* out = nullptr;
  void* save = nullptr;      // KeepOld
  const void* F = nullptr;   // Grid / ExpEuler (P1)
  SepParams sep;             // Sep / ExpEuler / adjoint
  double tau = 0;            // ExpEuler / adjoint
  void* ghat_out = nullptr;  // ExpEuler: optional copy of the transformed nonlinearity
  const void* F2 = nullptr;  // ExpEulerRec: phi_2 grid
  void* out2 = nullptr;      // ExpEulerRec: X
  double cre = 0, cim = 0;   // Axpy: c
  FlowParams flow;           // Flow
};

// One mode product out[a, i, b] = sum_k M[i, k] in[a, k, b] on a complex tensor
// viewed as (A, n, B); M is npad x npad (zero padded), row-major, in the layout of
// the precision (double / float / BF16 pieces).
struct MPLaunch {
  int prec = P_F64;
  int cfg = 0;  // tile configuration index
  int split = 0;       // 0 dense, 1 even/odd forward (Q^T), 2 even/odd backward (Q); see kernels.hpp
  int me = 0, mo = 0;  // split: even and odd block sizes (me + mo = n)
  int64_t A = 1;
  int n = 1;
  int npad = 1;
  int64_t B = 1;
  const void* M = nullptr;
  const void* in = nullptr;
  ProKind pk = ProKind::Id;
  ProParams pp;
  EpiKind ek = EpiKind::Store;
  EpiParams ep;
  bool wide = false;  // force the 64-bit-index loader (see mp_wide)
};

// Whether a mode product takes the WIDE tile configuration of its precision (64-bit element
// indices): an N-loader product (B > 1; T-loader offsets always fit) that is forced to, or
// whose k-tile rows, up to 32 of them at element stride B, span more than the 2 GiB the other
// configurations' buffer views address.
inline bool mp_wide(const MPLaunch& L) {
  const uint64_t esize = (L.prec == P_F64) ? 16 : 8;
  return L.B > 1 && (L.wide || (uint64_t)L.B * 32u * esize > 0x80000000ull);
}

constexpr int kNumCfg = 5;  // tile configurations per precision and structure
int cfg_rows(int prec, int cfg, int split = 0);
int cfg_cols(int prec, int cfg, int split = 0);  // complex columns per tile
int cfg_bufs(int prec, int cfg, int split = 0);  // LDS buffers of the operand tiles (1 or 2)
int cfg_tk_split(int prec, int cfg);              // k-tile length of an even/odd configuration
int cfg_update_tile(int prec, int cfg, bool otf);  // configuration that runs the update prologue
// True when the even/odd split kernels exist for the precision.
bool split_supported(int prec);

// True when the fused kernel exists for this (loader, prologue, epilogue) combination
// (ProKind::Update / UpdateOtf: backward even/odd products with the N loader only; prologues
// other than Id: forward products; EpiKind::Flow: backward products).
bool mp_supported(bool tloader, ProKind pk, EpiKind ek);

hipError_t launch_mp_f64(const MPLaunch& L, hipStream_t s);
hipError_t launch_mp_f32(const MPLaunch& L, hipStream_t s);
hipError_t launch_mp_bf16(const MPLaunch& L, hipStream_t s);
inline hipError_t launch_mode_product(const MPLaunch& L, hipStream_t s) {
  if (L.prec == P_F64) return launch_mp_f64(L, s);
  if (L.prec == P_F32) return launch_mp_f32(L, s);
  return launch_mp_bf16(L, s);
}

// Grouped FP32 even/odd mode products: the same mode product (same loader, prologue and
// epilogue kinds, direction, tile configuration `cfg`) of `count` independent problems in
// one launch.  group_build_f32 writes the item array for the per-problem descriptions
// L[0..count) (split = 1 forward or 2 backward) into host memory (group_item_bytes(pk, ek)
// bytes per item) and returns the total number of workgroups; the array must then be copied
// to the device and passed to launch_group_f32 with the same split (1 or 3 forward, 2
// backward).  Supported: forward (N loader, Nonlin or Id, Store), (T loader, Id, Store or
// ExpEuler); backward (either loader, Id, Store).  Nonlin is the plain form only: items with
// source terms or an extrapolated state make group_build_f32 return 0.
bool group_supported(bool tloader, ProKind pk, EpiKind ek, bool fwd);
constexpr int kGroupCfg = 5;  // tile configurations of the grouped kernels
int group_cfg_rows(int cfg);   // rows per tile of grouped configuration cfg
size_t group_item_bytes(ProKind pk, EpiKind ek);
uint32_t group_build_f32(int cfg, bool tloader, ProKind pk, EpiKind ek, const MPLaunch* L, int count,
                         void* items_host);
hipError_t launch_group_f32(int cfg, bool tloader, ProKind pk, EpiKind ek, int split, const void* items_dev,
                            int count, uint32_t nblocks, hipStream_t s);
// Persistent batched exponential Euler (batch_persist_kernel in kernels.hpp, FP32): one launch
// runs every phase of every step of all instances.  persist_build_f32 writes the item array of
// phase 0..3 (F0: forward axis 0 with the nonlinearity, F1: forward axis 1 with the fused update,
// B0, B1: backward; forward phases in the form with both even/odd blocks per tile) for the
// per-instance descriptions L[0..count) into host memory (persist_item_bytes(phase) bytes per
// item), the tiles of each instance into tiles[count], and returns the phase's tiles.
// persist_grid is the number of co-resident workgroups (0 when cfg has no instantiation).
struct PersistCtl {
  uint32_t next;   // next ticket
  uint32_t error;  // nonzero: a dependency wait ran out of polls
};

struct PersistArgs {
  PersistCtl* ctl;
  uint32_t* done;         // per instance: completed tiles over the whole launch
  const uint32_t* pre;    // per instance, 5 values: tiles of the instance before phase p (p = 0..3), per step (p = 4)
  const void* items[4];   // per phase: item arrays (GroupItem of the phase's prologue/epilogue)
  uint32_t phase0[5];     // first ticket of each phase within a step; phase0[4] = tickets per step
  uint32_t total;         // tickets of the launch
  int count;              // instances
  uint32_t spin_limit;    // polls of a dependency wait before giving up
};
bool persist_supported(int cfg);
size_t persist_item_bytes(int phase);
uint32_t persist_build_f32(int cfg, int phase, const MPLaunch* L, int count, void* items_host, uint32_t* tiles);
int persist_grid(int cfg);
hipError_t launch_persist_f32(int cfg, const PersistArgs& a, uint32_t grid, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t n, hipStream_t s);

// Grouped streaming epilogue (FP32): item k applies `ek` (ExpEuler) to v[k] viewed as
// (rows[k], nlast[k]) with parameters ep[k]; returns the total number of rows.
size_t pw_group_item_bytes(EpiKind ek);
uint32_t pw_group_build_f32(EpiKind ek, const int64_t* rows, const int* nlast, const void* const* v,
                            const EpiParams* ep, int count, void* items_host);
hipError_t launch_pw_group_f32(EpiKind ek, const void* items_dev, int count, uint32_t total_rows, hipStream_t s);

// Standalone pointwise passes (unfused fallbacks and helpers), complex tensors of N
// elements in the state type of `prec`.
hipError_t launch_pointwise_pro(int prec, int64_t N, const void* in, void* out, ProKind pk, const ProParams& p,
                                hipStream_t s);
// Applies epilogue `ek` to v[j] for every j, with the tensor viewed as (N / n_last, n_last).
hipError_t launch_pointwise_epi(int prec, int64_t N, int n_last, const void* v, EpiKind ek,
                                const EpiParams& p, hipStream_t s);
hipError_t launch_check_finite(int prec, int64_t N, const void* u, int* flag, hipStream_t s);
// Adjoint of exponential Euler (adjoint.hip).  Tensors of N elements viewed as
// (N / nlast, nlast); `partial` holds one row of 5 FP64 sums per tensor row, ordered
// (nu, eta, gamma, kappa, zeta), that these kernels ADD to (no atomics: row r is only
// touched by workgroup r).
hipError_t launch_fill_zero(double* x, int64_t count, hipStream_t s);
// p = tau conj(P1) o ahat
hipError_t launch_adj_init(int prec, int64_t N, const void* ahat, const void* P1, double tau, void* p,
                           hipStream_t s);
// wq <- (gamma - 2 conj(c)|u|^2) wq - c u^2 conj(wq),  c = kappa + i zeta; partial[r][2..4] +=
// Re sum conj(w) (u, -|u|^2 u, -i |u|^2 u)
hipError_t launch_adj_phys(int prec, int64_t N, int nlast, void* wq, const void* u, double gamma, double kappa,
                           double zeta, double* partial, hipStream_t s);
// S = sum conj(ahat) tau ell X;  ahat <- conj(E) o ahat + v;  p = tau conj(P1) o ahat;
// partial[r][0] += Re S, partial[r][1] += -Im S   (E, ell from the separable factors / eigenvalues)
hipError_t launch_adj_hat(int prec, int64_t N, int nlast, const void* v, void* ahat, void* p, const void* X,
                          const void* P1, const SepParams& sep, double tau, double* partial, hipStream_t s);

// Stage combination of Krogstad's scheme in eigenspace (streaming, FP64 arithmetic):
//   out[j] = E_j uh[j] + sum_{t < nt} F_t[j] (sum_{m < 5} c[t][m] v_m[j])
// E from sep (with sep.mu = d - 1; omitted when uh is null), F_t null means 1, v_m null means 0.
// out may alias any input (each element is read before it is written by the same thread).
struct CombParams {
  const void* uh = nullptr;
  SepParams sep;
  const void* F[3] = {nullptr, nullptr, nullptr};
  const void* v[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  double c[3][5] = {};
  int nt = 0;
  void* out = nullptr;
};
hipError_t launch_comb(int prec, int64_t N, int nlast, const CombParams& p, hipStream_t s);

// Refinement sweep of the inverse (refine.hip).  v, x, r: complex128 tensors of N elements;
// y: the state type of `prec` (complex64, or complex128 for FP64).
hipError_t launch_rf_sub(int64_t N, const void* v, const void* x, void* r, hipStream_t s);  // r = v - x
hipError_t launch_rf_to_state(int prec, int64_t N, const void* r, void* y, hipStream_t s);  // y = (state) r
hipError_t launch_rf_set(int prec, int64_t N, void* x, const void* y, hipStream_t s);       // x = y
hipError_t launch_rf_add(int prec, int64_t N, void* x, const void* y, hipStream_t s);       // x += y
// out[0] = sum |r_j|^2 in FP64; partial holds rf_norm_parts() doubles of scratch.
int rf_norm_parts();
hipError_t launch_rf_norm2(int64_t N, const void* r, double* partial, double* out, hipStream_t s);

// Sums `count` per-block partial rows of width `width` into acc[width] (acc += sum).
hipError_t launch_reduce_partials(const double* partial, int64_t count, int width, double* acc,
                                  hipStream_t s);
// other = prod over the axes != mu (mu = 0 or d-1) of the separable factors, for all
// `count` flat indices over the remaining axes (FP64, double2).
hipError_t launch_sep_table(const SepParams& sep, int mu, int64_t count, void* other, hipStream_t s);
// first_m1[j] = prod_{mu >= 1} (1 + facm1[mu][j_mu]) - 1 (accumulated without cancellation)
// and first_lam[j] = sum_{mu >= 1} lam[mu][j_mu], for the count = N / n_0 flat indices.
hipError_t launch_sep_table_m1(const SepParams& sep, int64_t count, void* first_m1, double* first_lam,
                               hipStream_t s);
// Elementwise f-grid from separable eigenvalues: F[j] = f(theta (nu + i eta) sum lam_mu[j_mu]),
// evaluated in FP64 on the device and stored in the state type.
hipError_t launch_fgrid(int prec, int kind, double theta_re, double theta_im, const SepParams& sep,
                        int64_t N, void* F, hipStream_t s);

}  // namespace fcgle
