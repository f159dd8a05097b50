// Internal definitions shared by the host translation units of the library: the plan
// object behind the opaque fcgle_plan handle, error helpers and small utilities.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fcgle.h"
#include "launch.h"

namespace fcgle {

// Records a message for fcgle_last_error() on the calling thread and returns `code`.
int fail(int code, const char* fmt, ...);

#define HIP_TRY(expr)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) return fail(FCGLE_ERR_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                                      __FILE__, __LINE__);                                      \
  } while (0)

#define FC_TRY(expr)            \
  do {                          \
    int r_ = (expr);            \
    if (r_ != FCGLE_OK) return r_; \
  } while (0)

// Restores the calling thread's current device on scope exit.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

inline hipStream_t as_stream(void* s) { return (hipStream_t)s; }

// hipMalloc that reports FCGLE_ERR_NOMEM with a message on failure.
int plan_alloc(void** p, size_t bytes);

// Batched independent problems (batch.hip).
struct BatchData;
void batch_free(BatchData* B);
int batch_autotune(fcgle_plan* plan, int reps, hipStream_t st);
int batch_describe(const fcgle_plan* plan, char* buf, size_t len);

struct GridBuf {
  int kind;
  double theta;
  void* F;
};

struct SepBuf {
  double theta;
  void* fac[4];       // double2[n_mu] each
  void* other_last;   // double2[N / n_{d-1}]: product over the axes before the last
  void* other_first;  // double2[N / n_0]: product over the axes after the first
  void* facm1[4];     // double2[n_mu]: expm1 of each factor's exponent
  void* first_m1;     // double2[N / n_0]: product over the axes after the first, minus 1
  double* first_lam;  // double[N / n_0]: sum of their eigenvalues
};

struct TimedLaunch {
  hipEvent_t e0, e1;
  int axis, fwd, sig;
};

// A captured run of `steps` exponential-Euler steps on the state buffer u with the eigenspace
// buffers uhat / uhat2 in that assignment, under plan configuration generation `gen`.
struct RunGraph {
  const void* u;
  void* uhat;
  void* uhat2;
  int64_t steps;
  uint64_t gen;
  hipGraphExec_t exec;
};

}  // namespace fcgle

struct fcgle_plan {
  int device = 0;
  fcgle::BatchData* batch = nullptr;  // set for plans made by fcgle_batch_setup
  int d = 0;
  int64_t n[4] = {1, 1, 1, 1};
  double alpha[4] = {0, 0, 0, 0};
  double h[4] = {0, 0, 0, 0};
  fcgle_params p{};
  int fd_order = 2;
  int prec = FCGLE_FP64;
  double tau = 0;
  int64_t N = 1;
  int elem = 16;
  int npad[4] = {0, 0, 0, 0};
  std::vector<double> Q[4], lam[4];  // host FP64: Q row-major, column k <-> lam[k]
  void* Mf[4] = {nullptr, nullptr, nullptr, nullptr};  // Q^T in the precision layout
  void* Mb[4] = {nullptr, nullptr, nullptr, nullptr};  // Q
  double* dlam[4] = {nullptr, nullptr, nullptr, nullptr};
  std::vector<fcgle::GridBuf> grids;
  std::vector<fcgle::SepBuf> seps;
  void* s[3] = {nullptr, nullptr, nullptr};  // scratch tensors
  void* uhat = nullptr;
  void* uhat2 = nullptr;  // second eigenspace state (update prologue writes here, then swapped)
  void* kg[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // Krogstad: ghat_n, ghat_2..4, stage
  bool uhat_valid = false;
  const void* uhat_src = nullptr;
  void* uprev = nullptr;
  bool hist_valid = false;
  const void* hist_src = nullptr;
  int ns = 0;
  double rate[4] = {0, 0, 0, 0};     // source rates c_k = rate + i rate_im
  double rate_im[4] = {0, 0, 0, 0};
  const void* S[4] = {nullptr, nullptr, nullptr, nullptr};
  int cfg[4][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};  // [axis][fwd], for the active structure
  int cfg_upd = -1;  // tiles of the axis-0 backward product with the update prologue (-1: cfg[0][0])
  bool fwd2[4] = {false, false, false, false};  // forward even/odd products with both blocks per tile
  // even/odd split of the mode products (persymmetric D): block sizes, leading dimension and
  // the stacked block matrices [Fe; Fo] (forward) and [Be; Bo] (backward)
  bool split = false;
  int me[4] = {0, 0, 0, 0}, mo[4] = {0, 0, 0, 0}, ldsp[4] = {0, 0, 0, 0};
  void* Mfs[4] = {nullptr, nullptr, nullptr, nullptr};
  void* Mbs[4] = {nullptr, nullptr, nullptr, nullptr};
  bool tuned = false;
  // bit 0: nonlinearity prologue, bit 1: epilogue of the last forward product, bit 3:
  // exponential-Euler update in the prologue of the first backward product (when supported)
  int fusion = 3;
  bool fwd_rev = false;  // forward operators run their mode products from axis d to axis 1
  bool wide_force = false;  // every N-loader mode product through 64-bit element indices (mp_wide)
  int* dflag = nullptr;
  // refinement sweep of the inverse (allocated on first use): FP64 Toeplitz D_mu (npad x npad),
  // the FP64 residual, a state-type work tensor, and norm partials + results
  void* Md[4] = {nullptr, nullptr, nullptr, nullptr};
  void* rf_r = nullptr;
  void* rf_y = nullptr;
  double* rf_part = nullptr;
  // adjoint work buffers (allocated on first use): eigenspace adjoint state, its P1-scaled
  // copy, the forward-transformed adjoint source, and the recomputed segment (u_k, X_k)
  void* adj[3] = {nullptr, nullptr, nullptr};
  std::vector<void*> traj_u, traj_x;
  double* partial = nullptr;
  int64_t partial_rows = 0;
  // captured exponential-Euler runs (fcgle_run), their capture stream, and the configuration
  // generation (bumped by every call that changes which kernels a step launches)
  std::vector<fcgle::RunGraph> run_graphs;
  hipStream_t cap_stream = nullptr;
  uint64_t gen = 0;
  uint64_t ready_gen = ~0ull;  // gen of the last directly run exponential-Euler step (its lazy set-up done)
  // timing
  int timing_cap = 0;
  std::vector<hipEvent_t> ev_pool;
  std::vector<fcgle::TimedLaunch> timed;
};
