/*
 * fcgle.h -- C ABI of the MI355X (gfx950) library for the matrix/tensor-oriented
 * integrators of the d-dimensional space-fractional complex Ginzburg--Landau
 * equation (Caliari & Cassini).
 *
 * The equation (Section 1, eq. FCGLE) is
 *     u_t = (nu + i eta) sum_mu d^{alpha_mu}_{x_mu} u + gamma u - (kappa + i zeta)|u|^2 u + s,
 * semidiscretised (Section 2) with centred fractional differences on n_mu inner
 * points per axis into u' = K u + g(t, u), where K = (nu + i eta)(D_1 (+) ... (+) D_d)
 * is a Kronecker sum (eq. Ksum) of dense symmetric Toeplitz matrices D_mu = Q_mu Lambda_mu Q_mu^T
 * (eqs. Dnalpha, diag).  Every time step applies a matrix function f(theta K) through
 * the Tucker form (Section 3, eq. fKu_diag):
 *     f(theta K) v = vec( (F o (V x_1 Q_1^T ... x_d Q_d^T)) x_1 Q_1 ... x_d Q_d ),
 * F_j = f(theta (nu + i eta) sum_mu lambda_{j_mu}).
 *
 * Conventions shared by all entry points
 * --------------------------------------
 *  - Tensors are C-ordered (n_1, ..., n_d), axis d fastest, complex interleaved
 *    (re, im).  The element type is complex128 for FCGLE_FP64 plans and
 *    complex64 for FCGLE_FP32 / FCGLE_BF16X3 / FCGLE_BF16X6 plans.
 *  - Arguments named *_dev are device pointers on the plan's device, owned by
 *    the caller, 16-byte aligned.  Arguments without the suffix are host memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    device work is ordered on it; no entry point synchronises except
 *    fcgle_setup / fcgle_batch_setup (host-to-device uploads), the fcgle_host_*
 *    helpers (host only) and the calls documented as synchronising.
 *  - Return value: FCGLE_OK (0) or a negative fcgle_status.  A readable message
 *    for the last failure on the calling thread is given by fcgle_last_error().
 *    No C++ exception crosses this boundary.
 *  - A plan is not thread-safe: calls on one plan must not overlap.
 */
#ifndef FCGLE_H
#define FCGLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fcgle_plan fcgle_plan;

/* Model parameters of eq. FCGLE (Section 1): nu >= 0, kappa >= 0 (the paper takes
 * both positive; 0 is accepted for conservation tests), eta, gamma, zeta real. */
typedef struct {
  double nu, eta, gamma, kappa, zeta;
} fcgle_params;

typedef enum {
  FCGLE_OK = 0,
  FCGLE_ERR_ARG = -1,         /* invalid argument (sizes, orders, NULL, tau mismatch ...) */
  FCGLE_ERR_UNSUPPORTED = -2, /* valid request that is not implemented                  */
  FCGLE_ERR_NOMEM = -3,       /* device or host allocation failed                       */
  FCGLE_ERR_HIP = -4,         /* a HIP runtime call failed                              */
  FCGLE_ERR_NONFINITE = -5,   /* NaN/Inf found by fcgle_check_finite                    */
  FCGLE_ERR_STATE = -6        /* call out of order (e.g. no source registered)          */
} fcgle_status;

/* Matrix functions f(z) (Section 3 and Section 4, eq. phi). */
typedef enum {
  FCGLE_INV = 0,  /* 1/(1 - z): linearly implicit steps          */
  FCGLE_EXP = 1,  /* e^z = phi_0                                  */
  FCGLE_PHI1 = 2, /* phi_1(z) = (e^z - 1)/z, phi_1(0) = 1         */
  FCGLE_PHI2 = 3, /* phi_2(z) = (phi_1(z) - 1)/z, phi_2(0) = 1/2  */
  FCGLE_PHI3 = 4  /* phi_3(z) = (phi_2(z) - 1/2)/z, phi_3(0) = 1/6 */
} fcgle_kind;

/* Time schemes for u' = K u + g(t, u). */
typedef enum {
  FCGLE_EXP_EULER = 0, /* u+ = e^{tau K} u + tau phi_1(tau K) g(t, u)                      */
  FCGLE_LAWSON = 1,    /* u+ = e^{tau K} (u + tau g(t, u))                                  */
  FCGLE_LIE = 2,       /* backward-forward Euler (Section 4): (I - tau K) u+ = u + tau g(t, u) */
  FCGLE_LBDF2 = 3,     /* linearised BDF2 with BFE start (Section 4, eq. lbdf2-v)          */
  FCGLE_STRANG = 4,    /* Strang splitting (Section 4, eq. Strang):
                          u+ = phi_{tau/2}(e^{tau K} phi_{tau/2}(u)), phi_t the exact flow of
                          w' = gamma w - (kappa + i zeta)|w|^2 w; no source term            */
  FCGLE_KROGSTAD = 5   /* Krogstad's fourth-order exponential Runge-Kutta scheme (Section 4,
                          eq. krogstad-v), phi_1..phi_3 at tau/2 and tau                    */
} fcgle_scheme;

/* Arithmetic of the mode-product contractions.  Setup (weights, eigenpairs,
 * f-grids) is always FP64. */
typedef enum {
  FCGLE_FP64 = 0,   /* complex128 state, FP64 MFMA                                       */
  FCGLE_FP32 = 1,   /* complex64 state, FP32 MFMA                                        */
  FCGLE_BF16X3 = 2, /* complex64 state, Q and U split in 2 BF16 pieces, 3 products, FP32 acc */
  FCGLE_BF16X6 = 3  /* complex64 state, 3 BF16 pieces, 6 products, FP32 acc               */
} fcgle_precision;

/* ---------------------------------------------------------------------------
 * Plan lifetime
 * ------------------------------------------------------------------------- */

/* Build a plan on the current HIP device.
 *   d          : number of space dimensions, 1 <= d <= 4
 *   n[d]       : inner points per axis, 2 <= n_mu <= 4096 (Section 2 grid)
 *   alpha[d]   : fractional orders, 1 < alpha_mu <= 2 (the paper requires < 2;
 *                2 gives the classical 3-point Laplacian and is kept for tests)
 *   h[d]       : grid spacings (b_mu - a_mu)/(n_mu + 1) > 0
 *   params     : model parameters (see fcgle_params)
 *   fd_order   : 2 (eq. FD2) or 4 (eq. FD4)
 *   precision  : fcgle_precision
 *   tau        : time step > 0; the f-grids are built for it
 *   out        : receives the plan (NULL on failure)
 * Forms the weights g_k by their recurrence (Section 2), the dense D_mu, their
 * eigendecomposition in FP64 on the host (Section 4, the paper's CPU-side
 * diagonalisation), and uploads Q_mu, Q_mu^T (in the plan's precision) and lambda_mu.
 * Synchronous.  Errors: ERR_ARG, ERR_NOMEM, ERR_HIP. */
int fcgle_setup(int d, const int64_t* n, const double* alpha, const double* h,
                const fcgle_params* params, int fd_order, int precision, double tau,
                fcgle_plan** out);

/* Release every device and host resource of the plan (NULL is a no-op).
 * Synchronises the plan's device before freeing. */
void fcgle_destroy(fcgle_plan* plan);

/* Message describing the last failure on the calling thread ("" if none).
 * The pointer stays valid until the next failing call on the same thread. */
const char* fcgle_last_error(void);

/* Eigenpairs of axis mu (0-based), D_mu = Q_mu Lambda_mu Q_mu^T (Section 2, eq. diag), in FP64:
 * Q[n_mu * n_mu] row-major with
 * column k the eigenvector of lambda[k]; lambda ascending (the plan itself keeps them in
 * even/odd block order, see fcgle_set_structure).  Host buffers.
 * Errors: ERR_ARG. */
int fcgle_get_eig(const fcgle_plan* plan, int mu, double* Q, double* lambda);

/* Register the source s(t) = sum_k exp(c_k t) S_k (Section 1, the term s of eq. FCGLE) with
 * complex rates c_k = rate[k] + i rate_im[k] (rate_im may be NULL: real rates), nterms <= 4,
 * each S_k a device tensor of the plan's state type that must stay alive while steps run.
 * exp(c_k t) is formed in FP64 on the host for every evaluation time.  nterms = 0 removes
 * the source.  Errors: ERR_ARG. */
int fcgle_set_source(fcgle_plan* plan, int nterms, const double* rate, const double* rate_im,
                     const void* const* S_dev);

/* ---------------------------------------------------------------------------
 * Matrix-function action and time steps
 * ------------------------------------------------------------------------- */

/* out = f(theta K) u (Section 3, eq. fKu_diag) for f = kind.  u_dev and out_dev
 * may be the same buffer.  The f-grid for (kind, theta) is built in FP64 on the
 * first call with that pair (synchronous upload); later calls only launch
 * kernels.  The exponential uses the separable grid exp(theta(nu+i eta)lambda_1) x ...
 * (the Kronecker-product form, eq. Neudeckerd).  Errors: ERR_ARG, ERR_NOMEM, ERR_HIP. */
int fcgle_apply_f(fcgle_plan* plan, int kind, double theta, const void* u_dev, void* out_dev,
                  void* stream);

/* The inverse of the linearly implicit steps, x = (I - theta (nu + i eta) K)^{-1} v (Section 3,
 * the resolvent R = 1/(1 - z) on the eigenvalue grid), refined to FP64 accuracy for plans of
 * any precision by classical iterative refinement: x_0 = R o v is formed with the plan's
 * precision (Q^T, the R-grid, Q); then `sweeps` times the residual
 * r = v - (I - theta (nu + i eta) K) x is formed in FP64 with FP64 MFMA mode products by the
 * Toeplitz matrices D_mu themselves (K u = sum_mu (nu + i eta) U x_mu D_mu, eq. kronsumv), and
 * x += R o r again with the plan's precision.
 * v_dev, x_dev: complex128 device tensors of N elements in C order, not aliased; v is read
 * only.  sweeps: 0..8.  rnorm (host, optional): sweeps + 1 values
 * ||v - (I - theta (nu + i eta) K) x_k||_2 / ||v||_2, k = 0..sweeps, from FP64 wavefront
 * reductions (one more residual; the call then synchronises the stream).  The first call
 * uploads D_mu in FP64 (npad^2 doubles per axis) and allocates two N-element work tensors.
 * Errors: ERR_ARG, ERR_NOMEM, ERR_HIP. */
int fcgle_apply_inv_refined(fcgle_plan* plan, double theta, const void* v_dev, void* x_dev, int sweeps,
                            double* rnorm, void* stream);

/* Forget the cached eigenspace state (u_hat = u x_1 Q_1^T ... x_d Q_d^T, the transformed
 * state of Section 3, eq. fKu_diag) and the LBDF2 history, then (if u_prev_dev is not NULL)
 * record u_prev_dev as u_{n-1}, the second starting value of the two-step scheme (Section 4,
 * eq. lbdf2-v), for the next FCGLE_LBDF2 step on u_dev.  Both caches are keyed by the device
 * address u_dev only: call it whenever the caller writes u_dev between steps, or hands the
 * library a new tensor that may occupy a freed buffer's address.  Errors: ERR_ARG. */
int fcgle_set_state(fcgle_plan* plan, const void* u_dev, const void* u_prev_dev, void* stream);

/* Advance u_dev in place from time t to t + tau by one step of `scheme`.
 * tau must equal the plan's tau (ERR_ARG otherwise).
 * FCGLE_EXP_EULER keeps u_hat = u x_mu Q_mu^T in the plan between calls on the
 * same u_dev, so a steady-state step costs one forward and one backward Tucker
 * operator; the first step on a buffer (or after fcgle_set_state) adds one
 * forward transform.  FCGLE_LBDF2 takes the BFE start when it has no history
 * for u_dev and keeps u_{n-1} in the plan afterwards.  FCGLE_STRANG keeps no state: a step
 * is the exact flow over tau/2, e^{tau K} as Q (E . (Q^T v)) with the separable E in the last
 * forward epilogue, and the flow over tau/2 again (streaming passes, or fused with fusion
 * bit 6); with fusion bit 1 its forward products run from the last axis to the first whatever
 * bit 2 says (the E epilogue is cheapest on axis 0).  A plan with a source term gives
 * ERR_UNSUPPORTED for it.  FCGLE_KROGSTAD keeps u_hat like FCGLE_EXP_EULER; a steady-state
 * step costs four forward and four backward Tucker operators (the nonlinearity at t, t + tau/2
 * twice and t + tau fused into the forward ones) and four streaming passes that combine the
 * stages in eigenspace with the phi_1..phi_3 grids and the separable E in FP64; the first step
 * allocates five more state tensors.  Errors: ERR_ARG, ERR_UNSUPPORTED, ERR_HIP, ERR_NOMEM. */
int fcgle_step(fcgle_plan* plan, int scheme, void* u_dev, double t, double tau, void* stream);

/* nsteps consecutive fcgle_step calls from t0 (t_k = t0 + k tau).  For FCGLE_STRANG the
 * trailing flow over tau/2 of each step and the leading one of the next run as one flow over
 * tau (the flow of an autonomous equation composes exactly), so intermediate states are not
 * formed; the result equals nsteps single steps up to rounding.  For FCGLE_EXP_EULER without
 * a source term and with timing off, runs of two or more steps replay them in blocks of 64,
 * 16, 4 and 2 steps from HIP graphs captured on first use of each block length (per state
 * buffer, eigenspace buffer assignment and plan configuration; fcgle_set_tiles / _fusion /
 * _structure / _source / _wide_loads and fcgle_autotune invalidate them; up to 8 are kept).
 * The first step runs directly unless the state of u_dev is cached and a step already ran
 * under the current configuration, and an odd remainder runs directly: the same kernels with
 * the same arguments, so the result is identical to nsteps single steps. */
int fcgle_run(fcgle_plan* plan, int scheme, void* u_dev, double t0, double tau, int64_t nsteps,
              void* stream);

/* Vector-Jacobian product of one FCGLE_EXP_EULER step u_{n+1} = E u_n + tau P1 g(t, u_n)
 * (E = e^{tau K}, P1 = phi_1(tau K)) for a real loss, cotangent convention
 * ubar = dL/dRe u + i dL/dIm u:
 *   w        = tau P1^H ubar_{n+1}
 *   ubar_n   = E^H ubar_{n+1} + (gamma - 2 conj(c)|u_n|^2) w - c u_n^2 conj(w),  c = kappa + i zeta
 *   pbar    += dL/d(nu, eta, gamma, kappa, zeta)
 * with dL/dnu = Re sum conj(Q^T ubar_{n+1}) tau ell (e^z Q^T u_n + tau phi_1'(z) Q^T g_n),
 * z = tau (nu + i eta) ell, phi_1' = phi_1 - phi_2 (from eq. phi), and i tau ell for eta.
 * u_n_dev: the state the step started from (not modified); ubar_next_dev: cotangent of
 * u_{n+1}; ubar_n_dev: output (may alias ubar_next_dev, must not alias u_n_dev); pbar_dev:
 * 5 doubles on the device, ADDED to.  The source must not depend on the parameters.
 * Equivalent to copying ubar_next into ubar_n and calling fcgle_vjp_run with m = 1.
 * Other schemes: ERR_UNSUPPORTED.  Errors: ERR_ARG, ERR_NOMEM, ERR_HIP. */
int fcgle_vjp(fcgle_plan* plan, int scheme, const void* u_n_dev, const void* ubar_next_dev,
              void* ubar_n_dev, double* pbar_dev, double t, double tau, void* stream);

/* Adjoint of m consecutive FCGLE_EXP_EULER steps u_0 -> u_m starting at time t0 from
 * u_start_dev = u_0 (a checkpoint; not modified).  The states u_0..u_{m-1} are recomputed
 * inside the call (m forward steps, kept in plan-owned buffers of 2m state tensors that are
 * allocated on first use and reused); the adjoint is then swept backwards with the adjoint
 * state in eigenspace, so each adjoint step costs one backward and one forward Tucker
 * operator plus two streaming passes.  On entry ubar_dev holds the cotangent of u_m, on
 * return that of u_0 (in place; distinct from u_start_dev).  pbar_dev (5 doubles, device) is
 * ADDED to, in the order (nu, eta, gamma, kappa, zeta); the per-row sums are formed in FP64
 * and reduced in a fixed order, so results do not depend on scheduling.  The plan's cached
 * eigenspace state and LBDF2 history are invalidated.  Other schemes: ERR_UNSUPPORTED.
 * Errors: ERR_ARG, ERR_NOMEM, ERR_HIP. */
int fcgle_vjp_run(fcgle_plan* plan, int scheme, const void* u_start_dev, int64_t m, void* ubar_dev,
                  double* pbar_dev, double t0, double tau, void* stream);

/* Scan a state tensor for NaN/Inf.  Synchronises `stream`.
 * Returns FCGLE_OK or FCGLE_ERR_NONFINITE (or ERR_ARG / ERR_HIP). */
int fcgle_check_finite(fcgle_plan* plan, const void* u_dev, void* stream);

/* ---------------------------------------------------------------------------
 * Introspection, tuning and timing
 * ------------------------------------------------------------------------- */

/* Number of elements N = prod n_mu and bytes per complex element (16 or 8). */
int fcgle_plan_shape(const fcgle_plan* plan, int64_t* N, int* elem_bytes);

/* Time every candidate tile configuration of each mode product on `stream`
 * (scratch inputs, max(3 reps, 10) launches each) and keep the fastest per axis and
 * direction; then time whole exponential-Euler steps (as many) for every placement of
 * the nonlinearity and of the update (fcgle_set_fusion), time the fastest four again in
 * three interleaved rounds and keep the best of them; finally compare each product's
 * runner-up tile with its choice in whole steps (three interleaved rounds) and keep the
 * faster.
 * For a batch plan: the same per grouped phase over all instances (`reps` launches).
 * Overwrites the plan's scratch buffers, so the cached eigenspace state and the LBDF2 history
 * are forgotten (as by fcgle_set_state): the next step of any scheme starts from u_dev alone.
 * Synchronous.  Errors: ERR_HIP. */
int fcgle_autotune(fcgle_plan* plan, int reps, void* stream);

/* Choose the tile configuration (0..4; rows x columns per tile depend on the precision and
 * structure, see fcgle_describe) of the mode product on `axis` in direction fwd (1: Q^T, 0: Q).
 * For a forward product of an even/odd plan, cfg 5..9 selects configuration
 * cfg - 5 in the form that computes both blocks in one tile (one load of each mirrored pair,
 * marked F by fcgle_describe).  Results do not depend on it beyond rounding order.
 * Errors: ERR_ARG, ERR_UNSUPPORTED (cfg >= 5 on a dense-structure plan). */
int fcgle_set_tiles(fcgle_plan* plan, int axis, int fwd, int cfg);

/* Structure of the mode products.  Every D_mu is symmetric Toeplitz, hence persymmetric
 * (J D J = D with J the exchange matrix), so Q_mu = Z diag(Ve, Vo) with Z built from
 * (e_k +- e_{n-1-k})/sqrt(2) and Ve, Vo the eigenvectors of two half-size blocks (the
 * set-up always diagonalises D_mu this way).  split = 1 (the default, every precision):
 * each mode product contracts the half-length sums and differences of mirrored fibre
 * entries with the half-size blocks -- half the multiply-adds of the dense product for the
 * same bytes moved; split = 0: dense Q_mu^T / Q_mu products.  Results agree to rounding.
 * Resets the tile choice to its default (autotune again after).  Errors: ERR_ARG. */
int fcgle_set_structure(fcgle_plan* plan, int split);

/* Loads of the mode products' tensor operand.  Every product reads its k-tiles through
 * 32-bit offsets from per-k-tile buffer views, except N-loader products (an axis other than
 * the last) whose 32 rows at element stride B = n_{mu+1} ... n_d span more than 2 GiB
 * (B > 2^23 for complex64, 2^22 for complex128): those use a tile configuration with 64-bit
 * element indices, chosen by the library and reported by fcgle_describe as
 * "loads=64-bit-index(axes ...)".  force = 1 takes that configuration for every N-loader
 * product (to test it on small tensors; results agree with the other configurations to
 * rounding order); force = 0 restores the automatic choice.
 * Errors: ERR_ARG. */
int fcgle_set_wide_loads(fcgle_plan* plan, int force);

/* Fusion switches: bit 0 fuses the pointwise prologue (nonlinearity) into the first
 * mode product of a Tucker operator, bit 1 fuses the pointwise epilogue (f-scale,
 * exponential-Euler update, LBDF2 history) into the last one; a cleared bit runs that
 * map as a separate streaming kernel.  Bit 2 runs the mode products of forward (Q^T)
 * operators from the last axis to the first (the products commute), so the epilogue lands
 * on a product along a slow axis.  Bit 3 moves the exponential-Euler update
 * uhat <- E uhat + tau P1 ghat out of the forward operator into the first backward product,
 * which applies it to ghat while loading its tile, stores the new state and contracts it
 * (even/odd plans with d >= 2; otherwise bit 3 is ignored).  Bit 5 (32), with
 * bit 3: that update forms P1 = phi_1(z) = (e^z - 1)/z in FP64 from separable tables (e^z - 1
 * accumulated from the per-axis expm1 without cancellation) instead of reading the stored P1
 * grid (n_1 <= 512; otherwise ignored).  Bit 6 (64) fuses the exact nonlinear flows of
 * FCGLE_STRANG into the first forward / the last backward mode product (cleared: streaming
 * passes, which are the faster form on MI355X at 256^3 since the flow's log1p and sincos would
 * stall the contraction).  Bit 4 is reserved.  Default 3; fcgle_autotune picks bits 0-5 by
 * timing whole exponential-Euler steps (and sets bit 1 when the update runs in the backward
 * prologue, where it has no effect on exponential Euler).  Errors: ERR_ARG. */
int fcgle_set_fusion(fcgle_plan* plan, int flags);

/* Human-readable plan summary (sizes, precision, chosen tiles) into buf. */
int fcgle_describe(const fcgle_plan* plan, char* buf, size_t len);

/* Enable (capacity > 0) or disable (0) per-launch HIP-event timing of the
 * mode-product kernels.  While enabled, each mode-product launch records an
 * event pair on its stream (up to `capacity` launches, further ones untimed).
 * Errors: ERR_NOMEM, ERR_HIP. */
int fcgle_timing_enable(fcgle_plan* plan, int capacity);

/* Copy out the recorded launches (synchronising on their events) and clear the
 * record.  For launch i < *count (at most cap): axis[i] = mode axis (0-based),
 * fwd[i] = 1 for a Q^T (forward) and 0 for a Q (backward) mode product, ms[i] =
 * its duration, sig[i] = the kernel instantiation it ran:
 *   sig = structure * 4096 + (((prec * 8 + tile_cfg) * 2 + t_loader) * 8 + prologue) * 8 + epilogue
 * (structure 0 dense, 1 even/odd Q^T, 2 even/odd Q, 3 even/odd Q^T with both blocks per tile;
 * prec 0..3 as fcgle_precision;
 * t_loader 1 for the fastest axis; prologue 0 none, 1 nonlinearity, 2 exponential-Euler
 * update, 3 the same with phi_1 on the fly, 4 exact nonlinear flow (Strang); epilogue 0 store,
 * 1 grid, 2 separable exp, 3 exp-Euler update, 4 keep-old, 5 exp-Euler update with adjoint
 * record, 6 FP64 axpy (refinement residual), 7 exact nonlinear flow (Strang)).
 * Errors: ERR_STATE if timing is off, ERR_HIP. */
int fcgle_timing_read(fcgle_plan* plan, int cap, int* axis, int* fwd, int* sig, double* ms,
                      int64_t* count);

/* ---------------------------------------------------------------------------
 * Batched independent 2-D instances
 * ------------------------------------------------------------------------- */

/* A batch of `count` independent 2-D problems (1 <= count <= 65535) of uneven sizes
 * n[2i] x n[2i+1] (2..4096 each), each with its own alpha[2i..2i+1], h[2i..2i+1] and
 * params[i], one shared tau, FD2, complex64 state, FP32 MFMA (precision must be
 * FCGLE_FP32, else ERR_UNSUPPORTED).  The eigendecompositions (Section 2, eq. diag) are
 * formed in FP64 on the host, spread over host threads; all per-instance device buffers
 * (Q, Q^T, eigenvalues, phi_1 grid, eigenspace state, two scratch tensors) live in one
 * device allocation.  The returned plan is accepted by fcgle_batch_run, fcgle_autotune,
 * fcgle_describe and fcgle_destroy only (ERR_ARG elsewhere).  Synchronous.
 * Errors: ERR_ARG, ERR_UNSUPPORTED, ERR_NOMEM, ERR_HIP. */
int fcgle_batch_setup(int count, const int64_t* n, const double* alpha, const double* h,
                      const fcgle_params* params, int precision, double tau, fcgle_plan** out);

/* nsteps exponential-Euler steps (the scheme of fcgle_step; each instance is its own problem
 * u' = K u + g(t, u) of Section 2, advanced through the Tucker form of Section 3, eq. fKu_diag,
 * with its own eigenpairs) of every instance, in place on
 * the caller's device buffers u_dev[i] (n[2i] * n[2i+1] complex64, C order), from t0.
 * Sources are not supported in batches.  The call forms each eigenspace state from u_dev
 * (two grouped launches), then replays a HIP graph that holds the whole trajectory (up to
 * 500 steps per graph; longer runs replay it): each phase of a step -- forward mode product
 * on axis 1 with the nonlinearity fused into its loads, forward mode product on axis 2
 * with the eigenspace update, the two backward mode products -- is one grouped launch
 * over all instances.  Graphs are captured on first use for each step count and reused;
 * the per-instance launch descriptions live in device arrays that are rebuilt (after a
 * device synchronisation) when the u_dev pointers change between calls.
 * scheme must be FCGLE_EXP_EULER (else ERR_UNSUPPORTED); tau must equal the plan's.
 * Errors: ERR_ARG, ERR_UNSUPPORTED, ERR_NOMEM, ERR_HIP. */
int fcgle_batch_run(fcgle_plan* plan, int scheme, void* const* u_dev, double t0, double tau,
                    int64_t nsteps, void* stream);

/* Form of fcgle_batch_run for a batch plan.  mode 0: the HIP graph of grouped launches above (the
 * only form in use).  mode 1 would run one persistent launch per call for all phases of all steps
 * (workgroups taking tiles in the order (step, phase, instance, tile) from an atomic ticket and
 * waiting, bounded by spin_limit polls, until the instance's previous phase is complete); that
 * form is switched off and gives ERR_UNSUPPORTED: its first GPU runs did not finish and the cause
 * is not established.  spin_limit: polls of such a wait (0 keeps the current limit).
 * Errors: ERR_ARG, ERR_UNSUPPORTED. */
int fcgle_batch_set_persistent(fcgle_plan* plan, int mode, int64_t spin_limit);

/* ---------------------------------------------------------------------------
 * Allocation-free variant
 * ------------------------------------------------------------------------- */

/* Bytes of each of the three work tensors of fcgle_apply_f_noalloc (16 MiB). */
#define FCGLE_NOALLOC_TENSOR_BYTES (16u << 20)

/* For callers that cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Computes what fcgle_apply_f(plan, kind, theta,
 * u_dev, out_dev, stream) computes, with the same kernels, but takes the three state-sized work
 * tensors of its Tucker operators from a fixed work space instead of the plan's own buffers,
 * and allocates nothing (no hipMalloc, hipFree or allocating library call).  The work space is
 * a device array of 3 * FCGLE_NOALLOC_TENSOR_BYTES bytes that every device the library runs on
 * holds from the load of the library's code object until the process ends; its address is
 * resolved when a plan is set up on the device.
 *   Limit: N * elem_bytes <= FCGLE_NOALLOC_TENSOR_BYTES (complex64 states up to 2^21 elements,
 *     e.g. 128^3; complex128 up to 2^20), else ERR_ARG.
 *   The f-grid for (kind, theta) (for FCGLE_EXP the separable factors for theta) must already
 *     exist on the plan, i.e. fcgle_apply_f ran once with the same pair (grids are built, and
 *     allocated, there); else ERR_STATE and nothing is launched.
 *   u_dev and out_dev may be the same buffer.  The work space needs no initial contents and
 *     keeps those of the last call.  It is shared by every call on one device: calls that may
 *     overlap there (other streams, threads or plans) race on it and must be serialised by the
 *     caller.
 * Errors: ERR_ARG, ERR_STATE, ERR_HIP. */
int fcgle_apply_f_noalloc(fcgle_plan* plan, int kind, double theta, const void* u_dev, void* out_dev,
                          void* stream);

/* ---------------------------------------------------------------------------
 * Host-only helpers (no device calls; usable without a GPU)
 * ------------------------------------------------------------------------- */

/* FD weights g_0..g_{n-1} of order fd_order (2: recurrence of Section 2;
 * 4: extrapolation of eq. FD4) into g[n].  Errors: ERR_ARG. */
int fcgle_host_fd_weights(double alpha, int64_t n, int fd_order, double* g);

/* D = -h^{-alpha} Toeplitz(g) and its FP64 eigendecomposition by this library's
 * own solver: the even/odd half-size blocks of the persymmetric D (see
 * fcgle_set_structure), each by Householder tridiagonalisation + implicit symmetric QR
 * with Wilkinson shifts and one extended-precision orthogonalisation sweep.  Q[n*n] row-major, column k = eigenvector of lambda[k]
 * (ascending).  Errors: ERR_ARG, ERR_NOMEM. */
int fcgle_host_eig(int64_t n, double alpha, double h, int fd_order, double* Q, double* lambda);

/* f(z) for `count` complex z (interleaved re, im) in FP64, as used for the
 * device f-grids: kind = fcgle_kind.  phi_l uses its Taylor series for |z| < 1
 * and the recurrence of eq. phi elsewhere.  Errors: ERR_ARG. */
int fcgle_host_fz(int kind, int64_t count, const double* z, double* out);

#ifdef __cplusplus
}
#endif

#endif /* FCGLE_H */
