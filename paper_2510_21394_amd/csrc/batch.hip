// Batched independent 2-D problems: many instances of uneven sizes and parameters advanced
// together by exponential Euler.  Each phase of a step (the nonlinearity fused into the
// axis-0 forward mode product, the axis-1 forward mode product with the eigenspace update,
// the two backward mode products) is ONE grouped launch over all instances, and the whole
// trajectory of a call is captured once into a HIP graph and replayed with one launch.
//
// Per instance (C-order (n1, n2), axis 2 fastest), with the eigenspace state
// uhat = Q_1^T U Q_2 (the tensor form of the Tucker operator, Section 3, eq. fKu_diag2):
//   F0: T   = g(U) x_1 Q_1^T                 (N loader, nonlinearity in the loads)
//   F1: uhat <- E o uhat + tau P1 o (T x_2 Q_2^T)   (T loader, fused or streaming update)
//   B0: T   = uhat x_1 Q_1
//   B1: U   = T x_2 Q_2
// A call first forms uhat from U (two more grouped launches), so calls are independent.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "fz.hpp"
#include "host_math.h"
#include "plan.h"

namespace fcgle {

namespace {

enum PhaseId { PH_T0 = 0, PH_T1, PH_F0, PH_F1, PH_B0, PH_B1, PH_COUNT };

struct BatchInst {
  int64_t n[2] = {0, 0};
  int npad[2] = {0, 0};   // leading dimension of each block matrix (>= me)
  int me[2] = {0, 0}, mo[2] = {0, 0};  // even / odd block sizes per axis
  double alpha[2] = {0, 0}, h[2] = {0, 0};
  fcgle_params p{};
  int64_t N = 0;
  std::vector<double> Q[2], lam[2];
  float* Mf[2] = {nullptr, nullptr};  // [Fe; Fo] per axis (forward, even/odd blocks)
  float* Mb[2] = {nullptr, nullptr};  // [Be; Bo] per axis (backward)
  double* dlam[2] = {nullptr, nullptr};
  double* fac[2] = {nullptr, nullptr};  // exp(tau (nu + i eta) lambda), complex FP64
  float2* P1 = nullptr;
  float2* uhat = nullptr;
  float2* tmp = nullptr;
  float2* tmp2 = nullptr;
};

// Instances can be split per phase into size classes by the half-block length of the axis the
// phase contracts (m_e <= kClassRows: one 128-row tile covers the block; larger: several), each
// class with its own tile configuration and grouped launch; the autotuner keeps that split or
// one class per phase, whichever runs a step faster.  Within a class the instances are ordered
// by work, largest first, so that their workgroups are dispatched first.
constexpr int kClasses = 2;
constexpr int kClassRows = 128;

struct Phase {
  int cfg = 1;
  int sp = 1;  // even/odd form: kSplitFwd or kSplitFwd2 (forward phases), kSplitBwd
  bool tl = false;
  ProKind pk = ProKind::Id;
  EpiKind ek = EpiKind::Store;
  void* items = nullptr;  // device item array
  uint32_t nblocks = 0;
  std::vector<int> members;  // instances of this size class, largest work first
};

struct CachedGraph {
  int64_t steps;
  hipGraphExec_t exec;
};

}  // namespace

struct BatchData {
  int count = 0;
  double tau = 0;
  std::vector<BatchInst> inst;
  void* pool = nullptr;
  Phase ph[PH_COUNT][kClasses];
  bool fuse = true;       // F1 with the fused update (else Store + streaming pass)
  bool classes = false;   // size classes per phase (else one class holding every instance)
  void* pw_items = nullptr;
  uint32_t pw_rows = 0;
  std::vector<const void*> bound;  // state pointers the item arrays were built for
  bool items_valid = false;
  bool tuned = false;
  hipStream_t cap = nullptr;
  std::vector<CachedGraph> graphs;
  // persistent form (batch_persist_kernel): one launch for all phases of every step
  bool persist = false;
  int pcfg = 0;                         // its tile configuration (persist_supported)
  uint32_t spin_limit = 1000000u;       // polls of a dependency wait (about 1 us each) before an error
  void* p_items[4] = {nullptr, nullptr, nullptr, nullptr};
  void* p_buf = nullptr;                // PersistCtl, done[count], pre[5 count]
  uint32_t p_phase0[5] = {0, 0, 0, 0, 0};
  int p_cfg_built = -1;                 // configuration the persistent items were built for
  int p_grid = 0;
};

void batch_free(BatchData* B) {
  if (!B) return;
  for (auto& g : B->graphs) (void)hipGraphExecDestroy(g.exec);
  for (auto& q : B->p_items)
    if (q) (void)hipFree(q);
  if (B->p_buf) (void)hipFree(B->p_buf);
  for (auto& pc : B->ph)
    for (auto& p : pc)
      if (p.items) (void)hipFree(p.items);
  if (B->pw_items) (void)hipFree(B->pw_items);
  if (B->pool) (void)hipFree(B->pool);
  if (B->cap) (void)hipStreamDestroy(B->cap);
  delete B;
}

namespace {

void clear_graphs(BatchData* B) {
  for (auto& g : B->graphs) (void)hipGraphExecDestroy(g.exec);
  B->graphs.clear();
}

MPLaunch inst_launch(const BatchData* B, const BatchInst& I, int phase, const Phase& ph, const void* u) {
  MPLaunch L;
  L.prec = P_F32;
  L.cfg = ph.cfg;
  const bool axis1 = (phase == PH_T1 || phase == PH_F1 || phase == PH_B1);
  const bool fwd = (phase == PH_T0 || phase == PH_T1 || phase == PH_F0 || phase == PH_F1);
  const int mu = axis1 ? 1 : 0;
  L.A = axis1 ? I.n[0] : 1;
  L.B = axis1 ? 1 : I.n[1];
  L.n = (int)I.n[mu];
  L.npad = I.npad[mu];
  L.split = fwd ? ph.sp : kSplitBwd;
  L.me = I.me[mu];
  L.mo = I.mo[mu];
  L.M = fwd ? (const void*)I.Mf[mu] : (const void*)I.Mb[mu];
  L.pk = ph.pk;
  L.ek = ph.ek;
  switch (phase) {
    case PH_T0:
      L.in = u;
      L.ep.out = I.tmp;
      break;
    case PH_T1:
      L.in = I.tmp;
      L.ep.out = I.uhat;
      break;
    case PH_F0:
      L.in = u;
      L.ep.out = I.tmp;
      L.pp.gamma = I.p.gamma;
      L.pp.kappa = I.p.kappa;
      L.pp.zeta = I.p.zeta;
      break;
    case PH_F1:
      L.in = I.tmp;
      if (ph.ek == EpiKind::ExpEuler) {
        L.ep.out = I.uhat;
        L.ep.F = I.P1;
        L.ep.tau = B->tau;
        L.ep.sep.d = 2;
        L.ep.sep.mu = 1;
        L.ep.sep.n[0] = (int)I.n[0];
        L.ep.sep.n[1] = (int)I.n[1];
        L.ep.sep.fac[0] = I.fac[0];
        L.ep.sep.fac[1] = I.fac[1];
      } else {
        L.ep.out = I.tmp2;
      }
      break;
    case PH_B0:
      L.in = I.uhat;
      L.ep.out = I.tmp;
      break;
    case PH_B1:
      L.in = I.tmp;
      L.ep.out = const_cast<void*>(u);
      break;
  }
  return L;
}

EpiParams update_params(const BatchData* B, const BatchInst& I) {
  EpiParams ep;
  ep.out = I.uhat;
  ep.F = I.P1;
  ep.tau = B->tau;
  ep.sep.d = 2;
  ep.sep.mu = 1;
  ep.sep.n[0] = (int)I.n[0];
  ep.sep.n[1] = (int)I.n[1];
  ep.sep.fac[0] = I.fac[0];
  ep.sep.fac[1] = I.fac[1];
  return ep;
}

int build_persist(BatchData* B, const void* const* u);

// Members of every phase's classes: by size class (split) or all in class 0, largest work first
// (the phase's multiply-adds are proportional to N m_e of its axis).  Invalidates the items.
void assign_classes(BatchData* B, bool split) {
  for (int p = 0; p < PH_COUNT; ++p) {
    const int mu = (p == PH_T1 || p == PH_F1 || p == PH_B1) ? 1 : 0;
    std::vector<int> order(B->count);
    for (int i = 0; i < B->count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      return B->inst[a].N * B->inst[a].me[mu] > B->inst[b].N * B->inst[b].me[mu];
    });
    for (int c = 0; c < kClasses; ++c) {
      Phase& ph = B->ph[p][c];
      ph.members.clear();
      for (int i : order)
        if ((split && B->inst[i].me[mu] > kClassRows) == (c == 1)) ph.members.push_back(i);
    }
  }
  B->classes = split;
  B->items_valid = false;
}

// (Re)build and upload every item array for the state pointers u[0..count).  Synchronises
// the device first: an item array may still be read by work in flight.
int build_items(BatchData* B, const void* const* u) {
  HIP_TRY(hipDeviceSynchronize());
  for (auto& ph : B->ph[PH_F1]) ph.ek = B->fuse ? EpiKind::ExpEuler : EpiKind::Store;
  std::vector<MPLaunch> L;
  for (int p = 0; p < PH_COUNT; ++p)
    for (Phase& ph : B->ph[p]) {
      const int nc = (int)ph.members.size();
      if (nc == 0) continue;
      L.resize(nc);
      for (int k = 0; k < nc; ++k) L[k] = inst_launch(B, B->inst[ph.members[k]], p, ph, u[ph.members[k]]);
      const size_t bytes = group_item_bytes(ph.pk, ph.ek) * (size_t)nc;
      if (bytes == 0) return fail(FCGLE_ERR_UNSUPPORTED, "batch: no grouped kernel for phase %d", p);
      std::vector<unsigned char> host(bytes);
      ph.nblocks = group_build_f32(ph.cfg, ph.tl, ph.pk, ph.ek, L.data(), nc, host.data());
      if (ph.nblocks == 0) return fail(FCGLE_ERR_UNSUPPORTED, "batch: no grouped kernel for the items of phase %d", p);
      if (!ph.items) {
        // largest item type over the epilogue choices of this phase
        const size_t cap =
            std::max(group_item_bytes(ph.pk, EpiKind::Store), group_item_bytes(ph.pk, EpiKind::ExpEuler));
        FC_TRY(plan_alloc(&ph.items, cap * (size_t)B->count));  // any class may hold every instance
      }
      HIP_TRY(hipMemcpy(ph.items, host.data(), bytes, hipMemcpyHostToDevice));
    }
  {
    std::vector<int64_t> rows(B->count);
    std::vector<int> nl(B->count);
    std::vector<const void*> v(B->count);
    std::vector<EpiParams> ep(B->count);
    for (int i = 0; i < B->count; ++i) {
      rows[i] = B->inst[i].n[0];
      nl[i] = (int)B->inst[i].n[1];
      v[i] = B->inst[i].tmp2;
      ep[i] = update_params(B, B->inst[i]);
    }
    const size_t bytes = pw_group_item_bytes(EpiKind::ExpEuler) * (size_t)B->count;
    std::vector<unsigned char> host(bytes);
    B->pw_rows = pw_group_build_f32(EpiKind::ExpEuler, rows.data(), nl.data(), v.data(), ep.data(), B->count,
                                    host.data());
    if (!B->pw_items) FC_TRY(plan_alloc(&B->pw_items, bytes));
    HIP_TRY(hipMemcpy(B->pw_items, host.data(), bytes, hipMemcpyHostToDevice));
  }
  if (B->persist) FC_TRY(build_persist(B, u));
  B->bound.assign(u, u + B->count);
  B->items_valid = true;
  return FCGLE_OK;
}

// Description of instance I in phase p (0 F0, 1 F1, 2 B0, 3 B1) of the persistent form: forward
// products with both even/odd blocks per tile, the update fused into F1's stores.
MPLaunch persist_launch(const BatchData* B, const BatchInst& I, int p, const void* u) {
  static const int kPh[4] = {PH_F0, PH_F1, PH_B0, PH_B1};
  MPLaunch L = inst_launch(B, I, kPh[p], B->ph[kPh[p]][0], u);
  if (p < 2) L.split = kSplitFwd2;
  L.cfg = B->pcfg;
  if (p == 0) {
    L.pk = ProKind::Nonlin;
    L.ek = EpiKind::Store;
  } else if (p == 1) {
    L.pk = ProKind::Id;
    L.ek = EpiKind::ExpEuler;
    L.ep = update_params(B, I);
    L.ep.sep.mu = 1;
  } else {
    L.pk = ProKind::Id;
    L.ek = EpiKind::Store;
  }
  return L;
}

// (Re)build the persistent form's item arrays, per-instance tile prefixes and control block for
// the state pointers u[0..count) (after the caller synchronised the device).
int build_persist(BatchData* B, const void* const* u) {
  const int n = B->count;
  std::vector<uint32_t> tiles[4];
  std::vector<MPLaunch> L(n);
  uint32_t phase_tiles[4];
  for (int p = 0; p < 4; ++p) {
    for (int i = 0; i < n; ++i) L[i] = persist_launch(B, B->inst[i], p, u[i]);
    std::vector<unsigned char> host(persist_item_bytes(p) * (size_t)n);
    tiles[p].resize(n);
    phase_tiles[p] = persist_build_f32(B->pcfg, p, L.data(), n, host.data(), tiles[p].data());
    if (phase_tiles[p] == 0) return fail(FCGLE_ERR_UNSUPPORTED, "batch: no persistent kernel for configuration %d", B->pcfg);
    if (!B->p_items[p]) FC_TRY(plan_alloc(&B->p_items[p], persist_item_bytes(p) * (size_t)n));
    HIP_TRY(hipMemcpy(B->p_items[p], host.data(), host.size(), hipMemcpyHostToDevice));
  }
  B->p_phase0[0] = 0;
  for (int p = 0; p < 4; ++p) B->p_phase0[p + 1] = B->p_phase0[p] + phase_tiles[p];
  std::vector<uint32_t> pre(5 * (size_t)n);
  for (int i = 0; i < n; ++i) {
    uint32_t acc = 0;
    for (int p = 0; p < 4; ++p) {
      pre[5 * i + p] = acc;
      acc += tiles[p][i];
    }
    pre[5 * i + 4] = acc;
  }
  const size_t ctl = 256, done = (size_t)round_up((int64_t)n * 4, 256);
  if (!B->p_buf) FC_TRY(plan_alloc(&B->p_buf, ctl + done + pre.size() * 4));
  HIP_TRY(hipMemcpy((unsigned char*)B->p_buf + ctl + done, pre.data(), pre.size() * 4, hipMemcpyHostToDevice));
  B->p_grid = persist_grid(B->pcfg);
  if (B->p_grid <= 0) return fail(FCGLE_ERR_HIP, "batch: no occupancy for the persistent kernel");
  B->p_cfg_built = B->pcfg;
  return FCGLE_OK;
}

// nsteps steps in persistent launches (each resets its control block with a fill kernel and runs
// at most as many steps as 32-bit tickets allow), then a synchronisation to report a dependency
// wait that ran out of polls.
int run_persist(BatchData* B, int64_t nsteps, hipStream_t st) {
  const size_t ctl = 256;
  PersistArgs a{};
  a.ctl = (PersistCtl*)B->p_buf;
  a.done = (uint32_t*)((unsigned char*)B->p_buf + ctl);
  a.pre = (const uint32_t*)((unsigned char*)B->p_buf + ctl + (size_t)round_up((int64_t)B->count * 4, 256));
  for (int p = 0; p < 4; ++p) a.items[p] = B->p_items[p];
  for (int p = 0; p < 5; ++p) a.phase0[p] = B->p_phase0[p];
  a.count = B->count;
  a.spin_limit = B->spin_limit;
  const int64_t per = B->p_phase0[4];
  const int64_t max_steps = std::max<int64_t>(1, 0x7fffffffLL / per);
  for (int64_t left = nsteps; left > 0;) {
    const int64_t k = std::min(left, max_steps);
    a.total = (uint32_t)(k * per);
    HIP_TRY(launch_fill_u32((uint32_t*)B->p_buf, (uint32_t)((ctl + B->count * 4) / 4), st));
    HIP_TRY(launch_persist_f32(B->pcfg, a, (uint32_t)std::min<int64_t>(B->p_grid, a.total), st));
    left -= k;
  }
  PersistCtl h{};
  HIP_TRY(hipMemcpyAsync(&h, B->p_buf, sizeof(h), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (h.error) return fail(FCGLE_ERR_HIP, "batch: a dependency wait of the persistent kernel ran out of polls");
  return FCGLE_OK;
}

int launch_class(const BatchData* B, int p, int c, hipStream_t st) {
  const Phase& ph = B->ph[p][c];
  if (ph.members.empty()) return FCGLE_OK;
  const bool fwd = (p == PH_T0 || p == PH_T1 || p == PH_F0 || p == PH_F1);
  HIP_TRY(launch_group_f32(ph.cfg, ph.tl, ph.pk, ph.ek, fwd ? ph.sp : kSplitBwd, ph.items, (int)ph.members.size(),
                           ph.nblocks, st));
  return FCGLE_OK;
}

int launch_phase(const BatchData* B, int p, hipStream_t st) {
  for (int c = 0; c < kClasses; ++c) FC_TRY(launch_class(B, p, c, st));
  return FCGLE_OK;
}

int launch_step(const BatchData* B, hipStream_t st) {
  FC_TRY(launch_phase(B, PH_F0, st));
  FC_TRY(launch_phase(B, PH_F1, st));
  if (!B->fuse) HIP_TRY(launch_pw_group_f32(EpiKind::ExpEuler, B->pw_items, B->count, B->pw_rows, st));
  FC_TRY(launch_phase(B, PH_B0, st));
  FC_TRY(launch_phase(B, PH_B1, st));
  return FCGLE_OK;
}

// Graph of `steps` consecutive steps, captured on the plan's private stream on first use.
int get_graph(BatchData* B, int64_t steps, hipGraphExec_t* out) {
  for (auto& g : B->graphs)
    if (g.steps == steps) {
      *out = g.exec;
      return FCGLE_OK;
    }
  HIP_TRY(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
  int rc = FCGLE_OK;
  for (int64_t k = 0; k < steps && rc == FCGLE_OK; ++k) rc = launch_step(B, B->cap);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(B->cap, &graph);
  if (rc != FCGLE_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return fail(FCGLE_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e2 != hipSuccess) return fail(FCGLE_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e2));
  B->graphs.push_back({steps, exec});
  *out = exec;
  return FCGLE_OK;
}

constexpr int64_t kGraphChunk = 500;  // steps per captured graph (longer runs replay it)

int batch_run_impl(fcgle_plan* P, void* const* u, int64_t nsteps, hipStream_t st) {
  BatchData* B = P->batch;
  bool same = B->items_valid && (int)B->bound.size() == B->count && (!B->persist || B->p_cfg_built == B->pcfg);
  for (int i = 0; same && i < B->count; ++i) same = (B->bound[i] == u[i]);
  if (!same) FC_TRY(build_items(B, (const void* const*)u));
  if (nsteps == 0) return FCGLE_OK;
  FC_TRY(launch_phase(B, PH_T0, st));
  FC_TRY(launch_phase(B, PH_T1, st));
  if (B->persist) return run_persist(B, nsteps, st);
  int64_t left = nsteps;
  while (left > 0) {
    const int64_t k = left > kGraphChunk ? kGraphChunk : left;
    hipGraphExec_t g;
    FC_TRY(get_graph(B, k, &g));
    HIP_TRY(hipGraphLaunch(g, st));
    left -= k;
  }
  return FCGLE_OK;
}

template <class Fn>
int time_phase(hipStream_t st, hipEvent_t e0, hipEvent_t e1, int reps, Fn fn, float* ms) {
  FC_TRY(fn());
  HIP_TRY(hipEventRecord(e0, st));
  for (int r = 0; r < reps; ++r) FC_TRY(fn());
  HIP_TRY(hipEventRecord(e1, st));
  HIP_TRY(hipEventSynchronize(e1));
  float t = 0;
  HIP_TRY(hipEventElapsedTime(&t, e0, e1));
  *ms = t / reps;
  return FCGLE_OK;
}

int autotune_impl(fcgle_plan* P, int reps, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  BatchData* B = P->batch;
  // bind the phases to plan-owned buffers (tmp2 stands in for the states)
  std::vector<const void*> scratch(B->count);
  for (int i = 0; i < B->count; ++i) {
    scratch[i] = B->inst[i].tmp2;
    HIP_TRY(hipMemsetAsync(B->inst[i].tmp2, 0, (size_t)B->inst[i].N * 8, st));
    HIP_TRY(hipMemsetAsync(B->inst[i].tmp, 0, (size_t)B->inst[i].N * 8, st));
    HIP_TRY(hipMemsetAsync(B->inst[i].uhat, 0, (size_t)B->inst[i].N * 8, st));
  }
  // per phase and size class: tile configuration, and for forward phases the even/odd form
  // (two row tiles, or both blocks in one tile)
  auto tune_class = [&](int p, int c, bool forms, float* best_ms) -> int {
    Phase& ph = B->ph[p][c];
    float best = 1e30f;
    int best_c = ph.cfg, best_sp = ph.sp;
    for (int f2 = 0; f2 < (forms ? 2 : 1); ++f2)
      for (int k = 0; k < kGroupCfg; ++k) {
        ph.cfg = k;
        if (forms) ph.sp = f2 ? kSplitFwd2 : kSplitFwd;
        FC_TRY(build_items(B, scratch.data()));
        float ms;
        FC_TRY(time_phase(st, e0, e1, reps, [&] { return launch_class(B, p, c, st); }, &ms));
        if (ms < best) {
          best = ms;
          best_c = k;
          best_sp = ph.sp;
        }
      }
    ph.cfg = best_c;
    ph.sp = best_sp;
    *best_ms = best;
    return FCGLE_OK;
  };
  struct Choice {
    int cfg[PH_COUNT][kClasses], sp[PH_COUNT][kClasses];
    bool fuse;
    float step_ms;
  } choice[2];
  for (int mode = 0; mode < 2; ++mode) {
    assign_classes(B, mode == 1);
    for (auto& pc : B->ph)
      for (auto& ph : pc) {
        ph.cfg = 1;
        ph.sp = kSplitFwd;
      }
    const int order[] = {PH_F0, PH_B0, PH_B1};
    for (int p : order)
      for (int c = 0; c < kClasses; ++c) {
        if (B->ph[p][c].members.empty()) continue;
        float ms;
        FC_TRY(tune_class(p, c, p == PH_F0, &ms));
      }
    // F1: fused update (each class at its best tile and form) against Store + streaming pass
    int keep_cfg[2][kClasses], keep_sp[2][kClasses];
    float total[2] = {0.f, 0.f};
    for (int f = 0; f < 2; ++f) {
      B->fuse = (f == 0);
      for (int c = 0; c < kClasses; ++c) {
        keep_cfg[f][c] = B->ph[PH_F1][c].cfg;
        keep_sp[f][c] = B->ph[PH_F1][c].sp;
        if (B->ph[PH_F1][c].members.empty()) continue;
        float ms;
        FC_TRY(tune_class(PH_F1, c, true, &ms));
        keep_cfg[f][c] = B->ph[PH_F1][c].cfg;
        keep_sp[f][c] = B->ph[PH_F1][c].sp;
        total[f] += ms;
      }
      if (!B->fuse) {
        FC_TRY(build_items(B, scratch.data()));
        float ms;
        FC_TRY(time_phase(st, e0, e1, reps, [&]() -> int {
          HIP_TRY(launch_pw_group_f32(EpiKind::ExpEuler, B->pw_items, B->count, B->pw_rows, st));
          return (int)FCGLE_OK;
        }, &ms));
        total[f] += ms;
      }
    }
    const int bf = total[0] <= total[1] ? 0 : 1;
    B->fuse = (bf == 0);
    for (int c = 0; c < kClasses; ++c) {
      B->ph[PH_F1][c].cfg = keep_cfg[bf][c];
      B->ph[PH_F1][c].sp = keep_sp[bf][c];
      B->ph[PH_T0][c].cfg = B->ph[PH_F0][c].cfg;
      B->ph[PH_T0][c].sp = B->ph[PH_F0][c].sp;
      B->ph[PH_T1][c].cfg = B->ph[PH_B1][c].cfg;
    }
    FC_TRY(build_items(B, scratch.data()));
    float ms;
    FC_TRY(time_phase(st, e0, e1, reps, [&] { return launch_step(B, st); }, &ms));
    Choice& ch = choice[mode];
    for (int p = 0; p < PH_COUNT; ++p)
      for (int c = 0; c < kClasses; ++c) {
        ch.cfg[p][c] = B->ph[p][c].cfg;
        ch.sp[p][c] = B->ph[p][c].sp;
      }
    ch.fuse = B->fuse;
    ch.step_ms = ms;
  }
  const int best_mode = choice[1].step_ms < choice[0].step_ms ? 1 : 0;
  assign_classes(B, best_mode == 1);
  for (int p = 0; p < PH_COUNT; ++p)
    for (int c = 0; c < kClasses; ++c) {
      B->ph[p][c].cfg = choice[best_mode].cfg[p][c];
      B->ph[p][c].sp = choice[best_mode].sp[p][c];
    }
  B->fuse = choice[best_mode].fuse;
  B->items_valid = false;
  clear_graphs(B);
  return FCGLE_OK;
}

}  // namespace

int batch_autotune(fcgle_plan* P, int reps, hipStream_t st) {
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  const int rc = autotune_impl(P, reps, st, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  P->batch->tuned = (rc == FCGLE_OK);
  P->batch->items_valid = false;
  return rc;
}

int batch_describe(const fcgle_plan* P, char* buf, size_t len) {
  const BatchData* B = P->batch;
  int64_t nmin = 1 << 30, nmax = 0;
  double flop = 0;
  for (const auto& I : B->inst) {
    nmin = std::min({nmin, I.n[0], I.n[1]});
    nmax = std::max({nmax, I.n[0], I.n[1]});
    for (int m = 0; m < 2; ++m)
      flop += 2.0 * 4.0 * (double)(I.me[m] * I.me[m] + I.mo[m] * I.mo[m]) * (double)I.N / (double)I.n[m];
  }
  static const char* names[] = {"t0", "t1", "f0", "f1", "b0", "b1"};
  std::string s = "batch count=" + std::to_string(B->count) + " n in [" + std::to_string(nmin) + "," +
                  std::to_string(nmax) + "] precision=fp32 structure=even-odd tiles(rows)=";
  for (int p = 0; p < PH_COUNT; ++p) {
    s += std::string(names[p]) + ":";
    bool first = true;
    for (int c = 0; c < kClasses; ++c) {
      const Phase& ph = B->ph[p][c];
      if (ph.members.empty()) continue;
      s += std::string(first ? "" : "|") + std::to_string(group_cfg_rows(ph.cfg)) + (ph.sp == kSplitFwd2 ? "F" : "");
      first = false;
    }
    s += (p + 1 < PH_COUNT ? "," : "");
  }
  if (B->classes) {
    int nl = 0;
    for (const auto& I : B->inst) nl += I.me[0] > kClassRows;
    s += " classes(m_e<=" + std::to_string(kClassRows) + "|larger, axis 0)=" + std::to_string(B->count - nl) + "|" +
         std::to_string(nl);
  } else {
    s += " classes=one";
  }
  s += std::string(" update=") + (B->fuse ? "fused" : "streaming");
  if (B->persist) s += " form=persistent(" + std::to_string(group_cfg_rows(B->pcfg)) + "-row tiles)";
  else s += " form=graph-of-grouped-launches";
  char tail[96];
  std::snprintf(tail, sizeof(tail), " flop/step=%.4g%s", flop, B->tuned ? " tuned" : " default");
  s += tail;
  std::snprintf(buf, len, "%s", s.c_str());
  return FCGLE_OK;
}

}  // namespace fcgle

using namespace fcgle;

extern "C" {

int fcgle_batch_setup(int count, const int64_t* n, const double* alpha, const double* h, const fcgle_params* params,
                      int precision, double tau, fcgle_plan** out) {
  if (!out) return fail(FCGLE_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (count < 1 || count > 65535) return fail(FCGLE_ERR_ARG, "batch: count = %d outside 1..65535", count);
  if (!n || !alpha || !h || !params) return fail(FCGLE_ERR_ARG, "batch: NULL argument");
  if (precision != FCGLE_FP32) return fail(FCGLE_ERR_UNSUPPORTED, "batch: only FCGLE_FP32 plans are built");
  if (!(tau > 0.0) || !std::isfinite(tau)) return fail(FCGLE_ERR_ARG, "tau must be > 0");
  for (int i = 0; i < count; ++i) {
    const fcgle_params& p = params[i];
    if (!(std::isfinite(p.nu) && std::isfinite(p.eta) && std::isfinite(p.gamma) && std::isfinite(p.kappa) &&
          std::isfinite(p.zeta)))
      return fail(FCGLE_ERR_ARG, "batch: non-finite parameter in instance %d", i);
    if (p.nu < 0.0 || p.kappa < 0.0) return fail(FCGLE_ERR_ARG, "batch: nu and kappa must be >= 0 (instance %d)", i);
    for (int m = 0; m < 2; ++m) {
      if (n[2 * i + m] < 2 || n[2 * i + m] > 4096)
        return fail(FCGLE_ERR_ARG, "batch: n[%d] = %lld outside 2..4096", 2 * i + m, (long long)n[2 * i + m]);
      if (!(alpha[2 * i + m] > 1.0 && alpha[2 * i + m] <= 2.0))
        return fail(FCGLE_ERR_ARG, "batch: alpha[%d] outside (1, 2]", 2 * i + m);
      if (!(h[2 * i + m] > 0.0) || !std::isfinite(h[2 * i + m]))
        return fail(FCGLE_ERR_ARG, "batch: h[%d] must be > 0", 2 * i + m);
    }
  }
  auto* P = new (std::nothrow) fcgle_plan();
  auto* B = new (std::nothrow) BatchData();
  if (!P || !B) {
    delete P;
    delete B;
    return fail(FCGLE_ERR_NOMEM, "host allocation failed");
  }
  P->batch = B;
  P->prec = FCGLE_FP32;
  P->elem = 8;
  P->tau = tau;
  P->d = 2;
  B->count = count;
  B->tau = tau;
  B->inst.resize(count);
  auto cleanup = [&](int rc) {
    (void)hipDeviceSynchronize();
    batch_free(B);
    P->batch = nullptr;
    delete P;
    return rc;
  };
  hipError_t e = hipGetDevice(&P->device);
  if (e != hipSuccess) return cleanup(fail(FCGLE_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e)));
  for (int i = 0; i < count; ++i) {
    BatchInst& I = B->inst[i];
    I.p = params[i];
    for (int m = 0; m < 2; ++m) {
      I.n[m] = n[2 * i + m];
      I.alpha[m] = alpha[2 * i + m];
      I.h[m] = h[2 * i + m];
      I.me[m] = (int)(I.n[m] - I.n[m] / 2);
      I.mo[m] = (int)(I.n[m] / 2);
      I.npad[m] = (int)round_up(I.me[m], 128);
    }
    I.N = I.n[0] * I.n[1];
  }
  // FP64 eigendecompositions on the host, spread over the host threads
  {
    const int jobs = 2 * count;
    std::vector<int> ok(jobs, 0);
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (unsigned w = 0; w < hw; ++w)
      th.emplace_back([&, w] {
        for (int j = (int)w; j < jobs; j += (int)hw) {
          BatchInst& I = B->inst[j / 2];
          const int m = j % 2;
          SplitEig se;
          ok[j] = toeplitz_eig_split(I.n[m], I.alpha[m], I.h[m], 2, se);
          if (ok[j]) {
            I.Q[m].swap(se.Q);
            I.lam[m].swap(se.lam);
          }
        }
      });
    for (auto& t : th) t.join();
    for (int j = 0; j < jobs; ++j)
      if (!ok[j]) return cleanup(fail(FCGLE_ERR_ARG, "batch: eigensolver did not converge (instance %d)", j / 2));
  }
  // one device pool for every per-instance buffer
  auto al = [](size_t b) { return (size_t)round_up((int64_t)b, 256); };
  size_t total = 0;
  for (const auto& I : B->inst) {
    for (int m = 0; m < 2; ++m)
      total += 2 * al((size_t)2 * I.npad[m] * I.npad[m] * sizeof(float)) + al(I.n[m] * sizeof(double)) +
               al(2 * I.n[m] * sizeof(double));
    total += 4 * al((size_t)I.N * 8);
  }
  if (plan_alloc(&B->pool, total) != FCGLE_OK) return cleanup(FCGLE_ERR_NOMEM);
  {
    unsigned char* base = (unsigned char*)B->pool;
    size_t off = 0;
    auto take = [&](size_t b) {
      void* p = base + off;
      off += al(b);
      return p;
    };
    for (auto& I : B->inst) {
      for (int m = 0; m < 2; ++m) {
        const size_t mb = (size_t)2 * I.npad[m] * I.npad[m] * sizeof(float);
        I.Mf[m] = (float*)take(mb);
        I.Mb[m] = (float*)take(mb);
        I.dlam[m] = (double*)take(I.n[m] * sizeof(double));
        I.fac[m] = (double*)take(2 * I.n[m] * sizeof(double));
      }
      I.P1 = (float2*)take((size_t)I.N * 8);
      I.uhat = (float2*)take((size_t)I.N * 8);
      I.tmp = (float2*)take((size_t)I.N * 8);
      I.tmp2 = (float2*)take((size_t)I.N * 8);
    }
  }
  // uploads: the even/odd block matrices (FP32), eigenvalues, separable exponential factors
  for (int i = 0; i < count; ++i) {
    BatchInst& I = B->inst[i];
    for (int m = 0; m < 2; ++m) {
      const int64_t nm = I.n[m];
      std::vector<double> Fd, Bd;
      split_block_matrices(nm, I.me[m], I.mo[m], I.Q[m], I.npad[m], Fd, Bd);
      const std::vector<float> qt(Fd.begin(), Fd.end()), q(Bd.begin(), Bd.end());
      std::vector<double> fac(2 * nm);
      for (int64_t j = 0; j < nm; ++j) {
        const zc z = fz_eval(1, zc{tau * I.p.nu * I.lam[m][j], tau * I.p.eta * I.lam[m][j]});
        fac[2 * j] = z.re;
        fac[2 * j + 1] = z.im;
      }
      e = hipMemcpy(I.Mf[m], qt.data(), qt.size() * sizeof(float), hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(I.Mb[m], q.data(), q.size() * sizeof(float), hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(I.dlam[m], I.lam[m].data(), nm * sizeof(double), hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(I.fac[m], fac.data(), fac.size() * sizeof(double), hipMemcpyHostToDevice);
      if (e != hipSuccess) return cleanup(fail(FCGLE_ERR_HIP, "batch upload: %s", hipGetErrorString(e)));
    }
    SepParams s;
    s.d = 2;
    s.n[0] = (int)I.n[0];
    s.n[1] = (int)I.n[1];
    s.lam[0] = I.dlam[0];
    s.lam[1] = I.dlam[1];
    e = launch_fgrid(P_F32, FCGLE_PHI1, tau * I.p.nu, tau * I.p.eta, s, I.N, I.P1, nullptr);
    if (e != hipSuccess) return cleanup(fail(FCGLE_ERR_HIP, "batch f-grid: %s", hipGetErrorString(e)));
  }
  e = hipDeviceSynchronize();
  if (e != hipSuccess) return cleanup(fail(FCGLE_ERR_HIP, "batch setup: %s", hipGetErrorString(e)));
  e = hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking);
  if (e != hipSuccess) return cleanup(fail(FCGLE_ERR_HIP, "hipStreamCreate: %s", hipGetErrorString(e)));
  // phase kinds, default tiles (128-row tiles suit the 96..512 sizes), one class per phase
  for (int p = 0; p < PH_COUNT; ++p)
    for (int c = 0; c < kClasses; ++c) {
      Phase& ph = B->ph[p][c];
      ph.cfg = 1;
      ph.tl = (p == PH_T1 || p == PH_F1 || p == PH_B1);
      ph.pk = (p == PH_F0) ? ProKind::Nonlin : ProKind::Id;
      ph.ek = (p == PH_F1) ? EpiKind::ExpEuler : EpiKind::Store;
    }
  assign_classes(B, false);
  B->fuse = true;
  *out = P;
  return FCGLE_OK;
}

int fcgle_batch_set_persistent(fcgle_plan* plan, int mode, int64_t spin_limit) {
  if (!plan || !plan->batch) return fail(FCGLE_ERR_ARG, "fcgle_batch_set_persistent needs a batch plan");
  if (mode != 0 && mode != 1) return fail(FCGLE_ERR_ARG, "mode must be 0 or 1");
  if (spin_limit < 0 || spin_limit > 0xffffffffLL) return fail(FCGLE_ERR_ARG, "spin_limit outside 0..2^32-1");
  BatchData* B = plan->batch;
  if (mode == 1)
    return fail(FCGLE_ERR_UNSUPPORTED, "batch: the persistent form is switched off (its first GPU runs did not "
                "finish; the cause is not established)");
  B->persist = false;
  if (spin_limit > 0) B->spin_limit = (uint32_t)spin_limit;
  B->items_valid = false;
  return FCGLE_OK;
}

int fcgle_batch_run(fcgle_plan* plan, int scheme, void* const* u_dev, double t0, double tau, int64_t nsteps,
                    void* stream) {
  if (!plan) return fail(FCGLE_ERR_ARG, "plan is NULL");
  if (!plan->batch) return fail(FCGLE_ERR_ARG, "fcgle_batch_run needs a plan made by fcgle_batch_setup");
  if (scheme != FCGLE_EXP_EULER) return fail(FCGLE_ERR_UNSUPPORTED, "batch: only FCGLE_EXP_EULER is built");
  if (tau != plan->tau) return fail(FCGLE_ERR_ARG, "tau %.17g differs from the plan's %.17g", tau, plan->tau);
  if (!std::isfinite(t0)) return fail(FCGLE_ERR_ARG, "t0 not finite");
  if (nsteps < 0) return fail(FCGLE_ERR_ARG, "nsteps < 0");
  if (!u_dev) return fail(FCGLE_ERR_ARG, "u_dev is NULL");
  for (int i = 0; i < plan->batch->count; ++i)
    if (!u_dev[i]) return fail(FCGLE_ERR_ARG, "u_dev[%d] is NULL", i);
  DeviceGuard g(plan->device);
  return batch_run_impl(plan, u_dev, nsteps, as_stream(stream));
}

}  // extern "C"
