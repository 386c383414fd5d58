// hevi_group_api.cpp -- groups of column batches advanced by one LHEVI ARK step
// per call (see hevi_group_* in include/hevi.h): launch plans, HIP-graph
// capture and the autotuner.  The arithmetic runs in hevi_group.hip (persistent
// multi-problem kernels) or, for the per-member plan, in the single-problem
// kernels of hevi_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "hevi.h"
#include "hevi_internal.h"
#include "hevi_objects.h"

using namespace hevi_host;

namespace {

struct Launch {
  int nlo, nhi;      // orders the kernel is compiled for
  int member;        // per-member plan: the member; else -1
  int32_t m;         // segments
  int64_t total;     // items
  size_t off;        // offset of plist (int32 x m, padded) + pstart (int64 x m+1) in d_sched
  int maxnz;         // largest n_z of the launch's members
  int tilt;          // some member's columns are not straight
};

}  // namespace

struct hevi_group {
  hevi_ctx* ctx = nullptr;
  int n = 0, s = 0;
  double dt = 0.0, lambda = 0.0;
  double Aexp[HEVI_MAX_STAGES * HEVI_MAX_STAGES] = {};
  double Aimp[HEVI_MAX_STAGES * HEVI_MAX_STAGES] = {};
  double b[HEVI_MAX_STAGES] = {};
  hevi_precision prec = HEVI_FP64;
  int sweeps = 4;
  double target = 1e-13;
  std::vector<hevi_group_member> mem;
  std::vector<hevi_factors*> fac;
  std::vector<HeviProbDev> probs;
  std::vector<HeviCallDev> calls;  // slot-major: calls[slot * n + member]
  HeviProbDev* d_probs = nullptr;
  HeviCallDev* d_calls = nullptr;
  HeviDevInfo* d_info = nullptr;
  uint32_t* d_ctr = nullptr;
  hevi_group_plan plan = {HEVI_LAUNCH_ONE, 0, 0};
  std::vector<Launch> launches;
  std::vector<Launch> factor_launches;  // per order, whatever the plan (not per-member)
  char* d_sched = nullptr;
  hipStream_t cap = nullptr;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
};

namespace {

// call slots: apply of stage i (i = 0..s-1), stage solve i (i = 1..s-1), combine
int slot_apply(const hevi_group* g, int i) { return i; }
int slot_stage(const hevi_group* g, int i) { return g->s + i - 1; }
int slot_combine(const hevi_group* g) { return 2 * g->s - 1; }

void drop_graphs(hevi_group* g) {
  for (auto& e : g->graph) {
    if (e) (void)hipGraphExecDestroy(e);
    e = nullptr;
  }
}

// relative cost of one tile: nodes x nodes per element
double tile_cost(const HeviShapeDev& sh) { return (double)sh.nz * (sh.N + 1); }

// (re)build the launch list of the current plan; the previous schedule buffer
// may still be read by queued work, so the device is drained first
hevi_status build_launches(hevi_group* g) {
  if (!ok(hipDeviceSynchronize())) return HEVI_E_DEVICE;
  std::vector<Launch> L, FL;
  std::vector<char> host;
  auto add_to = [&](std::vector<Launch>& out, int nlo, int nhi, std::vector<int> ids) {
    std::stable_sort(ids.begin(), ids.end(), [&](int a, int b) {
      return tile_cost(g->probs[a].sh) > tile_cost(g->probs[b].sh);
    });
    std::vector<int32_t> pl;
    std::vector<int64_t> ps{0};
    int maxnz = 1, tilt = 0;
    for (int p : ids) {
      if (g->probs[p].sh.ntiles == 0) continue;
      pl.push_back(p);
      ps.push_back(ps.back() + g->probs[p].sh.ntiles);
      maxnz = std::max(maxnz, g->probs[p].sh.nz);
      tilt |= g->probs[p].tilt;
    }
    if (pl.empty()) return;
    Launch l{nlo, nhi, -1, (int32_t)pl.size(), ps.back(), host.size(), maxnz, tilt};
    const size_t a = pl.size() * sizeof(int32_t), pad = (a + 7) / 8 * 8;
    host.resize(host.size() + pad + ps.size() * sizeof(int64_t));
    std::memcpy(host.data() + l.off, pl.data(), a);
    std::memcpy(host.data() + l.off + pad, ps.data(), ps.size() * sizeof(int64_t));
    out.push_back(l);
  };
  auto add = [&](int nlo, int nhi, std::vector<int> ids) { add_to(L, nlo, nhi, ids); };
  auto per_order = [&](std::vector<Launch>& out) {
    for (int N = HEVI_MAXN; N >= 1; --N) {
      std::vector<int> ids;
      for (int i = 0; i < g->n; ++i)
        if (g->probs[i].sh.N == N) ids.push_back(i);
      if (!ids.empty()) add_to(out, N, N, ids);
    }
  };
  if (g->plan.mode == HEVI_LAUNCH_ONE) {
    std::vector<int> all(g->n);
    for (int i = 0; i < g->n; ++i) all[i] = i;
    add(1, HEVI_MAXN, all);
  } else if (g->plan.mode == HEVI_LAUNCH_PER_ORDER) {
    per_order(L);
  } else {
    for (int i = 0; i < g->n; ++i)
      if (g->probs[i].sh.ntiles > 0)
        L.push_back(Launch{0, 0, i, 0, 0, 0, g->probs[i].sh.nz, g->probs[i].tilt});
  }
  // the factorisation runs per order in every multi-problem plan: one pass for the
  // orders up to HEVI_FUSED_FACTOR_MAX_N, and no kernel compiled for every order
  // (whose LU would need the registers of the largest)
  if (g->plan.mode != HEVI_LAUNCH_PER_MEMBER) per_order(FL);
  if (g->d_sched) (void)hipFree(g->d_sched);
  g->d_sched = nullptr;
  if (!host.empty()) {
    hevi_status s = dev_alloc(&g->d_sched, host.size());
    if (s) return s;
    if (!ok(hipMemcpy(g->d_sched, host.data(), host.size(), hipMemcpyHostToDevice)))
      return HEVI_E_DEVICE;
  }
  g->launches = L;
  g->factor_launches = FL;
  return HEVI_OK;
}

// One persistent multi-problem launch of phase ph over the members of l.
hipError_t multi(hevi_group* g, const Launch& l, int ph, int slot, hipStream_t st) {
  const int fp32 = g->prec == HEVI_FP32_REFINE;
  HeviSched s;
  const size_t pad = ((size_t)l.m * sizeof(int32_t) + 7) / 8 * 8;
  s.plist = (const int32_t*)(g->d_sched + l.off);
  s.pstart = (const int64_t*)(g->d_sched + l.off + pad);
  s.m = l.m;
  s.total = l.total;
  s.ctr = g->d_ctr;
  const int64_t want = g->plan.grid > 0 ? g->plan.grid : l.total;
  const int grid = (int)std::min<int64_t>(want, l.total);
  return hevi_launch_multi(ph, l.nlo, l.nhi, fp32, l.tilt, g->d_probs,
                           slot >= 0 ? g->d_calls + (size_t)slot * g->n : nullptr, s, grid,
                           fp32 ? g->sweeps : 0, g->target, l.maxnz, st);
}

hipError_t phase(hevi_group* g, int ph, int slot, hipStream_t st) {
  const int fp32 = g->prec == HEVI_FP32_REFINE;
  for (const Launch& l : g->launches) {
    hipError_t e = hipSuccess;
    if (l.member >= 0) {
      // per-member plan: the single-problem kernels
      const int p = l.member;
      const HeviProbDev& P = g->probs[p];
      const HeviCallDev* C = slot >= 0 ? &g->calls[(size_t)slot * g->n + p] : nullptr;
      switch (ph) {
        case HEVI_PH_APPLY:
          e = hevi_launch_apply(P.sh, 0, P.ops, C->x, C->xref, C->out, st);
          break;
        case HEVI_PH_FACTOR_ASSEMBLE:
          e = hevi_launch_factor(P.sh, 0, P.lambda, fp32, P.ops, P.sbuf, P.U, P.L, P.piv,
                                 P.info, st);
          break;
        case HEVI_PH_STAGE_RHS:
          e = hevi_launch_stage_solve(P.sh, 0, P.lambda, P.tilt, fp32, P.ops, P.U, P.L, P.piv, P.ws,
                                      C->E, C->Q, C->out, fp32 ? g->sweeps : 0, g->target, 0,
                                      P.info, st);
          break;
        case HEVI_PH_COMBINE:
          e = hevi_launch_combine(5 * (int64_t)P.sh.nz * P.sh.ncols, C->E, C->out, st);
          break;
        default:  // factor LU, bsolve and update run inside the calls above
          break;
      }
    } else {
      // FP64 stage solves of single-order launches whose columns fit the fused
      // kernel's LDS run as one fused pass; their band-solve and update phases are
      // then already done.  (A fused kernel over every order would need the
      // registers of the largest and spill.)
      const bool fused = !fp32 && l.nlo == l.nhi && l.maxnz <= HEVI_FUSED_MAX_NZ;
      if (fused && (ph == HEVI_PH_STAGE_BSOLVE || ph == HEVI_PH_STAGE_UPDATE)) continue;
      const int phx = (fused && ph == HEVI_PH_STAGE_RHS) ? HEVI_PH_STAGE_FUSED : ph;
      e = multi(g, l, phx, slot, st);
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// The factorisation of every member: per member in the per-member plan, else one
// launch per order (one pass up to HEVI_FUSED_FACTOR_MAX_N, assembly + LU above).
hipError_t factor(hevi_group* g, hipStream_t st) {
  if (g->plan.mode == HEVI_LAUNCH_PER_MEMBER) return phase(g, HEVI_PH_FACTOR_ASSEMBLE, -1, st);
  for (const Launch& l : g->factor_launches) {
    hipError_t e;
    if (l.nlo <= HEVI_FUSED_FACTOR_MAX_N) {
      e = multi(g, l, HEVI_PH_FACTOR_FUSED, -1, st);
    } else {
      e = multi(g, l, HEVI_PH_FACTOR_ASSEMBLE, -1, st);
      if (e == hipSuccess) e = multi(g, l, HEVI_PH_FACTOR_LU, -1, st);
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t enqueue_step(hevi_group* g, int refactor, hipStream_t st) {
  hipError_t e;
  if (refactor && (e = factor(g, st)) != hipSuccess) return e;
  if ((e = phase(g, HEVI_PH_APPLY, slot_apply(g, 0), st)) != hipSuccess) return e;
  for (int i = 1; i < g->s; ++i) {
    if ((e = phase(g, HEVI_PH_STAGE_RHS, slot_stage(g, i), st)) != hipSuccess) return e;
    if ((e = phase(g, HEVI_PH_STAGE_BSOLVE, slot_stage(g, i), st)) != hipSuccess) return e;
    if ((e = phase(g, HEVI_PH_STAGE_UPDATE, slot_stage(g, i), st)) != hipSuccess) return e;
    if ((e = phase(g, HEVI_PH_APPLY, slot_apply(g, i), st)) != hipSuccess) return e;
  }
  return phase(g, HEVI_PH_COMBINE, slot_combine(g), st);
}

bool valid_plan(const hevi_group_plan* p) {
  return p && p->mode >= HEVI_LAUNCH_ONE && p->mode <= HEVI_LAUNCH_PER_MEMBER && p->grid >= 0 &&
         (p->use_graph == 0 || p->use_graph == 1);
}

}  // namespace

extern "C" {

hevi_status hevi_group_create(hevi_ctx* ctx, int32_t n, const hevi_group_member* members,
                              const char* tableau, double dt, hevi_precision prec,
                              const hevi_refine* refine, hevi_group** out, hipStream_t stream) {
  if (!ctx || !out || !members || !tableau) return HEVI_E_INVALID;
  *out = nullptr;
  if (n < 1 || n > (1 << 20)) return HEVI_E_INVALID;
  if (!(dt > 0.0) || !std::isfinite(dt)) return HEVI_E_INVALID;
  if (prec != HEVI_FP64 && prec != HEVI_FP32_REFINE) return HEVI_E_INVALID;
  int32_t s = 0;
  double Ae[64], Ai[64], bb[8];
  if (hevi_tableau(tableau, &s, Ae, Ai, bb) != HEVI_OK) return HEVI_E_INVALID;
  if (s < 2 || s > HEVI_MAX_STAGES) return HEVI_E_INVALID;
  for (int i = 2; i < s; ++i)  // one factorisation serves every stage: constant a~_ii
    if (Ai[i * s + i] != Ai[1 * s + 1]) return HEVI_E_INVALID;
  int sweeps = 4;
  double target = 1e-13;
  if (refine) {
    if (refine->max_sweeps < 0 || refine->max_sweeps > 64 || !(refine->rel_residual_target >= 0) ||
        refine->full_sweeps != 0)
      return HEVI_E_INVALID;
    sweeps = refine->max_sweeps;
    target = refine->rel_residual_target;
  }
  for (int p = 0; p < n; ++p) {
    const hevi_group_member& m = members[p];
    if (!m.ops || m.ops->ctx->device != ctx->device) return HEVI_E_INVALID;
    if (m.ops->s3 || m.ops->ps) return HEVI_E_INVALID;  // the group kernels: set 2C at rest
    if (m.ops->sh.ncols == 0) continue;
    std::vector<const void*> outs{m.d_out};
    for (int i = 1; i < s; ++i) outs.push_back(m.d_Q[i]);
    for (int i = 0; i < s; ++i) outs.push_back(m.d_S[i]);
    if (!m.d_qn || !m.d_qref) return HEVI_E_INVALID;
    for (size_t a = 0; a < outs.size(); ++a) {
      if (!outs[a] || outs[a] == m.d_qn || outs[a] == m.d_qref) return HEVI_E_INVALID;
      for (size_t c = a + 1; c < outs.size(); ++c)
        if (outs[a] == outs[c]) return HEVI_E_INVALID;
    }
  }
  if (!ok(hipSetDevice(ctx->device))) return HEVI_E_DEVICE;
  hevi_group* g = new (std::nothrow) hevi_group;
  if (!g) return HEVI_E_NOMEM;
  g->ctx = ctx;
  g->n = n;
  g->s = s;
  g->dt = dt;
  g->prec = prec;
  g->sweeps = prec == HEVI_FP64 ? 0 : sweeps;
  g->target = target;
  for (int i = 0; i < s * s; ++i) {
    g->Aexp[i] = Ae[i];
    g->Aimp[i] = Ai[i];
  }
  for (int i = 0; i < s; ++i) g->b[i] = bb[i];
  g->lambda = Ai[1 * s + 1] * dt;
  g->mem.assign(members, members + n);
  hevi_status st;
  auto fail = [&](hevi_status e) {
    hevi_group_free(g);
    return e;
  };
  if ((st = dev_alloc(&g->d_info, sizeof(HeviDevInfo) * n)) ||
      (st = dev_alloc(&g->d_ctr, 2 * sizeof(uint32_t))))
    return fail(st);
  if (!ok(hipMemset(g->d_ctr, 0, 2 * sizeof(uint32_t))) ||
      !ok(hevi_launch_info_reset_n(g->d_info, n, stream)))
    return fail(HEVI_E_DEVICE);
  g->fac.assign(n, nullptr);
  g->probs.resize(n);
  for (int p = 0; p < n; ++p) {
    if ((st = hevi_factor(ctx, members[p].ops, g->lambda, prec, &g->fac[p], stream)))
      return fail(st);
    const hevi_ops* o = members[p].ops;
    const hevi_factors* f = g->fac[p];
    HeviProbDev& P = g->probs[p];
    std::memset(&P, 0, sizeof(P));
    P.sh = o->sh;
    P.fp32 = prec == HEVI_FP32_REFINE;
    P.tilt = o->tilted;
    P.lambda = g->lambda;
    P.ops = o->d_ops;
    P.sbuf = f->sbuf;
    P.U = f->U;
    P.L = f->L;
    P.piv = f->piv;
    P.ws = f->ws;
    P.info = g->d_info + p;
  }
  // operands of every call of the step, per member
  g->calls.assign((size_t)2 * s * n, HeviCallDev{});
  for (int p = 0; p < n; ++p) {
    const hevi_group_member& m = members[p];
    const bool empty = m.ops->sh.ncols == 0;
    auto Qv = [&](int j) -> const double* { return j == 0 ? m.d_qn : m.d_Q[j]; };
    for (int i = 0; i < s; ++i) {  // S_i = L (Q_i - q_ref)
      HeviCallDev& C = g->calls[(size_t)slot_apply(g, i) * n + p];
      C.x = Qv(i);
      C.xref = m.d_qref;
      C.out = m.d_S[i];
    }
    for (int i = 1; i < s; ++i) {
      HeviCallDev& C = g->calls[(size_t)slot_stage(g, i) * n + p];
      const double* ev[HEVI_MAXTERMS];
      double ec[HEVI_MAXTERMS];
      const double* qv[HEVI_MAXTERMS];
      double qc[HEVI_MAXTERMS];
      ev[0] = m.d_qn;
      ec[0] = 1.0;
      for (int j = 0; j < i; ++j) {
        ev[j + 1] = m.d_S[j];
        ec[j + 1] = dt * Ae[i * s + j];
        qv[j] = Qv(j);
        qc[j] = (Ai[i * s + j] - Ae[i * s + j]) / Ai[i * s + i];
      }
      if ((st = terms(i + 1, ev, ec, 1, empty, &C.E)) || (st = terms(i, qv, qc, 0, empty, &C.Q)))
        return fail(st);
      C.out = m.d_Q[i];
    }
    {
      HeviCallDev& C = g->calls[(size_t)slot_combine(g) * n + p];
      const double* v[HEVI_MAXTERMS];
      double c[HEVI_MAXTERMS];
      v[0] = m.d_qn;
      c[0] = 1.0;
      for (int i = 0; i < s; ++i) {
        v[i + 1] = m.d_S[i];
        c[i + 1] = dt * bb[i];
      }
      if ((st = terms(s + 1, v, c, 1, empty, &C.E))) return fail(st);
      C.out = m.d_out;
    }
  }
  if ((st = dev_alloc(&g->d_probs, sizeof(HeviProbDev) * n)) ||
      (st = dev_alloc(&g->d_calls, sizeof(HeviCallDev) * g->calls.size())))
    return fail(st);
  if (!ok(hipMemcpy(g->d_probs, g->probs.data(), sizeof(HeviProbDev) * n,
                    hipMemcpyHostToDevice)) ||
      !ok(hipMemcpy(g->d_calls, g->calls.data(), sizeof(HeviCallDev) * g->calls.size(),
                    hipMemcpyHostToDevice)))
    return fail(HEVI_E_DEVICE);
  if (!ok(hipStreamCreate(&g->cap))) return fail(HEVI_E_DEVICE);
  if ((st = build_launches(g))) return fail(st);
  *out = g;
  return HEVI_OK;
}

hevi_status hevi_group_set_plan(hevi_ctx* ctx, hevi_group* g, const hevi_group_plan* plan) {
  if (!ctx || !g || !valid_plan(plan)) return HEVI_E_INVALID;
  if (!ok(hipSetDevice(ctx->device))) return HEVI_E_DEVICE;
  const bool relaunch = plan->mode != g->plan.mode;
  if (!ok(hipDeviceSynchronize())) return HEVI_E_DEVICE;  // graphs may be in flight
  drop_graphs(g);
  g->plan = *plan;
  if (relaunch) return build_launches(g);
  return HEVI_OK;
}

hevi_status hevi_group_get_plan(const hevi_group* g, hevi_group_plan* plan) {
  if (!g || !plan) return HEVI_E_INVALID;
  *plan = g->plan;
  return HEVI_OK;
}

hevi_status hevi_group_step(hevi_ctx* ctx, hevi_group* g, int32_t refactor, hipStream_t stream) {
  if (!ctx || !g) return HEVI_E_INVALID;
  if (!ok(hipSetDevice(ctx->device))) return HEVI_E_DEVICE;
  const int r = refactor ? 1 : 0;
  if (!g->plan.use_graph) return ok(enqueue_step(g, r, stream)) ? HEVI_OK : HEVI_E_DEVICE;
  if (!g->graph[r]) {
    hipGraph_t graph = nullptr;
    if (!ok(hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal)))
      return HEVI_E_DEVICE;
    const hipError_t e = enqueue_step(g, r, g->cap);
    const hipError_t e2 = hipStreamEndCapture(g->cap, &graph);
    if (e != hipSuccess || e2 != hipSuccess || !graph) {
      if (graph) (void)hipGraphDestroy(graph);
      return HEVI_E_DEVICE;
    }
    const hipError_t e3 = hipGraphInstantiate(&g->graph[r], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) {
      g->graph[r] = nullptr;
      return HEVI_E_DEVICE;
    }
  }
  return ok(hipGraphLaunch(g->graph[r], stream)) ? HEVI_OK : HEVI_E_DEVICE;
}

hevi_status hevi_group_check(hevi_ctx* ctx, hevi_group* g, hevi_info* h_infos,
                             hipStream_t stream) {
  if (!ctx || !g || !h_infos) return HEVI_E_INVALID;
  if (!ok(hipSetDevice(ctx->device))) return HEVI_E_DEVICE;
  std::vector<HeviDevInfo> h(g->n);
  if (!ok(hipMemcpyAsync(h.data(), g->d_info, sizeof(HeviDevInfo) * g->n, hipMemcpyDeviceToHost,
                         stream)) ||
      !ok(hipStreamSynchronize(stream)) || !ok(hevi_launch_info_reset_n(g->d_info, g->n, stream)))
    return HEVI_E_DEVICE;
  int worst = 0;
  for (int p = 0; p < g->n; ++p) {
    info_to_host(h[p], &h_infos[p]);
    worst = std::max(worst, (int)h[p].status);
  }
  return (hevi_status)worst;
}

hevi_status hevi_group_autotune(hevi_ctx* ctx, hevi_group* g, int32_t reps,
                                hevi_tune_result* results, int32_t cap, int32_t* n_results,
                                hipStream_t stream) {
  if (!ctx || !g || reps < 1 || cap < 0 || (cap > 0 && !results)) return HEVI_E_INVALID;
  if (!ok(hipSetDevice(ctx->device))) return HEVI_E_DEVICE;
  std::vector<hevi_group_plan> cands;
  for (int graph = 0; graph <= 1; ++graph) {
    for (int mode : {HEVI_LAUNCH_ONE, HEVI_LAUNCH_PER_ORDER})
      for (int grid : {0, 1024, 2048, 4096}) cands.push_back({mode, grid, graph});
    cands.push_back({HEVI_LAUNCH_PER_MEMBER, 0, graph});
  }
  hipEvent_t e0, e1;
  if (!ok(hipEventCreate(&e0))) return HEVI_E_DEVICE;
  if (!ok(hipEventCreate(&e1))) {
    (void)hipEventDestroy(e0);
    return HEVI_E_DEVICE;
  }
  const hevi_group_plan keep = g->plan;
  hevi_group_plan best = keep;
  double best_ms = INFINITY;
  int nr = 0;
  hevi_status st = HEVI_OK;
  for (const hevi_group_plan& c : cands) {
    if ((st = hevi_group_set_plan(ctx, g, &c))) break;
    if ((st = hevi_group_step(ctx, g, 1, stream))) break;
    if (!ok(hipEventRecord(e0, stream))) { st = HEVI_E_DEVICE; break; }
    for (int r = 0; r < reps && !st; ++r) st = hevi_group_step(ctx, g, 1, stream);
    if (st) break;
    float ms = 0.f;
    if (!ok(hipEventRecord(e1, stream)) || !ok(hipEventSynchronize(e1)) ||
        !ok(hipEventElapsedTime(&ms, e0, e1))) {
      st = HEVI_E_DEVICE;
      break;
    }
    const double per = ms / reps;
    if (nr < cap) results[nr] = hevi_tune_result{c, per};
    ++nr;
    if (per < best_ms) {
      best_ms = per;
      best = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (n_results) *n_results = nr;
  const hevi_status s2 = hevi_group_set_plan(ctx, g, st ? &keep : &best);
  return st ? st : s2;
}

void hevi_group_free(hevi_group* g) {
  if (!g) return;
  (void)hipDeviceSynchronize();
  drop_graphs(g);
  if (g->cap) (void)hipStreamDestroy(g->cap);
  for (hevi_factors* f : g->fac) hevi_factors_free(f);
  if (g->d_probs) (void)hipFree(g->d_probs);
  if (g->d_calls) (void)hipFree(g->d_calls);
  if (g->d_info) (void)hipFree(g->d_info);
  if (g->d_ctr) (void)hipFree(g->d_ctr);
  if (g->d_sched) (void)hipFree(g->d_sched);
  delete g;
}

}  // extern "C"
