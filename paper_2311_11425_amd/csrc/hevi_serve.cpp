// hevi_serve.cpp -- continuous-batching server of LHEVI stage solves over
// resident factors (see hevi_serve_* in include/hevi.h).
//
// One worker thread per server owns a HIP stream.  It takes queued requests in
// arrival order (at most one per simulation per batch, so the per-simulation
// scratch is never shared inside a launch), stages the batch's problem and
// operand tables in pinned host memory, copies them to the device and runs the
// three stage-solve phases as persistent multi-problem launches
// (hevi_launch_multi), then copies the per-request reports back and records an
// event.  Up to kSlots batches are in flight; a slot's staging memory is reused
// only after its event has completed, so no copy reads memory that is being
// rewritten.  Completion is observed by polling the oldest slot's event.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hevi.h"
#include "hevi_internal.h"
#include "hevi_objects.h"

using namespace hevi_host;

namespace {

using Clock = std::chrono::steady_clock;

constexpr int kSlots = 3;       // batches in flight
constexpr int kMaxBatch = 128;  // requests per batch
constexpr int kSchedBytes = 2 * (kMaxBatch * 4 + (kMaxBatch + 1) * 8 + 8);

struct Sim {
  const hevi_ops* ops = nullptr;
  hevi_factors* fac = nullptr;
  size_t bytes = 0;
  HeviProbDev desc;    // info pointer set per batch
  int64_t pending = 0; // submitted and not completed
  bool releasing = false;
};

struct Req {
  uint64_t ticket;
  int32_t sim;
  HeviCallDev call;
  Clock::time_point t0;
};

struct Ticket {
  bool done = false;
  hevi_info info{};
  double latency = 0.0;
};

struct Slot {
  HeviProbDev* h_probs = nullptr;
  HeviCallDev* h_calls = nullptr;
  char* h_sched = nullptr;
  HeviDevInfo* h_info = nullptr;
  HeviProbDev* d_probs = nullptr;
  HeviCallDev* d_calls = nullptr;
  char* d_sched = nullptr;
  HeviDevInfo* d_info = nullptr;
  hipEvent_t ev = nullptr;
  std::vector<Req> reqs;
  bool busy = false;
};

}  // namespace

struct hevi_server {
  hevi_ctx* ctx = nullptr;
  size_t budget = 0, used = 0;
  int32_t max_inflight = 0;
  int sweeps = 4;        // refinement of FP32-factor simulations
  double target = 1e-13;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::map<int32_t, Sim> sims;
  int32_t next_sim = 0;
  std::deque<Req> queue;
  std::unordered_map<uint64_t, Ticket> tickets;
  uint64_t next_ticket = 1;
  int64_t inflight = 0;
  bool stop = false, broken = false;
  hipStream_t st = nullptr;
  uint32_t* d_ctr = nullptr;
  Slot slots[kSlots];
  int head = 0, nbusy = 0;  // oldest busy slot, busy slots
  std::thread worker;
};

namespace {

void complete(hevi_server* S, const Req& r, const hevi_info& info, Clock::time_point now) {
  Ticket& t = S->tickets[r.ticket];
  t.done = true;
  t.info = info;
  t.latency = std::chrono::duration<double>(now - r.t0).count();
  auto it = S->sims.find(r.sim);
  if (it != S->sims.end()) it->second.pending--;
  S->inflight--;
}

void fail_all(hevi_server* S) {
  // device failure: every queued and in-flight request completes with an error
  S->broken = true;
  hevi_info bad{};
  bad.status = HEVI_E_DEVICE;
  bad.first_bad_col = -1;
  const auto now = Clock::now();
  for (int k = 0; k < kSlots; ++k) {
    Slot& sl = S->slots[k];
    if (!sl.busy) continue;
    for (const Req& r : sl.reqs) complete(S, r, bad, now);
    sl.reqs.clear();
    sl.busy = false;
  }
  S->nbusy = 0;
  for (const Req& r : S->queue) complete(S, r, bad, now);
  S->queue.clear();
  S->cv_done.notify_all();
}

// retire completed batches, oldest first
void reap(hevi_server* S) {
  while (S->nbusy > 0) {
    Slot& sl = S->slots[S->head];
    const hipError_t q = hipEventQuery(sl.ev);
    if (q == hipErrorNotReady) return;
    if (q != hipSuccess) {
      fail_all(S);
      return;
    }
    const auto now = Clock::now();
    for (size_t j = 0; j < sl.reqs.size(); ++j) {
      hevi_info inf;
      info_to_host(sl.h_info[j], &inf);
      complete(S, sl.reqs[j], inf, now);
    }
    sl.reqs.clear();
    sl.busy = false;
    S->head = (S->head + 1) % kSlots;
    S->nbusy--;
    S->cv_done.notify_all();
  }
}

// take the next batch from the queue and enqueue its work (lock held)
void launch_batch(hevi_server* S) {
  Slot& sl = S->slots[(S->head + S->nbusy) % kSlots];
  std::vector<Req> pick;
  std::vector<int32_t> seen;
  for (auto it = S->queue.begin(); it != S->queue.end() && (int)pick.size() < kMaxBatch;) {
    if (std::find(seen.begin(), seen.end(), it->sim) != seen.end()) {
      ++it;
      continue;
    }
    seen.push_back(it->sim);
    pick.push_back(*it);
    it = S->queue.erase(it);
  }
  // launch classes: FP64 requests whose columns fit the fused stage kernel, other
  // FP64 requests, FP32-factor requests; most expensive tiles first within a class
  auto cls = [&](const HeviProbDev& d) {
    return d.fp32 ? 2 : (d.sh.nz <= HEVI_FUSED_MAX_NZ ? 0 : 1);
  };
  auto cost = [&](const Req& r) {
    const HeviShapeDev& sh = S->sims[r.sim].desc.sh;
    return (double)sh.nz * (sh.N + 1);
  };
  std::stable_sort(pick.begin(), pick.end(), [&](const Req& a, const Req& b) {
    const int pa = cls(S->sims[a.sim].desc), pb = cls(S->sims[b.sim].desc);
    if (pa != pb) return pa < pb;
    return cost(a) > cost(b);
  });
  const int n = (int)pick.size();
  for (int j = 0; j < n; ++j) {
    sl.h_probs[j] = S->sims[pick[j].sim].desc;
    sl.h_probs[j].info = sl.d_info + j;
    sl.h_calls[j] = pick[j].call;
  }
  // one schedule per launch class
  struct Sub {
    int lo, hi, fp32, nlo, nhi, maxnz, tilt;
    size_t off;
    int64_t total;
  };
  std::vector<Sub> subs;
  size_t off = 0;
  for (int j = 0; j < n;) {
    int k = j;
    const int fp32 = sl.h_probs[j].fp32, c = cls(sl.h_probs[j]);
    int nmin = HEVI_MAXN, nmax = 1, maxnz = 1, tilt = 0;
    while (k < n && cls(sl.h_probs[k]) == c) {
      nmin = std::min(nmin, sl.h_probs[k].sh.N);
      nmax = std::max(nmax, sl.h_probs[k].sh.N);
      maxnz = std::max(maxnz, sl.h_probs[k].sh.nz);
      tilt |= sl.h_probs[k].tilt;
      ++k;
    }
    const int m = k - j;
    int32_t* pl = (int32_t*)(sl.h_sched + off);
    const size_t pad = ((size_t)m * 4 + 7) / 8 * 8;
    int64_t* ps = (int64_t*)(sl.h_sched + off + pad);
    ps[0] = 0;
    for (int t = 0; t < m; ++t) {
      pl[t] = j + t;
      ps[t + 1] = ps[t] + sl.h_probs[j + t].sh.ntiles;
    }
    const bool one = nmin == nmax;
    subs.push_back(
        Sub{j, k, fp32, one ? nmin : 1, one ? nmin : HEVI_MAXN, maxnz, tilt, off, ps[m]});
    off += pad + (size_t)(m + 1) * 8;
    j = k;
  }
  sl.reqs = pick;
  sl.busy = true;
  S->nbusy++;
  bool okk = ok(hipMemcpyAsync(sl.d_probs, sl.h_probs, sizeof(HeviProbDev) * n,
                               hipMemcpyHostToDevice, S->st)) &&
             ok(hipMemcpyAsync(sl.d_calls, sl.h_calls, sizeof(HeviCallDev) * n,
                               hipMemcpyHostToDevice, S->st)) &&
             ok(hipMemcpyAsync(sl.d_sched, sl.h_sched, off, hipMemcpyHostToDevice, S->st)) &&
             ok(hevi_launch_info_reset_n(sl.d_info, n, S->st));
  for (const Sub& sb : subs) {
    if (!okk || sb.total == 0) continue;
    HeviSched s;
    const int m = sb.hi - sb.lo;
    const size_t pad = ((size_t)m * 4 + 7) / 8 * 8;
    s.plist = (const int32_t*)(sl.d_sched + sb.off);
    s.pstart = (const int64_t*)(sl.d_sched + sb.off + pad);
    s.m = m;
    s.total = sb.total;
    s.ctr = S->d_ctr;
    const int grid = (int)sb.total;
    const int sweeps = sb.fp32 ? S->sweeps : 0;
    if (!sb.fp32 && sb.nlo == sb.nhi && sb.maxnz <= HEVI_FUSED_MAX_NZ) {
      okk = okk && ok(hevi_launch_multi(HEVI_PH_STAGE_FUSED, sb.nlo, sb.nhi, 0, sb.tilt,
                                        sl.d_probs, sl.d_calls, s, grid, 0, 1e-13, sb.maxnz,
                                        S->st));
      continue;
    }
    for (int ph : {HEVI_PH_STAGE_RHS, HEVI_PH_STAGE_BSOLVE, HEVI_PH_STAGE_UPDATE})
      okk = okk && ok(hevi_launch_multi(ph, sb.nlo, sb.nhi, sb.fp32, sb.tilt, sl.d_probs,
                                        sl.d_calls, s, grid, sweeps, S->target, sb.maxnz,
                                        S->st));
  }
  okk = okk &&
        ok(hipMemcpyAsync(sl.h_info, sl.d_info, sizeof(HeviDevInfo) * n, hipMemcpyDeviceToHost,
                          S->st)) &&
        ok(hipEventRecord(sl.ev, S->st));
  if (!okk) fail_all(S);
}

void work(hevi_server* S) {
  (void)hipSetDevice(S->ctx->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    reap(S);
    if (S->stop && S->queue.empty() && S->nbusy == 0) break;
    if (!S->queue.empty() && S->nbusy < kSlots && !S->broken) {
      launch_batch(S);
      continue;
    }
    if (S->nbusy > 0) S->cv_work.wait_for(lk, std::chrono::microseconds(20));
    else S->cv_work.wait(lk);
  }
}

void free_slots(hevi_server* S) {
  for (Slot& sl : S->slots) {
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    if (sl.h_probs) (void)hipHostFree(sl.h_probs);
    if (sl.h_calls) (void)hipHostFree(sl.h_calls);
    if (sl.h_sched) (void)hipHostFree(sl.h_sched);
    if (sl.h_info) (void)hipHostFree(sl.h_info);
    if (sl.d_probs) (void)hipFree(sl.d_probs);
    if (sl.d_calls) (void)hipFree(sl.d_calls);
    if (sl.d_sched) (void)hipFree(sl.d_sched);
    if (sl.d_info) (void)hipFree(sl.d_info);
    sl = Slot();
  }
}

hevi_status retire(hevi_server* S, uint64_t ticket, hevi_info* info, double* latency_s) {
  auto it = S->tickets.find(ticket);
  const Ticket& t = it->second;
  if (info) *info = t.info;
  if (latency_s) *latency_s = t.latency;
  S->tickets.erase(it);
  return HEVI_OK;
}

}  // namespace

extern "C" {

hevi_status hevi_serve_create(hevi_ctx* ctx, size_t hbm_budget_bytes, int32_t max_inflight,
                              const hevi_refine* refine, hevi_server** out) {
  if (!ctx || !out || max_inflight < 1) return HEVI_E_INVALID;
  *out = nullptr;
  if (refine && (refine->max_sweeps < 0 || refine->max_sweeps > 64 ||
                 !(refine->rel_residual_target >= 0) || refine->full_sweeps != 0))
    return HEVI_E_INVALID;
  if (!ok(hipSetDevice(ctx->device))) return HEVI_E_DEVICE;
  hevi_server* S = new (std::nothrow) hevi_server;
  if (!S) return HEVI_E_NOMEM;
  S->ctx = ctx;
  S->budget = hbm_budget_bytes;
  S->max_inflight = max_inflight;
  if (refine) {
    S->sweeps = refine->max_sweeps;
    S->target = refine->rel_residual_target;
  }
  bool good = ok(hipStreamCreate(&S->st)) && !dev_alloc(&S->d_ctr, 2 * sizeof(uint32_t)) &&
              ok(hipMemset(S->d_ctr, 0, 2 * sizeof(uint32_t)));
  for (Slot& sl : S->slots) {
    if (!good) break;
    good = ok(hipHostMalloc((void**)&sl.h_probs, sizeof(HeviProbDev) * kMaxBatch, 0)) &&
           ok(hipHostMalloc((void**)&sl.h_calls, sizeof(HeviCallDev) * kMaxBatch, 0)) &&
           ok(hipHostMalloc((void**)&sl.h_sched, kSchedBytes, 0)) &&
           ok(hipHostMalloc((void**)&sl.h_info, sizeof(HeviDevInfo) * kMaxBatch, 0)) &&
           !dev_alloc(&sl.d_probs, sizeof(HeviProbDev) * kMaxBatch) &&
           !dev_alloc(&sl.d_calls, sizeof(HeviCallDev) * kMaxBatch) &&
           !dev_alloc(&sl.d_sched, kSchedBytes) &&
           !dev_alloc(&sl.d_info, sizeof(HeviDevInfo) * kMaxBatch) &&
           ok(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming));
  }
  if (!good) {
    free_slots(S);
    if (S->d_ctr) (void)hipFree(S->d_ctr);
    if (S->st) (void)hipStreamDestroy(S->st);
    delete S;
    return HEVI_E_NOMEM;
  }
  try {
    S->worker = std::thread(work, S);
  } catch (...) {
    free_slots(S);
    (void)hipFree(S->d_ctr);
    (void)hipStreamDestroy(S->st);
    delete S;
    return HEVI_E_NOMEM;
  }
  *out = S;
  return HEVI_OK;
}

hevi_status hevi_serve_register(hevi_server* S, const hevi_ops* ops, double lambda,
                                hevi_precision prec, int32_t* sim_id) {
  if (!S || !ops || !sim_id) return HEVI_E_INVALID;
  if (prec != HEVI_FP64 && prec != HEVI_FP32_REFINE) return HEVI_E_INVALID;
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) return HEVI_E_INVALID;
  if (ops->ctx->device != S->ctx->device) return HEVI_E_INVALID;
  if (ops->s3 || ops->ps) return HEVI_E_INVALID;  // batches run the set-2C group kernels
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->stop || S->broken) return HEVI_E_CLOSED;
  const size_t bytes = factor_storage_bytes(ops->sh, prec);
  if (S->used + bytes > S->budget) return HEVI_E_NOMEM;
  if (!ok(hipSetDevice(S->ctx->device))) return HEVI_E_DEVICE;
  hevi_factors* f = nullptr;
  hevi_status s = factor_stream_ordered(S->ctx, ops, lambda, prec, &f, S->st);
  if (s) return s;
  Sim sim;
  sim.ops = ops;
  sim.fac = f;
  sim.bytes = bytes;
  std::memset(&sim.desc, 0, sizeof(sim.desc));
  sim.desc.sh = ops->sh;
  sim.desc.fp32 = prec == HEVI_FP32_REFINE;
  sim.desc.tilt = ops->tilted;
  sim.desc.lambda = lambda;
  sim.desc.ops = ops->d_ops;
  sim.desc.sbuf = f->sbuf;
  sim.desc.U = f->U;
  sim.desc.L = f->L;
  sim.desc.piv = f->piv;
  sim.desc.ws = f->ws;
  const int32_t id = S->next_sim++;
  S->sims[id] = sim;
  S->used += bytes;
  *sim_id = id;
  return HEVI_OK;
}

hevi_status hevi_serve_submit(hevi_server* S, int32_t sim_id, int32_t n_e,
                              const double* const* h_dE, const double* h_e, int32_t n_prev,
                              const double* const* h_dQprev, const double* h_c, double* d_Qi,
                              uint64_t* ticket) {
  if (!S || !ticket) return HEVI_E_INVALID;
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->stop || S->broken) return HEVI_E_CLOSED;
  auto it = S->sims.find(sim_id);
  if (it == S->sims.end() || it->second.releasing) return HEVI_E_CLOSED;
  const bool empty = it->second.desc.sh.ncols == 0;
  Req r;
  std::memset(&r.call, 0, sizeof(r.call));
  hevi_status s;
  if ((s = terms(n_e, h_dE, h_e, 1, empty, &r.call.E))) return s;
  if ((s = terms(n_prev, h_dQprev, h_c, 0, empty, &r.call.Q))) return s;
  if (!empty) {
    if (!d_Qi) return HEVI_E_INVALID;
    for (int i = 0; i < r.call.E.n; ++i)
      if (r.call.E.v[i] == d_Qi) return HEVI_E_INVALID;
    for (int i = 0; i < r.call.Q.n; ++i)
      if (r.call.Q.v[i] == d_Qi) return HEVI_E_INVALID;
  }
  if (S->inflight >= S->max_inflight) return HEVI_E_BUSY;
  r.call.out = d_Qi;
  r.sim = sim_id;
  r.ticket = S->next_ticket++;
  r.t0 = Clock::now();
  S->tickets[r.ticket] = Ticket();
  S->queue.push_back(r);
  it->second.pending++;
  S->inflight++;
  *ticket = r.ticket;
  S->cv_work.notify_one();
  return HEVI_OK;
}

hevi_status hevi_serve_poll(hevi_server* S, uint64_t ticket, int32_t* done, hevi_info* info,
                            double* latency_s) {
  if (!S || !done) return HEVI_E_INVALID;
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->tickets.find(ticket);
  if (it == S->tickets.end()) return HEVI_E_CLOSED;
  *done = it->second.done ? 1 : 0;
  if (!it->second.done) return HEVI_OK;
  return retire(S, ticket, info, latency_s);
}

hevi_status hevi_serve_wait(hevi_server* S, uint64_t ticket, hevi_info* info,
                            double* latency_s) {
  if (!S) return HEVI_E_INVALID;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->tickets.find(ticket);
  if (it == S->tickets.end()) return HEVI_E_CLOSED;
  S->cv_done.wait(lk, [&] {
    auto f = S->tickets.find(ticket);
    return f == S->tickets.end() || f->second.done;
  });
  if (S->tickets.find(ticket) == S->tickets.end()) return HEVI_E_CLOSED;  // retired elsewhere
  return retire(S, ticket, info, latency_s);
}

hevi_status hevi_serve_release(hevi_server* S, int32_t sim_id) {
  if (!S) return HEVI_E_INVALID;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->sims.find(sim_id);
  if (it == S->sims.end() || it->second.releasing) return HEVI_E_CLOSED;
  it->second.releasing = true;
  S->cv_done.wait(lk, [&] { return S->sims[sim_id].pending == 0; });
  Sim sim = S->sims[sim_id];
  S->sims.erase(sim_id);
  S->used -= sim.bytes;
  lk.unlock();
  // its requests have completed; the buffers go back stream-ordered on the
  // server's stream (after everything queued there), so nothing waits here
  (void)hipSetDevice(S->ctx->device);
  hevi_factors_free(sim.fac);
  return HEVI_OK;
}

void hevi_serve_destroy(hevi_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->worker.joinable()) S->worker.join();
  (void)hipSetDevice(S->ctx->device);
  (void)hipStreamSynchronize(S->st);
  for (auto& kv : S->sims) hevi_factors_free(kv.second.fac);
  (void)hipStreamSynchronize(S->st);  // the stream-ordered frees, before the stream goes
  free_slots(S);
  if (S->d_ctr) (void)hipFree(S->d_ctr);
  if (S->st) (void)hipStreamDestroy(S->st);
  delete S;
}

}  // extern "C"
