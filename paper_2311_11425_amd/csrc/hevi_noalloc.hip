// hevi_noalloc.hip -- the allocation-free stage solve (hevi_solve_noalloc).
//
// For callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops): one call factors A = I - lambda L_z and runs
// one stage solve, with the factors, the stage solve's scratch and the kernel
// report placed in `scratch`, a fixed device array of this file.  The kernels
// are those of hevi_factor + hevi_stage_solve; they take pointers into the
// array as they take the factor object's buffers.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "hevi.h"
#include "hevi_internal.h"
#include "hevi_objects.h"

namespace {

// One copy per GPU, held until the process ends.  Host code never uses this
// name as an address: it works with the device address that
// hipGetSymbolAddress returned for the current device (scratch_of).
static __device__ __align__(256) unsigned char scratch[HEVI_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_ptr[kMaxDevices] = {};

unsigned char* scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_ptr[device];
}

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

// Places of the factor object's buffers inside the array for one shape.
struct Layout {
  size_t info, U, L, piv, ws, sbuf, total;
};

// full: the full-system refinement mode (its wider scratch)
Layout layout(const HeviShapeDev& sh, hevi_precision prec, bool full) {
  const size_t tn = hevi_host::tiles_nodes(sh);
  const size_t fs = prec == HEVI_FP64 ? sizeof(double) : sizeof(float);
  Layout l{};
  size_t o = 0;
  l.info = o; o += up256(sizeof(HeviDevInfo));
  l.U = o;    o += up256(tn * (4 * sh.N + 1) * fs);
  l.L = o;    o += up256(tn * 2 * sh.N * fs);
  l.piv = o;  o += up256(hevi_host::kFactorPlanes * tn);
  l.ws = o;   o += up256(tn * (full ? HEVI_NWS_FULL : HEVI_NWS) * sizeof(double));
  l.sbuf = o;
  if (hevi_host::needs_sbuf(sh, prec)) o += up256(tn * (4 * sh.N + 1) * sizeof(double));
  l.total = o;
  return l;
}

}  // namespace

// Called by hevi_create with `device` current: the array's address on it.
hevi_status hevi_host::hevi_noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return HEVI_E_DEVICE;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return HEVI_OK;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HEVI_E_DEVICE;
  g_ptr[device] = (unsigned char*)p;
  return HEVI_OK;
}

extern "C" {

hevi_status hevi_solve_noalloc(hevi_ctx* ctx, const hevi_ops* ops, double lambda,
                               hevi_precision prec, int32_t n_e, const double* const* h_dE,
                               const double* h_e, int32_t n_prev,
                               const double* const* h_dQprev, const double* h_c, double* d_Qi,
                               const hevi_refine* refine, hevi_info* h_info,
                               hipStream_t stream) {
  using namespace hevi_host;
  if (!ctx || !ops || ops->ps) return HEVI_E_INVALID;  // LHEVI-PS factors: hevi_factor
  if (prec != HEVI_FP64 && prec != HEVI_FP32_REFINE) return HEVI_E_INVALID;
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) return HEVI_E_INVALID;
  const HeviShapeDev& sh = ops->sh;
  HeviTerms E, Q;
  hevi_status s;
  const bool empty = sh.ncols == 0;
  if ((s = terms(n_e, h_dE, h_e, 1, empty, &E))) return s;
  if ((s = terms(n_prev, h_dQprev, h_c, 0, empty, &Q))) return s;
  if (!empty) {
    if (!d_Qi) return HEVI_E_INVALID;
    for (int i = 0; i < E.n; ++i)
      if (E.v[i] == d_Qi) return HEVI_E_INVALID;
    for (int i = 0; i < Q.n; ++i)
      if (Q.v[i] == d_Qi) return HEVI_E_INVALID;
  }
  int sweeps = 4, full = 0;
  double target = 1e-13;
  if (refine) {
    if (refine->max_sweeps < 0 || refine->max_sweeps > 64 || !(refine->rel_residual_target >= 0) ||
        refine->full_sweeps < 0 || refine->full_sweeps > 8)
      return HEVI_E_INVALID;
    sweeps = refine->max_sweeps;
    target = refine->rel_residual_target;
    full = refine->full_sweeps;
  }
  if (prec == HEVI_FP64) sweeps = 0;
  const Layout l = layout(sh, prec, full > 0);
  if (l.total > (size_t)HEVI_NOALLOC_SCRATCH_BYTES) return HEVI_E_SCRATCH;
  unsigned char* base = scratch_of(ctx->device);
  if (!base) return HEVI_E_DEVICE;
  if (!ok(hipSetDevice(ctx->device))) return HEVI_E_DEVICE;
  HeviDevInfo* info = (HeviDevInfo*)(base + l.info);
  void* U = base + l.U;
  void* L = base + l.L;
  uint8_t* piv = base + l.piv;
  double* ws = (double*)(base + l.ws);
  // FP64 factors assemble in place of U; FP32 factors of the fused orders need no buffer
  double* sbuf = needs_sbuf(sh, prec) ? (double*)(base + l.sbuf)
                                      : (prec == HEVI_FP64 ? (double*)U : nullptr);
  // the report starts at zero (a kernel, not a memset); every factor and scratch
  // entry the kernels read is written by this call's kernels first
  if (!ok(hevi_launch_info_reset(info, stream)) ||
      !ok(hevi_launch_factor(sh, ops->s3, lambda, prec == HEVI_FP32_REFINE, ops->d_ops, sbuf, U, L, piv,
                             info, stream)) ||
      !ok(hevi_launch_stage_solve(sh, ops->s3, lambda, ops->tilted, prec == HEVI_FP32_REFINE, ops->d_ops,
                                  U, L, piv, ws, E, Q, d_Qi, sweeps, target, full, info,
                                  stream)))
    return HEVI_E_DEVICE;
  if (h_info) {
    std::memset(h_info, 0, sizeof(*h_info));
    hevi_status r = read_info(info, stream, h_info, false);
    if (r == HEVI_E_DEVICE) return r;
  }
  return HEVI_OK;
}

}  // extern "C"
