// hevi_objects.h -- host-side objects of the C ABI and helpers shared by the
// ABI implementation files (hevi_api.cpp, hevi_group_api.cpp, hevi_serve.cpp).
// Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "hevi.h"
#include "hevi_internal.h"

struct hevi_ctx {
  int device;
};

struct hevi_ops {
  hevi_ctx* ctx;
  hevi_shape shape;
  hevi_consts consts;
  HeviShapeDev sh;
  double* d_ops;
  HeviDevInfo* d_info;
  int32_t* d_tilt;  // device flag set by the ops build
  int tilted;       // its value: some column's grad(zeta) is not one vector along it
  int s3;           // set 3C (state (rho, U, E); ops hold the J dP/drho plane)
  int ps;           // LHEVI-PS: linearised at a moving state (ops hold its velocity planes)
  HeviDevInfo* d_aux;  // reduction slot of hevi_newton_increment
};

struct hevi_factors {
  const hevi_ops* ops;
  double lambda;
  hevi_precision prec;
  void* U;
  void* L;
  uint8_t* piv;
  double* sbuf;  // FP64 assembly buffer (aliases U for FP64 factors)
  double* ws;    // per-node FP64 scratch of the stage solve (HEVI_NWS fields)
  // scratch of the full-system refinement mode (HEVI_NWS_FULL fields), allocated by the
  // first stage solve that asks for full sweeps
  mutable double* wsf;
  HeviDevInfo* d_info;
  hipStream_t alloc_stream;  // buffers allocated stream-ordered on it (server), or 0
  bool stream_ordered;
};

namespace hevi_host {

inline bool ok(hipError_t e) { return e == hipSuccess; }

template <typename P>
hevi_status dev_alloc(P** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 256;
  void* v = nullptr;
  if (!ok(hipMalloc(&v, bytes))) return HEVI_E_NOMEM;
  *p = (P*)v;
  return HEVI_OK;
}

// stream-ordered allocation on `st` (freed with hipFreeAsync on the same stream):
// neither call waits for the device
template <typename P>
hevi_status dev_alloc_on(P** p, size_t bytes, hipStream_t st) {
  *p = nullptr;
  if (bytes == 0) bytes = 256;
  void* v = nullptr;
  if (!ok(hipMallocAsync(&v, bytes, st))) return HEVI_E_NOMEM;
  *p = (P*)v;
  return HEVI_OK;
}

// hevi_factor with the factor object's buffers allocated stream-ordered on
// `stream` (and freed the same way by hevi_factors_free): the server's
// registrations and releases then never wait for the whole device
hevi_status factor_stream_ordered(hevi_ctx* ctx, const hevi_ops* ops, double lambda,
                                  hevi_precision prec, hevi_factors** out, hipStream_t stream);

HeviShapeDev dev_shape(const hevi_shape& s);
hevi_status check_shape(const hevi_shape* s);
size_t tiles_nodes(const HeviShapeDev& sh);
// copy a device report to the host (waits for the stream); optionally reset it
hevi_status read_info(HeviDevInfo* d_info, hipStream_t st, hevi_info* out, bool reset);
void info_to_host(const HeviDevInfo& h, hevi_info* out);
// validated linear-combination terms (lo = minimum count; empty = no columns)
hevi_status terms(int32_t n, const double* const* v, const double* coef, int lo, bool empty,
                  HeviTerms* t);
// byte planes beside the factors: pivot offsets, U row extents, row-scale exponents
constexpr size_t kFactorPlanes = 3;
// LHEVI-PS kernels hold one column in LDS, at most 64 KiB: the factorisation 12 operator
// fields (96 n_z bytes) and ~5 KiB of tables and staging, the stage solve two vectors and
// three byte planes (19 n = 95 n_z bytes): n_z up to 600
constexpr int kPsMaxNz = 600;
// FP32 factors of orders without the fused assembly + LU need an FP64 assembly
// buffer (FP64 factors assemble in place of U)
inline bool needs_sbuf(const HeviShapeDev& sh, hevi_precision prec) {
  return prec != HEVI_FP64 && sh.N > HEVI_FUSED_FACTOR_MAX_N;
}
// address of the allocation-free entry point's device array on `device` (current),
// taken once per device (hevi_create)
hevi_status hevi_noalloc_init(int device);
// bytes of the library-owned storage of one factor object
size_t factor_storage_bytes(const HeviShapeDev& sh, hevi_precision prec);

}  // namespace hevi_host
