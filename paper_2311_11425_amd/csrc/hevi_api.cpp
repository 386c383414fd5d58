// hevi_api.cpp -- C ABI of the batched LHEVI column solver (see include/hevi.h).
//
// Host side only: argument validation, ownership of device buffers, the ARK
// tableaux, and kernel launches on the caller's stream.  The arithmetic of the
// method runs in hevi_kernels.hip (GLL tables: compile-time constants, hevi_gll.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <new>
#include <vector>

#include "hevi.h"
#include "hevi_internal.h"
#include "hevi_objects.h"

namespace hevi_host {

HeviShapeDev dev_shape(const hevi_shape& s) {
  HeviShapeDev d;
  d.N = s.order_N;
  d.Ne = s.n_elem;
  d.nz = s.n_elem * s.order_N + 1;
  d.ncols = s.n_cols;
  d.ntiles = (s.n_cols + HEVI_TILE - 1) / HEVI_TILE;
  return d;
}

hevi_status check_shape(const hevi_shape* s) {
  if (!s) return HEVI_E_INVALID;
  if (s->order_N < 1 || s->order_N > HEVI_MAXN) return HEVI_E_SHAPE;
  if (s->n_elem < 1 || s->n_elem > 4096) return HEVI_E_SHAPE;
  if (s->n_cols < 0) return HEVI_E_SHAPE;
  const int64_t nz = (int64_t)s->n_elem * s->order_N + 1;
  if (nz > 32768) return HEVI_E_SHAPE;
  // grid dimension limit: one 64-column tile per block
  if ((s->n_cols + HEVI_TILE - 1) / HEVI_TILE > (int64_t)INT32_MAX) return HEVI_E_SHAPE;
  return HEVI_OK;
}

size_t tiles_nodes(const HeviShapeDev& sh) { return (size_t)sh.ntiles * (size_t)sh.nz * HEVI_TILE; }

void info_to_host(const HeviDevInfo& h, hevi_info* out) {
  out->status = h.status;
  out->max_sweeps_used = h.max_sweeps;
  out->first_bad_col = h.first_bad == INT64_MAX ? -1 : h.first_bad;
  out->n_bad_cols = h.n_bad;
  double r;
  std::memcpy(&r, &h.max_res_bits, sizeof(r));
  out->max_rel_correction = r;
}

hevi_status read_info(HeviDevInfo* d_info, hipStream_t st, hevi_info* out, bool reset) {
  HeviDevInfo h;
  if (!ok(hipMemcpyAsync(&h, d_info, sizeof(h), hipMemcpyDeviceToHost, st))) return HEVI_E_DEVICE;
  if (!ok(hipStreamSynchronize(st))) return HEVI_E_DEVICE;
  if (reset && !ok(hevi_launch_info_reset(d_info, st))) return HEVI_E_DEVICE;
  if (out) info_to_host(h, out);
  return (hevi_status)h.status;
}

size_t factor_storage_bytes(const HeviShapeDev& sh, hevi_precision prec) {
  const size_t tn = tiles_nodes(sh);
  const size_t fs = prec == HEVI_FP64 ? sizeof(double) : sizeof(float);
  // U, L, three byte planes (pivots, U row extents, row scales), stage scratch,
  // and for FP32 factors of orders without the fused factorisation an FP64
  // assembly buffer
  size_t b = tn * (4 * sh.N + 1) * fs + tn * 2 * sh.N * fs + kFactorPlanes * tn +
             tn * HEVI_NWS * sizeof(double);
  if (needs_sbuf(sh, prec)) b += tn * (4 * sh.N + 1) * sizeof(double);
  return b;
}

hevi_status terms(int32_t n, const double* const* v, const double* coef, int lo, bool empty,
                  HeviTerms* t) {
  // empty: the batch has no columns, so NULL device pointers are acceptable
  if (n < lo || n > HEVI_MAXTERMS) return HEVI_E_INVALID;
  if (n > 0 && (!v || !coef)) return HEVI_E_INVALID;
  t->n = n;
  for (int i = 0; i < n; ++i) {
    if ((!v[i] && !empty) || !std::isfinite(coef[i])) return HEVI_E_INVALID;
    t->v[i] = v[i];
    t->coef[i] = coef[i];
  }
  for (int i = n; i < HEVI_MAXTERMS; ++i) { t->v[i] = nullptr; t->coef[i] = 0.0; }
  return HEVI_OK;
}

}  // namespace hevi_host

using namespace hevi_host;

extern "C" {

const char* hevi_status_str(hevi_status s) {
  switch (s) {
    case HEVI_OK: return "ok";
    case HEVI_E_INVALID: return "invalid argument";
    case HEVI_E_SHAPE: return "unsupported shape";
    case HEVI_E_NOMEM: return "out of memory";
    case HEVI_E_DEVICE: return "HIP device error";
    case HEVI_E_SINGULAR: return "zero pivot";
    case HEVI_E_NOT_CONVERGED: return "refinement did not converge";
    case HEVI_E_BUSY: return "busy";
    case HEVI_E_CLOSED: return "closed";
    case HEVI_E_NONFINITE: return "non-finite value";
    case HEVI_E_SCRATCH: return "shape exceeds the fixed scratch of hevi_solve_noalloc";
  }
  return "unknown status";
}

hevi_status hevi_create(int device, hevi_ctx** out) {
  if (!out) return HEVI_E_INVALID;
  *out = nullptr;
  int n = 0;
  if (!ok(hipGetDeviceCount(&n)) || device < 0 || device >= n) return HEVI_E_DEVICE;
  hipDeviceProp_t prop;
  if (!ok(hipGetDeviceProperties(&prop, device))) return HEVI_E_DEVICE;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return HEVI_E_DEVICE;
  if (!ok(hipSetDevice(device))) return HEVI_E_DEVICE;
  if (hevi_noalloc_init(device) != HEVI_OK) return HEVI_E_DEVICE;
  hevi_ctx* c = new (std::nothrow) hevi_ctx;
  if (!c) return HEVI_E_NOMEM;
  c->device = device;
  *out = c;
  return HEVI_OK;
}

void hevi_destroy(hevi_ctx* ctx) { delete ctx; }

hevi_status hevi_build_column_ops(hevi_ctx* ctx, const hevi_shape* shape, const hevi_consts* k,
                                  const double* d_z, const double* d_J, const double* d_gz,
                                  const double* d_rho0, const double* d_Theta0, hevi_ops** out,
                                  hipStream_t stream) {
  return hevi_build_column_ops_set(ctx, shape, k, HEVI_SET_2C, d_z, d_J, d_gz, d_rho0, d_Theta0,
                                   out, stream);
}

hevi_status hevi_build_column_ops_set(hevi_ctx* ctx, const hevi_shape* shape,
                                      const hevi_consts* k, hevi_eqset eqset, const double* d_z,
                                      const double* d_J, const double* d_gz,
                                      const double* d_rho0, const double* d_Theta0,
                                      hevi_ops** out, hipStream_t stream) {
  if (!ctx || !out || !k) return HEVI_E_INVALID;
  if (eqset != HEVI_SET_2C && eqset != HEVI_SET_3C) return HEVI_E_INVALID;
  *out = nullptr;
  hevi_status s = check_shape(shape);
  if (s) return s;
  if (!(k->R > 0) || !(k->cp > k->R) || !(k->g >= 0) || !(k->p_A > 0) || !std::isfinite(k->R) ||
      !std::isfinite(k->cp) || !std::isfinite(k->g) || !std::isfinite(k->p_A))
    return HEVI_E_INVALID;
  if (shape->n_cols > 0 && (!d_z || !d_J || !d_gz || !d_rho0 || !d_Theta0)) return HEVI_E_INVALID;
  if (!ok(hipSetDevice(ctx->device))) return HEVI_E_DEVICE;
  hevi_ops* o = new (std::nothrow) hevi_ops;
  if (!o) return HEVI_E_NOMEM;
  o->ctx = ctx;
  o->shape = *shape;
  o->consts = *k;
  o->sh = dev_shape(*shape);
  o->d_ops = nullptr;
  o->d_info = nullptr;
  o->d_tilt = nullptr;
  o->d_aux = nullptr;
  o->tilted = 0;
  o->s3 = eqset == HEVI_SET_3C;
  o->ps = 0;
  // set 3C: one more per-node field (J dP/drho) after the tile-interleaved eight
  if ((s = dev_alloc(&o->d_ops, tiles_nodes(o->sh) * (HEVI_NOPS + o->s3) * sizeof(double))) ||
      (s = dev_alloc(&o->d_info, sizeof(HeviDevInfo))) ||
      (s = dev_alloc(&o->d_aux, sizeof(HeviDevInfo))) ||
      (s = dev_alloc(&o->d_tilt, sizeof(int32_t)))) {
    hevi_ops_free(o);
    return s;
  }
  // the geometry class (straight columns or not) selects the stage kernels, so it
  // is read back here, once
  int32_t tilt = 0;
  if (!ok(hipMemcpyAsync(o->d_tilt, &tilt, sizeof(tilt), hipMemcpyHostToDevice, stream)) ||
      !ok(hevi_launch_info_reset(o->d_info, stream)) ||
      !ok(hevi_launch_build_ops(o->sh, o->s3, k->R, k->cp, k->g, k->p_A, d_z, d_J, d_gz, d_rho0,
                                d_Theta0, o->d_ops, o->d_info, o->d_tilt, stream)) ||
      !ok(hipMemcpyAsync(&tilt, o->d_tilt, sizeof(tilt), hipMemcpyDeviceToHost, stream)) ||
      !ok(hipStreamSynchronize(stream))) {
    hevi_ops_free(o);
    return HEVI_E_DEVICE;
  }
  o->tilted = tilt != 0;
  *out = o;
  return HEVI_OK;
}

hevi_status hevi_build_column_ops_ps(hevi_ctx* ctx, const hevi_shape* shape,
                                     const hevi_consts* k, const double* d_z, const double* d_J,
                                     const double* d_gz, const double* d_rho0,
                                     const double* d_U0, const double* d_Theta0, hevi_ops** out,
                                     hipStream_t stream) {
  if (!ctx || !out || !k) return HEVI_E_INVALID;
  *out = nullptr;
  hevi_status s = check_shape(shape);
  if (s) return s;
  if (shape->order_N > HEVI_PS_MAXN) return HEVI_E_SHAPE;
  if (!(k->R > 0) || !(k->cp > k->R) || !(k->g >= 0) || !(k->p_A > 0) || !std::isfinite(k->R) ||
      !std::isfinite(k->cp) || !std::isfinite(k->g) || !std::isfinite(k->p_A))
    return HEVI_E_INVALID;
  if (shape->n_cols > 0 && (!d_z || !d_J || !d_gz || !d_rho0 || !d_U0 || !d_Theta0))
    return HEVI_E_INVALID;
  if (!ok(hipSetDevice(ctx->device))) return HEVI_E_DEVICE;
  hevi_ops* o = new (std::nothrow) hevi_ops;
  if (!o) return HEVI_E_NOMEM;
  o->ctx = ctx;
  o->shape = *shape;
  o->consts = *k;
  o->sh = dev_shape(*shape);
  o->d_ops = nullptr;
  o->d_info = nullptr;
  o->d_tilt = nullptr;
  o->d_aux = nullptr;
  o->tilted = 0;
  o->s3 = 0;
  o->ps = 1;
  // the eight fields, then the three velocity planes of the linearisation state
  if ((s = dev_alloc(&o->d_ops, tiles_nodes(o->sh) * (HEVI_NOPS + 3) * sizeof(double))) ||
      (s = dev_alloc(&o->d_info, sizeof(HeviDevInfo))) ||
      (s = dev_alloc(&o->d_aux, sizeof(HeviDevInfo))) ||
      (s = dev_alloc(&o->d_tilt, sizeof(int32_t)))) {
    hevi_ops_free(o);
    return s;
  }
  int32_t tilt = 0;
  if (!ok(hipMemcpyAsync(o->d_tilt, &tilt, sizeof(tilt), hipMemcpyHostToDevice, stream)) ||
      !ok(hevi_launch_info_reset(o->d_info, stream)) ||
      !ok(hevi_launch_build_ops(o->sh, 0, k->R, k->cp, k->g, k->p_A, d_z, d_J, d_gz, d_rho0,
                                d_Theta0, o->d_ops, o->d_info, o->d_tilt, stream)) ||
      !ok(hevi_launch_ps_state(o->sh, k->R, k->cp, k->p_A, d_rho0, d_U0, d_Theta0, o->d_ops,
                               o->d_info, stream)) ||
      !ok(hipMemcpyAsync(&tilt, o->d_tilt, sizeof(tilt), hipMemcpyDeviceToHost, stream)) ||
      !ok(hipStreamSynchronize(stream))) {
    hevi_ops_free(o);
    return HEVI_E_DEVICE;
  }
  o->tilted = tilt != 0;
  *out = o;
  return HEVI_OK;
}

hevi_status hevi_ops_relinearize(hevi_ctx* ctx, hevi_ops* ops, const double* d_rho0,
                                 const double* d_U0, const double* d_Theta0, hipStream_t stream) {
  if (!ctx || !ops || !ops->ps) return HEVI_E_INVALID;
  if (ops->sh.ncols > 0 && (!d_rho0 || !d_U0 || !d_Theta0)) return HEVI_E_INVALID;
  if (!ok(hipSetDevice(ctx->device))) return HEVI_E_DEVICE;
  const hevi_consts& k = ops->consts;
  if (!ok(hevi_launch_ps_state(ops->sh, k.R, k.cp, k.p_A, d_rho0, d_U0, d_Theta0, ops->d_ops,
                               ops->d_info, stream)))
    return HEVI_E_DEVICE;
  return HEVI_OK;
}

hevi_status hevi_ops_check(hevi_ctx* ctx, const hevi_ops* ops, int64_t* first_bad_col,
                           hipStream_t stream) {
  if (!ctx || !ops) return HEVI_E_INVALID;
  hevi_info inf;
  hevi_status s = read_info(ops->d_info, stream, &inf, false);
  if (first_bad_col) *first_bad_col = inf.first_bad_col;
  return s;
}

void hevi_ops_free(hevi_ops* ops) {
  if (!ops) return;
  if (ops->d_ops) (void)hipFree(ops->d_ops);
  if (ops->d_info) (void)hipFree(ops->d_info);
  if (ops->d_tilt) (void)hipFree(ops->d_tilt);
  if (ops->d_aux) (void)hipFree(ops->d_aux);
  delete ops;
}

hevi_status hevi_apply_op(hevi_ctx* ctx, const hevi_ops* ops, const double* d_x,
                          const double* d_xref, double* d_y, hipStream_t stream) {
  if (!ctx || !ops) return HEVI_E_INVALID;
  if (ops->sh.ncols > 0) {
    if (!d_x || !d_y) return HEVI_E_INVALID;
    if (d_y == d_x || (d_xref && d_y == d_xref)) return HEVI_E_INVALID;
  }
  if (!ok(hipSetDevice(ctx->device))) return HEVI_E_DEVICE;
  const hipError_t e = ops->ps ? hevi_launch_apply_ps(ops->sh, ops->d_ops, d_x, d_xref, d_y, stream)
                               : hevi_launch_apply(ops->sh, ops->s3, ops->d_ops, d_x, d_xref, d_y,
                                                   stream);
  if (!ok(e)) return HEVI_E_DEVICE;
  return HEVI_OK;
}

}  // extern "C"

namespace hevi_host {

hevi_status factor_impl(hevi_ctx* ctx, const hevi_ops* ops, double lambda, hevi_precision prec,
                        hevi_factors** out, hipStream_t stream, bool stream_ordered);

hevi_status factor_stream_ordered(hevi_ctx* ctx, const hevi_ops* ops, double lambda,
                                  hevi_precision prec, hevi_factors** out, hipStream_t stream) {
  return factor_impl(ctx, ops, lambda, prec, out, stream, true);
}

}  // namespace hevi_host

extern "C" {

hevi_status hevi_factor(hevi_ctx* ctx, const hevi_ops* ops, double lambda, hevi_precision prec,
                        hevi_factors** out, hipStream_t stream) {
  return factor_impl(ctx, ops, lambda, prec, out, stream, false);
}

}  // extern "C"

hevi_status hevi_host::factor_impl(hevi_ctx* ctx, const hevi_ops* ops, double lambda,
                                   hevi_precision prec, hevi_factors** out, hipStream_t stream,
                                   bool stream_ordered) {
  if (!ctx || !ops || !out) return HEVI_E_INVALID;
  *out = nullptr;
  if (prec != HEVI_FP64 && prec != HEVI_FP32_REFINE) return HEVI_E_INVALID;
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) return HEVI_E_INVALID;
  if (!ok(hipSetDevice(ctx->device))) return HEVI_E_DEVICE;
  hevi_factors* f = new (std::nothrow) hevi_factors;
  if (!f) return HEVI_E_NOMEM;
  std::memset(f, 0, sizeof(*f));
  f->ops = ops;
  f->prec = prec;
  f->stream_ordered = stream_ordered;
  f->alloc_stream = stream;
  const HeviShapeDev& sh = ops->sh;
  const size_t tn = tiles_nodes(sh);
  const size_t fs = prec == HEVI_FP64 ? sizeof(double) : sizeof(float);
  const int N = sh.N;
  auto alloc = [&](auto** p, size_t bytes) {
    return stream_ordered ? dev_alloc_on(p, bytes, stream) : dev_alloc(p, bytes);
  };
  hevi_status s;
  if (ops->ps) {
    // LHEVI-PS: the full 5 n_z band in FP64, column-contiguous, and four byte planes
    // (pivot offsets, row exponents, U column extents, L step extents)
    if (prec != HEVI_FP64) { delete f; return HEVI_E_INVALID; }
    if (N > HEVI_PS_MAXN || sh.nz > kPsMaxNz) { delete f; return HEVI_E_SHAPE; }
    const size_t n = 5 * (size_t)sh.nz, nc = (size_t)sh.ncols;
    if ((s = alloc(&f->U, nc * n * hevi_ps_band_width(N) * sizeof(double))) ||
        (s = alloc(&f->L, nc * n * hevi_ps_lower_width(N) * sizeof(double))) ||
        (s = alloc(&f->piv, 4 * nc * n)) || (s = alloc(&f->d_info, sizeof(HeviDevInfo)))) {
      hevi_factors_free(f);
      return s;
    }
  } else if ((s = alloc(&f->U, tn * (4 * N + 1) * fs)) || (s = alloc(&f->L, tn * 2 * N * fs)) ||
      (s = alloc(&f->piv, kFactorPlanes * tn)) ||
      (s = alloc(&f->ws, tn * HEVI_NWS * sizeof(double))) ||
      (s = alloc(&f->d_info, sizeof(HeviDevInfo)))) {
    hevi_factors_free(f);
    return s;
  }
  if (ops->ps) {
    f->sbuf = nullptr;
  } else if (!needs_sbuf(sh, prec)) {
    // FP64 factors assemble in place of U; the fused factorisation needs no buffer
    f->sbuf = prec == HEVI_FP64 ? (double*)f->U : nullptr;
  } else if ((s = alloc(&f->sbuf, tn * (4 * N + 1) * sizeof(double)))) {
    hevi_factors_free(f);
    return s;
  }
  if (!ok(hevi_launch_info_reset(f->d_info, stream))) {
    hevi_factors_free(f);
    return HEVI_E_DEVICE;
  }
  if ((s = hevi_refactor(ctx, f, lambda, stream))) {
    hevi_factors_free(f);
    return s;
  }
  *out = f;
  return HEVI_OK;
}

extern "C" {

hevi_status hevi_refactor(hevi_ctx* ctx, hevi_factors* f, double lambda, hipStream_t stream) {
  if (!ctx || !f) return HEVI_E_INVALID;
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) return HEVI_E_INVALID;
  if (!ok(hipSetDevice(ctx->device))) return HEVI_E_DEVICE;
  f->lambda = lambda;
  const hevi_ops* o = f->ops;
  const hipError_t e =
      o->ps ? hevi_launch_ps_factor(o->sh, lambda, o->d_ops, (double*)f->U, (double*)f->L, f->piv,
                                    f->d_info, stream)
            : hevi_launch_factor(o->sh, o->s3, lambda, f->prec == HEVI_FP32_REFINE, o->d_ops,
                                 f->sbuf, f->U, f->L, f->piv, f->d_info, stream);
  if (!ok(e)) return HEVI_E_DEVICE;
  return HEVI_OK;
}

hevi_status hevi_factors_check(hevi_ctx* ctx, const hevi_factors* f, hevi_info* info,
                               hipStream_t stream) {
  if (!ctx || !f) return HEVI_E_INVALID;
  return read_info(f->d_info, stream, info, true);
}

hevi_status hevi_factors_band_entries(hevi_ctx* ctx, const hevi_factors* f, int64_t* u_entries,
                                      hipStream_t stream) {
  if (!ctx || !f || !u_entries || f->ops->ps) return HEVI_E_INVALID;
  if (!ok(hipSetDevice(ctx->device))) return HEVI_E_DEVICE;
  const HeviShapeDev& sh = f->ops->sh;
  const size_t tn = tiles_nodes(sh);
  *u_entries = 0;
  if (tn == 0) return HEVI_OK;
  std::vector<uint8_t> h(tn);
  if (!ok(hipStreamSynchronize(stream)) ||
      !ok(hipMemcpy(h.data(), f->piv + tn, tn, hipMemcpyDeviceToHost)))
    return HEVI_E_DEVICE;
  int64_t u = 0;
  for (int64_t t = 0; t < sh.ntiles; ++t)
    for (int k = 0; k < sh.nz; ++k)
      for (int c = 0; c < HEVI_TILE; ++c)
        if (t * HEVI_TILE + c < sh.ncols) u += h[((size_t)t * sh.nz + k) * HEVI_TILE + c] + 1;
  *u_entries = u;
  return HEVI_OK;
}

void hevi_factors_free(hevi_factors* f) {
  if (!f) return;
  auto fr = [&](void* p) {
    if (!p) return;
    if (f->stream_ordered) (void)hipFreeAsync(p, f->alloc_stream);
    else (void)hipFree(p);
  };
  if (f->sbuf != (double*)f->U) fr(f->sbuf);
  fr(f->U);
  fr(f->L);
  fr(f->piv);
  fr(f->ws);
  if (f->wsf) (void)hipFree(f->wsf);
  fr(f->d_info);
  delete f;
}

hevi_status hevi_stage_solve(hevi_ctx* ctx, const hevi_factors* f, int32_t n_e,
                             const double* const* h_dE, const double* h_e, int32_t n_prev,
                             const double* const* h_dQprev, const double* h_c, double* d_Qi,
                             const hevi_refine* refine, hevi_info* h_info, hipStream_t stream) {
  if (!ctx || !f) return HEVI_E_INVALID;
  const hevi_ops* o = f->ops;
  HeviTerms E, Q;
  hevi_status s;
  const bool empty = o->sh.ncols == 0;
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
  if (f->prec == HEVI_FP64) sweeps = 0;
  if (!ok(hipSetDevice(ctx->device))) return HEVI_E_DEVICE;
  if (full > 0 && !o->ps && !f->wsf) {
    // the accuracy mode's wider scratch, once per factor object (this call allocates)
    hevi_status a = dev_alloc(&f->wsf, tiles_nodes(o->sh) * HEVI_NWS_FULL * sizeof(double));
    if (a) return a;
  }
  if (h_info && !ok(hevi_launch_info_reset(f->d_info, stream))) return HEVI_E_DEVICE;
  const hipError_t e =
      o->ps ? hevi_launch_ps_stage(o->sh, o->d_ops, (const double*)f->U, (const double*)f->L,
                                   f->piv, E, Q, d_Qi, f->d_info, stream)
            : hevi_launch_stage_solve(o->sh, o->s3, f->lambda, o->tilted,
                                      f->prec == HEVI_FP32_REFINE, o->d_ops, f->U, f->L, f->piv,
                                      full > 0 ? f->wsf : f->ws, E, Q, d_Qi, sweeps, target,
                                      full, f->d_info, stream);
  if (!ok(e)) return HEVI_E_DEVICE;
  if (h_info) {
    std::memset(h_info, 0, sizeof(*h_info));
    hevi_status r = read_info(f->d_info, stream, h_info, true);
    if (r == HEVI_E_DEVICE) return r;
  }
  return HEVI_OK;
}

hevi_status hevi_combine(hevi_ctx* ctx, const hevi_ops* ops, int32_t n_v,
                         const double* const* h_dV, const double* h_coef, double* d_out,
                         hipStream_t stream) {
  if (!ctx || !ops) return HEVI_E_INVALID;
  HeviTerms V;
  hevi_status s;
  if ((s = terms(n_v, h_dV, h_coef, 1, ops->sh.ncols == 0, &V))) return s;
  if (ops->sh.ncols > 0 && !d_out) return HEVI_E_INVALID;
  if (!ok(hipSetDevice(ctx->device))) return HEVI_E_DEVICE;
  const int64_t n = 5 * (int64_t)ops->sh.nz * ops->sh.ncols;
  if (!ok(hevi_launch_combine(n, V, d_out, stream))) return HEVI_E_DEVICE;
  return HEVI_OK;
}

hevi_status hevi_vertical_op(hevi_ctx* ctx, const hevi_ops* ops, const double* d_q, double* d_V,
                             hipStream_t stream) {
  if (!ctx || !ops || ops->s3) return HEVI_E_INVALID;
  if (ops->sh.ncols > 0 && (!d_q || !d_V || d_q == d_V)) return HEVI_E_INVALID;
  if (!ok(hipSetDevice(ctx->device))) return HEVI_E_DEVICE;
  const hevi_consts& k = ops->consts;
  if (!ok(hevi_launch_vertical_op(ops->sh, k.R, k.cp, k.p_A, ops->d_ops, d_q, d_V, stream)))
    return HEVI_E_DEVICE;
  return HEVI_OK;
}

hevi_status hevi_newton_increment(hevi_ctx* ctx, const hevi_ops* ops, const double* d_dq,
                                  const double* d_q, const double* d_qn, double* h_rel,
                                  hipStream_t stream) {
  if (!ctx || !ops || !h_rel) return HEVI_E_INVALID;
  if (ops->sh.ncols > 0 && (!d_dq || !d_q || !d_qn)) return HEVI_E_INVALID;
  if (!ok(hipSetDevice(ctx->device))) return HEVI_E_DEVICE;
  HeviDevInfo h;
  if (!ok(hevi_launch_info_reset(ops->d_aux, stream)) ||
      !ok(hevi_launch_newton_rel(ops->sh, d_dq, d_q, d_qn, ops->d_aux, stream)) ||
      !ok(hipMemcpyAsync(&h, ops->d_aux, sizeof(h), hipMemcpyDeviceToHost, stream)) ||
      !ok(hipStreamSynchronize(stream)))
    return HEVI_E_DEVICE;
  double r;
  std::memcpy(&r, &h.max_res_bits, sizeof(r));
  *h_rel = r;
  return HEVI_OK;
}

// ---- ARK tableaux (Sec. 6) ---------------------------------------------------
hevi_status hevi_tableau(const char* name, int32_t* s, double* a_exp, double* a_imp, double* b) {
  if (!name || !s || !a_exp || !a_imp || !b) return HEVI_E_INVALID;
  if (!std::strcmp(name, "ARK2") || !std::strcmp(name, "ARK2b") || !std::strcmp(name, "ARK2a")) {
    // ARK(2,3,2): gamma = 1 - 1/sqrt2, delta = 1/(2 sqrt2), free a_32
    const double r2 = std::sqrt(2.0);
    const double gm = 1.0 - 1.0 / r2, dl = 1.0 / (2.0 * r2);
    const double a32 = !std::strcmp(name, "ARK2a") ? (3.0 + 2.0 * r2) / 6.0 : 0.5;
    const double E[9] = {0, 0, 0, 2 * gm, 0, 0, 1 - a32, a32, 0};
    const double I[9] = {0, 0, 0, gm, gm, 0, dl, dl, gm};
    *s = 3;
    std::memcpy(a_exp, E, sizeof(E));
    std::memcpy(a_imp, I, sizeof(I));
    b[0] = dl; b[1] = dl; b[2] = gm;
    return HEVI_OK;
  }
  if (!std::strcmp(name, "ARS343")) {
    // ARS(3,4,3) (Ascher, Ruuth and Spiteri, 1997): gamma is the root in (1/3, 1/2)
    // of 6 g^3 - 18 g^2 + 9 g - 1; the last implicit row is b = (0, b1, b2, gamma)
    // with b1 = -3 g^2 / 2 + 4 g - 1/4, b2 = 3 g^2 / 2 - 5 g + 5/4; the explicit
    // coefficients are the published 10-digit values, a_31 = c_3 - a_32 and
    // a_41 = 1 - a_42 - a_43 (row sums equal to the implicit ones).  Doubles are
    // the correctly rounded values.
    const double g = 0.435866521508459, b1 = 1.20849664917601, b2 = -0.644363170684469;
    const double E[16] = {0, 0, 0, 0,
                          g, 0, 0, 0,
                          0.3212788860542295, 0.3966543747, 0, 0,
                          -0.1058582958, 0.5529291479, 0.5529291479, 0};
    const double I[16] = {0, 0, 0, 0,
                          0, g, 0, 0,
                          0, 0.2820667392457705, g, 0,
                          0, b1, b2, g};
    *s = 4;
    std::memcpy(a_exp, E, sizeof(E));
    std::memcpy(a_imp, I, sizeof(I));
    b[0] = 0.0; b[1] = b1; b[2] = b2; b[3] = g;
    return HEVI_OK;
  }
  if (!std::strcmp(name, "ARK4")) {
    // ARK4(3)6L[2]SA (Kennedy and Carpenter, 2003), the six-stage ARK(5,6,4):
    // gamma = 1/4, c = (0, 1/2, 83/250, 31/50, 17/20, 1), b = last implicit row
    const double q = 0.25;
    const double E[36] = {
        0, 0, 0, 0, 0, 0,
        0.5, 0, 0, 0, 0, 0,
        13861.0 / 62500.0, 6889.0 / 62500.0, 0, 0, 0, 0,
        -116923316275.0 / 2393684061468.0, -2731218467317.0 / 15368042101831.0,
        9408046702089.0 / 11113171139209.0, 0, 0, 0,
        -451086348788.0 / 2902428689909.0, -2682348792572.0 / 7519795681897.0,
        12662868775082.0 / 11960479115383.0, 3355817975965.0 / 11060851509271.0, 0, 0,
        647845179188.0 / 3216320057751.0, 73281519250.0 / 8382639484533.0,
        552539513391.0 / 3454668386233.0, 3354512671639.0 / 8306763924573.0,
        4040.0 / 17871.0, 0};
    const double I[36] = {
        0, 0, 0, 0, 0, 0,
        q, q, 0, 0, 0, 0,
        8611.0 / 62500.0, -1743.0 / 31250.0, q, 0, 0, 0,
        5012029.0 / 34652500.0, -654441.0 / 2922500.0, 174375.0 / 388108.0, q, 0, 0,
        15267082809.0 / 155376265600.0, -71443401.0 / 120774400.0,
        730878875.0 / 902184768.0, 2285395.0 / 8070912.0, q, 0,
        82889.0 / 524892.0, 0, 15625.0 / 83664.0, 69875.0 / 102672.0, -2260.0 / 8211.0, q};
    *s = 6;
    std::memcpy(a_exp, E, sizeof(E));
    std::memcpy(a_imp, I, sizeof(I));
    for (int i = 0; i < 6; ++i) b[i] = I[30 + i];
    return HEVI_OK;
  }
  if (!std::strcmp(name, "ARK3")) {
    // ARK3(2)4L[2]SA (Kennedy and Carpenter, 2003)
    const double g = 1767732205903.0 / 4055673282236.0;
    const double E[16] = {0, 0, 0, 0,
                          1767732205903.0 / 2027836641118.0, 0, 0, 0,
                          5535828885825.0 / 10492691773637.0,
                          788022342437.0 / 10882634858940.0, 0, 0,
                          6485989280629.0 / 16251701735622.0, -4246266847089.0 / 9704473918619.0,
                          10755448449292.0 / 10357097424841.0, 0};
    const double I[16] = {0, 0, 0, 0,
                          g, g, 0, 0,
                          2746238789719.0 / 10658868560708.0,
                          -640167445237.0 / 6845629431997.0, g, 0,
                          1471266399579.0 / 7840856788654.0, -4482444167858.0 / 7529755066697.0,
                          11266239266428.0 / 11593286722821.0, g};
    *s = 4;
    std::memcpy(a_exp, E, sizeof(E));
    std::memcpy(a_imp, I, sizeof(I));
    for (int i = 0; i < 4; ++i) b[i] = I[12 + i];
    return HEVI_OK;
  }
  return HEVI_E_INVALID;
}

hevi_status hevi_sizes(const hevi_shape* shape, hevi_precision prec, size_t* ops_bytes,
                       size_t* factor_bytes, size_t* paper_bytes, size_t* resident_bytes) {
  hevi_status s = check_shape(shape);
  if (s) return s;
  if (prec != HEVI_FP64 && prec != HEVI_FP32_REFINE) return HEVI_E_INVALID;
  const int N = shape->order_N;
  const size_t nz = (size_t)shape->n_elem * N + 1;
  const size_t fsz = prec == HEVI_FP64 ? 8 : 4;
  if (ops_bytes) *ops_bytes = nz * HEVI_NOPS * sizeof(double);
  if (factor_bytes) *factor_bytes = nz * ((4 * N + 1) + 2 * N) * fsz + kFactorPlanes * nz;
  if (resident_bytes) {
    // what a factor object holds per column (factor_storage_bytes of a one-tile
    // shape over its 64 columns): factors, byte planes, scratch, assembly buffer
    HeviShapeDev one{};
    one.N = N;
    one.Ne = shape->n_elem;
    one.nz = (int32_t)nz;
    one.ncols = HEVI_TILE;
    one.ntiles = 1;
    *resident_bytes = factor_storage_bytes(one, prec) / HEVI_TILE;
  }
  if (paper_bytes) {
    const size_t n = 5 * nz;
    const size_t ldab = 3 * 5 * (N + 1) - 2;
    *paper_bytes = n * ldab * 8 + n * 4;
  }
  return HEVI_OK;
}

}  // extern "C"
