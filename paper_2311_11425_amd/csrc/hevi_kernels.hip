// hevi_kernels.hip -- single-problem gfx950 kernels of the batched LHEVI column
// solver (one workgroup = one wavefront = one 64-column tile) and their launchers.
// The per-tile bodies and the method are described in hevi_device.h.
#include "hevi_device.h"

namespace {

// ---------------------------------------------------------------------------
// a1: compact per-node operator
template <int N>
__global__ __launch_bounds__(64) void k_build_ops(HeviShapeDev sh, double R, double cp, double g,
                                                  double pA, const double* __restrict__ z,
                                                  const double* __restrict__ J,
                                                  const double* __restrict__ gzeta,
                                                  const double* __restrict__ rho0,
                                                  const double* __restrict__ Th0,
                                                  double* __restrict__ ops, HeviDevInfo* info,
                                                  int32_t* tilted) {
  const Gll<N> tab{};
  const int lane = threadIdx.x;
  const int64_t tile = blockIdx.x;
  const int64_t c = tile * T + lane;
  const bool valid = c < sh.ncols;
  const int64_t cc = valid ? c : sh.ncols - 1;
  const int nz = sh.nz, Ne = sh.Ne;
  const int64_t nc = sh.ncols;
  const double gam = cp / (cp - R);
  bool bad = false;
  bool bent = false;  // grad(zeta) not the same vector at every node of the column
  double pg0 = 0.0, pg1 = 0.0, pg2 = 0.0;
  for (int k = 0; k < nz; ++k) {
    const double Jk = J[(size_t)k * nc + cc];
    const double r0 = rho0[(size_t)k * nc + cc];
    const double T0 = Th0[(size_t)k * nc + cc];
    const double g0 = gzeta[cix(nz, nc, 0, k, cc)];
    const double g1 = gzeta[cix(nz, nc, 1, k, cc)];
    const double g2 = gzeta[cix(nz, nc, 2, k, cc)];
    if (k > 0) bent = bent || g0 != pg0 || g1 != pg1 || g2 != pg2;
    pg0 = g0; pg1 = g1; pg2 = g2;
    // lumped mass and gravity numerator, summed over the (one or two)
    // elements that contain node k
    double M = 0.0, Gn = 0.0;
    const int i = k % N, e = k / N;
    for (int side = 0; side < 2; ++side) {
      int ee, ii;
      if (i != 0) {
        if (side) break;
        ee = e; ii = i;
      } else if (side == 0) {
        if (e == 0) continue;
        ee = e - 1; ii = N;
      } else {
        if (e >= Ne) continue;
        ee = e; ii = 0;
      }
      double dz = 0.0;
#pragma unroll
      for (int j = 0; j <= N; ++j)
        dz += tab.D[ii * (N + 1) + j] * z[(size_t)(ee * N + j) * nc + cc];
      M += tab.w[ii] * Jk;
      Gn += tab.w[ii] * Jk * g * dz;
    }
    const double P0 = pA * pow(R * T0 / pA, gam);
    const double th0 = T0 / r0;
    const double cT = gam * P0 / T0;
    const double gg = g0 * g0 + g1 * g1 + g2 * g2;
    bad |= !(Jk > 0.0) || !(r0 > 0.0) || !(T0 > 0.0) || !(gg > 0.0) || !isfinite(Jk) ||
           !isfinite(r0) || !isfinite(T0) || !isfinite(gg) || !isfinite(Gn) || !isfinite(cT);
    double* o = ops + tix(tile, nz, k, HEVI_NOPS, 0, lane);
    o[OP_MINV * T] = 1.0 / M;
    o[OP_J * T] = Jk;
    o[OP_JTH * T] = Jk * th0;
    o[OP_JCT * T] = Jk * cT;
    o[OP_GX * T] = g0;
    o[OP_GY * T] = g1;
    o[OP_GZ * T] = g2;
    o[OP_PHI * T] = Gn / M;
  }
  if (bad && valid) flag(info, 1 /*HEVI_E_INVALID*/, c);
  if (__any(bent && valid) && lane == 0) atomicOr(tilted, 1);
}

// ---------------------------------------------------------------------------
// Single-problem kernels: tile = blockIdx.x

// Streaming kernels take blocks of cw wavefronts (element chunks of one tile,
// cw <= kMaxChunks; see chunks_for).
// CHUNKED instances take the chunk count at run time (a kernel with cw fixed at 1
// keeps the element bounds as constants and needs fewer registers).
template <int N, bool HAS_REF, bool CHUNKED>
__global__ __launch_bounds__(CHUNKED ? 64 * kMaxChunks : 64, kStreamWaves<N>) void k_apply(
    HeviShapeDev sh, const double* __restrict__ ops, const double* __restrict__ x,
    const double* __restrict__ xref, double* __restrict__ y, int cw) {
  b_apply<N, HAS_REF>((int64_t)blockIdx.x, sh, Gll<N>{}, ops, x, xref, y, CHUNKED ? cw : 1);
}

template <int N>
__global__ __launch_bounds__(64) void k_factor_assemble(HeviShapeDev sh, double lambda,
                                                        const double* __restrict__ ops,
                                                        double* __restrict__ sbuf) {
  b_factor_assemble<N>((int64_t)blockIdx.x, sh, Gll<N>{}, lambda, ops, sbuf);
}

template <int N, typename FT>
__global__ __launch_bounds__(64) void k_factor_lu_split(HeviShapeDev sh, const double* sbuf,
                                                        FT* Ub, FT* __restrict__ Lb,
                                                        uint8_t* __restrict__ piv,
                                                        HeviDevInfo* info) {
  b_factor_lu_split<N, FT, kSplitLanes<N>>((int64_t)(blockIdx.x / kSplitLanes<N>),
                                           (int)(blockIdx.x % kSplitLanes<N>), sh, sbuf, Ub, Lb,
                                           piv, info);
}

template <int N, typename FT>
__global__ __launch_bounds__(64) void k_factor_fused(HeviShapeDev sh, double lambda,
                                                     const double* __restrict__ ops,
                                                     FT* __restrict__ Ub, FT* __restrict__ Lb,
                                                     uint8_t* __restrict__ piv,
                                                     HeviDevInfo* info) {
  constexpr int LPC = kSplitLanes<N>;
  __shared__ double lds[fused_lds_doubles<N>(LPC)];
  b_factor_fused_split<N, FT, LPC>((int64_t)(blockIdx.x / LPC), (int)(blockIdx.x % LPC), sh,
                                   Gll<N>{}, lambda, ops, Ub, Lb, piv, info, lds);
}

template <int N, typename FT>
__global__ __launch_bounds__(64) void k_stage_solve(HeviShapeDev sh, double lambda,
                                                    const double* __restrict__ ops,
                                                    const FT* __restrict__ Ub,
                                                    const FT* __restrict__ Lb,
                                                    const uint8_t* __restrict__ piv,
                                                    double* __restrict__ ws, HeviTerms E,
                                                    HeviTerms Q, double* __restrict__ Qi,
                                                    int max_sweeps, double rel_target,
                                                    int full_sweeps, HeviDevInfo* info) {
  b_stage_solve<N, FT>((int64_t)blockIdx.x,
      sh, Gll<N>{}, lambda, ops, Ub, Lb, piv, ws, E, Q, Qi, max_sweeps, rel_target, full_sweeps,
      info);
}

// The FP64 stage solve in one kernel: the three passes run back to back in the
// wavefront that owns the tile, with the reduced right-hand side r and the
// solution u (one array, used in place) in LDS instead of the global scratch.
// The element chunks of the tile's cw wavefronts write and read the one r/u array;
// the band solve runs in the first wavefront between the two barriers.
template <int N, bool TILT, bool CHUNKED>
__global__ __launch_bounds__(CHUNKED ? 64 * kMaxChunks : 64, kStreamWaves<N>) void k_stage_fused(
    HeviShapeDev sh, double lambda, const double* __restrict__ ops,
    const double* __restrict__ Ub, const double* __restrict__ Lb,
    const uint8_t* __restrict__ piv, double* __restrict__ ws, HeviTerms E, HeviTerms Q,
    double* __restrict__ Qi, HeviDevInfo* info, int cw_) {
  extern __shared__ double ru[];  // [n_z][64]
  const int64_t tile = blockIdx.x;
  const int cw = CHUNKED ? cw_ : 1;
  b_stage_rhs<N, true, TILT>(tile, sh, Gll<N>{}, lambda, ops, ws, E, Q, Qi, ru, cw);
  __syncthreads();
  if (threadIdx.x < T)
    band_solve<N, double, true>(Ub, Lb, piv, plane_size(sh), ws, tile, sh.nz, (int)threadIdx.x,
                                WS_R, WS_U, ru);
  __syncthreads();
  b_stage_update<N, true, TILT>(tile, sh, Gll<N>{}, lambda, ops, ws, Qi, info, ru, cw);
}

template <int N, bool TILT, bool CHUNKED>
__global__ __launch_bounds__(CHUNKED ? 64 * kMaxChunks : 64, kStreamWaves<N>) void k_stage_rhs(
    HeviShapeDev sh, double lambda, const double* __restrict__ ops, double* __restrict__ ws,
    HeviTerms E, HeviTerms Q, double* __restrict__ Qi, int cw) {
  b_stage_rhs<N, false, TILT>((int64_t)blockIdx.x, sh, Gll<N>{}, lambda, ops, ws, E, Q, Qi,
                              nullptr, CHUNKED ? cw : 1);
}

template <int N, typename FT, bool REFINE>
__global__ __launch_bounds__(64, kStreamWaves<N>) void k_stage_bsolve(HeviShapeDev sh, double lambda,
                                                        const double* __restrict__ ops,
                                                        const FT* __restrict__ Ub,
                                                        const FT* __restrict__ Lb,
                                                        const uint8_t* __restrict__ piv,
                                                        double* __restrict__ ws, int max_sweeps,
                                                        double rel_target, HeviDevInfo* info) {
  b_stage_bsolve<N, FT, REFINE>((int64_t)blockIdx.x,
      sh, Gll<N>{}, lambda, ops, Ub, Lb, piv, ws, max_sweeps, rel_target, info);
}

template <int N, bool TILT, bool CHUNKED>
__global__ __launch_bounds__(CHUNKED ? 64 * kMaxChunks : 64, kStreamWaves<N>) void k_stage_update(
    HeviShapeDev sh, double lambda, const double* __restrict__ ops, double* __restrict__ ws,
    double* __restrict__ Qi, HeviDevInfo* info, int cw) {
  b_stage_update<N, false, TILT>((int64_t)blockIdx.x, sh, Gll<N>{}, lambda, ops, ws, Qi, info,
                                 nullptr, CHUNKED ? cw : 1);
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_combine(int64_t n, HeviTerms V, double* __restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    double s = 0.0;
    for (int t = 0; t < V.n; ++t) s += V.coef[t] * __builtin_nontemporal_load(V.v[t] + i);
    __builtin_nontemporal_store(s, out + i);
  }
}

__global__ void k_info_reset(HeviDevInfo* info) {
  if (threadIdx.x == 0) {
    info->status = 0;
    info->max_sweeps = 0;
    info->first_bad = INT64_MAX;
    info->n_bad = 0;
    info->max_res_bits = 0;
  }
}

template <template <int> class F, typename... A>
hipError_t dispatch_N(int N, A&&... a) {
  switch (N) {
    case 1: return F<1>::run(a...);
    case 2: return F<2>::run(a...);
    case 3: return F<3>::run(a...);
    case 4: return F<4>::run(a...);
    case 5: return F<5>::run(a...);
    case 6: return F<6>::run(a...);
    case 7: return F<7>::run(a...);
    case 8: return F<8>::run(a...);
    default: return hipErrorInvalidValue;
  }
}

template <int N>
struct BuildOps {
  static hipError_t run(const HeviShapeDev& sh, double R, double cp, double g,
                        double pA, const double* z, const double* J, const double* gz,
                        const double* rho0, const double* Th0, double* ops, HeviDevInfo* info,
                        int32_t* tilted, hipStream_t st) {
    hipLaunchKernelGGL(k_build_ops<N>, dim3((unsigned)sh.ntiles), dim3(T), 0, st, sh, R, cp,
                       g, pA, z, J, gz, rho0, Th0, ops, info, tilted);
    return hipGetLastError();
  }
};

// Element chunks per tile of the streaming kernels.  A launch of few tiles is bound
// by each tile's latency along its elements: below 512 tiles (two per CU) each
// tile is split into up to kMaxChunks wavefronts, never more than it has elements.
// At 10,800 columns (169 tiles of 10 elements) one step took 0.957 ms with one
// wavefront per tile, 0.726 ms with 4 and 0.675 ms with 8.
int chunks_for(const HeviShapeDev& sh) {
  if (sh.ntiles >= 512) return 1;
  return sh.Ne < kMaxChunks ? sh.Ne : kMaxChunks;
}

template <int N>
struct Apply {
  static hipError_t run(const HeviShapeDev& sh, const double* ops,
                        const double* x, const double* xref, double* y, hipStream_t st) {
    const int cw = chunks_for(sh);
    const dim3 g((unsigned)sh.ntiles), b(T * cw);
    if (xref && cw > 1)
      hipLaunchKernelGGL((k_apply<N, true, true>), g, b, 0, st, sh, ops, x, xref, y, cw);
    else if (xref)
      hipLaunchKernelGGL((k_apply<N, true, false>), g, b, 0, st, sh, ops, x, xref, y, 1);
    else
      hipLaunchKernelGGL((k_apply<N, false, false>), dim3((unsigned)sh.ntiles), dim3(T), 0, st,
                         sh, ops, x, xref, y, 1);
    return hipGetLastError();
  }
};

template <int N>
struct Factor {
  static hipError_t run(const HeviShapeDev& sh, double lambda, int fp32,
                        const double* ops, double* sbuf, void* Ub, void* Lb, uint8_t* piv,
                        HeviDevInfo* info, hipStream_t st) {
    if constexpr (N > HEVI_FUSED_FACTOR_MAX_N) {
      // assembly into sbuf, then the register-window LU split over kSplitLanes<N>
      // lanes: kSplitLanes<N> workgroups per tile
      const dim3 g((unsigned)sh.ntiles);
      hipLaunchKernelGGL(k_factor_assemble<N>, g, dim3(T * CWF), 0, st, sh, lambda, ops, sbuf);
      const dim3 g4((unsigned)(sh.ntiles * kSplitLanes<N>));
      if (fp32)
        hipLaunchKernelGGL((k_factor_lu_split<N, float>), g4, dim3(T), 0, st, sh, sbuf,
                           (float*)Ub, (float*)Lb, piv, info);
      else
        hipLaunchKernelGGL((k_factor_lu_split<N, double>), g4, dim3(T), 0, st, sh, sbuf,
                           (double*)Ub, (double*)Lb, piv, info);
    } else {
      // assembly and LU in one pass, the window split over kSplitLanes<N> lanes:
      // kSplitLanes<N> workgroups per tile
      (void)sbuf;
      const dim3 g2((unsigned)(sh.ntiles * kSplitLanes<N>));
      if (fp32)
        hipLaunchKernelGGL((k_factor_fused<N, float>), g2, dim3(T), 0, st, sh, lambda, ops,
                           (float*)Ub, (float*)Lb, piv, info);
      else
        hipLaunchKernelGGL((k_factor_fused<N, double>), g2, dim3(T), 0, st, sh, lambda, ops,
                           (double*)Ub, (double*)Lb, piv, info);
    }
    return hipGetLastError();
  }
};

template <int N>
struct StageSolve {
  static hipError_t run(const HeviShapeDev& sh, double lambda, int tilt, int fp32,
                        const double* ops, const void* Ub, const void* Lb, const uint8_t* piv,
                        double* ws, const HeviTerms& E, const HeviTerms& Q, double* Qi,
                        int max_sweeps, double rel_target, int full_sweeps, HeviDevInfo* info,
                        hipStream_t st) {
    // element chunks for launches of few tiles (straight columns; the TILT kernels run
    // one wavefront per tile)
    const int cw = tilt ? 1 : chunks_for(sh);
    const dim3 g((unsigned)sh.ntiles), b(T), b4(T * cw);
    if (full_sweeps > 0) {
      // accuracy mode: one kernel with the full-system refinement sweeps
      if (fp32)
        hipLaunchKernelGGL((k_stage_solve<N, float>), g, b, 0, st, sh, lambda, ops,
                           (const float*)Ub, (const float*)Lb, piv, ws, E, Q, Qi, max_sweeps,
                           rel_target, full_sweeps, info);
      else
        hipLaunchKernelGGL((k_stage_solve<N, double>), g, b, 0, st, sh, lambda, ops,
                           (const double*)Ub, (const double*)Lb, piv, ws, E, Q, Qi, 0, rel_target,
                           full_sweeps, info);
      return hipGetLastError();
    }
    if (!fp32 && sh.nz <= HEVI_FUSED_MAX_NZ) {
      hipLaunchKernelGGL((tilt ? k_stage_fused<N, true, false>
                               : cw > 1 ? k_stage_fused<N, false, true> : k_stage_fused<N, false, false>),
                         g, b4, (size_t)sh.nz * T * sizeof(double), st, sh, lambda, ops,
                         (const double*)Ub, (const double*)Lb, piv, ws, E, Q, Qi, info, cw);
      return hipGetLastError();
    }
    hipLaunchKernelGGL((tilt ? k_stage_rhs<N, true, false>
                             : cw > 1 ? k_stage_rhs<N, false, true> : k_stage_rhs<N, false, false>),
                       g, b4, 0, st, sh, lambda, ops, ws, E, Q, Qi, cw);
    if (fp32)
      hipLaunchKernelGGL((k_stage_bsolve<N, float, true>), g, b, 0, st, sh, lambda, ops,
                         (const float*)Ub, (const float*)Lb, piv, ws, max_sweeps, rel_target, info);
    else
      hipLaunchKernelGGL((k_stage_bsolve<N, double, false>), g, b, 0, st, sh, lambda, ops,
                         (const double*)Ub, (const double*)Lb, piv, ws, 0, rel_target, info);
    hipLaunchKernelGGL((tilt ? k_stage_update<N, true, false>
                             : cw > 1 ? k_stage_update<N, false, true>
                                      : k_stage_update<N, false, false>),
                       g, b4, 0, st, sh, lambda, ops, ws, Qi, info, cw);
    return hipGetLastError();
  }
};

}  // namespace

hipError_t hevi_launch_build_ops(const HeviShapeDev& sh, double R, double cp,
                                 double g, double pA, const double* z, const double* J,
                                 const double* gz, const double* rho0, const double* Th0,
                                 double* ops, HeviDevInfo* info, int32_t* tilted,
                                 hipStream_t st) {
  if (sh.ntiles == 0) return hipSuccess;
  return dispatch_N<BuildOps>(sh.N, sh, R, cp, g, pA, z, J, gz, rho0, Th0, ops, info, tilted,
                              st);
}

hipError_t hevi_launch_apply(const HeviShapeDev& sh, const double* ops,
                             const double* x, const double* xref, double* y, hipStream_t st) {
  if (sh.ntiles == 0) return hipSuccess;
  return dispatch_N<Apply>(sh.N, sh, ops, x, xref, y, st);
}

hipError_t hevi_launch_factor(const HeviShapeDev& sh, double lambda, int fp32,
                              const double* ops, double* sbuf, void* Ub, void* Lb, uint8_t* piv,
                              HeviDevInfo* info, hipStream_t st) {
  if (sh.ntiles == 0) return hipSuccess;
  return dispatch_N<Factor>(sh.N, sh, lambda, fp32, ops, sbuf, Ub, Lb, piv, info, st);
}

hipError_t hevi_launch_stage_solve(const HeviShapeDev& sh, double lambda, int tilt,
                                   int fp32, const double* ops, const void* Ub, const void* Lb,
                                   const uint8_t* piv, double* ws, const HeviTerms& E,
                                   const HeviTerms& Q, double* Qi, int max_sweeps,
                                   double rel_target, int full_sweeps, HeviDevInfo* info,
                                   hipStream_t st) {
  if (sh.ntiles == 0) return hipSuccess;
  return dispatch_N<StageSolve>(sh.N, sh, lambda, tilt, fp32, ops, Ub, Lb, piv, ws, E, Q, Qi,
                                max_sweeps, rel_target, full_sweeps, info, st);
}

hipError_t hevi_launch_combine(int64_t n, const HeviTerms& V, double* out, hipStream_t st) {
  if (n == 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_combine, dim3((unsigned)blocks), dim3(256), 0, st, n, V, out);
  return hipGetLastError();
}

hipError_t hevi_launch_info_reset(HeviDevInfo* info, hipStream_t st) {
  hipLaunchKernelGGL(k_info_reset, dim3(1), dim3(64), 0, st, info);
  return hipGetLastError();
}
