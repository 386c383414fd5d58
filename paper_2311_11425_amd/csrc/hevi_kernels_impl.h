// hevi_kernels_impl.h -- single-problem gfx950 kernels of the batched LHEVI
// column solver (one workgroup = one wavefront = one 64-column tile, or a few
// wavefronts per tile for launches of few tiles) and their launch logic, as
// templates over the order N and the equation set (S3: set 3C).  Included by
// hevi_kernels.hip (set 2C) and hevi_kernels3c.hip (set 3C), which instantiate one
// set each and so compile in parallel.  The bodies and the method are described
// in hevi_device.h.
#pragma once
#include "hevi_device.h"

namespace {

// ---------------------------------------------------------------------------
// Single-problem kernels: tile = blockIdx.x

// Streaming kernels take blocks of cw wavefronts (element chunks of one tile,
// cw <= kMaxChunks; see chunks_for).
// CHUNKED instances take the chunk count at run time (a kernel with cw fixed at 1
// keeps the element bounds as constants and needs fewer registers).
template <int N, bool HAS_REF, bool CHUNKED, bool S3>
__global__ __launch_bounds__(CHUNKED ? 64 * kMaxChunks : 64, kStreamWaves<N>) void k_apply(
    HeviShapeDev sh, const double* __restrict__ ops, const double* __restrict__ x,
    const double* __restrict__ xref, double* __restrict__ y, int cw) {
  b_apply<N, HAS_REF, S3>((int64_t)blockIdx.x, sh, Gll<N>{}, ops, x, xref, y, CHUNKED ? cw : 1);
}

template <int N, bool S3>
__global__ __launch_bounds__(64) void k_factor_assemble(HeviShapeDev sh, double lambda,
                                                        const double* __restrict__ ops,
                                                        double* __restrict__ sbuf) {
  b_factor_assemble<N, S3>((int64_t)blockIdx.x, sh, Gll<N>{}, lambda, ops, sbuf);
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

template <int N, typename FT, bool S3, int LPC = kSplitLanes<N>>
__global__ __launch_bounds__(64) void k_factor_fused(HeviShapeDev sh, double lambda,
                                                     const double* __restrict__ ops,
                                                     FT* __restrict__ Ub, FT* __restrict__ Lb,
                                                     uint8_t* __restrict__ piv,
                                                     HeviDevInfo* info) {
  __shared__ double lds[fused_lds_doubles<N>(LPC)];
  b_factor_fused_split<N, FT, LPC, S3>((int64_t)(blockIdx.x / LPC), (int)(blockIdx.x % LPC),
                                       sh, Gll<N>{}, lambda, ops, Ub, Lb, piv, info, lds);
}

template <int N, typename FT, bool S3>
__global__ __launch_bounds__(64) void k_stage_solve(HeviShapeDev sh, double lambda,
                                                    const double* __restrict__ ops,
                                                    const FT* __restrict__ Ub,
                                                    const FT* __restrict__ Lb,
                                                    const uint8_t* __restrict__ piv,
                                                    double* __restrict__ ws, HeviTerms E,
                                                    HeviTerms Q, double* __restrict__ Qi,
                                                    int max_sweeps, double rel_target,
                                                    int full_sweeps, HeviDevInfo* info) {
  b_stage_solve<N, FT, S3>((int64_t)blockIdx.x,
      sh, Gll<N>{}, lambda, ops, Ub, Lb, piv, ws, E, Q, Qi, max_sweeps, rel_target, full_sweeps,
      info);
}

// The FP64 stage solve in one kernel: the three passes run back to back in the
// wavefront that owns the tile, with the reduced right-hand side r and the
// solution u (one array, used in place) in LDS instead of the global scratch.
// The element chunks of the tile's cw wavefronts write and read the one r/u array;
// the band solve runs in the first wavefront between the two barriers.
// The band solve's form in the fused kernel (see band_solve): kChunkedPipe in chunked
// launches (few tiles), kFusedPipe otherwise.
constexpr int kChunkedPipe = 3;
constexpr int kFusedPipe = 1;

template <int N, bool TILT, bool CHUNKED, bool S3>
__global__ __launch_bounds__(CHUNKED ? 64 * kMaxChunks : 64, kStreamWaves<N>) void k_stage_fused(
    HeviShapeDev sh, double lambda, const double* __restrict__ ops,
    const double* __restrict__ Ub, const double* __restrict__ Lb,
    const uint8_t* __restrict__ piv, double* __restrict__ ws, HeviTerms E, HeviTerms Q,
    double* __restrict__ Qi, HeviDevInfo* info, int cw_) {
  extern __shared__ double ru[];  // [n_z][64]
  const int64_t tile = blockIdx.x;
  const int cw = CHUNKED ? cw_ : 1;
  b_stage_rhs<N, true, TILT, S3>(tile, sh, Gll<N>{}, lambda, ops, ws, E, Q, Qi, ru, cw);
  __syncthreads();
  if (threadIdx.x < T)
    band_solve<N, double, true, HEVI_NWS, CHUNKED ? kChunkedPipe : kFusedPipe>(
        Ub, Lb, piv, plane_size(sh), ws, tile, sh.nz, (int)threadIdx.x, WS_R, WS_U, ru);
  __syncthreads();
  b_stage_update<N, true, TILT, S3>(tile, sh, Gll<N>{}, lambda, ops, ws, Qi, info, ru, cw);
}

template <int N, bool TILT, bool CHUNKED, bool S3>
__global__ __launch_bounds__(CHUNKED ? 64 * kMaxChunks : 64, kStreamWaves<N>) void k_stage_rhs(
    HeviShapeDev sh, double lambda, const double* __restrict__ ops, double* __restrict__ ws,
    HeviTerms E, HeviTerms Q, double* __restrict__ Qi, int cw) {
  b_stage_rhs<N, false, TILT, S3>((int64_t)blockIdx.x, sh, Gll<N>{}, lambda, ops, ws, E, Q, Qi,
                              nullptr, CHUNKED ? cw : 1);
}

template <int N, typename FT, bool REFINE, bool S3>
__global__ __launch_bounds__(64, kStreamWaves<N>) void k_stage_bsolve(HeviShapeDev sh, double lambda,
                                                        const double* __restrict__ ops,
                                                        const FT* __restrict__ Ub,
                                                        const FT* __restrict__ Lb,
                                                        const uint8_t* __restrict__ piv,
                                                        double* __restrict__ ws, int max_sweeps,
                                                        double rel_target, HeviDevInfo* info) {
  b_stage_bsolve<N, FT, REFINE, S3>((int64_t)blockIdx.x,
      sh, Gll<N>{}, lambda, ops, Ub, Lb, piv, ws, max_sweeps, rel_target, info);
}

template <int N, bool TILT, bool CHUNKED, bool S3>
__global__ __launch_bounds__(CHUNKED ? 64 * kMaxChunks : 64, kStreamWaves<N>) void k_stage_update(
    HeviShapeDev sh, double lambda, const double* __restrict__ ops, double* __restrict__ ws,
    double* __restrict__ Qi, HeviDevInfo* info, int cw) {
  b_stage_update<N, false, TILT, S3>((int64_t)blockIdx.x, sh, Gll<N>{}, lambda, ops, ws, Qi, info,
                                 nullptr, CHUNKED ? cw : 1);
}

template <template <int, bool> class F, bool S3, typename... A>
hipError_t dispatch_NS(int N, A&&... a) {
  switch (N) {
    case 1: return F<1, S3>::run(a...);
    case 2: return F<2, S3>::run(a...);
    case 3: return F<3, S3>::run(a...);
    case 4: return F<4, S3>::run(a...);
    case 5: return F<5, S3>::run(a...);
    case 6: return F<6, S3>::run(a...);
    case 7: return F<7, S3>::run(a...);
    case 8: return F<8, S3>::run(a...);
    default: return hipErrorInvalidValue;
  }
}

// Element chunks per tile of the streaming kernels.  A launch of few tiles is bound
// by each tile's latency along its elements: below 512 tiles (two per CU) each
// tile is split into up to kMaxChunks wavefronts, never more than it has elements.
// At 10,800 columns (169 tiles of 10 elements) one step took 0.957 ms with one
// wavefront per tile, 0.726 ms with 4 and 0.675 ms with 8.
constexpr int64_t kChunkTiles = 512;
int chunks_for(const HeviShapeDev& sh) {
  if (sh.ntiles >= kChunkTiles) return 1;
  return sh.Ne < kMaxChunks ? sh.Ne : kMaxChunks;
}

template <int N, bool S3>
struct Apply {
  static hipError_t run(const HeviShapeDev& sh, const double* ops,
                        const double* x, const double* xref, double* y, hipStream_t st) {
    const int cw = chunks_for(sh);
    const dim3 g((unsigned)sh.ntiles), b(T * cw);
    if (xref && cw > 1)
      hipLaunchKernelGGL((k_apply<N, true, true, S3>), g, b, 0, st, sh, ops, x, xref, y, cw);
    else if (xref)
      hipLaunchKernelGGL((k_apply<N, true, false, S3>), g, b, 0, st, sh, ops, x, xref, y, 1);
    else
      hipLaunchKernelGGL((k_apply<N, false, false, S3>), dim3((unsigned)sh.ntiles), dim3(T), 0, st,
                         sh, ops, x, xref, y, 1);
    return hipGetLastError();
  }
};

template <int N, bool S3>
struct Factor {
  static hipError_t run(const HeviShapeDev& sh, double lambda, int fp32,
                        const double* ops, double* sbuf, void* Ub, void* Lb, uint8_t* piv,
                        HeviDevInfo* info, hipStream_t st) {
    if constexpr (N > HEVI_FUSED_FACTOR_MAX_N) {
      // assembly into sbuf, then the register-window LU split over kSplitLanes<N>
      // lanes: kSplitLanes<N> workgroups per tile
      const dim3 g((unsigned)sh.ntiles);
      hipLaunchKernelGGL((k_factor_assemble<N, S3>), g, dim3(T * CWF), 0, st, sh, lambda, ops, sbuf);
      const dim3 g4((unsigned)(sh.ntiles * kSplitLanes<N>));
      if (fp32)
        hipLaunchKernelGGL((k_factor_lu_split<N, float>), g4, dim3(T), 0, st, sh, sbuf,
                           (float*)Ub, (float*)Lb, piv, info);
      else
        hipLaunchKernelGGL((k_factor_lu_split<N, double>), g4, dim3(T), 0, st, sh, sbuf,
                           (double*)Ub, (double*)Lb, piv, info);
    } else {
      // assembly and LU in one pass, the window split over kSplitLanes<N> lanes:
      // kSplitLanes<N> workgroups per tile.  A launch of few tiles (as the streaming
      // kernels' chunking) splits the window over 4 lanes, for twice the wavefronts.
      (void)sbuf;
      constexpr int L2 = kSplitLanes<N>;
      if (L2 < 4 && sh.ntiles < kChunkTiles) {
        const dim3 g4((unsigned)(sh.ntiles * 4));
        if (fp32)
          hipLaunchKernelGGL((k_factor_fused<N, float, S3, 4>), g4, dim3(T), 0, st, sh, lambda,
                             ops, (float*)Ub, (float*)Lb, piv, info);
        else
          hipLaunchKernelGGL((k_factor_fused<N, double, S3, 4>), g4, dim3(T), 0, st, sh, lambda,
                             ops, (double*)Ub, (double*)Lb, piv, info);
        return hipGetLastError();
      }
      const dim3 g2((unsigned)(sh.ntiles * L2));
      if (fp32)
        hipLaunchKernelGGL((k_factor_fused<N, float, S3>), g2, dim3(T), 0, st, sh, lambda, ops,
                           (float*)Ub, (float*)Lb, piv, info);
      else
        hipLaunchKernelGGL((k_factor_fused<N, double, S3>), g2, dim3(T), 0, st, sh, lambda, ops,
                           (double*)Ub, (double*)Lb, piv, info);
    }
    return hipGetLastError();
  }
};

template <int N, bool S3>
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
        hipLaunchKernelGGL((k_stage_solve<N, float, S3>), g, b, 0, st, sh, lambda, ops,
                           (const float*)Ub, (const float*)Lb, piv, ws, E, Q, Qi, max_sweeps,
                           rel_target, full_sweeps, info);
      else
        hipLaunchKernelGGL((k_stage_solve<N, double, S3>), g, b, 0, st, sh, lambda, ops,
                           (const double*)Ub, (const double*)Lb, piv, ws, E, Q, Qi, 0, rel_target,
                           full_sweeps, info);
      return hipGetLastError();
    }
    if (!fp32 && sh.nz <= HEVI_FUSED_MAX_NZ) {
      hipLaunchKernelGGL((tilt ? k_stage_fused<N, true, false, S3>
                               : cw > 1 ? k_stage_fused<N, false, true, S3> : k_stage_fused<N, false, false, S3>),
                         g, b4, (size_t)sh.nz * T * sizeof(double), st, sh, lambda, ops,
                         (const double*)Ub, (const double*)Lb, piv, ws, E, Q, Qi, info, cw);
      return hipGetLastError();
    }
    hipLaunchKernelGGL((tilt ? k_stage_rhs<N, true, false, S3>
                             : cw > 1 ? k_stage_rhs<N, false, true, S3> : k_stage_rhs<N, false, false, S3>),
                       g, b4, 0, st, sh, lambda, ops, ws, E, Q, Qi, cw);
    if (fp32)
      hipLaunchKernelGGL((k_stage_bsolve<N, float, true, S3>), g, b, 0, st, sh, lambda, ops,
                         (const float*)Ub, (const float*)Lb, piv, ws, max_sweeps, rel_target, info);
    else
      hipLaunchKernelGGL((k_stage_bsolve<N, double, false, S3>), g, b, 0, st, sh, lambda, ops,
                         (const double*)Ub, (const double*)Lb, piv, ws, 0, rel_target, info);
    hipLaunchKernelGGL((tilt ? k_stage_update<N, true, false, S3>
                             : cw > 1 ? k_stage_update<N, false, true, S3>
                                      : k_stage_update<N, false, false, S3>),
                       g, b4, 0, st, sh, lambda, ops, ws, Qi, info, cw);
    return hipGetLastError();
  }
};

}  // namespace
