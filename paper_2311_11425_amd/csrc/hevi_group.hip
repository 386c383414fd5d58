// hevi_group.hip -- multi-problem persistent kernels for gfx950.
//
// A group of column batches (problems) of different polynomial order N, element
// count and column count is processed by ONE launch per phase: a fixed grid of
// one-wavefront workgroups pulls work items (one 64-column tile of one problem)
// from a device counter until the list is exhausted.  The list is ordered by
// the host (most expensive tiles first), so the tail of the launch is made of
// cheap tiles and the chip stays busy until the end.  Each item runs the same
// per-tile body as the single-problem kernels (hevi_device.h), specialised on
// the problem's order by a switch, so results are those of the single-problem
// path.
//
// Counter protocol: ctr[0] is the next item, ctr[1] counts workgroups that have
// taken their last (failed) item.  The workgroup that brings ctr[1] to the grid
// size resets both to zero, so consecutive launches on one stream (and replays
// of a captured graph) need no memset.
#include <type_traits>

#include "hevi_device.h"

namespace {

__device__ __forceinline__ int64_t grab(uint32_t* ctr) {
  uint32_t v = 0;
  if (threadIdx.x == 0) v = atomicAdd(ctr, 1u);
  return (int64_t)__builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ void finish(uint32_t* ctr) {
  if (threadIdx.x == 0) {
    __threadfence();
    const uint32_t d = atomicAdd(ctr + 1, 1u);
    if (d == gridDim.x - 1) {
      atomicExch(ctr, 0u);
      atomicExch(ctr + 1, 0u);
    }
  }
}

// segment of item (uniform binary search over the m + 1 segment starts)
__device__ __forceinline__ int segment(const HeviSched& s, int64_t item) {
  int lo = 0, hi = s.m - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (s.pstart[mid] <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int NLO, int NHI, class F>
__device__ __forceinline__ void switch_N(int n, F&& f) {
  if constexpr (NLO <= NHI) {
    if (n == NLO) f(std::integral_constant<int, NLO>{});
    else switch_N<NLO + 1, NHI>(n, f);
  }
}

// The persistent loop shared by every phase: body(p, tile) for each item.
template <class Body>
__device__ __forceinline__ void persist(const HeviSched& s, Body&& body) {
  for (;;) {
    const int64_t item = grab(s.ctr);
    if (item >= s.total) break;
    const int j = segment(s, item);
    const int p = __builtin_amdgcn_readfirstlane(s.plist[j]);
    body(p, item - s.pstart[j]);
  }
  finish(s.ctr);
}

template <int NLO, int NHI>
__global__ __launch_bounds__(64) void km_apply(const HeviProbDev* __restrict__ probs,
                                               const HeviCallDev* __restrict__ calls,
                                               HeviSched s) {
  persist(s, [&](int p, int64_t tile) {
    const HeviProbDev& P = probs[p];
    const HeviCallDev& C = calls[p];
    switch_N<NLO, NHI>(P.sh.N, [&](auto n) {
      constexpr int NN = decltype(n)::value;
      b_apply<NN, true>(tile, P.sh, Gll<NN>{}, P.ops, C.x, C.xref, C.out);
    });
  });
}

template <int NLO, int NHI>
__global__ __launch_bounds__(64) void km_factor_assemble(const HeviProbDev* __restrict__ probs,
                                                         HeviSched s) {
  persist(s, [&](int p, int64_t tile) {
    const HeviProbDev& P = probs[p];
    switch_N<NLO, NHI>(P.sh.N, [&](auto n) {
      constexpr int NN = decltype(n)::value;
      b_factor_assemble<NN>(tile, P.sh, Gll<NN>{}, P.lambda, P.ops, P.sbuf);
    });
  });
}

// The band LU of one order (launched per order only), the parts of each tile in turn.
template <int NLO, int NHI, typename FT>
__global__ __launch_bounds__(64) void km_factor_lu(const HeviProbDev* __restrict__ probs,
                                                   HeviSched s) {
  persist(s, [&](int p, int64_t tile) {
    const HeviProbDev& P = probs[p];
    switch_N<NLO, NHI>(P.sh.N, [&](auto n) {
      constexpr int NN = decltype(n)::value;
      for (int part = 0; part < kSplitLanes<NN>; ++part)
        b_factor_lu_split<NN, FT, kSplitLanes<NN>>(tile, part, P.sh, P.sbuf, (FT*)P.U, (FT*)P.L,
                                                   P.piv, P.info);
    });
  });
}

// Assembly and LU in one pass for one order N <= HEVI_FUSED_FACTOR_MAX_N (launched
// per order only): the parts of each tile in turn, each lane's LDS rows reused.
template <int N, typename FT>
__global__ __launch_bounds__(64) void km_factor_fused(const HeviProbDev* __restrict__ probs,
                                                      HeviSched s) {
  constexpr int LPC = kSplitLanes<N>;
  __shared__ double lds[fused_lds_doubles<N>(LPC)];
  persist(s, [&](int p, int64_t tile) {
    const HeviProbDev& P = probs[p];
    for (int part = 0; part < LPC; ++part)
      b_factor_fused_split<N, FT, LPC>(tile, part, P.sh, Gll<N>{}, P.lambda, P.ops, (FT*)P.U,
                                       (FT*)P.L, P.piv, P.info, lds);
  });
}

template <int NLO, int NHI, bool TILT>
__global__ __launch_bounds__(64) void km_stage_rhs(const HeviProbDev* __restrict__ probs,
                                                   const HeviCallDev* __restrict__ calls,
                                                   HeviSched s) {
  persist(s, [&](int p, int64_t tile) {
    const HeviProbDev& P = probs[p];
    const HeviCallDev& C = calls[p];
    switch_N<NLO, NHI>(P.sh.N, [&](auto n) {
      constexpr int NN = decltype(n)::value;
      b_stage_rhs<NN, false, TILT>(tile, P.sh, Gll<NN>{}, P.lambda, P.ops, P.ws, C.E, C.Q, C.out);
    });
  });
}

template <int NLO, int NHI, typename FT, bool REFINE>
__global__ __launch_bounds__(64) void km_stage_bsolve(const HeviProbDev* __restrict__ probs,
                                                      HeviSched s, int max_sweeps,
                                                      double rel_target) {
  persist(s, [&](int p, int64_t tile) {
    const HeviProbDev& P = probs[p];
    switch_N<NLO, NHI>(P.sh.N, [&](auto n) {
      constexpr int NN = decltype(n)::value;
      b_stage_bsolve<NN, FT, REFINE>(tile, P.sh, Gll<NN>{}, P.lambda, P.ops, (const FT*)P.U,
                                     (const FT*)P.L, P.piv, P.ws, max_sweeps, rel_target,
                                     P.info);
    });
  });
}

template <int NLO, int NHI, bool TILT>
__global__ __launch_bounds__(64) void km_stage_update(const HeviProbDev* __restrict__ probs,
                                                      const HeviCallDev* __restrict__ calls,
                                                      HeviSched s) {
  persist(s, [&](int p, int64_t tile) {
    const HeviProbDev& P = probs[p];
    const HeviCallDev& C = calls[p];
    switch_N<NLO, NHI>(P.sh.N, [&](auto n) {
      constexpr int NN = decltype(n)::value;
      b_stage_update<NN, false, TILT>(tile, P.sh, Gll<NN>{}, P.lambda, P.ops, P.ws, C.out, P.info);
    });
  });
}

// FP64 stage solve of a tile in one pass (as k_stage_fused): r/u in LDS
template <int NLO, int NHI, bool TILT>
__global__ __launch_bounds__(64) void km_stage_fused(const HeviProbDev* __restrict__ probs,
                                                     const HeviCallDev* __restrict__ calls,
                                                     HeviSched s) {
  extern __shared__ double ru[];  // [max n_z][64]
  persist(s, [&](int p, int64_t tile) {
    const HeviProbDev& P = probs[p];
    const HeviCallDev& C = calls[p];
    switch_N<NLO, NHI>(P.sh.N, [&](auto n) {
      constexpr int NN = decltype(n)::value;
      b_stage_rhs<NN, true, TILT>(tile, P.sh, Gll<NN>{}, P.lambda, P.ops, P.ws, C.E, C.Q, C.out,
                                  ru);
      __syncthreads();
      band_solve<NN, double, true>((const double*)P.U, (const double*)P.L, P.piv,
                                   plane_size(P.sh), P.ws, tile,
                                   P.sh.nz, (int)threadIdx.x, WS_R, WS_U, ru);
      __syncthreads();
      b_stage_update<NN, true, TILT>(tile, P.sh, Gll<NN>{}, P.lambda, P.ops, P.ws, C.out, P.info,
                                     ru);
      __syncthreads();
    });
  });
}

// out = sum_t coef_t V_t over the 5 n_z values of each column of the tile;
// the same summation order as k_combine.
__global__ __launch_bounds__(64) void km_combine(const HeviProbDev* __restrict__ probs,
                                                 const HeviCallDev* __restrict__ calls,
                                                 HeviSched s) {
  persist(s, [&](int p, int64_t tile) {
    const HeviProbDev& P = probs[p];
    const HeviCallDev& C = calls[p];
    const int64_t c = tile * T + (threadIdx.x & (T - 1));
    if (c >= P.sh.ncols) return;
    const int rows = 5 * P.sh.nz;
    const HeviTerms& V = C.E;
#pragma unroll 4
    for (int r = 0; r < rows; ++r) {
      const size_t i = (size_t)r * P.sh.ncols + c;
      double acc = 0.0;
      for (int t = 0; t < V.n; ++t) acc += V.coef[t] * V.v[t][i];
      C.out[i] = acc;
    }
  });
}

__global__ void k_info_reset_n(HeviDevInfo* info, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    info[i].status = 0;
    info[i].max_sweeps = 0;
    info[i].first_bad = INT64_MAX;
    info[i].n_bad = 0;
    info[i].max_res_bits = 0;
  }
}

template <int NLO, int NHI>
hipError_t launch_range(int phase, int fp32, int tilt, const HeviProbDev* probs,
                        const HeviCallDev* calls,
                        const HeviSched& s, int grid, int max_sweeps, double rel_target,
                        int max_nz, hipStream_t st) {
  const dim3 g((unsigned)grid), b(T);
  switch (phase) {
    case HEVI_PH_APPLY:
      hipLaunchKernelGGL((km_apply<NLO, NHI>), g, b, 0, st, probs, calls, s);
      break;
    case HEVI_PH_FACTOR_ASSEMBLE:  // the factor phases run per order only
      if constexpr (NLO != NHI) return hipErrorInvalidValue;
      else hipLaunchKernelGGL((km_factor_assemble<NLO, NHI>), g, b, 0, st, probs, s);
      break;
    case HEVI_PH_FACTOR_LU:
      if constexpr (NLO != NHI) {
        return hipErrorInvalidValue;
      } else {
        if (fp32) hipLaunchKernelGGL((km_factor_lu<NLO, NHI, float>), g, b, 0, st, probs, s);
        else hipLaunchKernelGGL((km_factor_lu<NLO, NHI, double>), g, b, 0, st, probs, s);
      }
      break;
    case HEVI_PH_FACTOR_FUSED:
      if constexpr (NLO != NHI || NHI > HEVI_FUSED_FACTOR_MAX_N) {
        return hipErrorInvalidValue;
      } else {
        if (fp32) hipLaunchKernelGGL((km_factor_fused<NHI, float>), g, b, 0, st, probs, s);
        else hipLaunchKernelGGL((km_factor_fused<NHI, double>), g, b, 0, st, probs, s);
      }
      break;
    case HEVI_PH_STAGE_RHS:
      if (tilt) hipLaunchKernelGGL((km_stage_rhs<NLO, NHI, true>), g, b, 0, st, probs, calls, s);
      else hipLaunchKernelGGL((km_stage_rhs<NLO, NHI, false>), g, b, 0, st, probs, calls, s);
      break;
    case HEVI_PH_STAGE_BSOLVE:
      if (fp32)
        hipLaunchKernelGGL((km_stage_bsolve<NLO, NHI, float, true>), g, b, 0, st, probs, s,
                           max_sweeps, rel_target);
      else
        hipLaunchKernelGGL((km_stage_bsolve<NLO, NHI, double, false>), g, b, 0, st, probs, s, 0,
                           rel_target);
      break;
    case HEVI_PH_STAGE_UPDATE:
      if (tilt)
        hipLaunchKernelGGL((km_stage_update<NLO, NHI, true>), g, b, 0, st, probs, calls, s);
      else
        hipLaunchKernelGGL((km_stage_update<NLO, NHI, false>), g, b, 0, st, probs, calls, s);
      break;
    case HEVI_PH_STAGE_FUSED:
      // single-order launches only (see the callers)
      if constexpr (NLO != NHI) {
        return hipErrorInvalidValue;
      } else {
        if (fp32 || max_nz > HEVI_FUSED_MAX_NZ) return hipErrorInvalidValue;
        const size_t lds = (size_t)max_nz * T * sizeof(double);
        if (tilt)
          hipLaunchKernelGGL((km_stage_fused<NLO, NHI, true>), g, b, lds, st, probs, calls, s);
        else
          hipLaunchKernelGGL((km_stage_fused<NLO, NHI, false>), g, b, lds, st, probs, calls, s);
      }
      break;
    case HEVI_PH_COMBINE:
      hipLaunchKernelGGL(km_combine, g, b, 0, st, probs, calls, s);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t hevi_launch_multi(int phase, int nlo, int nhi, int fp32, int tilt,
                             const HeviProbDev* probs, const HeviCallDev* calls,
                             const HeviSched& s, int grid, int max_sweeps, double rel_target,
                             int max_nz, hipStream_t st) {
  if (s.total == 0) return hipSuccess;
  if (grid < 1) return hipErrorInvalidValue;
  if (nlo == 1 && nhi == HEVI_MAXN)
    return launch_range<1, HEVI_MAXN>(phase, fp32, tilt, probs, calls, s, grid, max_sweeps,
                                      rel_target, max_nz, st);
  if (nlo != nhi) return hipErrorInvalidValue;
  switch (nlo) {
#define HEVI_ONE_N(n)                                                                          \
  case n:                                                                                      \
    return launch_range<n, n>(phase, fp32, tilt, probs, calls, s, grid, max_sweeps,        \
                              rel_target, max_nz, st);
    HEVI_ONE_N(1) HEVI_ONE_N(2) HEVI_ONE_N(3) HEVI_ONE_N(4)
    HEVI_ONE_N(5) HEVI_ONE_N(6) HEVI_ONE_N(7) HEVI_ONE_N(8)
#undef HEVI_ONE_N
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t hevi_launch_info_reset_n(HeviDevInfo* info, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_info_reset_n, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, st, info, n);
  return hipGetLastError();
}
