// hevi_internal.h -- launch interface between the C ABI layer (hevi_api.cpp)
// and the gfx950 kernels (hevi_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#define HEVI_MAXN 8       // highest supported polynomial order
#define HEVI_TILE 64      // columns per wavefront: one lane per column
#define HEVI_NOPS 8       // compact per-node operator fields
#define HEVI_NWS 6        // per-node FP64 scratch fields of a stage solve (r, u, Drho u,
                          // DTh u, residual, correction)
#define HEVI_NWS_FULL 21  // ... of the full-system refinement mode (5-field b, x, s added)
#define HEVI_MAXTERMS 16  // max vectors in a linear combination
#define HEVI_MAXSTAGES 8  // max stages of an ARK tableau in a group step

// compact per-node operator fields (tile-interleaved, see hevi_kernels.hip)
enum { OP_MINV = 0, OP_J = 1, OP_JTH = 2, OP_JCT = 3, OP_GX = 4, OP_GY = 5, OP_GZ = 6, OP_PHI = 7 };

// kernel-side report of a call, reduced with device atomics
struct HeviDevInfo {
  int32_t status;          // worst status code seen
  int32_t max_sweeps;      // refinement sweeps of the worst column
  int64_t first_bad;       // lowest flagged column (INT64_MAX if none)
  int64_t n_bad;           // number of flagged columns
  uint64_t max_res_bits;   // bit pattern of the max (non-negative) relative residual
};

struct HeviTerms {         // sum_t coef[t] * v[t] over state vectors
  int32_t n;
  const double* v[HEVI_MAXTERMS];
  double coef[HEVI_MAXTERMS];
};

struct HeviShapeDev {
  int32_t N, Ne, nz;
  int64_t ncols, ntiles;
};

// *tilted becomes nonzero if grad(zeta) is not the same vector (bitwise) at every
// node of some column: the stage solves then need the tangential part of the
// pressure gradient (the TILT kernels).  s3: set 3C (Th0 holds the total energy
// E0; ops then has room for the extra J dP/drho plane, HEVI_NOPS + 1 fields per node).
hipError_t hevi_launch_build_ops(const HeviShapeDev& sh, int s3, double R, double cp,
                                 double g, double pA, const double* z, const double* J,
                                 const double* gz, const double* rho0, const double* Th0,
                                 double* ops, HeviDevInfo* info, int32_t* tilted,
                                 hipStream_t st);

// s3: the operator is of set 3C (instances in hevi_kernels3c.hip)
hipError_t hevi_launch_apply(const HeviShapeDev& sh, int s3, const double* ops,
                             const double* x, const double* xref, double* y, hipStream_t st);

// fp32 != 0 selects FP32 factor storage.  sbuf: FP64 assembly buffer of
// (4N+1) entries per node (may alias Ub when FP64).
hipError_t hevi_launch_factor(const HeviShapeDev& sh, int s3, double lambda, int fp32,
                              const double* ops, double* sbuf, void* Ub, void* Lb, uint8_t* piv,
                              HeviDevInfo* info, hipStream_t st);

// tilt: the operator's columns are not all straight (see hevi_launch_build_ops)
hipError_t hevi_launch_stage_solve(const HeviShapeDev& sh, int s3, double lambda, int tilt,
                                   int fp32, const double* ops, const void* Ub, const void* Lb,
                                   const uint8_t* piv, double* ws, const HeviTerms& E,
                                   const HeviTerms& Q, double* Qi, int max_sweeps,
                                   double rel_target, int full_sweeps, HeviDevInfo* info,
                                   hipStream_t st);

// the set-3C instances (hevi_kernels3c.hip)
hipError_t hevi_launch_apply_3c(const HeviShapeDev& sh, const double* ops, const double* x,
                                const double* xref, double* y, hipStream_t st);
hipError_t hevi_launch_factor_3c(const HeviShapeDev& sh, double lambda, int fp32,
                                 const double* ops, double* sbuf, void* Ub, void* Lb,
                                 uint8_t* piv, HeviDevInfo* info, hipStream_t st);
hipError_t hevi_launch_stage_solve_3c(const HeviShapeDev& sh, double lambda, int tilt, int fp32,
                                      const double* ops, const void* Ub, const void* Lb,
                                      const uint8_t* piv, double* ws, const HeviTerms& E,
                                      const HeviTerms& Q, double* Qi, int max_sweeps,
                                      double rel_target, int full_sweeps, HeviDevInfo* info,
                                      hipStream_t st);

// LHEVI-PS (hevi_ps.hip): the full 5 n_z band, one wavefront per column, N <= 5.
// Operators hold the velocity planes of the linearisation state after the eight
// fields (HEVI_NOPS + 3 planes); factors U [ncols][n][WS], L [ncols][n][KLS], then four
// byte planes [ncols][n] (pivot offsets, row-scale exponents, U and L extents), n = 5 n_z,
// KLS = hevi_ps_lower_width(N), WS = hevi_ps_band_width(N) (the band widths rounded up to
// whole 128-byte lines).
#define HEVI_PS_MAXN 5
int hevi_ps_band_width(int N);
int hevi_ps_lower_width(int N);
hipError_t hevi_launch_ps_factor(const HeviShapeDev& sh, double lambda, const double* ops,
                                 double* U, double* L, uint8_t* piv, HeviDevInfo* info,
                                 hipStream_t st);
hipError_t hevi_launch_ps_stage(const HeviShapeDev& sh, const double* ops, const double* U,
                                const double* L, const uint8_t* piv, const HeviTerms& E,
                                const HeviTerms& Q, double* Qi, HeviDevInfo* info,
                                hipStream_t st);
hipError_t hevi_launch_apply_ps(const HeviShapeDev& sh, const double* ops, const double* x,
                                const double* xref, double* y, hipStream_t st);
hipError_t hevi_launch_ps_state(const HeviShapeDev& sh, double R, double cp, double pA,
                                const double* rho0, const double* U0, const double* Th0,
                                double* ops, HeviDevInfo* info, hipStream_t st);

// NHEVI-LU: the nonlinear set-2C vertical operator V(q) (any order), and the Newton
// measure max ||dq_v|| / ||q_v - q^n_v|| into info->max_res_bits
hipError_t hevi_launch_vertical_op(const HeviShapeDev& sh, double R, double cp, double pA,
                                   const double* ops, const double* q, double* V,
                                   hipStream_t st);
hipError_t hevi_launch_newton_rel(const HeviShapeDev& sh, const double* dq, const double* q,
                                  const double* qn, HeviDevInfo* info, hipStream_t st);

hipError_t hevi_launch_combine(int64_t n, const HeviTerms& V, double* out, hipStream_t st);

hipError_t hevi_launch_info_reset(HeviDevInfo* info, hipStream_t st);

// ---------------------------------------------------------------------------
// Multi-problem persistent launches (hevi_group.hip).  A launch covers several
// problems (column batches of possibly different order N, element count and
// column count); its work items are the 64-column tiles of all of them.

// one problem: shape, operator and factor storage (device-resident table)
struct HeviProbDev {
  HeviShapeDev sh;
  int32_t fp32;           // factors stored in FP32
  int32_t tilt;           // host use: the operator has columns that are not straight
  double lambda;
  const double* ops;
  double* sbuf;           // FP64 assembly buffer (aliases U for FP64 factors)
  void* U;
  void* L;
  uint8_t* piv;
  double* ws;             // stage-solve scratch
  HeviDevInfo* info;      // per-problem report
};

// operands of one call for one problem
struct HeviCallDev {
  HeviTerms E;            // stage solve: q^E terms; combine: the terms
  HeviTerms Q;            // stage solve: previous stage values and c_j
  const double* x;        // apply: x
  const double* xref;     // apply: x_ref (required)
  double* out;            // apply: y; stage solve: Q_i; combine: output
};

// work list of one launch: segment j is problem plist[j] with items
// pstart[j] .. pstart[j+1]-1 (its tiles in order)
struct HeviSched {
  const int32_t* plist;
  const int64_t* pstart;  // m + 1 entries, pstart[0] = 0, pstart[m] = total
  int32_t m;
  int64_t total;
  uint32_t* ctr;          // {next item, finished workgroups}; zero before a launch, zero after it
};

enum HeviPhase {
  HEVI_PH_APPLY = 0,
  HEVI_PH_FACTOR_ASSEMBLE = 1,
  HEVI_PH_FACTOR_LU = 2,
  HEVI_PH_STAGE_RHS = 3,
  HEVI_PH_STAGE_BSOLVE = 4,
  HEVI_PH_STAGE_UPDATE = 5,
  HEVI_PH_COMBINE = 6,
  HEVI_PH_STAGE_FUSED = 7,   // FP64 rhs + band solve + update, r/u in LDS
  HEVI_PH_FACTOR_FUSED = 8,  // assembly + LU in one pass (N <= HEVI_FUSED_FACTOR_MAX_N)
  HEVI_NPHASES = 9
};

// The fused stage kernel holds n_z doubles per column of its 64-column tile in LDS
// (n_z * 512 bytes per one-wave workgroup).  It beats the three separate kernels while
// three such workgroups fit in a CU's 160 KiB of LDS (n_z <= 106): with only two, half
// of the CU's SIMDs sit idle and its bandwidth-bound RHS part runs ~2.4x slower (1.6M
// uneven columns, N 3..7: 16.0/26.7/37.0 ms per stage fused at n_z 113, against
// 14.0/18.5/23.0 ms for the three kernels).
#define HEVI_FUSED_MAX_NZ 106

// Orders whose factorisation runs as one pass (assembly into LDS inside the LU
// wavefront); above, the element data would not fit beside the LU window and
// the assembly is a kernel of its own.
#define HEVI_FUSED_FACTOR_MAX_N 6

// One persistent launch of `phase` with `grid` workgroups of one wavefront.
// nlo..nhi: the orders the kernel is compiled for ((n, n) for n = 1..8, or
// (1, HEVI_MAXN)); every problem in the schedule must have nlo <= N <= nhi.
// fp32 / refine select the factor type and the reduced refinement of the
// stage solve (max_sweeps, rel_target).  tilt: some problem of the launch has
// columns that are not straight (the stage phases then use the TILT kernels).
// max_nz: the largest n_z of the launch's problems (sizes the LDS of
// HEVI_PH_STAGE_FUSED).
hipError_t hevi_launch_multi(int phase, int nlo, int nhi, int fp32, int tilt,
                             const HeviProbDev* probs, const HeviCallDev* calls,
                             const HeviSched& s, int grid, int max_sweeps, double rel_target,
                             int max_nz, hipStream_t st);

hipError_t hevi_launch_info_reset_n(HeviDevInfo* info, int n, hipStream_t st);
