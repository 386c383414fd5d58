// hevi_kernels3c.hip -- the set-3C (total energy) instances of the single-problem
// kernels of hevi_kernels_impl.h, in a file of their own so that they compile in
// parallel with the set-2C ones (hevi_kernels.hip).
#include "hevi_kernels_impl.h"

hipError_t hevi_launch_apply_3c(const HeviShapeDev& sh, const double* ops, const double* x,
                                const double* xref, double* y, hipStream_t st) {
  if (sh.ntiles == 0) return hipSuccess;
  return dispatch_NS<Apply, true>(sh.N, sh, ops, x, xref, y, st);
}

hipError_t hevi_launch_factor_3c(const HeviShapeDev& sh, double lambda, int fp32,
                                 const double* ops, double* sbuf, void* Ub, void* Lb,
                                 uint8_t* piv, HeviDevInfo* info, hipStream_t st) {
  if (sh.ntiles == 0) return hipSuccess;
  return dispatch_NS<Factor, true>(sh.N, sh, lambda, fp32, ops, sbuf, Ub, Lb, piv, info, st);
}

hipError_t hevi_launch_stage_solve_3c(const HeviShapeDev& sh, double lambda, int tilt, int fp32,
                                      const double* ops, const void* Ub, const void* Lb,
                                      const uint8_t* piv, double* ws, const HeviTerms& E,
                                      const HeviTerms& Q, double* Qi, int max_sweeps,
                                      double rel_target, int full_sweeps, HeviDevInfo* info,
                                      hipStream_t st) {
  if (sh.ntiles == 0) return hipSuccess;
  return dispatch_NS<StageSolve, true>(sh.N, sh, lambda, tilt, fp32, ops, Ub, Lb, piv, ws, E, Q,
                                       Qi, max_sweeps, rel_target, full_sweeps, info, st);
}
