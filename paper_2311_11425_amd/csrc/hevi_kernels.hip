// hevi_kernels.hip -- launchers of the single-problem gfx950 kernels of the
// batched LHEVI column solver: the operator build, the set-2C instances of the
// kernels of hevi_kernels_impl.h (set 3C: hevi_kernels3c.hip), the linear
// combination and the report reset.  The per-tile bodies and the method are
// described in hevi_device.h.
#include "hevi_kernels_impl.h"

namespace {

// ---------------------------------------------------------------------------
// a1: compact per-node operator.  Set 2C (s3 == 0): Th0 is Theta0, the flux
// coefficient theta0 = Theta0/rho0 and c_Theta = dP/dTheta from P = P_A (R Theta /
// P_A)^gamma (Appendix A.1, eq. set2c_pressure).  Set 3C: Th0 is the total energy
// E0; at rest P0 = (gamma-1)(E0 - rho0 Phi), Phi = g z (eq. set3c_pressure), the
// flux coefficient is (E0 + P0)/rho0, dP/dE = gamma - 1 and the extra plane
// holds J dP/drho = -J (gamma-1) Phi (eq. set3c_jacobian at U = 0).
template <int N>
__global__ __launch_bounds__(64) void k_build_ops(HeviShapeDev sh, double R, double cp, double g,
                                                  double pA, const double* __restrict__ z,
                                                  const double* __restrict__ J,
                                                  const double* __restrict__ gzeta,
                                                  const double* __restrict__ rho0,
                                                  const double* __restrict__ Th0,
                                                  double* __restrict__ ops, HeviDevInfo* info,
                                                  int32_t* tilted, int s3) {
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
    double th0, cT, P0;
    if (s3) {
      const double phi = g * z[(size_t)k * nc + cc];
      P0 = (gam - 1.0) * (T0 - r0 * phi);
      th0 = (T0 + P0) / r0;
      cT = gam - 1.0;
      ops[pr_offset(sh) + ((size_t)tile * nz + k) * T + lane] = -Jk * cT * phi;
    } else {
      P0 = pA * pow(R * T0 / pA, gam);
      th0 = T0 / r0;
      cT = gam * P0 / T0;
    }
    const double gg = g0 * g0 + g1 * g1 + g2 * g2;
    bad |= !(Jk > 0.0) || !(r0 > 0.0) || !(T0 > 0.0) || !(P0 > 0.0) || !(gg > 0.0) ||
           !isfinite(Jk) || !isfinite(r0) || !isfinite(T0) || !isfinite(gg) || !isfinite(Gn) ||
           !isfinite(cT) || !isfinite(th0);
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
                        int32_t* tilted, int s3, hipStream_t st) {
    hipLaunchKernelGGL(k_build_ops<N>, dim3((unsigned)sh.ntiles), dim3(T), 0, st, sh, R, cp,
                       g, pA, z, J, gz, rho0, Th0, ops, info, tilted, s3);
    return hipGetLastError();
  }
};

}  // namespace

hipError_t hevi_launch_build_ops(const HeviShapeDev& sh, int s3, double R, double cp,
                                 double g, double pA, const double* z, const double* J,
                                 const double* gz, const double* rho0, const double* Th0,
                                 double* ops, HeviDevInfo* info, int32_t* tilted,
                                 hipStream_t st) {
  if (sh.ntiles == 0) return hipSuccess;
  return dispatch_N<BuildOps>(sh.N, sh, R, cp, g, pA, z, J, gz, rho0, Th0, ops, info, tilted,
                              s3, st);
}

hipError_t hevi_launch_apply(const HeviShapeDev& sh, int s3, const double* ops,
                             const double* x, const double* xref, double* y, hipStream_t st) {
  if (sh.ntiles == 0) return hipSuccess;
  if (s3) return hevi_launch_apply_3c(sh, ops, x, xref, y, st);
  return dispatch_NS<Apply, false>(sh.N, sh, ops, x, xref, y, st);
}

hipError_t hevi_launch_factor(const HeviShapeDev& sh, int s3, double lambda, int fp32,
                              const double* ops, double* sbuf, void* Ub, void* Lb, uint8_t* piv,
                              HeviDevInfo* info, hipStream_t st) {
  if (sh.ntiles == 0) return hipSuccess;
  if (s3) return hevi_launch_factor_3c(sh, lambda, fp32, ops, sbuf, Ub, Lb, piv, info, st);
  return dispatch_NS<Factor, false>(sh.N, sh, lambda, fp32, ops, sbuf, Ub, Lb, piv, info, st);
}

hipError_t hevi_launch_stage_solve(const HeviShapeDev& sh, int s3, double lambda, int tilt,
                                   int fp32, const double* ops, const void* Ub, const void* Lb,
                                   const uint8_t* piv, double* ws, const HeviTerms& E,
                                   const HeviTerms& Q, double* Qi, int max_sweeps,
                                   double rel_target, int full_sweeps, HeviDevInfo* info,
                                   hipStream_t st) {
  if (sh.ntiles == 0) return hipSuccess;
  if (s3)
    return hevi_launch_stage_solve_3c(sh, lambda, tilt, fp32, ops, Ub, Lb, piv, ws, E, Q, Qi,
                                      max_sweeps, rel_target, full_sweeps, info, st);
  return dispatch_NS<StageSolve, false>(sh.N, sh, lambda, tilt, fp32, ops, Ub, Lb, piv, ws, E,
                                        Q, Qi, max_sweeps, rel_target, full_sweeps, info, st);
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
