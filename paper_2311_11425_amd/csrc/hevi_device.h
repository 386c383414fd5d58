// hevi_device.h -- device code of the batched LHEVI column solver for gfx950:
// per-tile bodies of every kernel, shared by the single-problem kernels
// (hevi_kernels.hip) and the multi-problem persistent kernels (hevi_group.hip).
//
// Mapping.  One lane owns one vertical column; a 64-lane wavefront owns a tile
// of 64 consecutive columns (the LU kernels split a column over lanes).  The caller's arrays are column-fastest
// struct-of-arrays, so every per-node access of a wavefront is one coalesced
// 512-byte FP64 request.  Library-owned arrays (compact operator, factors,
// scratch) are tile-interleaved: element (tile, node k, field f, lane) sits at
// ((tile * nz + k) * F + f) * 64 + lane, so a wavefront streams one contiguous
// region per tile.
//
// Method (Giraldo et al., arXiv 2311.11425).  L_z is the set-2C vertical
// operator (Appendix A.2) linearised about a state at rest and discretised as
// in Sec. 3 / Appendix A.3: per element, strong derivative w_i D_ij J_j f_j for
// the momentum and rho-theta rows, weak derivative -w_j D_ji J_j f_j for the
// continuity row, direct-stiffness summation along the column, division by the
// lumped mass; gravity rho dPhi/dzeta grad(zeta) in the momentum rows; the
// momentum rows of the bottom and top nodes are replaced by the rigid lid.
// With u = grad(zeta).U (contravariant vertical momentum):
//   (L x)_rho   = Drho u      = M^-1 sum_e sum_j w_j D_ji J_j u_j
//   (L x)_Theta = DTh u       = -M^-1 sum_e w_i sum_j D_ij (J theta0)_j u_j
//   (L x)_U     = PG(Theta) - Phi' grad(zeta) rho
//               = -M^-1 sum_e w_i sum_j D_ij (J c_Theta grad(zeta))_j Theta_j
//                 - Phi'_k grad(zeta)_k rho_k                 (interior nodes)
// The rho-rho and Theta-Theta blocks of A = I - Lambda L_z are identities, so
// eliminating rho, Theta and the tangential momentum exactly leaves
//   S u = r,  S = I - Lambda^2 grad(zeta).(PG DTh - Phi' grad(zeta) Drho),
//   r = grad(zeta).(b_U + Lambda (PG b_Theta - Phi' grad(zeta) b_rho)),
// a band matrix of half-bandwidth 2N in u (identity rows at the rigid-lid
// nodes, where u = 0).  Back-substitution recovers
//   x_rho = b_rho + Lambda Drho u,  x_Theta = b_Theta + Lambda DTh u,
//   x_U   = b_U + Lambda (PG x_Theta - Phi' grad(zeta) x_rho).
// S is LU-factored with partial pivoting (band LU, the paper's LAPACK scheme
// of Sec. 4.2.3 applied to the reduced matrix).
//
// Set 3C (total energy E in place of Theta; Appendix A.1 eq. set3c and the
// Jacobian eq. set3c_jacobian at rest) has the same structure: its E row is DTh
// with (J theta0) replaced by J (E0 + P0)/rho0, and its linearised pressure
// (gamma-1)(E - Phi rho) adds dP/drho = -(gamma-1) Phi, a rho column in the pressure
// gradient: (L x)_U = PG(x_E) + PGr(x_rho) - Phi' grad(zeta) x_rho, PGr the
// pressure gradient with (J dP/drho) in place of (J c_Theta), so
//   S = I - Lambda^2 grad(zeta).(PG DTh + PGr Drho - Phi' grad(zeta) Drho),
// the same band.  The bodies take a template flag S3; with S3 the operator holds
// the extra per-node field J dP/drho as a plane of its own after the eight
// tile-interleaved fields (pr_plane).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "hevi_gll.h"
#include "hevi_internal.h"

namespace {

constexpr int T = HEVI_TILE;

__device__ __forceinline__ size_t tix(int64_t tile, int nz, int k, int nf, int f, int lane) {
  return ((size_t)(tile * nz + k) * nf + f) * T + lane;
}

// caller layout: field f (or vector component) v, node k, column c
__device__ __forceinline__ size_t cix(int nz, int64_t ncols, int v, int k, int64_t c) {
  return ((size_t)v * nz + k) * (size_t)ncols + (size_t)c;
}

__device__ __forceinline__ void flag(HeviDevInfo* info, int code, int64_t col) {
  atomicMax(&info->status, code);
  atomicMin((unsigned long long*)&info->first_bad, (unsigned long long)col);
  atomicAdd((unsigned long long*)&info->n_bad, 1ull);
}

// Streaming accesses carry the non-temporal hint: state vectors, factors and
// the factorisation's scratch are each touched once per kernel, so they should
// not evict the compact operator, which every kernel of a step reads again and
// which fits in the last-level cache at the production column count.
template <typename FT>
__device__ __forceinline__ double ld(const FT* p) { return (double)__builtin_nontemporal_load(p); }
__device__ __forceinline__ double ldn(const double* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void stn(double* p, double v) { __builtin_nontemporal_store(v, p); }
template <typename FT>
__device__ __forceinline__ void stnt(FT* p, FT v) { __builtin_nontemporal_store(v, p); }

// ---------------------------------------------------------------------------
// Element-streaming helpers.  Node eN is shared by elements e-1 and e; a sum
// over elements is finished for node eN after element e, so each helper
// carries the partial sum of the last node of an element into the next.

struct OpsView {
  const double* ops;
  int64_t tile;
  int nz, lane;
  const double* pr = nullptr;  // set 3C: J dP/drho plane (pr_plane), else unused
  __device__ __forceinline__ double operator()(int k, int f) const {
    return ops[tix(tile, nz, k, HEVI_NOPS, f, lane)];
  }
  // J dP/drho at node k (set 3C only)
  __device__ __forceinline__ double jpr(int k) const { return pr[((size_t)tile * nz + k) * T + lane]; }
};

// Set 3C: the ninth per-node operator field J dP/drho, stored [tile][k][lane]
// after the eight tile-interleaved fields of the compact operator.  LHEVI-PS
// operators hold instead three planes there: the velocity u0 = U0/rho0 of the
// linearisation state (ps_plane(ops, sh, m), m = 0..2).
__device__ __forceinline__ size_t pr_offset(const HeviShapeDev& sh) {
  return (size_t)sh.ntiles * sh.nz * HEVI_NOPS * T;
}
__device__ __forceinline__ const double* pr_plane(const double* ops, const HeviShapeDev& sh) {
  return ops + pr_offset(sh);
}
__device__ __forceinline__ size_t plane_elems(const HeviShapeDev& sh) {
  return (size_t)sh.ntiles * sh.nz * T;
}
__device__ __forceinline__ const double* ps_plane(const double* ops, const HeviShapeDev& sh,
                                                  int m) {
  return ops + pr_offset(sh) + (size_t)m * plane_elems(sh);
}

// v_rho = Drho u and v_Th = DTh u for all nodes; u read from scratch field
// fu, results written to fields fr, ft.
template <int N, int NWS = HEVI_NWS>
__device__ void div_pass(Gll<N> tab, const OpsView& op, int Ne, double* ws, int64_t tile,
                         int lane, int fu, int fr, int ft) {
  const int nz = op.nz;
  double cr = 0.0, ct = 0.0;
  for (int e = 0; e < Ne; ++e) {
    double Ju[N + 1], Jtu[N + 1];
#pragma unroll
    for (int j = 0; j <= N; ++j) {
      const int k = e * N + j;
      const double u = ws[tix(tile, nz, k, NWS, fu, lane)];
      Ju[j] = op(k, OP_J) * u;
      Jtu[j] = op(k, OP_JTH) * u;
    }
#pragma unroll
    for (int a = 0; a <= N; ++a) {
      double sr = 0.0, st = 0.0;
#pragma unroll
      for (int j = 0; j <= N; ++j) {
        sr += tab.w[j] * tab.D[j * (N + 1) + a] * Ju[j];
        st += tab.D[a * (N + 1) + j] * Jtu[j];
      }
      st *= tab.w[a];
      if (a == 0) { sr += cr; st += ct; }
      if (a == N && e < Ne - 1) { cr = sr; ct = st; continue; }
      const int k = e * N + a;
      const double mi = op(k, OP_MINV);
      ws[tix(tile, nz, k, NWS, fr, lane)] = mi * sr;
      ws[tix(tile, nz, k, NWS, ft, lane)] = -mi * st;
    }
  }
}

// Pressure gradient + gravity of (v_rho, v_Th) (fields fr, ft):
//   G_k = -M^-1 sum_e w_i sum_j D_ij (J c_Theta grad zeta)_j v_Th,j - Phi'_k grad(zeta)_k v_rho,k
// (S3: the pressure is J (c v_Th + dP/drho v_rho)); writes grad(zeta)_k . G_k into
// field fo (zero at the rigid-lid nodes).
template <int N, bool S3 = false, int NWS = HEVI_NWS>
__device__ void pg_pass(Gll<N> tab, const OpsView& op, int Ne, double* ws, int64_t tile,
                        int lane, int fr, int ft, int fo) {
  const int nz = op.nz;
  double c0 = 0.0, c1 = 0.0, c2 = 0.0;
  for (int e = 0; e < Ne; ++e) {
    double f0[N + 1], f1[N + 1], f2[N + 1];
#pragma unroll
    for (int j = 0; j <= N; ++j) {
      const int k = e * N + j;
      double v = op(k, OP_JCT) * ws[tix(tile, nz, k, NWS, ft, lane)];
      if constexpr (S3) v += op.jpr(k) * ws[tix(tile, nz, k, NWS, fr, lane)];
      f0[j] = v * op(k, OP_GX);
      f1[j] = v * op(k, OP_GY);
      f2[j] = v * op(k, OP_GZ);
    }
#pragma unroll
    for (int a = 0; a <= N; ++a) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
      for (int j = 0; j <= N; ++j) {
        const double d = tab.D[a * (N + 1) + j];
        s0 += d * f0[j];
        s1 += d * f1[j];
        s2 += d * f2[j];
      }
      s0 *= tab.w[a]; s1 *= tab.w[a]; s2 *= tab.w[a];
      if (a == 0) { s0 += c0; s1 += c1; s2 += c2; }
      if (a == N && e < Ne - 1) { c0 = s0; c1 = s1; c2 = s2; continue; }
      const int k = e * N + a;
      const bool lid = (k == 0) || (k == nz - 1);
      const double mi = op(k, OP_MINV), ph = op(k, OP_PHI);
      const double gx = op(k, OP_GX), gy = op(k, OP_GY), gzz = op(k, OP_GZ);
      const double vr = ws[tix(tile, nz, k, NWS, fr, lane)];
      const double G0 = -mi * s0 - ph * gx * vr;
      const double G1 = -mi * s1 - ph * gy * vr;
      const double G2 = -mi * s2 - ph * gzz * vr;
      ws[tix(tile, nz, k, NWS, fo, lane)] = lid ? 0.0 : gx * G0 + gy * G1 + gzz * G2;
    }
  }
}

// ---------------------------------------------------------------------------
// Element-chunked kernels: a block of cw wavefronts owns one 64-column tile;
// wavefront w owns a contiguous chunk of elements [e0, e1) and the nodes
// e0*N .. e1*N - 1 (plus the top node for the last chunk).  A node on a chunk
// boundary also receives a contribution from the last element of the previous
// chunk; the wavefront recomputes that element's contribution itself instead of
// exchanging partial sums, so the wavefronts run independently.  With enough
// tiles to fill the chip one wavefront per tile measured fastest (the chunk
// recomputation costs more than the extra wavefronts gain); a launch of few
// tiles is bound by one tile's latency along its elements instead, and the
// single-problem launchers then split tiles into up to kMaxChunks chunks
// (chunks_for).
constexpr int kMaxChunks = 8;

// Waves per SIMD the streaming kernels (apply, stage passes) are compiled for: two
// up to N = 4, whose element working set fits in 256 VGPRs; one above, where a
// 256-VGPR cap spilled hundreds of bytes per lane to scratch.
template <int N>
constexpr int kStreamWaves = N <= 4 ? 2 : 1;

struct Chunk {
  int lane, e0, e1;
  int64_t tile;
};

// chunk of wavefront threadIdx.x / 64 among cw wavefronts: elements split as evenly
// as integers allow (the first Ne % cw chunks take one more)
__device__ __forceinline__ Chunk chunk_of(int Ne, int64_t tile, int cw = 1) {
  Chunk ch;
  ch.lane = threadIdx.x & (T - 1);
  const int wv = threadIdx.x / T;
  const int q = Ne / cw, r = Ne % cw;
  ch.e0 = wv * q + min(wv, r);
  ch.e1 = ch.e0 + q + (wv < r ? 1 : 0);
  ch.tile = tile;
  return ch;
}

// a0: y = L_z (x - x_ref).  Each element iteration loads everything it needs
// unconditionally (clamped indices), computes, then stores the owned nodes, so
// the loads of an element are in flight together.
template <int N, bool HAS_REF, bool S3 = false, bool PS = false>
__device__ __forceinline__ void b_apply(int64_t tile_, HeviShapeDev sh, Gll<N> tab,
                                        const double* __restrict__ ops,
                                        const double* __restrict__ x,
                                        const double* __restrict__ xref, double* __restrict__ y,
                                        int cw = 1) {
  const int Ne = sh.Ne, nz = sh.nz;
  const Chunk ch = chunk_of(Ne, tile_, cw);
  if (ch.e0 >= ch.e1) return;
  const int lane = ch.lane;
  const int64_t tile = ch.tile;
  const int64_t c = tile * T + lane;
  const bool valid = c < sh.ncols;
  const int64_t cc = valid ? c : sh.ncols - 1;
  const int64_t nc = sh.ncols;
  OpsView op{ops, tile, nz, lane, S3 ? pr_plane(ops, sh) : nullptr};
  auto X = [&](int v, int k) {
    const size_t i = cix(nz, nc, v, k, cc);
    if constexpr (HAS_REF) return ldn(x + i) - ldn(xref + i);
    else return ldn(x + i);
  };
  double cr = 0.0, ct = 0.0, c0 = 0.0, c1 = 0.0, c2 = 0.0;
  // node eN is shared by elements e-1 and e: its values are carried over instead
  // of being loaded again (the first element loads all N+1 nodes).  Each node's
  // loads are reduced at once to what the element sums use (u times J and J theta0,
  // the pressure J (c x_T [+ dP/drho x_rho])), so few values stay live.
  double kg0 = 0.0, kg1 = 0.0, kg2 = 0.0, kmi = 0.0, kph = 0.0, kxr = 0.0;
  double kJu = 0.0, kJtu = 0.0, kp = 0.0, kf0 = 0.0, kf1 = 0.0, kf2 = 0.0;
  // LHEVI-PS: the velocity planes of the linearisation state
  const double* u0p = PS ? ps_plane(ops, sh, 0) : nullptr;
  const size_t pe = PS ? plane_elems(sh) : 0;
  auto element = [&](const int e, auto first) {
    constexpr bool FIRST = decltype(first)::value;
    // ---- loads ----
    double g0[N + 1], g1[N + 1], g2[N + 1], mi[N + 1], ph[N + 1], xr[N + 1];
    double Ju[N + 1], Jtu[N + 1], pp[N + 1], f0[N + 1], f1[N + 1], f2[N + 1];
#pragma unroll
    for (int j = 0; j <= N; ++j) {
      if (!FIRST && j == 0) {
        g0[0] = kg0; g1[0] = kg1; g2[0] = kg2; mi[0] = kmi; ph[0] = kph; xr[0] = kxr;
        Ju[0] = kJu; Jtu[0] = kJtu; pp[0] = kp;
        f0[0] = kf0; f1[0] = kf1; f2[0] = kf2;
        continue;
      }
      const int k = e * N + j;
      g0[j] = op(k, OP_GX); g1[j] = op(k, OP_GY); g2[j] = op(k, OP_GZ);
      mi[j] = op(k, OP_MINV); ph[j] = op(k, OP_PHI);
      xr[j] = X(0, k);
      const double x1 = X(1, k), x2 = X(2, k), x3 = X(3, k), xt = X(4, k);
      const double u = g0[j] * x1 + g1[j] * x2 + g2[j] * x3;
      Ju[j] = op(k, OP_J) * u;
      if constexpr (PS) {
        // fluxes linearised at (rho0, U0, Theta0), u0 = U0/rho0, w = grad(zeta).u0:
        //   J F_Theta' = J theta0 (u - w rho') + J w Theta'
        //   J F_U'     = J c_Theta Theta' grad(zeta) + J (w U' + u0 (u - w rho'))
        const size_t ip = ((size_t)tile * nz + k) * T + lane;
        const double a0 = u0p[ip], a1 = u0p[ip + pe], a2 = u0p[ip + 2 * pe];
        const double Jk = op(k, OP_J);
        const double w = g0[j] * a0 + g1[j] * a1 + g2[j] * a2;
        const double uw = u - w * xr[j];
        Jtu[j] = op(k, OP_JTH) * uw + Jk * w * xt;
        const double pc = op(k, OP_JCT) * xt;
        f0[j] = pc * g0[j] + Jk * (w * x1 + a0 * uw);
        f1[j] = pc * g1[j] + Jk * (w * x2 + a1 * uw);
        f2[j] = pc * g2[j] + Jk * (w * x3 + a2 * uw);
      } else {
        Jtu[j] = op(k, OP_JTH) * u;
        pp[j] = op(k, OP_JCT) * xt;
        if constexpr (S3) pp[j] += op.jpr(k) * xr[j];
      }
    }
    // ---- element sums ----
    if constexpr (!PS) {
#pragma unroll
      for (int j = 0; j <= N; ++j) {
        f0[j] = pp[j] * g0[j]; f1[j] = pp[j] * g1[j]; f2[j] = pp[j] * g2[j];
      }
    }
    double yo[N + 1][5];
#pragma unroll
    for (int a = 0; a <= N; ++a) {
      double sr = 0.0, st = 0.0, s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
      for (int j = 0; j <= N; ++j) {
        const double d = tab.D[a * (N + 1) + j];
        sr += tab.w[j] * tab.D[j * (N + 1) + a] * Ju[j];
        st += d * Jtu[j];
        s0 += d * f0[j]; s1 += d * f1[j]; s2 += d * f2[j];
      }
      const double wa = tab.w[a];
      st *= wa; s0 *= wa; s1 *= wa; s2 *= wa;
      if (a == 0) { sr += cr; st += ct; s0 += c0; s1 += c1; s2 += c2; }
      if (a == N) { cr = sr; ct = st; c0 = s0; c1 = s1; c2 = s2; }
      const int k = e * N + a;
      const bool lid = (k == 0) || (k == nz - 1);
      yo[a][0] = mi[a] * sr;
      yo[a][4] = -mi[a] * st;
      yo[a][1] = lid ? 0.0 : -mi[a] * s0 - ph[a] * g0[a] * xr[a];
      yo[a][2] = lid ? 0.0 : -mi[a] * s1 - ph[a] * g1[a] * xr[a];
      yo[a][3] = lid ? 0.0 : -mi[a] * s2 - ph[a] * g2[a] * xr[a];
    }
    // ---- stores of the owned nodes ----
    if (e >= ch.e0 && valid) {
      const int amax = (e == Ne - 1) ? N : N - 1;
#pragma unroll
      for (int a = 0; a <= N; ++a) {
        if (a <= amax) {
#pragma unroll
          for (int v = 0; v < 5; ++v) stn(y + cix(nz, nc, v, e * N + a, c), yo[a][v]);
        }
      }
    }
    kg0 = g0[N]; kg1 = g1[N]; kg2 = g2[N]; kmi = mi[N]; kph = ph[N]; kxr = xr[N];
    kJu = Ju[N]; kJtu = Jtu[N];
    if constexpr (PS) { kf0 = f0[N]; kf1 = f1[N]; kf2 = f2[N]; }
    else kp = pp[N];
  };
  int e = max(ch.e0 - 1, 0);
  element(e, std::true_type{});
  for (++e; e < ch.e1; ++e) element(e, std::false_type{});
}

// ---------------------------------------------------------------------------
// a2 + a3: assemble S = I - lambda^2 K and factor it (band LU, partial pivoting)
//
// Storage per node j (tile-interleaved): U row j, entries (j, j+t) for
// t = 0..4N (zero beyond the last column); L multipliers of step j for rows
// j+1..j+2N; pivot offset p in 0..2N (row j was swapped with row j+p).
// sbuf holds, during assembly, row r of -lambda^2 K at band offset c - r + 2N.

// Row a (node r = eN + a) of element e's part of K as band offsets o = column - r +
// 2N.  The pressure gradient of DTh u contributes
//   sum_i P_ai DTh_iq,  P_ai = -M^-1_r w_a D_ai (J c_Theta)_i grad(zeta)_r . grad(zeta)_i,
// where DTh row i (node eN + i) is -M^-1_i C_iq (J theta0)_q over the nodes
// q = (e-1)N .. (e+2)N: C = w_i D_i(q-eN) for the element's own nodes, plus the
// neighbours' terms at the shared end nodes (element e-1's row N into node eN when
// `left`, element e+1's row 0 into node (e+1)N when `right`).  Every DTh entry is
// proportional to (J theta0)_q, so the row is acc_q = (J theta0)_q sum_i Pm_i C_iq
// with Pm_i = -P_ai M^-1_i.  Gravity adds -Phi'_r |grad zeta_r|^2 M^-1_r times Drho
// row a.  Jth[q] is J theta0 at node (e-1)N + q (zero outside the column); mi, gx,
// gy, gz, jc, jn and ph are MINV, GX, GY, GZ, JCT, J and PHI at nodes eN .. eN+N.
template <int N>
__device__ __forceinline__ void k_row(Gll<N> tab, int a, bool left, bool right,
                                      const double (&Jth)[3 * N + 1], const double (&mi)[N + 1],
                                      const double (&gx)[N + 1], const double (&gy)[N + 1],
                                      const double (&gz)[N + 1], const double (&jc)[N + 1],
                                      const double (&jn)[N + 1], const double (&ph)[N + 1],
                                      double (&acc)[4 * N + 1]) {
  // every product and sum rounded on its own: the assembly kernel and the fused
  // factorisation then produce the same bits whatever the surrounding code
#pragma clang fp contract(off)
  constexpr int B = 2 * N, W = 4 * N + 1, NC = 3 * N + 1;
  const double mr = mi[a];
  double Pm[N + 1];
#pragma unroll
  for (int i = 0; i <= N; ++i) {
    const double dot = gx[a] * gx[i] + gy[a] * gy[i] + gz[a] * gz[i];
    Pm[i] = mr * tab.w[a] * tab.D[a * (N + 1) + i] * jc[i] * dot * mi[i];
  }
#pragma unroll
  for (int o = 0; o < W; ++o) acc[o] = 0.0;
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    double sq = 0.0;
    if (q >= N && q <= B) {
#pragma unroll
      for (int i = 0; i <= N; ++i) sq += Pm[i] * (tab.w[i] * tab.D[i * (N + 1) + q - N]);
    }
    if (q <= N && left) sq += Pm[0] * (tab.w[N] * tab.D[N * (N + 1) + q]);
    if (q >= B && right) sq += Pm[N] * (tab.w[0] * tab.D[q - B]);
    acc[q + N - a] = sq * Jth[q];
  }
  const double gr = -ph[a] * (gx[a] * gx[a] + gy[a] * gy[a] + gz[a] * gz[a]) * mr;
#pragma unroll
  for (int i2 = 0; i2 <= N; ++i2) acc[B + i2 - a] += gr * tab.w[i2] * tab.D[i2 * (N + 1) + a] * jn[i2];
}

// Set 3C: the rho column of the pressure adds to row a the term
//   sum_i Pr_ai Drho_iq,  Pr_ai = -M^-1_r w_a D_ai (J dP/drho)_i grad(zeta)_r . grad(zeta)_i,
// where Drho row i (node eN + i) is M^-1_i C'_iq J_q: C' = w_q D_(q-eN)i for the
// element's own nodes, element e-1's w_q D_qN at node eN when `left`, element e+1's
// w_(q-2N) D_(q-2N)0 at node (e+1)N when `right` (the weak form).  So
// acc_q -= J_q sum_i Prm_i C'_iq with Prm_i = -Pr_ai M^-1_i.  Jq[q] is J at node
// (e-1)N + q (zero outside the column), jp J dP/drho at nodes eN .. eN+N.
template <int N>
__device__ __forceinline__ void k_row_pr(Gll<N> tab, int a, bool left, bool right,
                                         const double (&Jq)[3 * N + 1], const double (&mi)[N + 1],
                                         const double (&gx)[N + 1], const double (&gy)[N + 1],
                                         const double (&gz)[N + 1], const double (&jp)[N + 1],
                                         double (&acc)[4 * N + 1]) {
#pragma clang fp contract(off)
  constexpr int B = 2 * N, NC = 3 * N + 1;
  const double mr = mi[a];
  double Pm[N + 1];
#pragma unroll
  for (int i = 0; i <= N; ++i) {
    const double dot = gx[a] * gx[i] + gy[a] * gy[i] + gz[a] * gz[i];
    Pm[i] = mr * tab.w[a] * tab.D[a * (N + 1) + i] * jp[i] * dot * mi[i];
  }
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    double sq = 0.0;
    if (q >= N && q <= B) {
#pragma unroll
      for (int i = 0; i <= N; ++i) sq += Pm[i] * (tab.w[q - N] * tab.D[(q - N) * (N + 1) + i]);
    }
    if (q <= N && left) sq += Pm[0] * (tab.w[q] * tab.D[q * (N + 1) + N]);
    if (q >= B && right) sq += Pm[N] * (tab.w[q - B] * tab.D[(q - B) * (N + 1)]);
    acc[q + N - a] -= sq * Jq[q];
  }
}

// Assembly of -lambda^2 K (element-chunked, see Chunk): row r of the band is
// written once, by the wavefront owning node r.
constexpr int CWF = 1;  // chunk wavefronts of the assembly kernel

template <int N, bool S3 = false>
__device__ __forceinline__ void b_factor_assemble(int64_t tile_, HeviShapeDev sh,
                                                  Gll<N> tab, double lambda,
                                                  const double* __restrict__ ops,
                                                  double* __restrict__ sbuf) {
#pragma clang fp contract(off)
  constexpr int W = 4 * N + 1;      // S band width = U row width kl + ku + 1
  constexpr int NC = 3 * N + 1;     // columns touched by DTh rows of one element
  const int Ne = sh.Ne, nz = sh.nz;
  const Chunk ch = chunk_of(Ne, tile_);
  if (ch.e0 >= ch.e1) return;
  const int lane = ch.lane;
  const int64_t tile = ch.tile;
  OpsView op{ops, tile, nz, lane, S3 ? pr_plane(ops, sh) : nullptr};
  const double l2 = lambda * lambda;
  double carry[W];
#pragma unroll
  for (int o = 0; o < W; ++o) carry[o] = 0.0;
  for (int e = max(ch.e0 - 1, 0); e < ch.e1; ++e) {
    double Jth[NC], mi[N + 1], gx[N + 1], gy[N + 1], gz[N + 1], jc[N + 1], jn[N + 1], ph[N + 1];
    double Jq[NC], jp[N + 1];
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const int k = (e - 1) * N + q;
      const double v = op(min(max(k, 0), nz - 1), OP_JTH);
      Jth[q] = (k >= 0 && k < nz) ? v : 0.0;
      if constexpr (S3) {
        const double vj = op(min(max(k, 0), nz - 1), OP_J);
        Jq[q] = (k >= 0 && k < nz) ? vj : 0.0;
      }
    }
#pragma unroll
    for (int i = 0; i <= N; ++i) {
      const int k = e * N + i;
      mi[i] = op(k, OP_MINV); gx[i] = op(k, OP_GX); gy[i] = op(k, OP_GY); gz[i] = op(k, OP_GZ);
      jc[i] = op(k, OP_JCT); jn[i] = op(k, OP_J); ph[i] = op(k, OP_PHI);
      if constexpr (S3) jp[i] = op.jpr(k);
    }
#pragma unroll
    for (int a = 0; a <= N; ++a) {
      if (e < ch.e0 && a < N) continue;  // only the boundary row of the recomputed element
      const int r = e * N + a;
      double acc[W];
      k_row<N>(tab, a, e > 0, e < Ne - 1, Jth, mi, gx, gy, gz, jc, jn, ph, acc);
      if constexpr (S3) k_row_pr<N>(tab, a, e > 0, e < Ne - 1, Jq, mi, gx, gy, gz, jp, acc);
      if (a == 0) {
#pragma unroll
        for (int o = 0; o < W; ++o) acc[o] += carry[o];
      }
      if (a == N && e < Ne - 1) {
#pragma unroll
        for (int o = 0; o < W; ++o) carry[o] = acc[o];
        continue;
      }
      double* row = sbuf + tix(tile, nz, r, W, 0, lane);
#pragma unroll
      for (int o = 0; o < W; ++o) stn(row + o * T, -l2 * acc[o]);
    }
  }
}

// Band LU with partial pivoting of S, per column.  At step j the active window
// holds rows j..j+2N and columns j..j+4N of the partly eliminated matrix (the
// U rows fill in up to 4N right of the diagonal).  Step j picks the largest
// |entry| of column j among rows j..j+2N (lowest row on ties), exchanges it
// with row j, stores U row j, the 2N multipliers and the pivot offset, and
// eliminates column j from the rows below; then the window moves one row down
// and one column right and row j+2N+1 of S enters at the bottom.  The window
// starts empty at j = -(2N+1), the first 2N+1 steps only shift rows 0..2N in
// (their loads go through the same prefetch ring as every later row).  The
// window is kept in registers, split over the lanes of a group
// (b_factor_lu_split, and b_factor_fused_split with the assembly folded in).
template <int N>
__device__ __forceinline__ double s_fix(int r, int nz, int s, double raw) {
  // entry (r, r - 2N + s) of S from the stored -lambda^2 K value: identity rows
  // at the rigid-lid nodes, zero columns for their (identically zero) unknowns
  constexpr int B = 2 * N;
  const int cabs = r - B + s;
  if (r >= nz) return 0.0;
  if (r == 0 || r == nz - 1) return s == B ? 1.0 : 0.0;
  if (cabs <= 0 || cabs >= nz - 1) return 0.0;
  return raw + (s == B ? 1.0 : 0.0);
}

// Lane exchanges inside groups of LPC = 2 or 4 consecutive lanes (DPP quad_perm):
// from_first: every lane gets the group's first lane's value; from_next: lane h
// gets lane h+1's value (the group's last lane gets its own).
template <int LPC>
__device__ __forceinline__ int from_first(int v) {
  return __builtin_amdgcn_mov_dpp(v, LPC == 2 ? 0xA0 : 0x00, 0xF, 0xF, false);
}
template <int LPC>
__device__ __forceinline__ int from_next(int v) {
  return __builtin_amdgcn_mov_dpp(v, LPC == 2 ? 0xF5 : 0xF9, 0xF, 0xF, false);
}
template <int LPC>
__device__ __forceinline__ double from_first(double v) {
  const int lo = from_first<LPC>(__double2loint(v)), hi = from_first<LPC>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
template <int LPC>
__device__ __forceinline__ double from_next(double v) {
  const int lo = from_next<LPC>(__double2loint(v)), hi = from_next<LPC>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
// maximum over the LPC = 2 or 4 lanes of the group (DPP quad_perm swaps)
template <int LPC>
__device__ __forceinline__ int group_max(int v) {
  v = max(v, __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false));  // lanes 1,0,3,2
  if constexpr (LPC == 4) v = max(v, __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false));
  return v;
}

// The pivot array holds three byte planes of plane_size(sh) bytes each, laid out
// like the factors: the pivot offset of step j; the band offset of the last
// nonzero entry of U row j (U entries beyond it are exact zeros, which the
// solves do not read: about half of each row at N = 4); and the binary exponent
// e_r of row r's scale 2^-e_r (signed byte, see scale_row).
__device__ __forceinline__ size_t plane_size(const HeviShapeDev& sh) {
  return (size_t)sh.ntiles * sh.nz * T;
}
constexpr int kPlanes = 3;

// Row equilibration of S by powers of two (LAPACK's row scaling of the band
// system before the LU, with the scale rounded to a power of two so that
// scaling is exact).  Row r is multiplied by 2^-e_r, e_r the binary exponent of
// its largest |entry| (the group's lanes share the row), before it enters the
// LU window, and the solves multiply r_r by the same 2^-e_r.  Pivoting then
// compares entries relative to their rows' size.  Rows of S near element
// boundaries, where the GLL spacing is smallest, are up to ~10x larger than the
// others; without the scaling they win pivot searches they should not, and
// the reduced solution loses about two digits at the ne = 30 shape.
template <int LPC, int H>
__device__ __forceinline__ void scale_row(double (&row)[H], int r, int nz, int h, int64_t tile,
                                          int lane, uint8_t* __restrict__ piv, size_t plane) {
  double m = 0.0;
#pragma unroll
  for (int i = 0; i < H; ++i) m = fmax(m, fabs(row[i]));
  int ex = -4096;  // a lane whose part of the row is zero does not count
  if (m > 0.0) (void)frexp(m, &ex);
  ex = group_max<LPC>(ex);
  ex = ex == -4096 ? 0 : min(max(ex, -120), 120);  // a zero row keeps scale 1
#pragma unroll
  for (int i = 0; i < H; ++i) row[i] = ldexp(row[i], -ex);
  if (h == 0 && r < nz) piv[2 * plane + tix(tile, nz, r, 1, 0, lane)] = (uint8_t)(int8_t)ex;
}

// The band LU with each column's window split over LPC consecutive lanes: lane
// h holds window columns hH .. hH+H-1, H = ceil((4N+1) / LPC) (columns past 4N
// are always zero), so the window stays in VGPRs.  The group shares the pivot
// index and the multipliers of its first lane, and passes the column crossing
// each split to the left with DPP moves.  A wavefront handles 64 / LPC columns:
// part `part` of a 64-column tile.
constexpr int kLuLanes = 2;  // lanes per column of the register-window LU up to N = 4

// Lanes per column of the register-window LU by order: 2 up to N = 4, 4 above,
// where a two-lane window would not fit in registers.
template <int N>
constexpr int kSplitLanes = N <= 4 ? kLuLanes : 4;

// One step of the split-window LU: elimination step j (if j >= 0), then the
// window moves one row down and one column right.  Its bottom row is left for
// the caller to fill with row j + 2N + 1.
template <int N, typename FT, int LPC>
__device__ __forceinline__ void split_step(double (&Wn)[2 * N + 1][(4 * N + LPC) / LPC], int j,
                                           int nz, int h, int s0, int64_t tile, int lane,
                                           FT* Ub, FT* __restrict__ Lb,
                                           uint8_t* __restrict__ piv, size_t plane,
                                           bool& singular) {
  constexpr int B = 2 * N, W = 4 * N + 1, H = (W + LPC - 1) / LPC;
  if (j >= 0) {  // elimination step j (rows 0..2N are only shifted in)
    // pivot search on window column 0 (first lane of the group)
    int p = 0;
    double best = fabs(Wn[0][0]);
#pragma unroll
    for (int t = 1; t <= B; ++t) {
      const double v = fabs(Wn[t][0]);
      if (j + t < nz && v > best) { best = v; p = t; }
    }
    if (h == 0 && !(best > 0.0)) { singular = true; Wn[0][0] = 1.0; p = 0; }
    p = from_first<LPC>(p);
    if (__ballot(p != 0) != 0) {
#pragma unroll
      for (int m = 0; m < H; ++m) {
        const double v0 = Wn[0][m];
        double vp = v0;
#pragma unroll
        for (int t = 1; t <= B; ++t) vp = (p == t) ? Wn[t][m] : vp;
        Wn[0][m] = vp;
#pragma unroll
        for (int t = 1; t <= B; ++t) Wn[t][m] = (p == t) ? v0 : Wn[t][m];
      }
    }
    // the last nonzero entry of U row j (the pivot itself is nonzero)
    int ue = 0;
#pragma unroll
    for (int m = 0; m < H; ++m)
      if (s0 + m < W && Wn[0][m] != 0.0) ue = s0 + m;
    ue = group_max<LPC>(ue);
    FT* urow = Ub + tix(tile, nz, j, W, 0, lane);
#pragma unroll
    for (int m = 0; m < H; ++m)
      if (s0 + m < W) stnt(urow + (s0 + m) * T, (FT)Wn[0][m]);
    const double inv = 1.0 / Wn[0][0];
    double l[B + 1];
#pragma unroll
    for (int t = 1; t <= B; ++t) l[t] = from_first<LPC>(Wn[t][0] * inv);
    if (h == 0) {
      const size_t pi = tix(tile, nz, j, 1, 0, lane);
      piv[pi] = (uint8_t)p;
      piv[plane + pi] = (uint8_t)ue;
      FT* lrow = Lb + tix(tile, nz, j, B, 0, lane);
#pragma unroll
      for (int t = 1; t <= B; ++t) stnt(lrow + (t - 1) * T, (FT)l[t]);
    }
#pragma unroll
    for (int t = 1; t <= B; ++t)
#pragma unroll
      for (int m = 0; m < H; ++m) Wn[t][m] -= l[t] * Wn[0][m];
  }
  // move the window one row down and one column right: each lane's last
  // column comes from the next lane's first, the group's last lane's is zero
  double cross[B];
#pragma unroll
  for (int t = 0; t < B; ++t) cross[t] = from_next<LPC>(Wn[t + 1][0]);
#pragma unroll
  for (int t = 0; t < B; ++t) {
#pragma unroll
    for (int m = 0; m < H - 1; ++m) Wn[t][m] = Wn[t + 1][m + 1];
    Wn[t][H - 1] = h < LPC - 1 ? cross[t] : 0.0;
  }
}

template <int N, typename FT, int LPC>
__device__ __forceinline__ void b_factor_lu_split(int64_t tile, int part, HeviShapeDev sh,
                                                  const double* sbuf, FT* Ub,
                                                  FT* __restrict__ Lb,
                                                  uint8_t* __restrict__ piv, HeviDevInfo* info) {
  constexpr int B = 2 * N, W = 4 * N + 1, H = (W + LPC - 1) / LPC, PFL = 2;
  const int h = threadIdx.x % LPC;                           // window part of this lane
  const int lane = part * (T / LPC) + (threadIdx.x / LPC);   // the column's lane in its tile
  const int64_t c = tile * T + lane;
  const bool valid = c < sh.ncols;
  const int nz = sh.nz;
  const int s0 = h * H;                                      // first window column of this lane
  // Wn[t][m] = entry (j + t, j + s0 + m); empty at j = -(2N+1), rows shifted in
  double Wn[B + 1][H];
#pragma unroll
  for (int t = 0; t <= B; ++t)
#pragma unroll
    for (int m = 0; m < H; ++m) Wn[t][m] = 0.0;
  double ring[PFL][H];
#pragma unroll
  for (int d = 0; d < PFL; ++d) {
    const int r = min(d, nz - 1);
#pragma unroll
    for (int m = 0; m < H; ++m)
      ring[d][m] = ldn(sbuf + tix(tile, nz, r, W, min(s0 + m, W - 1), lane));
  }
  bool singular = false;
  for (int j0 = -(B + 1); j0 < nz; j0 += PFL) {
#pragma unroll
    for (int d = 0; d < PFL; ++d) {
      const int j = j0 + d;
      if (j < nz) {
        split_step<N, FT, LPC>(Wn, j, nz, h, s0, tile, lane, Ub, Lb, piv, plane_size(sh),
                               singular);
        // new bottom row j + 2N + 1 from the ring; refill the slot
        const int rn = j + B + 1;
#pragma unroll
        for (int m = 0; m < H; ++m)
          Wn[B][m] = s0 + m < W ? s_fix<N>(rn, nz, s0 + m, ring[d][m]) : 0.0;
        scale_row<LPC, H>(Wn[B], rn, nz, h, tile, lane, piv, plane_size(sh));
        const int rf = min(rn + PFL, nz - 1);
#pragma unroll
        for (int m = 0; m < H; ++m)
          ring[d][m] = ldn(sbuf + tix(tile, nz, rf, W, min(s0 + m, W - 1), lane));
      }
    }
  }
  if (singular && valid) flag(info, 5 /*HEVI_E_SINGULAR*/, c);
}

// Assembly and split-window LU in one pass (N <= HEVI_FUSED_FACTOR_MAX_N): the
// wavefront computes each element's rows of S itself (k_row, as b_factor_assemble
// does), keeps this lane's part of them in LDS until they enter the window, and loads the
// operator fields of the next element while they do.  S never goes through
// memory: per column the pass reads the compact operator and writes the factors.
// lds holds fused_lds_doubles<N>(LPC) doubles: (N + 1) rows of H per lane.
template <int N>
constexpr int fused_lds_doubles(int lpc) {
  return (N + 1) * ((4 * N + lpc) / lpc) * 64;
}

template <int N, typename FT, int LPC, bool S3 = false>
__device__ __forceinline__ void b_factor_fused_split(int64_t tile, int part, HeviShapeDev sh,
                                                     Gll<N> tab, double lambda,
                                                     const double* __restrict__ ops,
                                                     FT* __restrict__ Ub, FT* __restrict__ Lb,
                                                     uint8_t* __restrict__ piv,
                                                     HeviDevInfo* info, double* lds) {
  constexpr int B = 2 * N, W = 4 * N + 1, H = (W + LPC - 1) / LPC, NC = 3 * N + 1;
  const int h = threadIdx.x % LPC;
  const int lane = part * (T / LPC) + (threadIdx.x / LPC);
  const int64_t c = tile * T + lane;
  const bool valid = c < sh.ncols;
  const int nz = sh.nz, Ne = sh.Ne;
  const int s0 = h * H;
  const OpsView op{ops, tile, nz, lane, S3 ? pr_plane(ops, sh) : nullptr};
  const double l2 = lambda * lambda;
  const size_t plane = plane_size(sh);
  double* slot = lds + threadIdx.x;  // row a, window column m of this lane: slot[(a * H + m) * T]
  double Wn[B + 1][H];
#pragma unroll
  for (int t = 0; t <= B; ++t)
#pragma unroll
    for (int m = 0; m < H; ++m) Wn[t][m] = 0.0;
  // operator fields of element e: J theta0 at nodes (e-1)N .. (e+2)N (zero outside
  // the column), the others at nodes eN .. eN+N
  auto jth_at = [&](int k) {
    const double v = op(min(max(k, 0), nz - 1), OP_JTH);
    return (k >= 0 && k < nz) ? v : 0.0;
  };
  auto j_at = [&](int k) {
    const double v = op(min(max(k, 0), nz - 1), OP_J);
    return (k >= 0 && k < nz) ? v : 0.0;
  };
  double jth[NC], mi[N + 1], gx[N + 1], gy[N + 1], gz[N + 1], jc[N + 1], jn[N + 1], ph[N + 1];
  double jq[NC], jp[N + 1];  // set 3C: J at the nodes of jth, J dP/drho
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    jth[q] = jth_at(q - N);
    if constexpr (S3) jq[q] = j_at(q - N);
  }
#pragma unroll
  for (int i = 0; i <= N; ++i) {
    const int k = min(i, nz - 1);
    mi[i] = op(k, OP_MINV); gx[i] = op(k, OP_GX); gy[i] = op(k, OP_GY); gz[i] = op(k, OP_GZ);
    jc[i] = op(k, OP_JCT); jn[i] = op(k, OP_J); ph[i] = op(k, OP_PHI);
    if constexpr (S3) jp[i] = op.jpr(k);
  }
  double carry[H];  // this lane's part of row N of the previous element
#pragma unroll
  for (int m = 0; m < H; ++m) carry[m] = 0.0;
  bool singular = false;
  int j = -(B + 1);  // the step whose window takes in the next row
  for (int e = 0; e < Ne; ++e) {
    // rows eN .. eN+N-1 of S (and the top row after the last element) into LDS,
    // rounded as the assembly kernel and the LU's s_fix round them
#pragma unroll
    for (int a = 0; a <= N; ++a) {
#pragma clang fp contract(off)
      double acc[W];
      k_row<N>(tab, a, e > 0, e < Ne - 1, jth, mi, gx, gy, gz, jc, jn, ph, acc);
      if constexpr (S3) k_row_pr<N>(tab, a, e > 0, e < Ne - 1, jq, mi, gx, gy, gz, jp, acc);
      double x[H];
#pragma unroll
      for (int m = 0; m < H; ++m) {
        double v = acc[m];
#pragma unroll
        for (int hh = 1; hh < LPC; ++hh)
          if (h == hh) v = hh * H + m < W ? acc[hh * H + m] : 0.0;
        x[m] = a == 0 ? v + carry[m] : v;
      }
      if (a == N && e < Ne - 1) {
#pragma unroll
        for (int m = 0; m < H; ++m) carry[m] = x[m];
      } else {
        const int r = e * N + a;
#pragma unroll
        for (int m = 0; m < H; ++m)
          slot[(a * H + m) * T] = s0 + m < W ? s_fix<N>(r, nz, s0 + m, -l2 * x[m]) : 0.0;
      }
    }
    // the next element's new operator fields, in flight while the rows enter
    double pj[N], pmi[N], pgx[N], pgy[N], pgz[N], pjc[N], pjn[N], pph[N], pjq[N], pjp[N];
#pragma unroll
    for (int t = 0; t < N; ++t) {
      pj[t] = jth_at((e + 2) * N + 1 + t);
      const int k = min((e + 1) * N + 1 + t, nz - 1);
      pmi[t] = op(k, OP_MINV); pgx[t] = op(k, OP_GX); pgy[t] = op(k, OP_GY);
      pgz[t] = op(k, OP_GZ); pjc[t] = op(k, OP_JCT); pjn[t] = op(k, OP_J); pph[t] = op(k, OP_PHI);
      if constexpr (S3) {
        pjq[t] = j_at((e + 2) * N + 1 + t);
        pjp[t] = op.jpr(k);
      }
    }
    const int na = e == Ne - 1 ? N + 1 : N;
#pragma unroll
    for (int a = 0; a <= N; ++a) {
      if (a < na) {
        split_step<N, FT, LPC>(Wn, j, nz, h, s0, tile, lane, Ub, Lb, piv, plane, singular);
#pragma unroll
        for (int m = 0; m < H; ++m) Wn[B][m] = slot[(a * H + m) * T];
        scale_row<LPC, H>(Wn[B], j + B + 1, nz, h, tile, lane, piv, plane);
        ++j;
      }
    }
#pragma unroll
    for (int q = 0; q <= B; ++q) jth[q] = jth[q + N];
#pragma unroll
    for (int t = 0; t < N; ++t) jth[B + 1 + t] = pj[t];
    mi[0] = mi[N]; gx[0] = gx[N]; gy[0] = gy[N]; gz[0] = gz[N];
    jc[0] = jc[N]; jn[0] = jn[N]; ph[0] = ph[N];
#pragma unroll
    for (int t = 0; t < N; ++t) {
      mi[1 + t] = pmi[t]; gx[1 + t] = pgx[t]; gy[1 + t] = pgy[t]; gz[1 + t] = pgz[t];
      jc[1 + t] = pjc[t]; jn[1 + t] = pjn[t]; ph[1 + t] = pph[t];
    }
    if constexpr (S3) {
#pragma unroll
      for (int q = 0; q <= B; ++q) jq[q] = jq[q + N];
      jp[0] = jp[N];
#pragma unroll
      for (int t = 0; t < N; ++t) {
        jq[B + 1 + t] = pjq[t];
        jp[1 + t] = pjp[t];
      }
    }
  }
  // rows past the top are zero
  while (j < nz) {
    split_step<N, FT, LPC>(Wn, j, nz, h, s0, tile, lane, Ub, Lb, piv, plane, singular);
#pragma unroll
    for (int m = 0; m < H; ++m) Wn[B][m] = 0.0;
    ++j;
  }
  if (singular && valid) flag(info, 5 /*HEVI_E_SINGULAR*/, c);
}

// ---------------------------------------------------------------------------
// a4 + a5 + a6: one stage solve
//
// scratch fields per node
// R: reduced right-hand side, U: reduced solution u, VR/VT: Drho u / DTh u,
// T/D: reduced residual / correction; B, X, S: 5-field vectors (rho, U, Theta)
// of the full-residual refinement (right-hand side, solution, residual)
enum { WS_R = 0, WS_U = 1, WS_VR = 2, WS_VT = 3, WS_T = 4, WS_D = 5, WS_B = 6, WS_X = 11,
       WS_S = 16 };

// solve S x = rhs with the band LU factors (rhs field fi, result field fo).
// The sweeps are sequential in the row index, so each wavefront keeps the factor
// rows of the next rows in flight (PF forward, PB backward) in a register ring,
// refilled as soon as a slot is consumed, while it works on the current row.  The
// fused stage kernels (LDSRU) hold r/u in LDS and have the registers for a third
// backward slot; the others spill with it.
//
// PIPE (bit 0 forward, bit 1 backward) selects the pipelined form of a sweep, same
// arithmetic.  For the ring to stay in flight the loads must be unconditional and nothing
// may use a value right after loading it: a guarded load (a branch), a step behind a
// branch, or a load whose value is used at once makes the compiler wait for every
// outstanding load, the one just issued included.  So in the pipelined form the groups of
// PF (PB) steps always run whole (the steps past the last row compute on clamped rows and
// store nothing), a row's scale is applied when its entry enters the window, and the
// FP64 U rows are read by buffer loads whose lanes past the row's extent take an offset
// outside the buffer (zero returned, no memory access) instead of guarded loads.  In a
// launch of few tiles each wavefront's memory latency is exposed and the pipelined form
// is faster (the 10,800-column share: 0.596 against 0.660 ms per step); when the chip is
// full the guarded form measured faster (0.389 against 0.404 ms per stage solve at ne = 30).
template <int N, typename FT, bool LDSRU = false, int NWS = HEVI_NWS, int PIPE = 0>
__device__ __forceinline__ void band_solve(const FT* __restrict__ Ub, const FT* __restrict__ Lb,
                                           const uint8_t* __restrict__ piv, size_t plane,
                                           double* ws, int64_t tile, int nz, int lane, int fi,
                                           int fo, double* ru = nullptr) {
  // right-hand side and solution: scratch fields fi / fo, or (LDSRU) one array
  // ru[k * 64 + lane] in LDS used in place
  auto S = [&](int k, int f) -> double& {
    if constexpr (LDSRU) return ru[k * T + lane];
    else return ws[tix(tile, nz, k, NWS, f, lane)];
  };
  constexpr int B = 2 * N, K = 4 * N, PF = 3, PB = LDSRU ? 3 : 2;
  // U row extents (see plane_size): entries past them are zeros and, with FP64
  // factors, are not fetched; each ring slot knows the extent of the row it loads
  // next.  The FP32-factor solves run inside refinement sweeps, where the extra code of
  // the skipping pushed the kernel into scratch spills: they load the full rows.
  constexpr bool SKIP = std::is_same<FT, double>::value;
  const uint8_t* ue_p = piv + plane;
  auto pidx = [&](int k) { return tix(tile, nz, k, 1, 0, lane); };
  // right-hand side entry k times its row's scale 2^-e_k (see scale_row)
  auto rhs = [&](int k) {
    const int kk = min(k, nz - 1);
    const int ex = (int)(int8_t)piv[2 * plane + pidx(kk)];
    return k < nz ? ldexp(S(kk, fi), -ex) : 0.0;
  };
  // the same as two parts: the entry (zero past the last row) and the exponent
  auto rex = [&](int k) { return (int)(int8_t)piv[2 * plane + pidx(min(k, nz - 1))]; };
  auto rval = [&](int k) { return k < nz ? S(min(k, nz - 1), fi) : 0.0; };
  if constexpr ((PIPE & 1) != 0) {
    // ---- forward: row swaps and unit-lower elimination ----
    double y[B + 1];
#pragma unroll
    for (int t = 0; t <= B; ++t) y[t] = ldexp(rval(t), -rex(t));
    double lr[PF][B], rin[PF];
    int pv[PF], rie[PF];
#pragma unroll
    for (int d = 0; d < PF; ++d) {
      const int jj = d < nz ? d : nz - 1;
      pv[d] = piv[pidx(jj)];
#pragma unroll
      for (int t = 0; t < B; ++t) lr[d][t] = ld(Lb + tix(tile, nz, jj, B, t, lane));
      rin[d] = rval(d + B + 1);
      rie[d] = rex(d + B + 1);
    }
    for (int j0 = 0; j0 < nz; j0 += PF) {
#pragma unroll
      for (int d = 0; d < PF; ++d) {
        const int j = j0 + d;
        const int p = pv[d];
        const double v0 = y[0];
        double vp = v0;
#pragma unroll
        for (int t = 1; t <= B; ++t) vp = (p == t) ? y[t] : vp;
#pragma unroll
        for (int t = 1; t <= B; ++t) y[t] = (p == t) ? v0 : y[t];
        if (j < nz) S(j, fo) = vp;
#pragma unroll
        for (int t = 1; t <= B; ++t) y[t] -= lr[d][t - 1] * vp;
#pragma unroll
        for (int t = 0; t < B; ++t) y[t] = y[t + 1];
        y[B] = ldexp(rin[d], -rie[d]);
        // refill the consumed slot with row j + PF
        const int jn = j + PF;
        const int jj = jn < nz ? jn : nz - 1;
        pv[d] = piv[pidx(jj)];
#pragma unroll
        for (int t = 0; t < B; ++t) lr[d][t] = ld(Lb + tix(tile, nz, jj, B, t, lane));
        rin[d] = rval(jn + B + 1);
        rie[d] = rex(jn + B + 1);
      }
    }
  } else {
    // ---- forward: row swaps and unit-lower elimination ----
    double y[B + 1];
#pragma unroll
    for (int t = 0; t <= B; ++t) y[t] = rhs(t);
    double lr[PF][B], rin[PF];
    int pv[PF];
#pragma unroll
    for (int d = 0; d < PF; ++d) {
      const int jj = d < nz ? d : nz - 1;
      pv[d] = piv[pidx(jj)];
#pragma unroll
      for (int t = 0; t < B; ++t) lr[d][t] = ld(Lb + tix(tile, nz, jj, B, t, lane));
      rin[d] = rhs(d + B + 1);
    }
    for (int j0 = 0; j0 < nz; j0 += PF) {
#pragma unroll
      for (int d = 0; d < PF; ++d) {
        const int j = j0 + d;
        if (j < nz) {
          const int p = pv[d];
          const double v0 = y[0];
          double vp = v0;
#pragma unroll
          for (int t = 1; t <= B; ++t) vp = (p == t) ? y[t] : vp;
#pragma unroll
          for (int t = 1; t <= B; ++t) y[t] = (p == t) ? v0 : y[t];
          S(j, fo) = vp;
#pragma unroll
          for (int t = 1; t <= B; ++t) y[t] -= lr[d][t - 1] * vp;
#pragma unroll
          for (int t = 0; t < B; ++t) y[t] = y[t + 1];
          y[B] = rin[d];
          // refill the consumed slot with row j + PF
          const int jn = j + PF;
          const int jj = jn < nz ? jn : nz - 1;
          pv[d] = piv[pidx(jj)];
#pragma unroll
          for (int t = 0; t < B; ++t) lr[d][t] = ld(Lb + tix(tile, nz, jj, B, t, lane));
          rin[d] = rhs(jn + B + 1);
        }
      }
    }
  }
  if constexpr ((PIPE & 2) != 0) {
    // ---- backward: upper-triangular substitution ----
    double xw[K + 1];
#pragma unroll
    for (int t = 0; t <= K; ++t) xw[t] = 0.0;
    double ur[PB][K + 1], yin[PB];
    int unext[PB];
    // FP64 rows: buffer loads over this tile's U block (unused with FP32 factors)
    const __amdgpu_buffer_rsrc_t urs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(Ub + tix(tile, nz, 0, K + 1, 0, 0)), (short)0,
        (int)((size_t)nz * (K + 1) * T * sizeof(FT)), 0x00020000);
    auto urow = [&](double (&dst)[K + 1], int jj, int ue) {
#pragma unroll
      for (int t = 0; t <= K; ++t) {
        if constexpr (SKIP) {
          const unsigned off =
              t <= ue ? (unsigned)(tix(0, nz, jj, K + 1, t, lane) * sizeof(double)) : 0x80000000u;
          dst[t] = __builtin_bit_cast(double,
                                      __builtin_amdgcn_raw_buffer_load_b64(urs, off, 0, 2 /*nt*/));
        } else {
          dst[t] = ld(Ub + tix(tile, nz, jj, K + 1, t, lane));
        }
      }
    };
#pragma unroll
    for (int d = 0; d < PB; ++d) {
      const int jr = nz - 1 - d;
      const int jj = jr >= 0 ? jr : 0;
      urow(ur[d], jj, SKIP ? (int)ue_p[pidx(jj)] : K);
      unext[d] = SKIP ? ue_p[pidx(max(jr - PB, 0))] : K;
      yin[d] = S(jj, fo);
    }
    for (int j0 = nz - 1; j0 >= 0; j0 -= PB) {
#pragma unroll
      for (int d = 0; d < PB; ++d) {
        const int j = j0 - d;
        double s = yin[d];
#pragma unroll
        for (int t = 1; t <= K; ++t) s -= ur[d][t] * xw[t];
        const double xj = s / ur[d][0];
        if (j >= 0) S(j, fo) = xj;
#pragma unroll
        for (int t = K; t >= 2; --t) xw[t] = xw[t - 1];
        xw[1] = xj;
        // refill the consumed slot with row j - PB (steps below the first row work on
        // row 0 again and store nothing)
        const int jr = j - PB;
        const int jj = jr >= 0 ? jr : 0;
        urow(ur[d], jj, unext[d]);
        if constexpr (SKIP) unext[d] = ue_p[pidx(max(jr - PB, 0))];
        yin[d] = S(jj, fo);
      }
    }
  } else {
    // ---- backward: upper-triangular substitution ----
    double xw[K + 1];
#pragma unroll
    for (int t = 0; t <= K; ++t) xw[t] = 0.0;
    double ur[PB][K + 1], yin[PB];
    int unext[PB];
#pragma unroll
    for (int d = 0; d < PB; ++d) {
      const int jr = nz - 1 - d;
      const int jj = jr >= 0 ? jr : 0;
      const int ue = SKIP ? ue_p[pidx(jj)] : K;
#pragma unroll
      for (int t = 0; t <= K; ++t) {
        double v = 0.0;
        if (!SKIP || t <= ue) v = ld(Ub + tix(tile, nz, jj, K + 1, t, lane));
        ur[d][t] = v;
      }
      unext[d] = SKIP ? ue_p[pidx(max(jr - PB, 0))] : K;
      yin[d] = S(jj, fo);
    }
    for (int j0 = nz - 1; j0 >= 0; j0 -= PB) {
#pragma unroll
      for (int d = 0; d < PB; ++d) {
        const int j = j0 - d;
        if (j >= 0) {
          double s = yin[d];
#pragma unroll
          for (int t = 1; t <= K; ++t) s -= ur[d][t] * xw[t];
          const double xj = s / ur[d][0];
          S(j, fo) = xj;
#pragma unroll
          for (int t = K; t >= 2; --t) xw[t] = xw[t - 1];
          xw[1] = xj;
          // refill the consumed slot with row j - PB
          const int jr = j - PB;
          const int jj = jr >= 0 ? jr : 0;
          const int ue = unext[d];
#pragma unroll
          for (int t = 0; t <= K; ++t) {
            double v = 0.0;
            if (!SKIP || t <= ue) v = ld(Ub + tix(tile, nz, jj, K + 1, t, lane));
            ur[d][t] = v;
          }
          if constexpr (SKIP) unext[d] = ue_p[pidx(max(jr - PB, 0))];
          yin[d] = S(jj, fo);
        }
      }
    }
  }
}

// Reduced refinement for FP32-stored factors: d = r - S u with S applied
// matrix-free in FP64, correction delta from the factors, u += delta, until the
// correction is small, ||delta|| <= target ||u|| (a residual test would stop
// early: ||u_err|| can exceed ||d|| / ||r|| by the condition number of S), or
// max_sweeps.  Per column; the wavefront sweeps while any column needs one.
template <int N, typename FT, bool S3 = false, int NWS = HEVI_NWS>
__device__ void reduced_refine(Gll<N> tab, const OpsView& op, int Ne, double* ws,
                               int64_t tile, int lane, bool valid, double lambda,
                               const FT* __restrict__ Ub, const FT* __restrict__ Lb,
                               const uint8_t* __restrict__ piv, size_t plane, int max_sweeps,
                               double rel_target, int* sweeps_out, double* corr_out) {
  const int nz = op.nz;
  int sweeps = 0;
  double corr = INFINITY;
  for (;;) {
    const bool need = !(corr <= rel_target) && sweeps < max_sweeps;
    if (!__any(valid && need)) break;
    div_pass<N, NWS>(tab, op, Ne, ws, tile, lane, WS_U, WS_VR, WS_VT);
    pg_pass<N, S3, NWS>(tab, op, Ne, ws, tile, lane, WS_VR, WS_VT, WS_T);
    const double l2 = lambda * lambda;
    for (int k = 0; k < nz; ++k) {
      const double u = ws[tix(tile, nz, k, NWS, WS_U, lane)];
      const double Ku = ws[tix(tile, nz, k, NWS, WS_T, lane)];
      const double Su = (k == 0 || k == nz - 1) ? u : u - l2 * Ku;
      ws[tix(tile, nz, k, NWS, WS_T, lane)] = ws[tix(tile, nz, k, NWS, WS_R, lane)] - Su;
    }
    band_solve<N, FT, false, NWS>(Ub, Lb, piv, plane, ws, tile, nz, lane, WS_T, WS_D);
    if (need) {
      double d2 = 0.0, u2 = 0.0;
      for (int k = 0; k < nz; ++k) {
        const size_t iu = tix(tile, nz, k, NWS, WS_U, lane);
        const double d = ws[tix(tile, nz, k, NWS, WS_D, lane)];
        const double u = ws[iu] + d;
        ws[iu] = u;
        d2 += d * d;
        u2 += u * u;
      }
      corr = u2 > 0.0 ? sqrt(d2 / u2) : (d2 > 0.0 ? INFINITY : 0.0);
      ++sweeps;
    }
  }
  *sweeps_out = sweeps;
  *corr_out = corr;
}

// Reduced right-hand side r = grad(zeta).(b_U + lambda (PG b_Theta - Phi' grad(zeta) b_rho))
// of a 5-field vector b stored in scratch fields fb..fb+4 (zero at the lid nodes).
template <int N, bool S3 = false, int NWS = HEVI_NWS>
__device__ double reduced_rhs_pass(Gll<N> tab, const OpsView& op, int Ne, double* ws,
                                   int64_t tile, int lane, double lambda, int fb) {
  const int nz = op.nz;
  double c0 = 0.0, c1 = 0.0, c2 = 0.0, rn2 = 0.0;
  for (int e = 0; e < Ne; ++e) {
    double f0[N + 1], f1[N + 1], f2[N + 1];
#pragma unroll
    for (int j = 0; j <= N; ++j) {
      const int k = e * N + j;
      double p = op(k, OP_JCT) * ws[tix(tile, nz, k, NWS, fb + 4, lane)];
      if constexpr (S3) p += op.jpr(k) * ws[tix(tile, nz, k, NWS, fb + 0, lane)];
      f0[j] = p * op(k, OP_GX); f1[j] = p * op(k, OP_GY); f2[j] = p * op(k, OP_GZ);
    }
#pragma unroll
    for (int a = 0; a <= N; ++a) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
      for (int j = 0; j <= N; ++j) {
        const double d = tab.D[a * (N + 1) + j];
        s0 += d * f0[j]; s1 += d * f1[j]; s2 += d * f2[j];
      }
      s0 *= tab.w[a]; s1 *= tab.w[a]; s2 *= tab.w[a];
      if (a == 0) { s0 += c0; s1 += c1; s2 += c2; }
      if (a == N && e < Ne - 1) { c0 = s0; c1 = s1; c2 = s2; continue; }
      const int k = e * N + a;
      double r = 0.0;
      if (k != 0 && k != nz - 1) {
        const double gx = op(k, OP_GX), gy = op(k, OP_GY), gzz = op(k, OP_GZ);
        const double mi = op(k, OP_MINV), ph = op(k, OP_PHI);
        const double br = ws[tix(tile, nz, k, NWS, fb + 0, lane)];
        const double g1 = lambda * (-mi * s0 - ph * gx * br);
        const double g2 = lambda * (-mi * s1 - ph * gy * br);
        const double g3 = lambda * (-mi * s2 - ph * gzz * br);
        r = gx * (ws[tix(tile, nz, k, NWS, fb + 1, lane)] + g1) +
            gy * (ws[tix(tile, nz, k, NWS, fb + 2, lane)] + g2) +
            gzz * (ws[tix(tile, nz, k, NWS, fb + 3, lane)] + g3);
      }
      rn2 += r * r;
      ws[tix(tile, nz, k, NWS, WS_R, lane)] = r;
    }
  }
  return rn2;
}

// Back-substitution of the block elimination: with u (field WS_U) and the
// right-hand side b (fields fb..), d_rho = b_rho + lambda Drho u,
// d_Th = b_Th + lambda DTh u, d_U = b_U + lambda (PG d_Th - Phi' grad(zeta) d_rho)
// (interior), d_U = P(b_U) at the lid (P removes the normal component).
// Writes d into fields fx.. or adds it to them (accumulate).
template <int N, bool S3 = false, int NWS = HEVI_NWS>
__device__ void recover_pass(Gll<N> tab, const OpsView& op, int Ne, double* ws,
                             int64_t tile, int lane, double lambda, int fb, int fx,
                             bool accumulate) {
  const int nz = op.nz;
  div_pass<N, NWS>(tab, op, Ne, ws, tile, lane, WS_U, WS_VR, WS_VT);
  auto W = [&](int k, int f) -> double& { return ws[tix(tile, nz, k, NWS, f, lane)]; };
  double c0 = 0.0, c1 = 0.0, c2 = 0.0;
  for (int e = 0; e < Ne; ++e) {
    double f0[N + 1], f1[N + 1], f2[N + 1];
#pragma unroll
    for (int j = 0; j <= N; ++j) {
      const int k = e * N + j;
      const double dth = W(k, fb + 4) + lambda * W(k, WS_VT);
      double p = op(k, OP_JCT) * dth;
      if constexpr (S3) p += op.jpr(k) * (W(k, fb + 0) + lambda * W(k, WS_VR));
      f0[j] = p * op(k, OP_GX); f1[j] = p * op(k, OP_GY); f2[j] = p * op(k, OP_GZ);
    }
#pragma unroll
    for (int a = 0; a <= N; ++a) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
      for (int j = 0; j <= N; ++j) {
        const double d = tab.D[a * (N + 1) + j];
        s0 += d * f0[j]; s1 += d * f1[j]; s2 += d * f2[j];
      }
      s0 *= tab.w[a]; s1 *= tab.w[a]; s2 *= tab.w[a];
      if (a == 0) { s0 += c0; s1 += c1; s2 += c2; }
      if (a == N && e < Ne - 1) { c0 = s0; c1 = s1; c2 = s2; continue; }
      const int k = e * N + a;
      const double gx = op(k, OP_GX), gy = op(k, OP_GY), gzz = op(k, OP_GZ);
      const double dr = W(k, fb + 0) + lambda * W(k, WS_VR);
      const double dt = W(k, fb + 4) + lambda * W(k, WS_VT);
      double d1, d2, d3;
      const double b1 = W(k, fb + 1), b2 = W(k, fb + 2), b3 = W(k, fb + 3);
      if (k == 0 || k == nz - 1) {
        const double inv = 1.0 / sqrt(gx * gx + gy * gy + gzz * gzz);
        const double n0 = gx * inv, n1 = gy * inv, n2 = gzz * inv;
        const double dd = n0 * b1 + n1 * b2 + n2 * b3;
        d1 = b1 - n0 * dd; d2 = b2 - n1 * dd; d3 = b3 - n2 * dd;
      } else {
        const double mi = op(k, OP_MINV), ph = op(k, OP_PHI);
        d1 = b1 + lambda * (-mi * s0 - ph * gx * dr);
        d2 = b2 + lambda * (-mi * s1 - ph * gy * dr);
        d3 = b3 + lambda * (-mi * s2 - ph * gzz * dr);
        // normal part from grad(zeta).d_U = u (see b_stage_update)
        const double tn = (W(k, WS_U) - (gx * d1 + gy * d2 + gzz * d3)) /
                          (gx * gx + gy * gy + gzz * gzz);
        d1 += gx * tn; d2 += gy * tn; d3 += gzz * tn;
      }
      if (accumulate) {
        W(k, fx + 0) += dr; W(k, fx + 1) += d1; W(k, fx + 2) += d2; W(k, fx + 3) += d3;
        W(k, fx + 4) += dt;
      } else {
        W(k, fx + 0) = dr; W(k, fx + 1) = d1; W(k, fx + 2) = d2; W(k, fx + 3) = d3;
        W(k, fx + 4) = dt;
      }
    }
  }
}

// Full-system residual s = P(b) - A x = P(b) - x + lambda L_z x in FP64 for the
// vectors b (fields fb..) and x (fields fx..); rigid-lid momentum rows of A are
// identity rows, so there s_U = P(b_U) - x_U.  Writes fields fs..
template <int N, bool S3 = false, int NWS = HEVI_NWS>
__device__ void residual_pass(Gll<N> tab, const OpsView& op, int Ne, double* ws,
                              int64_t tile, int lane, double lambda, int fb, int fx, int fs) {
  const int nz = op.nz;
  auto W = [&](int k, int f) -> double& { return ws[tix(tile, nz, k, NWS, f, lane)]; };
  double cr = 0.0, ct = 0.0, c0 = 0.0, c1 = 0.0, c2 = 0.0;
  for (int e = 0; e < Ne; ++e) {
    double Ju[N + 1], Jtu[N + 1], f0[N + 1], f1[N + 1], f2[N + 1];
#pragma unroll
    for (int j = 0; j <= N; ++j) {
      const int k = e * N + j;
      const double gx = op(k, OP_GX), gy = op(k, OP_GY), gzz = op(k, OP_GZ);
      const double u = gx * W(k, fx + 1) + gy * W(k, fx + 2) + gzz * W(k, fx + 3);
      Ju[j] = op(k, OP_J) * u;
      Jtu[j] = op(k, OP_JTH) * u;
      double p = op(k, OP_JCT) * W(k, fx + 4);
      if constexpr (S3) p += op.jpr(k) * W(k, fx + 0);
      f0[j] = p * gx; f1[j] = p * gy; f2[j] = p * gzz;
    }
#pragma unroll
    for (int a = 0; a <= N; ++a) {
      double sr = 0.0, st = 0.0, s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
      for (int j = 0; j <= N; ++j) {
        const double d = tab.D[a * (N + 1) + j];
        sr += tab.w[j] * tab.D[j * (N + 1) + a] * Ju[j];
        st += d * Jtu[j];
        s0 += d * f0[j]; s1 += d * f1[j]; s2 += d * f2[j];
      }
      const double wa = tab.w[a];
      st *= wa; s0 *= wa; s1 *= wa; s2 *= wa;
      if (a == 0) { sr += cr; st += ct; s0 += c0; s1 += c1; s2 += c2; }
      if (a == N && e < Ne - 1) { cr = sr; ct = st; c0 = s0; c1 = s1; c2 = s2; continue; }
      const int k = e * N + a;
      const double mi = op(k, OP_MINV);
      const double gx = op(k, OP_GX), gy = op(k, OP_GY), gzz = op(k, OP_GZ);
      W(k, fs + 0) = W(k, fb + 0) - W(k, fx + 0) + lambda * (mi * sr);
      W(k, fs + 4) = W(k, fb + 4) - W(k, fx + 4) + lambda * (-mi * st);
      const double b1 = W(k, fb + 1), b2 = W(k, fb + 2), b3 = W(k, fb + 3);
      if (k == 0 || k == nz - 1) {
        const double inv = 1.0 / sqrt(gx * gx + gy * gy + gzz * gzz);
        const double n0 = gx * inv, n1 = gy * inv, n2 = gzz * inv;
        const double dd = n0 * b1 + n1 * b2 + n2 * b3;
        W(k, fs + 1) = b1 - n0 * dd - W(k, fx + 1);
        W(k, fs + 2) = b2 - n1 * dd - W(k, fx + 2);
        W(k, fs + 3) = b3 - n2 * dd - W(k, fx + 3);
      } else {
        const double ph = op(k, OP_PHI), xr = W(k, fx + 0);
        W(k, fs + 1) = b1 - W(k, fx + 1) + lambda * (-mi * s0 - ph * gx * xr);
        W(k, fs + 2) = b2 - W(k, fx + 2) + lambda * (-mi * s1 - ph * gy * xr);
        W(k, fs + 3) = b3 - W(k, fx + 3) + lambda * (-mi * s2 - ph * gzz * xr);
      }
    }
  }
}

// Stage solve with full-system FP64 iterative refinement (accuracy mode,
// hevi_refine.full_sweeps > 0), one lane per column, every field in scratch: the
// HEVI_NWS_FULL-field scratch of this mode (the other stage kernels use HEVI_NWS).
template <int N, typename FT, bool S3 = false>
__device__ __forceinline__ void b_stage_solve(int64_t tile_, HeviShapeDev sh, Gll<N> tab,
                                              double lambda, const double* __restrict__ ops,
                                              const FT* __restrict__ Ub, const FT* __restrict__ Lb,
                                              const uint8_t* __restrict__ piv,
                                              double* __restrict__ ws, const HeviTerms& E,
                                              const HeviTerms& Q, double* __restrict__ Qi,
                                              int max_sweeps, double rel_target, int full_sweeps,
                                              HeviDevInfo* info) {
  const int lane = threadIdx.x;
  const int64_t tile = tile_;
  const int64_t c = tile * T + lane;
  const bool valid = c < sh.ncols;
  const int64_t cc = valid ? c : sh.ncols - 1;
  const int nz = sh.nz, Ne = sh.Ne;
  const int64_t nc = sh.ncols;
  OpsView op{ops, tile, nz, lane, S3 ? pr_plane(ops, sh) : nullptr};
  bool nonfinite = false;

  // ---- pass 1: q^E, q^ = q^E + sum c_j Q_j, reduced right-hand side r ----
  double c0 = 0.0, c1 = 0.0, c2 = 0.0;
  for (int e = 0; e < Ne; ++e) {
    // q^E and q^ at the element's nodes; the term loop is outermost so that
    // each term issues (N+1)*5 independent coalesced loads
    double qE[N + 1][5], b[N + 1][5];
#pragma unroll
    for (int j = 0; j <= N; ++j)
#pragma unroll
      for (int v = 0; v < 5; ++v) qE[j][v] = 0.0;
    for (int t = 0; t < E.n; ++t) {
      const double* src = E.v[t];
      const double cf = E.coef[t];
#pragma unroll
      for (int j = 0; j <= N; ++j)
#pragma unroll
        for (int v = 0; v < 5; ++v) qE[j][v] += cf * ldn(src + cix(nz, nc, v, e * N + j, cc));
    }
#pragma unroll
    for (int j = 0; j <= N; ++j)
#pragma unroll
      for (int v = 0; v < 5; ++v) b[j][v] = qE[j][v];
    for (int t = 0; t < Q.n; ++t) {
      const double* src = Q.v[t];
      const double cf = Q.coef[t];
#pragma unroll
      for (int j = 0; j <= N; ++j)
#pragma unroll
        for (int v = 0; v < 5; ++v) b[j][v] += cf * ldn(src + cix(nz, nc, v, e * N + j, cc));
    }
    double f0[N + 1], f1[N + 1], f2[N + 1];
#pragma unroll
    for (int j = 0; j <= N; ++j) {
      const int k = e * N + j;
      double p = op(k, OP_JCT) * b[j][4];
      if constexpr (S3) p += op.jpr(k) * b[j][0];
      f0[j] = p * op(k, OP_GX); f1[j] = p * op(k, OP_GY); f2[j] = p * op(k, OP_GZ);
    }
#pragma unroll
    for (int a = 0; a <= N; ++a) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
      for (int j = 0; j <= N; ++j) {
        const double d = tab.D[a * (N + 1) + j];
        s0 += d * f0[j]; s1 += d * f1[j]; s2 += d * f2[j];
      }
      s0 *= tab.w[a]; s1 *= tab.w[a]; s2 *= tab.w[a];
      if (a == 0) { s0 += c0; s1 += c1; s2 += c2; }
      if (a == N && e < Ne - 1) { c0 = s0; c1 = s1; c2 = s2; continue; }
      const int k = e * N + a;
      const double gx = op(k, OP_GX), gy = op(k, OP_GY), gzz = op(k, OP_GZ);
      double r = 0.0;  // u = 0 at the rigid lid
      if (k != 0 && k != nz - 1) {
        const double mi = op(k, OP_MINV), ph = op(k, OP_PHI);
        const double g1 = lambda * (-mi * s0 - ph * gx * b[a][0]);
        const double g2 = lambda * (-mi * s1 - ph * gy * b[a][0]);
        const double g3 = lambda * (-mi * s2 - ph * gzz * b[a][0]);
        r = gx * (b[a][1] + g1) + gy * (b[a][2] + g2) + gzz * (b[a][3] + g3);
      }
      ws[tix(tile, nz, k, HEVI_NWS_FULL, WS_R, lane)] = r;
      // keep q^ (offset-free) for the full-system residual; Q_i holds q^E
#pragma unroll
      for (int v = 0; v < 5; ++v) ws[tix(tile, nz, k, HEVI_NWS_FULL, WS_B + v, lane)] = b[a][v];
      if (valid) {
#pragma unroll
        for (int v = 0; v < 5; ++v) stn(Qi + cix(nz, nc, v, k, c), qE[a][v]);
      }
    }
  }

  // ---- pass 2: S u = r (+ reduced FP64 refinement when the factors are FP32) ----
  band_solve<N, FT, false, HEVI_NWS_FULL>(Ub, Lb, piv, plane_size(sh), ws, tile, nz, lane, WS_R, WS_U);
  int sweeps = 0;
  double relres = 0.0;
  if (max_sweeps > 0)
    reduced_refine<N, FT, S3, HEVI_NWS_FULL>(tab, op, Ne, ws, tile, lane, valid, lambda, Ub, Lb, piv,
                              plane_size(sh), max_sweeps,
                              rel_target, &sweeps, &relres);

  {
    // ---- full-system FP64 iterative refinement on x = q_tt (offset-free) ----
    recover_pass<N, S3, HEVI_NWS_FULL>(tab, op, Ne, ws, tile, lane, lambda, WS_B, WS_X, false);
    for (int it = 0; it < full_sweeps; ++it) {
      residual_pass<N, S3, HEVI_NWS_FULL>(tab, op, Ne, ws, tile, lane, lambda, WS_B, WS_X, WS_S);
      reduced_rhs_pass<N, S3, HEVI_NWS_FULL>(tab, op, Ne, ws, tile, lane, lambda, WS_S);
      band_solve<N, FT, false, HEVI_NWS_FULL>(Ub, Lb, piv, plane_size(sh), ws, tile, nz, lane, WS_R, WS_U);
      if (max_sweeps > 0) {
        // the correction only needs the accuracy of the outer sweep
        int sw = 0;
        double cr = 0.0;
        reduced_refine<N, FT, S3, HEVI_NWS_FULL>(tab, op, Ne, ws, tile, lane, valid, lambda, Ub, Lb, piv,
                                  plane_size(sh), 1,
                                  rel_target, &sw, &cr);
        sweeps += sw;
      }
      recover_pass<N, S3, HEVI_NWS_FULL>(tab, op, Ne, ws, tile, lane, lambda, WS_S, WS_X, true);
    }
    // Q_i = q_tt - sum_j c_j Q_j = q^E + x - q^
    if (valid) {
      for (int k = 0; k < nz; ++k) {
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          const size_t i = cix(nz, nc, v, k, c);
          const double q = Qi[i] + ws[tix(tile, nz, k, HEVI_NWS_FULL, WS_X + v, lane)] -
                           ws[tix(tile, nz, k, HEVI_NWS_FULL, WS_B + v, lane)];
          Qi[i] = q;
          if (!isfinite(q)) nonfinite = true;
        }
      }
    }
  }

  if (valid) {
    if (nonfinite) flag(info, 9 /*HEVI_E_NONFINITE*/, c);
    if (max_sweeps > 0) {
      if (!(relres <= rel_target)) flag(info, 6 /*HEVI_E_NOT_CONVERGED*/, c);
      atomicMax(&info->max_sweeps, sweeps);
      const double rr = isfinite(relres) ? relres : 1.0e300;
      atomicMax((unsigned long long*)&info->max_res_bits,
                (unsigned long long)__double_as_longlong(rr));
    }
  }
}

// ---------------------------------------------------------------------------
// Momentum of the stage solution.  With u known, x_U = b_U + lambda G(x),
// G = PG x_Theta - Phi' grad(zeta) x_rho, splits into its part along
// grad(zeta), fixed by grad(zeta).x_U = u, and the tangential part of
// lambda PG x_Theta (gravity acts along grad(zeta) only):
//   x_U = P_t b_U + lambda (PG x_Theta)_t + grad(zeta) u / |grad(zeta)|^2.
// The stage passes evaluate PG x_Theta as PG b_Theta (pass 1) plus
// lambda PG DTh u (pass 3): two vectors ~|b_Theta| / |x_Theta| (about 100 at
// the later ARK stages) larger than their sum, each the derivative of a large
// field.  Taken whole, their rounding would swamp x_U.  Their tangential parts
// are formed term by term from the tangential part of each grad(zeta)_j at the
// output node k, which is exactly zero where grad(zeta)_j equals grad(zeta)_k
// (straight columns): pg_tangent returns
//   t_a = w_a sum_j D_aj p_j (|g_a|^2 g_j - (g_a . g_j) g_a) / |g_a|^2,
// g_j = grad(zeta) at node j of the element, p_j = (J c_Theta)_j Theta_j, so that
// (PG Theta)_t at node a is -M^-1 (sum of t_a over the elements containing it).
template <int N>
__device__ __forceinline__ double gdot(const double (&g0)[N + 1], const double (&g1)[N + 1],
                                       const double (&g2)[N + 1], int a, int j) {
#pragma clang fp contract(off)
  return g0[a] * g0[j] + g1[a] * g1[j] + g2[a] * g2[j];
}

// True if grad(zeta) is the same vector at every node of the element in every
// column of the wavefront (then every t_a is exactly zero).
template <int N>
__device__ __forceinline__ bool wave_straight(const double (&g0)[N + 1], const double (&g1)[N + 1],
                                              const double (&g2)[N + 1]) {
  bool same = true;
#pragma unroll
  for (int j = 1; j <= N; ++j)
    same = same && g0[j] == g0[0] && g1[j] == g1[0] && g2[j] == g2[0];
  return __all(same);
}

template <int N>
__device__ __forceinline__ void pg_tangent(Gll<N> tab, int a, const double (&p)[N + 1],
                                           const double (&g0)[N + 1], const double (&g1)[N + 1],
                                           const double (&g2)[N + 1], double& t0, double& t1,
                                           double& t2) {
  // products rounded on their own: |g_a|^2 g_j - (g_a . g_j) g_a is then exactly
  // zero whenever g_j == g_a
#pragma clang fp contract(off)
  const double gga = gdot<N>(g0, g1, g2, a, a);
  t0 = 0.0; t1 = 0.0; t2 = 0.0;
#pragma unroll
  for (int j = 0; j <= N; ++j) {
    if (j == a) continue;  // its tangential part is zero
    const double dj = gdot<N>(g0, g1, g2, a, j);
    const double dp = tab.D[a * (N + 1) + j] * p[j];
    t0 += dp * (gga * g0[j] - dj * g0[a]);
    t1 += dp * (gga * g1[j] - dj * g1[a]);
    t2 += dp * (gga * g2[j] - dj * g2[a]);
  }
  const double sc = tab.w[a] / gga;
  t0 *= sc; t1 *= sc; t2 *= sc;
}

// ---------------------------------------------------------------------------
// Fast stage solve as three kernels: k_stage_rhs (element-chunked),
// k_stage_bsolve (one lane per column), k_stage_update (element-chunked).

// pass 1: q^E = sum e_t E_t and q^ = q^E + sum c_j Q_j at the owned nodes; writes
// the reduced right-hand side r = grad(zeta).(q^_U + lambda (PG q^_Theta - Phi'
// grad(zeta) q^_rho)) (0 at the lid) and
// Q_i <- (q^E_rho, q^E_U - n (n . q^_U) + lambda (PG q^_Theta)_t [interior], q^E_Theta)
// with n = grad(zeta)/|grad(zeta)| and ( )_t the tangential part (see pg_tangent).
// The term loop is outermost so that each term issues (N+1)*5 independent loads.
template <int N, bool LDSRU, bool TILT, bool S3 = false>
__device__ __forceinline__ void b_stage_rhs(int64_t tile_, HeviShapeDev sh, Gll<N> tab,
                                            double lambda, const double* __restrict__ ops,
                                            double* __restrict__ ws, const HeviTerms& E,
                                            const HeviTerms& Q, double* __restrict__ Qi,
                                            double* ru = nullptr, int cw = 1) {
  const int Ne = sh.Ne, nz = sh.nz;
  const Chunk ch = chunk_of(Ne, tile_, cw);
  if (ch.e0 >= ch.e1) return;
  const int lane = ch.lane;
  const int64_t tile = ch.tile;
  const int64_t c = tile * T + lane;
  const bool valid = c < sh.ncols;
  const int64_t cc = valid ? c : sh.ncols - 1;
  const int64_t nc = sh.ncols;
  OpsView op{ops, tile, nz, lane, S3 ? pr_plane(ops, sh) : nullptr};
  if (ch.e0 == 0) ws[tix(tile, nz, 0, HEVI_NWS, WS_T, lane)] = 0.0;  // per-column flag
  double c0 = 0.0, c1 = 0.0, c2 = 0.0, d0 = 0.0, d1 = 0.0, d2 = 0.0;
  // node eN is shared by elements e-1 and e: its sums and operator values are
  // carried over instead of being loaded again (the first element loads all)
  double kqE[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, kb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  double kg0 = 0.0, kg1 = 0.0, kg2 = 0.0, kmi = 0.0, kph = 0.0, kpt = 0.0;
  auto element = [&](const int e, auto first) {
    constexpr bool FIRST = decltype(first)::value;
    double qE[N + 1][5], b[N + 1][5];
    // E's first vector (q^n in an ARK stage) is loaded once; a Q term naming the
    // same vector (Q_1 = q^n) reuses it
    double e0[N + 1][5];
#pragma unroll
    for (int j = FIRST ? 0 : 1; j <= N; ++j)
#pragma unroll
      for (int v = 0; v < 5; ++v) e0[j][v] = ldn(E.v[0] + cix(nz, nc, v, e * N + j, cc));
#pragma unroll
    for (int j = 0; j <= N; ++j)
#pragma unroll
      for (int v = 0; v < 5; ++v) qE[j][v] = (!FIRST && j == 0) ? kqE[v] : E.coef[0] * e0[j][v];
#pragma unroll 2
    for (int t = 1; t < E.n; ++t) {
      const double* src = E.v[t];
      const double cf = E.coef[t];
#pragma unroll
      for (int j = FIRST ? 0 : 1; j <= N; ++j)
#pragma unroll
        for (int v = 0; v < 5; ++v) qE[j][v] += cf * ldn(src + cix(nz, nc, v, e * N + j, cc));
    }
#pragma unroll
    for (int j = 0; j <= N; ++j)
#pragma unroll
      for (int v = 0; v < 5; ++v) b[j][v] = (!FIRST && j == 0) ? kb[v] : qE[j][v];
    const bool alias0 = Q.n > 0 && Q.v[0] == E.v[0];
    if (alias0) {
      const double cf = Q.coef[0];
#pragma unroll
      for (int j = FIRST ? 0 : 1; j <= N; ++j)
#pragma unroll
        for (int v = 0; v < 5; ++v) b[j][v] += cf * e0[j][v];
    }
#pragma unroll 2
    for (int t = alias0 ? 1 : 0; t < Q.n; ++t) {
      const double* src = Q.v[t];
      const double cf = Q.coef[t];
#pragma unroll
      for (int j = FIRST ? 0 : 1; j <= N; ++j)
#pragma unroll
        for (int v = 0; v < 5; ++v) b[j][v] += cf * ldn(src + cix(nz, nc, v, e * N + j, cc));
    }
    double g0[N + 1], g1[N + 1], g2[N + 1], mi[N + 1], ph[N + 1], pt[N + 1];
#pragma unroll
    for (int j = 0; j <= N; ++j) {
      if (!FIRST && j == 0) {
        g0[0] = kg0; g1[0] = kg1; g2[0] = kg2; mi[0] = kmi; ph[0] = kph; pt[0] = kpt;
        continue;
      }
      const int k = e * N + j;
      g0[j] = op(k, OP_GX); g1[j] = op(k, OP_GY); g2[j] = op(k, OP_GZ);
      mi[j] = op(k, OP_MINV); ph[j] = op(k, OP_PHI);
      pt[j] = op(k, OP_JCT) * b[j][4];
      if constexpr (S3) pt[j] += op.jpr(k) * b[j][0];
    }
    // TILT: some column's grad(zeta) varies; elsewhere every tangential term is zero
    const bool straight = !TILT || wave_straight<N>(g0, g1, g2);
    double ro[N + 1], ho[N + 1][3];
#pragma unroll
    for (int a = 0; a <= N; ++a) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
      for (int j = 0; j <= N; ++j) {
        const double d = tab.D[a * (N + 1) + j] * pt[j];
        s0 += d * g0[j]; s1 += d * g1[j]; s2 += d * g2[j];
      }
      s0 *= tab.w[a]; s1 *= tab.w[a]; s2 *= tab.w[a];
      double t0 = 0.0, t1 = 0.0, t2 = 0.0;
      if constexpr (TILT) {
        if (!straight) pg_tangent<N>(tab, a, pt, g0, g1, g2, t0, t1, t2);
      }
      if (a == 0) { s0 += c0; s1 += c1; s2 += c2; t0 += d0; t1 += d1; t2 += d2; }
      if (a == N) { c0 = s0; c1 = s1; c2 = s2; d0 = t0; d1 = t1; d2 = t2; }
      const int k = e * N + a;
      const double gx = g0[a], gy = g1[a], gzz = g2[a];
      // normal part of q^_U removed (lid: the rigid-lid projection; interior: pass 3
      // adds the normal part of the solution, grad(zeta) u / |grad(zeta)|^2)
      const double gg = gx * gx + gy * gy + gzz * gzz;
      const double bn = (gx * b[a][1] + gy * b[a][2] + gzz * b[a][3]) / gg;
      ho[a][0] = qE[a][1] - gx * bn; ho[a][1] = qE[a][2] - gy * bn; ho[a][2] = qE[a][3] - gzz * bn;
      if (k == 0 || k == nz - 1) {
        ro[a] = 0.0;
      } else {
        const double q1 = lambda * (-mi[a] * s0 - ph[a] * gx * b[a][0]);
        const double q2 = lambda * (-mi[a] * s1 - ph[a] * gy * b[a][0]);
        const double q3 = lambda * (-mi[a] * s2 - ph[a] * gzz * b[a][0]);
        ro[a] = gx * (b[a][1] + q1) + gy * (b[a][2] + q2) + gzz * (b[a][3] + q3);
        // tangential part of lambda PG q^_Theta
        const double lm = lambda * mi[a];
        ho[a][0] -= lm * t0; ho[a][1] -= lm * t1; ho[a][2] -= lm * t2;
      }
    }
    if (e >= ch.e0) {
      const int amax = (e == Ne - 1) ? N : N - 1;
#pragma unroll
      for (int a = 0; a <= N; ++a) {
        if (a <= amax) {
          const int k = e * N + a;
          if constexpr (LDSRU) ru[k * T + lane] = ro[a];
          else ws[tix(tile, nz, k, HEVI_NWS, WS_R, lane)] = ro[a];
          if (valid) {
            stn(Qi + cix(nz, nc, 0, k, c), qE[a][0]);
            stn(Qi + cix(nz, nc, 1, k, c), ho[a][0]);
            stn(Qi + cix(nz, nc, 2, k, c), ho[a][1]);
            stn(Qi + cix(nz, nc, 3, k, c), ho[a][2]);
            stn(Qi + cix(nz, nc, 4, k, c), qE[a][4]);
          }
        }
      }
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) { kqE[v] = qE[N][v]; kb[v] = b[N][v]; }
    kg0 = g0[N]; kg1 = g1[N]; kg2 = g2[N]; kmi = mi[N]; kph = ph[N]; kpt = pt[N];
  };
  int e = max(ch.e0 - 1, 0);
  element(e, std::true_type{});
  for (++e; e < ch.e1; ++e) element(e, std::false_type{});
}

// pass 2: S u = r, one lane per column (+ reduced FP64 refinement for FP32 factors)
template <int N, typename FT, bool REFINE, bool S3 = false>
__device__ __forceinline__ void b_stage_bsolve(int64_t tile_, HeviShapeDev sh, Gll<N> tab,
                                               double lambda, const double* __restrict__ ops,
                                               const FT* __restrict__ Ub, const FT* __restrict__ Lb,
                                               const uint8_t* __restrict__ piv,
                                               double* __restrict__ ws, int max_sweeps,
                                               double rel_target, HeviDevInfo* info) {
  const int lane = threadIdx.x;
  const int64_t tile = tile_;
  const int64_t c = tile * T + lane;
  const bool valid = c < sh.ncols;
  const int nz = sh.nz;
  band_solve<N, FT>(Ub, Lb, piv, plane_size(sh), ws, tile, nz, lane, WS_R, WS_U);
  if (REFINE && max_sweeps > 0) {
    OpsView op{ops, tile, nz, lane, S3 ? pr_plane(ops, sh) : nullptr};
    int sweeps = 0;
    double corr = 0.0;
    reduced_refine<N, FT, S3>(tab, op, sh.Ne, ws, tile, lane, valid, lambda, Ub, Lb, piv,
                              plane_size(sh), max_sweeps,
                              rel_target, &sweeps, &corr);
    if (valid) {
      if (!(corr <= rel_target)) flag(info, 6 /*HEVI_E_NOT_CONVERGED*/, c);
      atomicMax(&info->max_sweeps, sweeps);
      const double rr = isfinite(corr) ? corr : 1.0e300;
      atomicMax((unsigned long long*)&info->max_res_bits,
                (unsigned long long)__double_as_longlong(rr));
    }
  }
}

// pass 3: v_rho = Drho u, v_Th = DTh u; Q_i += (lambda v_rho, lambda^2 (PG v_Th)_t +
// grad(zeta) u / |grad(zeta)|^2 [interior], lambda v_Th), ( )_t the tangential part.
// An element needs u on its neighbours too (the DSS of Drho u, DTh u at its end
// nodes), so each iteration loads u and the operator on nodes (e-1)N .. (e+2)N.
template <int N, bool LDSRU, bool TILT, bool S3 = false>
__device__ __forceinline__ void b_stage_update(int64_t tile_, HeviShapeDev sh, Gll<N> tab,
                                               double lambda, const double* __restrict__ ops,
                                               double* __restrict__ ws, double* __restrict__ Qi,
                                               HeviDevInfo* info, double* ru = nullptr,
                                               int cw = 1) {
  constexpr int NC = 3 * N + 1;
  const int Ne = sh.Ne, nz = sh.nz;
  const Chunk ch = chunk_of(Ne, tile_, cw);
  if (ch.e0 >= ch.e1) return;
  const int lane = ch.lane;
  const int64_t tile = ch.tile;
  const int64_t c = tile * T + lane;
  const bool valid = c < sh.ncols;
  const int64_t cc = valid ? c : sh.ncols - 1;
  const int64_t nc = sh.ncols;
  OpsView op{ops, tile, nz, lane, S3 ? pr_plane(ops, sh) : nullptr};
  const double l2 = lambda * lambda;
  bool nonfinite = false;
  double c0 = 0.0, c1 = 0.0, c2 = 0.0;
  // consecutive elements share nodes eN .. (e+2)N of the u window and node eN of
  // the operator and Q_i: those values are carried over instead of loaded again
  double kJu[2 * N + 1], kJtu[2 * N + 1], kq[5];
  double kg0 = 0.0, kg1 = 0.0, kg2 = 0.0, kmi = 0.0, kjc = 0.0, kjp = 0.0;
  auto element = [&](const int e, auto first) {
    constexpr bool FIRST = decltype(first)::value;
    // ---- loads: u, J, J theta0 on nodes (e-1)N .. (e+2)N; operator and Q_i on the element
    double Ju[NC], Jtu[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      if (!FIRST && q <= 2 * N) {
        Ju[q] = kJu[q];
        Jtu[q] = kJtu[q];
        continue;
      }
      const int k = (e - 1) * N + q;
      const int kk = min(max(k, 0), nz - 1);
      const double u = LDSRU ? ru[kk * T + lane] : ws[tix(tile, nz, kk, HEVI_NWS, WS_U, lane)];
      const double in = (k >= 0 && k < nz) ? 1.0 : 0.0;
      Ju[q] = in * op(kk, OP_J) * u;
      Jtu[q] = in * op(kk, OP_JTH) * u;
    }
    double g0[N + 1], g1[N + 1], g2[N + 1], mi[N + 1], jc[N + 1], jp[N + 1], q[N + 1][5];
#pragma unroll
    for (int j = 0; j <= N; ++j) {
      if (!FIRST && j == 0) {
        g0[0] = kg0; g1[0] = kg1; g2[0] = kg2; mi[0] = kmi; jc[0] = kjc; jp[0] = kjp;
#pragma unroll
        for (int v = 0; v < 5; ++v) q[0][v] = kq[v];
        continue;
      }
      const int k = e * N + j;
      g0[j] = op(k, OP_GX); g1[j] = op(k, OP_GY); g2[j] = op(k, OP_GZ);
      mi[j] = op(k, OP_MINV); jc[j] = op(k, OP_JCT);
      jp[j] = S3 ? op.jpr(k) : 0.0;
#pragma unroll
      for (int v = 0; v < 5; ++v) q[j][v] = ldn(Qi + cix(nz, nc, v, k, cc));
    }
    // node N as loaded (before this element's update) is node 0 of the next
#pragma unroll
    for (int v = 0; v < 5; ++v) kq[v] = q[N][v];
    kg0 = g0[N]; kg1 = g1[N]; kg2 = g2[N]; kmi = mi[N]; kjc = jc[N]; kjp = jp[N];
#pragma unroll
    for (int t = 0; t <= 2 * N; ++t) { kJu[t] = Ju[N + t]; kJtu[t] = Jtu[N + t]; }
    // ---- v_rho, v_Th at the element's nodes (contributions of elements e-1, e, e+1)
    double sr[N + 1], st[N + 1];
#pragma unroll
    for (int a = 0; a <= N; ++a) {
      double r = 0.0, t = 0.0;
#pragma unroll
      for (int j = 0; j <= N; ++j) {
        r += tab.w[j] * tab.D[j * (N + 1) + a] * Ju[N + j];
        t += tab.D[a * (N + 1) + j] * Jtu[N + j];
      }
      sr[a] = r;
      st[a] = tab.w[a] * t;
    }
    {
      // element e-1 into node 0 (its node N), element e+1 into node N (its node 0)
      double r0 = 0.0, t0 = 0.0, rN = 0.0, tN = 0.0;
#pragma unroll
      for (int j = 0; j <= N; ++j) {
        r0 += tab.w[j] * tab.D[j * (N + 1) + N] * Ju[j];
        t0 += tab.D[N * (N + 1) + j] * Jtu[j];
        rN += tab.w[j] * tab.D[j * (N + 1) + 0] * Ju[2 * N + j];
        tN += tab.D[0 * (N + 1) + j] * Jtu[2 * N + j];
      }
      sr[0] += r0; st[0] += tab.w[N] * t0;
      sr[N] += rN; st[N] += tab.w[0] * tN;
    }
    double vr[N + 1], vt[N + 1], pt[N + 1];
#pragma unroll
    for (int j = 0; j <= N; ++j) {
      vr[j] = mi[j] * sr[j];
      vt[j] = -mi[j] * st[j];
      pt[j] = jc[j] * vt[j];
      if constexpr (S3) pt[j] += jp[j] * vr[j];
    }
    // ---- stage update: rho and Theta; momentum = the tangential part of
    // lambda^2 PG v_Th plus the normal part grad(zeta) u / |grad(zeta)|^2 (see
    // pg_tangent; pass 1 left q^E_U with q^_U's normal part removed)
    // TILT: some column's grad(zeta) varies; elsewhere every tangential term is zero
    const bool straight = !TILT || wave_straight<N>(g0, g1, g2);
#pragma unroll
    for (int a = 0; a <= N; ++a) {
      double t0 = 0.0, t1 = 0.0, t2 = 0.0;
      if constexpr (TILT) {
        if (!straight) pg_tangent<N>(tab, a, pt, g0, g1, g2, t0, t1, t2);
      }
      if (a == 0) { t0 += c0; t1 += c1; t2 += c2; }
      if (a == N) { c0 = t0; c1 = t1; c2 = t2; }
      const int k = e * N + a;
      const bool lid = (k == 0) || (k == nz - 1);
      q[a][0] += lambda * vr[a];
      q[a][4] += lambda * vt[a];
      if (!lid) {
        const double uk = LDSRU ? ru[k * T + lane] : ws[tix(tile, nz, k, HEVI_NWS, WS_U, lane)];
        const double un = uk / (g0[a] * g0[a] + g1[a] * g1[a] + g2[a] * g2[a]);
        const double lm = l2 * mi[a];
        q[a][1] += g0[a] * un - lm * t0;
        q[a][2] += g1[a] * un - lm * t1;
        q[a][3] += g2[a] * un - lm * t2;
      }
    }
    if (e >= ch.e0 && valid) {
      const int amax = (e == Ne - 1) ? N : N - 1;
#pragma unroll
      for (int a = 0; a <= N; ++a) {
        if (a <= amax) {
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            stn(Qi + cix(nz, nc, v, e * N + a, c), q[a][v]);
            if (!isfinite(q[a][v])) nonfinite = true;
          }
        }
      }
    }
  };
  {
    int e = max(ch.e0 - 1, 0);
    element(e, std::true_type{});
    for (++e; e < ch.e1; ++e) element(e, std::false_type{});
  }
  if (nonfinite) {
    // count each column once: the first wavefront to flag it wins the exchange
    unsigned long long* fl =
        (unsigned long long*)&ws[tix(tile, nz, 0, HEVI_NWS, WS_T, lane)];
    if (atomicCAS(fl, 0ull, 1ull) == 0ull) flag(info, 9 /*HEVI_E_NONFINITE*/, c);
    else {
      atomicMax(&info->status, 9);
      atomicMin((unsigned long long*)&info->first_bad, (unsigned long long)c);
    }
  }
}

}  // namespace
