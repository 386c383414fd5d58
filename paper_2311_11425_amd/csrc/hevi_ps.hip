// hevi_ps.hip -- LHEVI-PS column solves (Sec. 4.3.1): the linear operator is the
// Jacobian of the set-2C vertical operator at a moving state q0 = (rho0, U0, Theta0)
// (a previous solution), not at a state at rest.
//
// With U0 != 0 the flux Jacobian K(q0) (Appendix A.3, eq. set2c_jacobian at a
// general state) has advection entries w = grad(zeta).u0 on its diagonal blocks,
// so the rho-theta and momentum blocks of A = I - lambda L_z are no longer
// identities and the exact elimination of the reference-state path does not
// apply.  These kernels factor the whole 5 n_z band instead, as the paper does with
// LAPACK's banded LU (Sec. 4.2.2): unknown (node k, variable v) at 5k + v, KL =
// 5(N+1) - 1 sub- and super-diagonals, U rows of width W = 2 KL + 1 (partial
// pivoting fills KL more super-diagonals).
//
// Mapping: one wavefront per column.  Lane l holds window column l of the
// (KL + 1) x W active window of the band LU (rows j..j+KL, columns j..j+W-1) in
// registers; step j takes the pivot from lane 0's column (largest magnitude, lowest
// row on ties), broadcasts the multipliers, eliminates, stores U row j (W lanes),
// the KL multipliers and the pivot offset, and shifts the window one lane to the
// left, computing the entering row of A on the fly from the compact operator.
// The stage solve runs the substitutions with the window of the vector in
// registers and q^E, q^ and the solution of the column in LDS.
//
// Rows are equilibrated as they enter the window: each row of A is scaled by 2^-e,
// e the binary exponent of its largest entry (exact; LAPACK's row equilibration with
// power-of-two scales).  The rows of A mix variables of very different size (the
// continuity, momentum and rho-theta rows), and unscaled pivoting on them lost a digit
// at the ne = 30 shape; the solves scale the right-hand side the same way.
//
// Factor storage per column (column-contiguous): U by columns of the band, [n][WS] with
// entry (c, l) = U[c - l][c] (what the column-oriented back substitution reads, in order;
// the entries above the first row, l > c, and the padding are not written); L [n][KLS]
// (multipliers of step j for rows j+1..j+KL); WS and KLS are W and KL rounded up to whole
// 128-byte lines; four byte planes, each [ncols][n]: the pivot offsets, the row exponents
// e (signed), the extent of each U column (largest offset l of a nonzero entry) and of
// each step's multipliers (largest i of a nonzero one), n = 5 n_z.  At N = 4, n_z = 41:
// 158,260 bytes per column.
#include "hevi_device.h"

namespace {

template <int N>
constexpr int kPsKL = 5 * (N + 1) - 1;
template <int N>
constexpr int kPsW = 2 * kPsKL<N> + 1;
// Stored widths: a U column and an L row padded to whole 128-byte cache lines, so that a
// read up to an extent touches only the lines the extent needs.
template <int N>
constexpr int kPsWS = (kPsW<N> + 15) / 16 * 16;
template <int N>
constexpr int kPsKLS = (kPsKL<N> + 15) / 16 * 16;

// Whole-wavefront lane shift by DPP (wave_shl:1, a VALU move): lane i takes lane i+1's
// value, lane 63 takes 0.
__device__ __forceinline__ double shift_down1(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x130, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x130, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

// Exchange of register a[0] with a[p], p uniform, as one branch to the matching case
// (a chain of selects over every slot otherwise).
template <int I, int KL>
__device__ __forceinline__ void swap_first(double (&a)[KL + 1], int p) {
  if constexpr (I <= KL) {
    if (p == I) {
      const double t = a[0];
      a[0] = a[I];
      a[I] = t;
      return;
    }
    swap_first<I + 1, KL>(a, p);
  }
}

__device__ __forceinline__ double bcast(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// DPP moves of a double within the wavefront: dpp_z fills lanes whose source is invalid
// with zero (no copy of the old value needed), dpp_d keeps their own value.  The maximum
// over all 64 lanes of values >= -1 whose maximum is >= 0 (magnitudes, with -1 marking
// lanes out of the search) by an inclusive scan: row_shr:1,2,4,8 leave each 16-lane row's
// maximum (or 0) in its lane 15, row_bcast:15 and row_bcast:31 carry it into the following
// rows, so lane 63 ends with the maximum of the wavefront.
template <int CTRL>
__device__ __forceinline__ double dpp_z(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(v), __double2loint(v), CTRL, ROWS,
                                             0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(v), __double2hiint(v), CTRL, ROWS,
                                             0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp_z<0x111>(v));
  v = fmax(v, dpp_z<0x112>(v));
  v = fmax(v, dpp_z<0x114>(v));
  v = fmax(v, dpp_z<0x118>(v));
  v = fmax(v, dpp_d<0x142, 0xA>(v));
  v = fmax(v, dpp_d<0x143, 0xC>(v));
  return bcast(v, 63);
}

// The operator of one column as the PS kernels read it (lane-dependent nodes).
struct PsCol {
  const double* ops;
  const double* u0;  // velocity planes of the linearisation state
  size_t pe;         // elements per plane
  int64_t tile;
  int nz, Ne, cl;    // cl: the column's lane within its tile
  __device__ __forceinline__ double op(int k, int f) const {
    return ops[tix(tile, nz, k, HEVI_NOPS, f, cl)];
  }
  __device__ __forceinline__ double u(int k, int m) const {
    return u0[(size_t)m * pe + ((size_t)tile * nz + k) * T + cl];
  }
};

// The operator of one column copied into LDS at the start of the factorisation
// (field-major, s[f * nz + k]): J, grad(zeta), u0, J c_Theta, J theta0, M^-1, the
// gravity coefficient and w = grad(zeta).u0 per node.  The entering rows of every step
// then read LDS instead of memory.
enum { PN_J = 0, PN_G = 1, PN_U = 4, PN_JCT = 7, PN_JTH = 8, PN_MINV = 9, PN_PHI = 10,
       PN_W = 11, PN_FIELDS = 12 };
struct PsNodes {
  const double* s;
  int nz;
  __device__ __forceinline__ double f(int fld, int k) const { return s[fld * nz + k]; }
};

__device__ void ps_load_nodes(const PsCol& P, double* s) {
  const int nz = P.nz, lane = threadIdx.x;
  for (int q = lane; q < (PN_FIELDS - 1) * nz; q += T) {
    const int fld = q / nz, k = q - fld * nz;
    double v;
    if (fld == PN_J) v = P.op(k, OP_J);
    else if (fld < PN_U) v = P.op(k, OP_GX + (fld - PN_G));
    else if (fld < PN_JCT) v = P.u(k, fld - PN_U);
    else if (fld == PN_JCT) v = P.op(k, OP_JCT);
    else if (fld == PN_JTH) v = P.op(k, OP_JTH);
    else if (fld == PN_MINV) v = P.op(k, OP_MINV);
    else v = P.op(k, OP_PHI);
    s[q] = v;
  }
  __syncthreads();
  for (int k = lane; k < nz; k += T)
    s[PN_W * nz + k] = s[PN_G * nz + k] * s[PN_U * nz + k] +
                       s[(PN_G + 1) * nz + k] * s[(PN_U + 1) * nz + k] +
                       s[(PN_G + 2) * nz + k] * s[(PN_U + 2) * nz + k];
  __syncthreads();
}

// Entry (r, c) of A = I - lambda L_z (zero outside the matrix or the band):
//   L_z = -M^-1 B - gravity,  B_(k,a),(kc,b) = sum over the elements e holding both
//   nodes of  w_i D_ij J_kc K_kc[a][b]  (a > 0, strong)  or  -w_j D_ji J_kc K_kc[0][b]
//   (the continuity row, weak), i, j the local indices of k, kc in e; the momentum rows
//   of the bottom and top nodes are identity rows (rigid lid).  K at the state q0,
//   u0 = U0/rho0, w = grad(zeta).u0:
//   K[rho][U_m] = g_m;  K[U_l][rho] = -u0_l w, K[U_l][U_m] = delta_lm w + u0_l g_m,
//   K[U_l][Theta] = g_l c_Theta;  K[Theta][rho] = -theta0 w, K[Theta][U_m] = theta0 g_m,
//   K[Theta][Theta] = w.
template <int N>
__device__ double ps_entry(const PsNodes& P, int Ne, const double* Dsh, const double* wsh,
                           double lambda, int r, int c) {
  const int nz = P.nz, n = 5 * nz;
  if (r < 0 || r >= n || c < 0 || c >= n) return 0.0;
  const int k = r / 5, a = r - 5 * k, kc = c / 5, b = c - 5 * kc;
  const double delta = r == c ? 1.0 : 0.0;
  if (a >= 1 && a <= 3 && (k == 0 || k == nz - 1)) return delta;
  const int dk = kc - k;
  if (dk > N || dk < -N) return delta;
  const double J = P.f(PN_J, kc);
  const double w = P.f(PN_W, kc);
  const double gb = (b >= 1 && b <= 3) ? P.f(PN_G + b - 1, kc) : 0.0;
  double JK;
  if (a == 0) {
    JK = J * gb;
  } else if (a <= 3) {
    const double ul = P.f(PN_U + a - 1, kc);
    if (b == 0) JK = -J * ul * w;
    else if (b <= 3) JK = J * ((a == b ? w : 0.0) + ul * gb);
    else JK = P.f(PN_G + a - 1, kc) * P.f(PN_JCT, kc);
  } else {
    const double Jth = P.f(PN_JTH, kc);
    if (b == 0) JK = -Jth * w;
    else if (b <= 3) JK = Jth * gb;
    else JK = J * w;
  }
  double Bs = 0.0;
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    // the element in which k is local node N (side 0) or local node < N (side 1)
    const int e = side == 0 ? ((k % N == 0) ? k / N - 1 : -1) : k / N;
    if (e < 0 || e >= Ne) continue;
    const int i = k - e * N, j = kc - e * N;
    if (j < 0 || j > N) continue;
    const double coef = a == 0 ? -wsh[j] * Dsh[j * (N + 1) + i] : wsh[i] * Dsh[i * (N + 1) + j];
    Bs += coef * JK;
  }
  double L = -P.f(PN_MINV, k) * Bs;
  if (kc == k && b == 0 && a >= 1 && a <= 3) L -= P.f(PN_PHI, k) * P.f(PN_G + a - 1, k);
  return delta - lambda * L;
}

// The five rows of node k (variables a = 0..4) of A at the columns c0 + lane, as
// ps_entry gives them, with the lane's node lookups and element coefficients shared by
// the five rows.
template <int N>
__device__ void ps_node_rows(const PsNodes& P, int Ne, const double* Dsh, const double* wsh,
                             double lambda, int k, int c0, double (&row)[5]) {
  const int nz = P.nz, n = 5 * nz;
  const int c = c0 + (int)threadIdx.x;
  const int kc = c / 5, b = c - 5 * kc, dk = kc - k;
  const bool band = c < n && dk <= N && dk >= -N;
  const int kq = band ? kc : k;  // an in-range node for the loads
  const double J = P.f(PN_J, kq), w = P.f(PN_W, kq);
  const double g[3] = {P.f(PN_G, kq), P.f(PN_G + 1, kq), P.f(PN_G + 2, kq)};
  const double u[3] = {P.f(PN_U, kq), P.f(PN_U + 1, kq), P.f(PN_U + 2, kq)};
  const double jct = P.f(PN_JCT, kq), jth = P.f(PN_JTH, kq);
  const double gb = b == 1 ? g[0] : b == 2 ? g[1] : b == 3 ? g[2] : 0.0;
  // per element side: the strong (rows a >= 1) and weak (row a = 0) coefficients
  double cs[2], cw[2];
  bool on[2];
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int e = side == 0 ? ((k % N == 0) ? k / N - 1 : -1) : k / N;
    const int i = k - e * N, jj = kc - e * N;
    on[side] = band && e >= 0 && e < Ne && jj >= 0 && jj <= N;
    const int ic = min(max(i, 0), N), jc = min(max(jj, 0), N);
    cs[side] = wsh[ic] * Dsh[ic * (N + 1) + jc];
    cw[side] = -wsh[jc] * Dsh[jc * (N + 1) + ic];
  }
  const double minv = P.f(PN_MINV, k), phi = P.f(PN_PHI, k);
#pragma unroll
  for (int a = 0; a < 5; ++a) {
    const int r = 5 * k + a;
    const double delta = r == c ? 1.0 : 0.0;
    double JK;
    if (a == 0) {
      JK = J * gb;
    } else if (a <= 3) {
      const double ul = u[a - 1];
      JK = b == 0 ? -J * ul * w
                  : b <= 3 ? J * ((a == b ? w : 0.0) + ul * gb) : g[a - 1] * jct;
    } else {
      JK = b == 0 ? -jth * w : b <= 3 ? jth * gb : J * w;
    }
    double Bs = 0.0;
#pragma unroll
    for (int side = 0; side < 2; ++side)
      if (on[side]) Bs += (a == 0 ? cw[side] : cs[side]) * JK;
    double L = -minv * Bs;
    if (a >= 1 && a <= 3 && kc == k && b == 0) L -= phi * P.f(PN_G + a - 1, k);
    double v;
    if (r >= n || c >= n) v = 0.0;
    else if ((a >= 1 && a <= 3 && (k == 0 || k == nz - 1)) || !band) v = delta;  // rigid lid
    else v = delta - lambda * L;
    row[a] = v;
  }
}

// Workgroups are dealt to the 8 XCDs round-robin (workgroup b runs on XCD b mod 8),
// and each XCD has its own L2.  A wavefront reads its column's entries of the
// column-fastest caller vectors and of the tile-interleaved operator, 8 bytes of
// each cache line that 16 (or 64) neighbouring columns share, so neighbouring
// columns must run on the same XCD: XCD x takes the contiguous columns
// x*chunk .. x*chunk + chunk - 1 (grid = 8 * chunk, chunk = ceil(ncols / 8)).
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t ps_column(int64_t ncols) {
  const int64_t chunk = (ncols + kXcds - 1) / kXcds;
  return (int64_t)(blockIdx.x % kXcds) * chunk + blockIdx.x / kXcds;
}
__host__ __forceinline__ unsigned ps_grid(int64_t ncols) {
  return (unsigned)(kXcds * ((ncols + kXcds - 1) / kXcds));
}

// Scales the row held across the lanes (one entry per lane) by 2^-e, e the binary
// exponent of its largest magnitude (clamped to a signed byte), and returns e.
__device__ __forceinline__ int ps_scale_row(double& v) {
  const double m = wave_max(fabs(v));
  int e = 0;
  if (m > 0.0 && isfinite(m)) {
    frexp(m, &e);
    e = min(max(e, -120), 120);
  }
  v = ldexp(v, -e);
  return e;
}

template <int N>
__device__ __forceinline__ void load_tables(double* Dsh, double* wsh) {
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < (N + 1) * (N + 1); ++q) Dsh[q] = Gll<N>::D[q];
#pragma unroll
    for (int q = 0; q <= N; ++q) wsh[q] = Gll<N>::w[q];
  }
  __syncthreads();
}

// Waves per SIMD of the factorisation (its window, multipliers and the entering node's
// rows take 96-134 registers for N = 1..5; at N = 4 the limit of 5 waves spills).
template <int N>
constexpr int kPsFactorWaves = N <= 3 ? 5 : N == 4 ? 4 : 3;

template <int N>
__global__ __launch_bounds__(64, kPsFactorWaves<N>) void k_ps_factor(HeviShapeDev sh, double lambda,
                                                  const double* __restrict__ ops,
                                                  double* __restrict__ Ub,
                                                  double* __restrict__ Lb,
                                                  uint8_t* __restrict__ piv, HeviDevInfo* info) {
  constexpr int KL = kPsKL<N>, W = kPsW<N>;
  static_assert(W <= 64, "one wavefront holds the window");
  __shared__ double Dsh[(N + 1) * (N + 1)], wsh[N + 1];
  __shared__ double col0[T];         // the pivot column spread over the lanes
  __shared__ double mb[T];           // the step's multipliers, for their broadcast
  __shared__ double ub[8 * W];       // the last 8 rows of U, before they are stored
  extern __shared__ double nodes[];  // PN_FIELDS * n_z
  load_tables<N>(Dsh, wsh);
  const int lane = threadIdx.x;
  const int64_t col = ps_column(sh.ncols);
  if (col >= sh.ncols) return;
  const int nz = sh.nz, n = 5 * nz, Ne = sh.Ne;
  ps_load_nodes(PsCol{ops, ps_plane(ops, sh, 0), plane_elems(sh), col / T, nz, Ne,
                      (int)(col % T)},
                nodes);
  const PsNodes P{nodes, nz};
  constexpr int WS = kPsWS<N>, KLS = kPsKLS<N>;
  double* Uc = Ub + (size_t)col * n * WS;
  double* Lr = Lb + (size_t)col * n * KLS;
  const size_t plane = (size_t)sh.ncols * n;
  uint8_t* pr = piv + (size_t)col * n;
  int8_t* er = (int8_t*)piv + plane + (size_t)col * n;
  uint8_t* uxr = piv + 2 * plane + (size_t)col * n;
  uint8_t* lxr = piv + 3 * plane + (size_t)col * n;
  double a[KL + 1];
#pragma unroll
  for (int i = 0; i <= KL; ++i) {
    a[i] = lane < W ? ps_entry<N>(P, Ne, Dsh, wsh, lambda, i, lane) : 0.0;
    const int e = ps_scale_row(a[i]);
    if (lane == 0 && i < n) er[i] = (int8_t)e;
  }
  // extent of the window column held by this lane: the offset from the diagonal of its
  // first nonzero U entry, -1 until a row has one (set when that row leaves the window)
  int xt = -1;
  double nr[5];  // rows of the node whose rows are entering the window
  bool singular = false;
  for (int j = 0; j < n; ++j) {
    // pivot of column j (lane 0's registers): largest magnitude among rows j..j+KL inside
    // the matrix, the lowest row on ties.  The column goes across the lanes through LDS;
    // a wave reduction finds the largest magnitude, a ballot the lowest lane holding it.
    const int rmax = min(KL, n - 1 - j);
    if (lane == 0) {
#pragma unroll
      for (int i = 0; i <= KL; ++i) col0[i] = a[i];
    }
    __syncthreads();
    const double cl = lane <= KL ? col0[lane] : 0.0;
    const double v = lane <= rmax ? fabs(cl) : -1.0;
    const double vm = wave_max(v);
    const unsigned long long hit = __ballot(lane <= rmax && v == vm);
    const int p = hit ? (int)__builtin_ctzll(hit) : 0;
    // the nonzero rows of the column after the exchange; the highest one below the pivot
    // is the extent of the step's multipliers
    unsigned long long nzm = __ballot(lane <= rmax && v != 0.0);
    if (p != 0) {
      const unsigned long long b0 = nzm & 1ull, bp = (nzm >> p) & 1ull;
      nzm = (nzm & ~(1ull | (1ull << p))) | bp | (b0 << p);
    }
    nzm &= ~1ull;
    const int lx = nzm ? 63 - __builtin_clzll(nzm) : 0;
    __syncthreads();  // col0 is rewritten by the next step
    if (p != 0) swap_first<1, KL>(a, p);
    if (xt < 0 && a[0] != 0.0) xt = lane;
    // the pivot column after the exchange, entry i in lane i, and its multipliers: stored
    // by lanes 1..KL in one coalesced store and broadcast through LDS
    const double c0 = bcast(cl, 0), pv = bcast(cl, p);
    const double cs = lane == 0 ? pv : (lane == p ? c0 : cl);
    if (pv == 0.0) singular = true;
    const double rp = pv != 0.0 ? 1.0 / pv : 0.0;
    const double mv = cs * rp;
    if (lane >= 1 && lane <= KL) {
      mb[lane] = mv;
      Lr[(size_t)j * KLS + lane - 1] = mv;
    }
    // U row j into the column-band layout (entry (j, j+l) at column j+l, offset l), through
    // LDS: rows are staged for 8 steps, then written as runs of up to 8 consecutive entries
    // per column (row-by-row stores into that layout would touch W separate cache lines per
    // step with 8 bytes each)
    if (lane < W) ub[(j & 7) * W + lane] = a[0];
    if ((j & 7) == 7 || j == n - 1) {
      const int r0 = j & ~7, nr = j - r0 + 1;
      for (int t = lane; t < (W + 7) * 8; t += T) {
        const int cc = t >> 3, k = t & 7, o = cc - k, c = r0 + cc;
        if (k < nr && o >= 0 && o < W && c < n) Uc[(size_t)c * WS + o] = ub[k * W + o];
      }
    }
    if (lane == 0) {
      pr[j] = (uint8_t)p;
      lxr[j] = (uint8_t)lx;
      uxr[j] = (uint8_t)max(xt, 0);
    }
    __syncthreads();
    // the rank-1 update in tiers of 8 rows; the rows past the step's multiplier extent lx
    // have zero multipliers (the update would leave them as they are) and are skipped
#pragma unroll
    for (int t = 0; 8 * t < KL; ++t) {
      if (t > 0 && lx <= 8 * t) break;
#pragma unroll
      for (int q = 1; q <= 8; ++q) {
        const int i = 8 * t + q;
        if (i <= KL) a[i] = fma(-mb[i], a[0], a[i]);
      }
    }
    __syncthreads();  // mb is rewritten by the next step
    // next window: rows j+1..j+1+KL, columns j+1..j+W (lanes >= W hold zeros)
#pragma unroll
    for (int i = 0; i < KL; ++i) a[i] = shift_down1(a[i + 1]);
    xt = __builtin_amdgcn_mov_dpp(xt, 0x130, 0xF, 0xF, true);
    if (lane == W - 1) xt = -1;
    // the entering row j+1+KL = 5 m + (j mod 5): the node's five rows are computed when its
    // first one enters (at columns j+1+lane) and the later ones shift with the window
    if (j % 5 == 0) {
      ps_node_rows<N>(P, Ne, Dsh, wsh, lambda, (j + 1 + KL) / 5, j + 1, nr);
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) nr[q] = shift_down1(nr[q + 1]);
    }
    a[KL] = lane < W ? nr[0] : 0.0;
    const int e = ps_scale_row(a[KL]);
    if (lane == 0 && j + 1 + KL < n) er[j + 1 + KL] = (int8_t)e;
  }
  if (singular && lane == 0) flag(info, 5 /*HEVI_E_SINGULAR*/, col);
}

// One stage solve: q^E = sum e_t E_t, q^ = q^E + sum c_j Q_j, A x = P(q^) with the
// band factors (P the rigid-lid projection of the momentum at the bottom and top
// nodes), Q_i = x + (q^E - q^) (= x - sum c_j Q_j, Sec. 4.3 eq. lhevi-ark-final-3).
// Dynamic LDS: 2 n doubles (q^E - q^, and P(q^) overwritten by the solution) and 3 n bytes
// (pivot offsets, U and L extents).  The factor
// rows are read kPsRing steps ahead into register rings, so each step's loads are in
// flight long before the dependent chain of the substitution reaches them, and only up
// to the extents the factorisation recorded: the loads are buffer loads whose lanes past
// the extent take an offset outside the buffer, which returns zero without a memory
// access (at ne = 30, 38% of the stored U entries and 56% of L's are nonzero).
constexpr int kPsRing = 8;

typedef unsigned int PsU2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double ps_bload(__amdgpu_buffer_rsrc_t rs, unsigned off) {
  const PsU2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
  return __hiloint2double((int)v.y, (int)v.x);
}
constexpr unsigned kPsOff = 0x80000000u;  // beyond any buffer of these kernels

// 1/u from the hardware estimate and two Newton steps y <- y + y (1 - u y) (each
// doubles the correct bits), within an ulp of the rounded reciprocal for normal u; the
// quotient correction that follows does not need it rounded.  A zero u (a singular
// factor, flagged by the factorisation) gives a non-finite result.
__device__ __forceinline__ double ps_recip(double u) {
  double y = __builtin_amdgcn_rcp(u);
  y = fma(y, fma(-u, y, 1.0), y);
  y = fma(y, fma(-u, y, 1.0), y);
  return y;
}

template <int N>
__global__ __launch_bounds__(64) void k_ps_stage(HeviShapeDev sh, const double* __restrict__ ops,
                                                 const double* __restrict__ Ub,
                                                 const double* __restrict__ Lb,
                                                 const uint8_t* __restrict__ piv, HeviTerms E,
                                                 HeviTerms Q, double* __restrict__ Qi,
                                                 HeviDevInfo* info) {
  constexpr int KL = kPsKL<N>, W = kPsW<N>, WS = kPsWS<N>, KLS = kPsKLS<N>;
  extern __shared__ double sm[];
  const int lane = threadIdx.x;
  const int64_t col = ps_column(sh.ncols);
  if (col >= sh.ncols) return;
  const int nz = sh.nz, n = 5 * nz;
  const int64_t nc = sh.ncols;
  double* qd = sm;      // q^E - q^
  double* xs = sm + n;  // P(q^), then the solution
  // byte planes of the factorisation: pivot offsets, row exponents, U column extents and
  // L step extents; all but the exponents are copied to LDS (global loads between the
  // ring loads would make the compiler wait for the whole ring)
  uint8_t* pr = (uint8_t*)(sm + 2 * n);
  uint8_t* uxr = pr + n;
  uint8_t* lxr = uxr + n;
  const size_t plane = (size_t)nc * n;
  const int8_t* er = (const int8_t*)piv + plane + (size_t)col * n;
  {
    const uint8_t* pg = piv + (size_t)col * n;
    for (int r = lane; r < n; r += T) {
      pr[r] = pg[r];
      uxr[r] = pg[2 * plane + r];
      lxr[r] = pg[3 * plane + r];
    }
  }
  for (int r = lane; r < n; r += T) {
    const int k = r / 5, v = r - 5 * k;
    const size_t ix = cix(nz, nc, v, k, col);
    double e = 0.0;
    for (int t = 0; t < E.n; ++t) e += E.coef[t] * E.v[t][ix];
    double h = e;
    for (int t = 0; t < Q.n; ++t) h += Q.coef[t] * Q.v[t][ix];
    qd[r] = e - h;
    xs[r] = h;
  }
  __syncthreads();
  if (lane < 2) {
    const int k = lane == 0 ? 0 : nz - 1;
    const int64_t tile = col / T;
    const int cl = (int)(col % T);
    const double g0 = ops[tix(tile, nz, k, HEVI_NOPS, OP_GX, cl)];
    const double g1 = ops[tix(tile, nz, k, HEVI_NOPS, OP_GY, cl)];
    const double g2 = ops[tix(tile, nz, k, HEVI_NOPS, OP_GZ, cl)];
    const double inv = 1.0 / sqrt(g0 * g0 + g1 * g1 + g2 * g2);
    const double n0 = g0 * inv, n1 = g1 * inv, n2 = g2 * inv;
    double* b = xs + 5 * k;
    const double d = n0 * b[1] + n1 * b[2] + n2 * b[3];
    b[1] -= n0 * d; b[2] -= n1 * d; b[3] -= n2 * d;
  }
  __syncthreads();
  // the right-hand side in the scale of the equilibrated rows
  for (int r = lane; r < n; r += T) xs[r] = ldexp(xs[r], -(int)er[r]);
  __syncthreads();
  constexpr int D = kPsRing;
  const __amdgpu_buffer_rsrc_t lrs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(Lb + (size_t)col * n * KLS), (short)0, n * KLS * (int)sizeof(double), 0x00020000);
  const __amdgpu_buffer_rsrc_t urs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(Ub + (size_t)col * n * WS), (short)0, n * WS * (int)sizeof(double), 0x00020000);
  // Forward: the row exchanges and L, y[j + i] in lane i (i = 0..KL).  Each block of 64
  // steps takes its pivot offsets, the extents of the rows its ring loads fetch and the
  // entering values y[j + 1 + KL] from lane-spread registers (read from LDS once per
  // block), and collects its results y[j] the same way, so no step waits on LDS.  The ring
  // loads are unconditional (a guarded load becomes a branch, across which the compiler
  // waits for every outstanding load, the one just issued included); rows past the last
  // step have extent 0, so all their lanes read zero.
  const bool lrow = lane >= 1 && lane <= KL;
  auto loff = [&](int j, int x) -> unsigned {
    return lane >= 1 && lane <= x ? (unsigned)((j * KLS + lane - 1) * (int)sizeof(double)) : kPsOff;
  };
  double lr[D];
#pragma unroll
  for (int d = 0; d < D; ++d) lr[d] = ps_bload(lrs, loff(d, d < n ? (int)lxr[d] : 0));
  double y = (lane <= KL && lane < n) ? xs[lane] : 0.0;
  for (int j0 = 0; j0 < n; j0 += T) {
    const int pb = j0 + lane < n ? (int)pr[j0 + lane] : 0;
    const int lx = j0 + lane + D < n ? (int)lxr[j0 + lane + D] : 0;
    const int je = j0 + lane + KL + 1;
    const double eb = je < n ? xs[je] : 0.0;
    double ob = 0.0;
    const int nb = min(T, n - j0);
    // whole groups of D steps (a conditional step would again make the compiler wait for
    // every outstanding load): past the last row every y is zero (no exchange, zero
    // entering values, no multipliers), so the extra steps have x_j = 0, change nothing,
    // and their results are not stored
    for (int d0 = 0; d0 < nb; d0 += D) {
#pragma unroll
      for (int e = 0; e < D; ++e) {
        const int d = d0 + e;
        const int j = j0 + d;
        const int p = __builtin_amdgcn_readlane(pb, d);
        if (p != 0) {
          const double yp = bcast(y, p), y0 = bcast(y, 0);
          if (lane == 0) y = yp;
          if (lane == p) y = y0;
        }
        const double xj = bcast(y, 0);
        if (lrow) y -= lr[e] * xj;
        // the slot's next row, loaded into the register just used (a load into another
        // register followed by a copy would wait for it here)
        lr[e] = ps_bload(lrs, loff(j + D, __builtin_amdgcn_readlane(lx, d)));
        if (lane == d) ob = xj;
        y = shift_down1(y);
        const double ent = bcast(eb, d);
        y = lane == KL ? ent : y;
      }
    }
    // entries j0..j0+63 of xs are no longer read (the entering values are read up to a block
    // ahead); a wavefront's LDS accesses complete in order
    if (lane < nb) xs[j0 + lane] = ob;
  }
  __syncthreads();
  // Backward, column-oriented: lane l holds the partial sum of row j - l (l = 0..W-1);
  // step j: x_j = r_j / U_jj, then r[j - l] -= U[j - l][j] x_j, one FMA per lane, and the
  // rows shift one lane down with row j - W entering at lane W-1.  Column j of U is one
  // contiguous W-vector of the column-band layout, read up to its extent (lanes past it,
  // lanes l > j among them, read zero).  Lanes >= W read zero and their sums are replaced
  // by the entering row (lane W-1 takes lane W's) before any use.  The extra steps below
  // the first row read nothing (extent -1) and are not stored.
  auto uoff = [&](int j, int x) -> unsigned {
    return lane <= x ? (unsigned)((j * WS + lane) * (int)sizeof(double)) : kPsOff;
  };
  double ur[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const int jn = n - 1 - d;
    ur[d] = ps_bload(urs, uoff(jn, jn >= 0 ? (int)uxr[jn] : -1));
  }
  double r = (lane < W && n - 1 - lane >= 0) ? xs[n - 1 - lane] : 0.0;
  double un = bcast(ur[0], 0);
  double rn = ps_recip(un);
  for (int jt = n - 1; jt >= 0; jt -= T) {
    const int ju = jt - D - lane;
    const int ux = ju >= 0 ? (int)uxr[ju] : -1;
    const int jr = jt - W - lane;
    const double eb = jr >= 0 ? xs[jr] : 0.0;
    double ob = 0.0;
    const int nb = min(T, jt + 1);
    for (int d0 = 0; d0 < nb; d0 += D) {
#pragma unroll
      for (int e = 0; e < D; ++e) {
        const int d = d0 + e;
        const int j = jt - d;
        // x_j = r_j / U_jj with only a product and two FMAs on the chain through r: the
        // reciprocal of U_jj is computed a step ahead, off the chain, and one residual
        // correction of the product (Markstein's final step of division with a fused
        // multiply-add) gives the rounded quotient but in rare cases of the last bit
        const double u = un, ri = rn;
        const double r0 = bcast(r, 0);
        double xj = r0 * ri;
        xj = fma(fma(-xj, u, r0), ri, xj);
        r = fma(-ur[e], xj, r);
        ur[e] = ps_bload(urs, uoff(j - D, __builtin_amdgcn_readlane(ux, d)));
        un = bcast(ur[(e + 1) % D], 0);  // the next step's U_jj, loaded D - 1 steps ago
        rn = ps_recip(un);
        if (lane == d) ob = xj;
        r = shift_down1(r);
        const double ent = bcast(eb, d);
        r = lane == W - 1 ? ent : r;
        // keep each step's ring load in its step (the scheduler would otherwise gather the
        // group's loads at its end and shorten the prefetch distance)
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    // xs[jt - 63 .. jt]: read for the last time as entering values a block earlier
    if (lane < nb) xs[jt - lane] = ob;
  }
  __syncthreads();
  bool nonfinite = false;
  for (int r = lane; r < n; r += T) {
    const int k = r / 5, v = r - 5 * k;
    const double q = xs[r] + qd[r];
    Qi[cix(nz, nc, v, k, col)] = q;
    if (!isfinite(q)) nonfinite = true;
  }
  if (__any(nonfinite) && lane == 0) flag(info, 9 /*HEVI_E_NONFINITE*/, col);
}

// New linearisation state for an LHEVI-PS operator (no allocation): theta0 and
// c_Theta = gamma P(Theta0)/Theta0 (Appendix A.1, eq. set2c_pressure) times J into
// their fields, the velocity u0 = U0/rho0 into the state planes.
__global__ __launch_bounds__(64) void k_ps_state(HeviShapeDev sh, double R, double cp,
                                                 double pA, const double* __restrict__ rho0,
                                                 const double* __restrict__ U0,
                                                 const double* __restrict__ Th0,
                                                 double* __restrict__ ops, HeviDevInfo* info) {
  const int lane = threadIdx.x;
  const int64_t tile = blockIdx.x;
  const int64_t c = tile * T + lane;
  const bool valid = c < sh.ncols;
  const int64_t cc = valid ? c : sh.ncols - 1;
  const int nz = sh.nz;
  const int64_t nc = sh.ncols;
  const double gam = cp / (cp - R);
  const size_t pe = plane_elems(sh);
  double* u0p = ops + pr_offset(sh);
  bool bad = false;
  for (int k = 0; k < nz; ++k) {
    const double r0 = rho0[(size_t)k * nc + cc];
    const double T0 = Th0[(size_t)k * nc + cc];
    double* o = ops + tix(tile, nz, k, HEVI_NOPS, 0, lane);
    const double Jk = o[OP_J * T];
    const double P0 = pA * pow(R * T0 / pA, gam);
    const double th0 = T0 / r0, cT = gam * P0 / T0;
    o[OP_JTH * T] = Jk * th0;
    o[OP_JCT * T] = Jk * cT;
    const size_t ip = ((size_t)tile * nz + k) * T + lane;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const double v = U0[cix(nz, nc, m, k, cc)] / r0;
      u0p[(size_t)m * pe + ip] = v;
      bad |= !isfinite(v);
    }
    bad |= !(r0 > 0.0) || !(T0 > 0.0) || !isfinite(r0) || !isfinite(T0) || !isfinite(cT);
  }
  if (bad && valid) flag(info, 1 /*HEVI_E_INVALID*/, c);
}

template <int N, bool HAS_REF>
__global__ __launch_bounds__(64, kStreamWaves<N>) void k_apply_ps(
    HeviShapeDev sh, const double* __restrict__ ops, const double* __restrict__ x,
    const double* __restrict__ xref, double* __restrict__ y) {
  b_apply<N, HAS_REF, false, true>((int64_t)blockIdx.x, sh, Gll<N>{}, ops, x, xref, y, 1);
}

// NHEVI-LU (Sec. 4.2.2): the nonlinear set-2C vertical operator V(q) (Appendix A.2)
// with the discretisation of the linear one: fluxes F_rho = J U^z, F_U = J (U U^z/rho +
// P(Theta) grad zeta), F_Theta = J Theta U^z/rho (U^z = grad(zeta).U, P = P_A (R
// Theta/P_A)^gamma, eq. set2c_pressure), the continuity row weak, the others strong,
// DSS, lumped mass, gravity -rho Phi' grad(zeta), zero momentum rows at the rigid
// lid.  One lane per column, elements in order, the sums of a shared node carried.
template <int N>
__global__ __launch_bounds__(64) void k_vertical_op(HeviShapeDev sh, double R, double gam,
                                                    double pA, const double* __restrict__ ops,
                                                    const double* __restrict__ q,
                                                    double* __restrict__ V) {
  const Gll<N> tab{};
  const int lane = threadIdx.x;
  const int64_t tile = blockIdx.x;
  const int64_t c = tile * T + lane;
  const bool valid = c < sh.ncols;
  const int64_t cc = valid ? c : sh.ncols - 1;
  const int nz = sh.nz, Ne = sh.Ne;
  const int64_t nc = sh.ncols;
  OpsView op{ops, tile, nz, lane};
  double cr = 0.0, c0 = 0.0, c1 = 0.0, c2 = 0.0, ct = 0.0;
  for (int e = 0; e < Ne; ++e) {
    double Fr[N + 1], F0[N + 1], F1[N + 1], F2[N + 1], Ft[N + 1], rho[N + 1];
#pragma unroll
    for (int j = 0; j <= N; ++j) {
      const int k = e * N + j;
      const double g0 = op(k, OP_GX), g1 = op(k, OP_GY), g2 = op(k, OP_GZ), Jk = op(k, OP_J);
      const double r = q[cix(nz, nc, 0, k, cc)];
      const double u0 = q[cix(nz, nc, 1, k, cc)], u1 = q[cix(nz, nc, 2, k, cc)];
      const double u2 = q[cix(nz, nc, 3, k, cc)], th = q[cix(nz, nc, 4, k, cc)];
      const double Uz = g0 * u0 + g1 * u1 + g2 * u2;
      const double P = pA * pow(R * th / pA, gam);
      const double a = Uz / r;
      rho[j] = r;
      Fr[j] = Jk * Uz;
      F0[j] = Jk * (u0 * a + P * g0);
      F1[j] = Jk * (u1 * a + P * g1);
      F2[j] = Jk * (u2 * a + P * g2);
      Ft[j] = Jk * th * a;
    }
#pragma unroll
    for (int i = 0; i <= N; ++i) {
      double sr = 0.0, s0 = 0.0, s1 = 0.0, s2 = 0.0, st = 0.0;
#pragma unroll
      for (int j = 0; j <= N; ++j) {
        const double d = tab.D[i * (N + 1) + j];
        sr += tab.w[j] * tab.D[j * (N + 1) + i] * Fr[j];
        s0 += d * F0[j]; s1 += d * F1[j]; s2 += d * F2[j]; st += d * Ft[j];
      }
      const double wi = tab.w[i];
      s0 *= wi; s1 *= wi; s2 *= wi; st *= wi;
      if (i == 0) { sr += cr; s0 += c0; s1 += c1; s2 += c2; st += ct; }
      if (i == N && e < Ne - 1) { cr = sr; c0 = s0; c1 = s1; c2 = s2; ct = st; continue; }
      const int k = e * N + i;
      const double mi = op(k, OP_MINV), ph = op(k, OP_PHI);
      const bool lid = (k == 0) || (k == nz - 1);
      if (valid) {
        V[cix(nz, nc, 0, k, c)] = mi * sr;
        V[cix(nz, nc, 1, k, c)] = lid ? 0.0 : -mi * s0 - ph * op(k, OP_GX) * rho[i];
        V[cix(nz, nc, 2, k, c)] = lid ? 0.0 : -mi * s1 - ph * op(k, OP_GY) * rho[i];
        V[cix(nz, nc, 3, k, c)] = lid ? 0.0 : -mi * s2 - ph * op(k, OP_GZ) * rho[i];
        V[cix(nz, nc, 4, k, c)] = -mi * st;
      }
    }
  }
}

// Newton stopping measure: max over columns and variables of ||dq_v|| / ||q_v - q^n_v||
// (norms over the column's nodes; q the updated iterate), reduced into info->max_res_bits.
__global__ __launch_bounds__(64) void k_newton_rel(HeviShapeDev sh, const double* __restrict__ dq,
                                                   const double* __restrict__ q,
                                                   const double* __restrict__ qn,
                                                   HeviDevInfo* info) {
  const int64_t c = (int64_t)blockIdx.x * T + threadIdx.x;
  if (c >= sh.ncols) return;
  const int nz = sh.nz;
  const int64_t nc = sh.ncols;
  double worst = 0.0;
  for (int v = 0; v < 5; ++v) {
    double d2 = 0.0, q2 = 0.0;
    for (int k = 0; k < nz; ++k) {
      const size_t i = cix(nz, nc, v, k, c);
      const double d = dq[i], w = q[i] - qn[i];
      d2 += d * d;
      q2 += w * w;
    }
    const double rel = q2 > 0.0 ? sqrt(d2 / q2) : (d2 > 0.0 ? INFINITY : 0.0);
    worst = fmax(worst, rel);
  }
  if (!isfinite(worst)) worst = 1.0e300;
  atomicMax((unsigned long long*)&info->max_res_bits, (unsigned long long)__double_as_longlong(worst));
}

template <int N>
struct VerticalOp {
  static hipError_t run(const HeviShapeDev& sh, double R, double gam, double pA,
                        const double* ops, const double* q, double* V, hipStream_t st) {
    hipLaunchKernelGGL(k_vertical_op<N>, dim3((unsigned)sh.ntiles), dim3(T), 0, st, sh, R, gam,
                       pA, ops, q, V);
    return hipGetLastError();
  }
};

template <template <int> class F, typename... A>
hipError_t dispatch_ps(int N, A&&... a) {
  switch (N) {
    case 1: return F<1>::run(a...);
    case 2: return F<2>::run(a...);
    case 3: return F<3>::run(a...);
    case 4: return F<4>::run(a...);
    case 5: return F<5>::run(a...);
    default: return hipErrorInvalidValue;
  }
}

template <int N>
struct PsFactor {
  static hipError_t run(const HeviShapeDev& sh, double lambda, const double* ops, double* U,
                        double* L, uint8_t* piv, HeviDevInfo* info, hipStream_t st) {
    hipLaunchKernelGGL(k_ps_factor<N>, dim3(ps_grid(sh.ncols)), dim3(T),
                       (size_t)PN_FIELDS * sh.nz * sizeof(double), st, sh, lambda, ops, U, L, piv,
                       info);
    return hipGetLastError();
  }
};

template <int N>
struct PsStage {
  static hipError_t run(const HeviShapeDev& sh, const double* ops, const double* U,
                        const double* L, const uint8_t* piv, const HeviTerms& E,
                        const HeviTerms& Q, double* Qi, HeviDevInfo* info, hipStream_t st) {
    const size_t n = 5 * (size_t)sh.nz;
    hipLaunchKernelGGL(k_ps_stage<N>, dim3(ps_grid(sh.ncols)), dim3(T),
                       2 * n * sizeof(double) + 3 * n, st, sh, ops, U, L, piv, E, Q, Qi, info);
    return hipGetLastError();
  }
};

template <int N>
struct PsApply {
  static hipError_t run(const HeviShapeDev& sh, const double* ops, const double* x,
                        const double* xref, double* y, hipStream_t st) {
    if (xref)
      hipLaunchKernelGGL((k_apply_ps<N, true>), dim3((unsigned)sh.ntiles), dim3(T), 0, st, sh,
                         ops, x, xref, y);
    else
      hipLaunchKernelGGL((k_apply_ps<N, false>), dim3((unsigned)sh.ntiles), dim3(T), 0, st, sh,
                         ops, x, xref, y);
    return hipGetLastError();
  }
};

}  // namespace

int hevi_ps_band_width(int N) { return (2 * (5 * (N + 1) - 1) + 1 + 15) / 16 * 16; }
int hevi_ps_lower_width(int N) { return (5 * (N + 1) - 1 + 15) / 16 * 16; }

hipError_t hevi_launch_ps_factor(const HeviShapeDev& sh, double lambda, const double* ops,
                                 double* U, double* L, uint8_t* piv, HeviDevInfo* info,
                                 hipStream_t st) {
  if (sh.ncols == 0) return hipSuccess;
  return dispatch_ps<PsFactor>(sh.N, sh, lambda, ops, U, L, piv, info, st);
}

hipError_t hevi_launch_ps_stage(const HeviShapeDev& sh, const double* ops, const double* U,
                                const double* L, const uint8_t* piv, const HeviTerms& E,
                                const HeviTerms& Q, double* Qi, HeviDevInfo* info,
                                hipStream_t st) {
  if (sh.ncols == 0) return hipSuccess;
  return dispatch_ps<PsStage>(sh.N, sh, ops, U, L, piv, E, Q, Qi, info, st);
}

hipError_t hevi_launch_apply_ps(const HeviShapeDev& sh, const double* ops, const double* x,
                                const double* xref, double* y, hipStream_t st) {
  if (sh.ntiles == 0) return hipSuccess;
  return dispatch_ps<PsApply>(sh.N, sh, ops, x, xref, y, st);
}

hipError_t hevi_launch_ps_state(const HeviShapeDev& sh, double R, double cp, double pA,
                                const double* rho0, const double* U0, const double* Th0,
                                double* ops, HeviDevInfo* info, hipStream_t st) {
  if (sh.ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ps_state, dim3((unsigned)sh.ntiles), dim3(T), 0, st, sh, R, cp, pA, rho0,
                     U0, Th0, ops, info);
  return hipGetLastError();
}

hipError_t hevi_launch_vertical_op(const HeviShapeDev& sh, double R, double cp, double pA,
                                   const double* ops, const double* q, double* V,
                                   hipStream_t st) {
  if (sh.ntiles == 0) return hipSuccess;
  if (sh.N > HEVI_PS_MAXN) {
    // orders 6..8 share the same body
    switch (sh.N) {
      case 6: return VerticalOp<6>::run(sh, R, cp / (cp - R), pA, ops, q, V, st);
      case 7: return VerticalOp<7>::run(sh, R, cp / (cp - R), pA, ops, q, V, st);
      case 8: return VerticalOp<8>::run(sh, R, cp / (cp - R), pA, ops, q, V, st);
      default: return hipErrorInvalidValue;
    }
  }
  return dispatch_ps<VerticalOp>(sh.N, sh, R, cp / (cp - R), pA, ops, q, V, st);
}

hipError_t hevi_launch_newton_rel(const HeviShapeDev& sh, const double* dq, const double* q,
                                  const double* qn, HeviDevInfo* info, hipStream_t st) {
  if (sh.ncols == 0) return hipSuccess;
  hipLaunchKernelGGL(k_newton_rel, dim3((unsigned)sh.ntiles), dim3(T), 0, st, sh, dq, q, qn,
                     info);
  return hipGetLastError();
}
