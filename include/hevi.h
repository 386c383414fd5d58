/*
 * hevi.h -- C ABI of the batched LHEVI vertical column solver for MI355X (gfx950).
 *
 * The library solves, for many independent vertical columns at once, the
 * linear implicit problem of the LHEVI additive Runge-Kutta method of
 * Giraldo et al. (arXiv 2311.11425):
 *
 *     (I - Lambda L_z) q_tt = q^,   Lambda = a~_ii dt          (Sec. 4.3,
 *                                                       eq. lhevi-ark-final-2)
 *
 * where L_z is the set-2C vertical operator (Appendix A.2) linearised about a
 * hydrostatic reference state at rest and discretised on the Gauss-Lobatto-
 * Legendre points of each column (Sec. 3; Appendix A.3), with a rigid lid at
 * the bottom and top nodes.  The matrix is factored once and the factors are
 * reused by every implicit stage (Sec. 5.3: the forward reduction is paid when
 * the operator is rebuilt, the back-substitution once per stage).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Shapes.   order_N = polynomial order of the vertical elements (1..8),
 *           n_elem = number of vertical elements (>= 1),
 *           n_z = n_elem * order_N + 1 unique GLL nodes per column,
 *           n_cols = number of columns (>= 0).
 * Layout.   All device arrays owned by the caller are FP64, struct-of-arrays,
 *           column index fastest:  a per-node field f is f[k * n_cols + c];
 *           grad(zeta) is gz[(m * n_z + k) * n_cols + c], m = x, y, z;
 *           a state vector q (rho, rho u, rho v, rho w, rho theta) is
 *           q[(v * n_z + k) * n_cols + c].  8-byte alignment is required,
 *           256-byte alignment gives the best coalescing.
 * Ownership. d_* pointers are caller-owned device memory; the library never
 *           frees them and keeps no reference to them after the call's work
 *           has run on the stream.  hevi_ops / hevi_factors / hevi_server are
 *           library-owned, freed only by the matching *_free / *_destroy;
 *           ops must outlive every factor object built from them.
 * Streams.  Work is enqueued on the caller's HIP stream and returns
 *           immediately unless stated otherwise; inputs must stay valid until
 *           the stream reaches the call.  A NULL stream is the default stream.
 * Errors.   The return value reports synchronous validation (bad arguments,
 *           shapes, allocation failures).  Problems found by a kernel (zero
 *           pivot, non-finite value, refinement not converged) are reported
 *           through hevi_info, which is filled only when the caller passes a
 *           non-NULL hevi_info (that makes the call wait for its stream).  On a
 *           synchronous error no device work is enqueued and outputs are
 *           untouched; outputs of columns flagged by a kernel are unspecified.
 * Threads.  A context may be used by one host thread at a time; distinct
 *           contexts are independent.  The server API is thread-safe.
 */
#ifndef HEVI_H
#define HEVI_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HEVI_OK = 0,
  HEVI_E_INVALID = 1,       /* bad argument value (NULL pointer, NaN constant ...) */
  HEVI_E_SHAPE = 2,         /* unsupported or inconsistent shape                   */
  HEVI_E_NOMEM = 3,         /* device or host allocation failed / over budget      */
  HEVI_E_DEVICE = 4,        /* HIP runtime error                                   */
  HEVI_E_SINGULAR = 5,      /* exactly zero pivot in some column                   */
  HEVI_E_NOT_CONVERGED = 6, /* mixed path: refinement target not reached           */
  HEVI_E_BUSY = 7,          /* server: no slot or memory free right now            */
  HEVI_E_CLOSED = 8,        /* server: shut down or unknown id                     */
  HEVI_E_NONFINITE = 9,     /* a kernel produced or read a non-finite value        */
  HEVI_E_SCRATCH = 10       /* hevi_solve_noalloc: the shape needs more than its
                               fixed scratch (HEVI_NOALLOC_SCRATCH_BYTES)             */
} hevi_status;

typedef enum {
  HEVI_FP64 = 0,        /* factors and solve in FP64                                  */
  HEVI_FP32_REFINE = 1  /* FP32-stored factors, FP64 right-hand side, FP64 residual
                           of the reduced system, iterative refinement               */
} hevi_precision;

/* Physical constants: gas constant R, specific heat c_p, gravity g, reference
 * pressure P_A of the equation of state P = P_A (R Theta / P_A)^gamma,
 * gamma = c_p / (c_p - R) (Appendix A.1; P_A = 1e5 Pa in Sec. 2.1). */
typedef struct { double R, cp, g, p_A; } hevi_consts;

typedef struct { int32_t order_N, n_elem; int64_t n_cols; } hevi_shape;

/* Refinement controls of a stage solve.
 * max_sweeps / rel_residual_target: FP32-factor path only -- sweeps of
 *   iterative refinement of the reduced system (FP64 residual r - S u applied
 *   matrix-free, correction d from the FP32 factors, u += d) until the last
 *   correction satisfies ||d|| <= rel_residual_target ||u||.
 * full_sweeps: either precision -- sweeps of iterative refinement of the full
 *   system with the FP64 residual q^ - A q_tt formed on offset-free vectors, in
 *   a slower kernel that keeps every vector in scratch (an accuracy reference;
 *   the default path already solves the row-equilibrated reduced system and
 *   recovers the momentum from u without differencing large terms).  The first
 *   stage solve with full_sweeps > 0 on a factor object allocates that kernel's
 *   wider scratch (15 more FP64 per node), which the object keeps until freed. */
typedef struct { int32_t max_sweeps; double rel_residual_target; int32_t full_sweeps; } hevi_refine;

typedef struct {
  int32_t status;            /* worst kernel-detected hevi_status of the call       */
  int32_t max_sweeps_used;   /* refinement sweeps of the worst column (mixed path)  */
  int64_t first_bad_col;     /* lowest flagged column, -1 if none                   */
  int64_t n_bad_cols;        /* number of flagged columns                           */
  double max_rel_correction; /* max over columns of the last ||d|| / ||u|| (FP32)    */
} hevi_info;

typedef struct hevi_ctx hevi_ctx;
typedef struct hevi_ops hevi_ops;
typedef struct hevi_factors hevi_factors;
typedef struct hevi_server hevi_server;

/* ---- context ----------------------------------------------------------- */
/* Create a context on HIP device `device` (makes it current for the calling
 * thread).  Returns HEVI_E_DEVICE if the device does not exist or is not a
 * gfx950 part. */
hevi_status hevi_create(int device, hevi_ctx **out);
void hevi_destroy(hevi_ctx *ctx);
const char *hevi_status_str(hevi_status s);

/* ---- column operators (a1/a2) -------------------------------------------
 * Column set-up of Sec. 3 and Appendix A: GLL nodes, weights and
 * differentiation matrix of order N; per node the lumped mass M_k (quadrature
 * weight times J, direct-stiffness-summed along the column), theta0 =
 * Theta0/rho0 and c_Theta = dP/dTheta = gamma P0/Theta0 from the set-2C
 * equation of state, and the gravity coefficient dPhi/dzeta with Phi = g z
 * (Sec. 2.1), integrated and summed like every other term.
 * Inputs (per node, [k][c]): height d_z, metric Jacobian d_J (> 0), reference
 * density d_rho0 (> 0) and density potential temperature d_Theta0 (> 0);
 * d_gz = grad(zeta) ([m][k][c], nonzero).  The result is a library-owned
 * compact per-node operator (8 FP64 per node).  Invalid per-node values are
 * reported by hevi_ops_check.  The call waits for `stream` once: whether every
 * column's grad(zeta) is one vector along the column (straight columns, whose
 * pressure gradient has no part tangential to grad(zeta)) selects the stage-solve
 * kernels used with these ops. */
hevi_status hevi_build_column_ops(hevi_ctx *ctx, const hevi_shape *shape,
                                  const hevi_consts *consts, const double *d_z,
                                  const double *d_J, const double *d_gz,
                                  const double *d_rho0, const double *d_Theta0,
                                  hevi_ops **out, hipStream_t stream);

/* Equation sets (Appendix A.1): set 2C carries Theta = rho theta, set 3C the total
 * energy E = rho (c_v T + u.u/2 + Phi) as the fifth state variable. */
typedef enum {
  HEVI_SET_2C = 0,
  HEVI_SET_3C = 1
} hevi_eqset;

/* hevi_build_column_ops for either equation set; HEVI_SET_2C is exactly
 * hevi_build_column_ops.  For HEVI_SET_3C, d_q0 is the reference total energy E0
 * ([k][c]) and the operator is the set-3C vertical operator linearised at rest
 * (Appendix A.3, eq. set3c_jacobian at U = 0): pressure P0 = (gamma - 1)(E0 -
 * rho0 Phi) with Phi = g z (eq. set3c_pressure; must be > 0), energy flux
 * coefficient (E0 + P0)/rho0, dP/dE = gamma - 1 and dP/drho = -(gamma - 1) Phi,
 * whose rho column joins the pressure gradient of the momentum rows (the reduced
 * system keeps its band, see hevi_factor).  Every state vector handed to calls on
 * these ops is then (rho, U, E).  A set-3C operator holds 9 FP64 per node.  Group
 * steps and the server take set-2C operators only (HEVI_E_INVALID). */
hevi_status hevi_build_column_ops_set(hevi_ctx *ctx, const hevi_shape *shape,
                                      const hevi_consts *consts, hevi_eqset eqset,
                                      const double *d_z, const double *d_J,
                                      const double *d_gz, const double *d_rho0,
                                      const double *d_q0, hevi_ops **out,
                                      hipStream_t stream);
/* LHEVI-PS (Sec. 4.3.1): the linear operator is the Jacobian of the set-2C vertical
 * operator at a moving state q0 = (rho0, U0, Theta0), a previous solution, instead of a
 * state at rest: the flux Jacobian K(q0) of Appendix A.3 (eq. set2c_jacobian, re-derived
 * from the fluxes of Appendix A.2) with u0 = U0/rho0 and w = grad(zeta).u0 gives the
 * advection entries K[U_l][rho] = -u0_l w, K[U_l][U_m] = delta_lm w + u0_l gz_m,
 * K[Theta][rho] = -theta0 w, K[Theta][Theta] = w besides the rest-state ones.  d_U0 is
 * the state's momentum [m][k][c] (its normal part should vanish at the bottom and top
 * nodes, as the rigid lid requires); the other inputs as hevi_build_column_ops.  The
 * rho-theta and momentum blocks of I - lambda L_z are then not identities, so these
 * operators factor the whole 5 n_z band with partial pivoting (the paper's LAPACK band
 * LU, Sec. 4.2.2; kl = ku = 5(N+1) - 1): hevi_factor / hevi_refactor store U by band
 * columns (2 kl + 1 entries, padded to whole 128-byte lines), the kl multipliers of each
 * step (padded likewise), and per unknown the pivot offset, row-scale exponent and the
 * extents of U's column and L's row (at N = 4, n_z = 41: 158,260 bytes per column), FP64 only
 * (HEVI_FP32_REFINE gives HEVI_E_INVALID), N <= 5 and n_z <= 600 (else HEVI_E_SHAPE);
 * hevi_stage_solve solves directly (its refine argument is ignored), hevi_apply_op applies
 * L_z(q0).  hevi_factors_band_entries, hevi_solve_noalloc, groups and the server take
 * reference-state operators only (HEVI_E_INVALID).  The operator holds 11 FP64 per node. */
hevi_status hevi_build_column_ops_ps(hevi_ctx *ctx, const hevi_shape *shape,
                                     const hevi_consts *consts, const double *d_z,
                                     const double *d_J, const double *d_gz,
                                     const double *d_rho0, const double *d_U0,
                                     const double *d_Theta0, hevi_ops **out,
                                     hipStream_t stream);
/* New linearisation state for an LHEVI-PS operator, in place (no allocation, no wait):
 * the state-dependent fields are rewritten from (rho0, U0, Theta0); the geometry stays.
 * The paper refreshes the state every few steps (5 by default, Sec. 4.3.1); follow it
 * with hevi_refactor.  Invalid values are reported by hevi_ops_check. */
hevi_status hevi_ops_relinearize(hevi_ctx *ctx, hevi_ops *ops, const double *d_rho0,
                                 const double *d_U0, const double *d_Theta0,
                                 hipStream_t stream);
/* NHEVI-LU (Sec. 4.2.2): each implicit stage solves F(q) = q - Lambda V(q) - R = 0 by
 * Newton's method, rebuilding and factoring the Jacobian I - Lambda dV/dq at every
 * iterate.  hevi_vertical_op evaluates the nonlinear set-2C vertical operator
 *   V(q) = -(div(J U^z), div(J (U U^z/rho + P(Theta) grad zeta)) + rho Phi' grad zeta,
 *            div(J Theta U^z/rho)) / J     (Appendix A.2; P of eq. set2c_pressure)
 * with the discretisation of L_z (continuity row weak, the others strong, DSS, lumped
 * mass, zero momentum rows at the rigid lid), for any set-2C operator's geometry (the
 * state is q, [v][k][c]; d_V must not alias d_q).  The Newton step then is
 * hevi_ops_relinearize(ops, q_rho, q_U, q_Theta) + hevi_refactor + hevi_stage_solve with
 * E = {R, q, V(q)}, e = {1, -1, Lambda} (the increment, rigid-lid projected) +
 * hevi_combine.  hevi_newton_increment waits for `stream` and returns the stopping
 * measure max over columns and variables of ||dq_v|| / ||q_v - q^n_v|| (node norms, q the
 * updated iterate; the paper stops at 1e-5, Sec. 7.1). */
hevi_status hevi_vertical_op(hevi_ctx *ctx, const hevi_ops *ops, const double *d_q, double *d_V,
                             hipStream_t stream);
hevi_status hevi_newton_increment(hevi_ctx *ctx, const hevi_ops *ops, const double *d_dq,
                                  const double *d_q, const double *d_qn, double *h_rel,
                                  hipStream_t stream);
/* Waits for `stream` and reports the first column whose inputs were invalid
 * (non-positive J/rho0/Theta0, zero grad(zeta), non-finite values). */
hevi_status hevi_ops_check(hevi_ctx *ctx, const hevi_ops *ops, int64_t *first_bad_col,
                           hipStream_t stream);
void hevi_ops_free(hevi_ops *ops);

/* ---- operator application (a0) ------------------------------------------
 * y = L_z (x - x_ref) for every column (x_ref may be NULL), with the rigid-lid
 * rows of the end nodes zero.  This is the discrete vertical operator of
 * Appendix A.2 linearised at rest; it serves as the synthetic explicit
 * tendency S(q) = L_z (q - q_ref) of the benchmark.  Vectors [v][k][c].  y must
 * not alias x or x_ref. */
hevi_status hevi_apply_op(hevi_ctx *ctx, const hevi_ops *ops, const double *d_x,
                          const double *d_xref, double *d_y, hipStream_t stream);

/* ---- factorisation (a3) ---------------------------------------------------
 * Factor A = I - lambda L_z (with rigid-lid identity rows) for every column.
 * Representation: the exact block elimination of rho, Theta and the tangential
 * momentum (their diagonal blocks are identities) leaves a band system of
 * half-bandwidth 2N in the contravariant vertical momentum u = grad(zeta).U;
 * that system is row-equilibrated by powers of two (each row scaled by the
 * binary exponent of its largest entry, exactly) and LU-factored with partial
 * pivoting (largest magnitude in the pivot column, lowest row on ties): the
 * band LU the paper uses through LAPACK (Sec. 4.2.3), applied to the reduced
 * matrix with LAPACK-style row equilibration.  Factors are FP64, or FP32 for
 * HEVI_FP32_REFINE (elimination in FP64, then rounded).  lambda >= 0.
 * hevi_factor allocates; hevi_refactor reuses the storage of `f` for a new
 * lambda (no allocation).  A zero pivot is reported as HEVI_E_SINGULAR by
 * hevi_factors_check. */
hevi_status hevi_factor(hevi_ctx *ctx, const hevi_ops *ops, double lambda,
                        hevi_precision prec, hevi_factors **out, hipStream_t stream);
hevi_status hevi_refactor(hevi_ctx *ctx, hevi_factors *f, double lambda, hipStream_t stream);
/* U entries the solves read, summed over the valid columns: each U row up to its
 * last nonzero entry, pivot included (the rest of the 4N + 1 band entries are
 * exact zeros, which the factorisation records and the solves skip; L is read in
 * full).  Waits for the stream and copies one byte per node to the host (a
 * diagnostic, not for the stepping loop). */
hevi_status hevi_factors_band_entries(hevi_ctx *ctx, const hevi_factors *f, int64_t *u_entries,
                                      hipStream_t stream);
hevi_status hevi_factors_check(hevi_ctx *ctx, const hevi_factors *f, hevi_info *info,
                               hipStream_t stream);
void hevi_factors_free(hevi_factors *f);

/* ---- stage solve (a4 + a5 + a6) -------------------------------------------
 * One implicit LHEVI stage for every column (Sec. 4.3, eq. lhevi-ark-final-3):
 *     q^E = sum_t e[t] E_t            (e.g. E = {q^n, S(Q_1), ...},
 *                                      e = {1, dt a_i1, ...})
 *     q^  = q^E + sum_j c[j] Q_j      (c_j = (a~_ij - a_ij) / a~_ii)
 *     q_tt = (I - lambda L_z)^{-1} q^  (rigid-lid projection of q^ first)
 *     Q_i  = q_tt - sum_j c[j] Q_j
 * h_dE / h_dQprev are HOST arrays of n_e / n_prev DEVICE pointers to state
 * vectors [v][k][c]; h_e / h_c are host coefficient arrays.  n_e in [1, 16],
 * n_prev in [0, 16]; n_prev = 0 with n_e = 1, e = {1} solves A x = b directly.
 * d_Qi must not alias any input.  `refine` (NULL = {4, 1e-13, 0}) is described
 * at hevi_refine; max_sweeps is ignored for FP64 factors.
 * If h_info != NULL the call waits for the stream and fills it. */
hevi_status hevi_stage_solve(hevi_ctx *ctx, const hevi_factors *f, int32_t n_e,
                             const double *const *h_dE, const double *h_e, int32_t n_prev,
                             const double *const *h_dQprev, const double *h_c, double *d_Qi,
                             const hevi_refine *refine, hevi_info *h_info, hipStream_t stream);

/* ---- allocation-free stage solve -------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  One call factors
 * A = I - lambda L_z of `ops` (as hevi_factor with precision `prec`) and runs
 * one stage solve with those factors (arguments and results as in
 * hevi_stage_solve; zero pivots are reported through h_info as well).  It calls
 * no hipMalloc, hipFree or other allocating routine: the factors, the stage
 * solve's scratch and the kernel report live in a fixed device array of
 * HEVI_NOALLOC_SCRATCH_BYTES per GPU, set up by hevi_create and held until the
 * process ends.  A shape that needs more (about 15.5 KB per column at order 4
 * with 41 nodes in FP64, so up to ~8,600 such columns) returns HEVI_E_SCRATCH
 * before any work is enqueued.  Every call on one GPU uses that GPU's one
 * array: calls that overlap in time on one GPU (several streams, several host
 * threads, several contexts) race and must be serialised by the caller.  The
 * results equal those of hevi_factor + hevi_stage_solve bit for bit. */
#define HEVI_NOALLOC_SCRATCH_BYTES (128u << 20)
hevi_status hevi_solve_noalloc(hevi_ctx *ctx, const hevi_ops *ops, double lambda,
                               hevi_precision prec, int32_t n_e, const double *const *h_dE,
                               const double *h_e, int32_t n_prev,
                               const double *const *h_dQprev, const double *h_c, double *d_Qi,
                               const hevi_refine *refine, hevi_info *h_info,
                               hipStream_t stream);

/* ---- linear combination (end of step, a6) ---------------------------------
 * out = sum_t coef[t] V_t over n_v state vectors (n_v in [1, 16]), e.g. the
 * update q^{n+1} = q^n + dt sum_i b_i S(Q_i) (Sec. 4.1, with b = b~). */
hevi_status hevi_combine(hevi_ctx *ctx, const hevi_ops *ops, int32_t n_v,
                         const double *const *h_dV, const double *h_coef, double *d_out,
                         hipStream_t stream);

/* ---- tableaux ---------------------------------------------------------------
 * IMEX ARK tableaux of the paper's integrators (Sec. 6): "ARK2" / "ARK2b" =
 * ARK(2,3,2) with a_32 = 1/2, "ARK2a" with a_32 = (3 + 2 sqrt 2)/6 (Sec. 4.1),
 * "ARK3" = ARK3(2)4L[2]SA and "ARK4" = ARK4(3)6L[2]SA of Kennedy and Carpenter,
 * "ARS343" = ARS(3,4,3) of Ascher, Ruuth and Spiteri (further integrators of
 * Sec. 6).  Writes s and the
 * row-major s x s explicit / implicit matrices and weights (capacity 8 stages).
 * Returns HEVI_E_INVALID for an unknown name. */
hevi_status hevi_tableau(const char *name, int32_t *s, double *a_exp, double *a_imp,
                         double *b);

/* ---- introspection ---------------------------------------------------------- */
/* Bytes per column of: the compact operator; the factors (FP64 or FP32 U and L
 * entries plus three byte planes: pivot offsets, U row extents, row-scale
 * exponents); the paper's LAPACK band layout (ldab = 3 * 5 (N+1) - 2 rows of
 * 8-byte entries per unknown plus a 4-byte pivot, Sec. 4.2.3); and everything a
 * factor object holds resident (factors, the stage solve's FP64 scratch of 6 values
 * per node and, for FP32 factors of order N > 6, an FP64 assembly buffer; not the
 * full-sweep scratch allocated on demand): the figure the server
 * charges against its HBM budget, per column of the 64-column tiles it
 * allocates.  Any output pointer may be NULL. */
hevi_status hevi_sizes(const hevi_shape *shape, hevi_precision prec, size_t *ops_bytes_per_col,
                       size_t *factor_bytes_per_col, size_t *paper_band_bytes_per_col,
                       size_t *resident_bytes_per_col);

/* ---- groups: one ARK step for many column batches ---------------------------
 * A group advances n member problems -- column batches with their own
 * operator, of any order N, element count and column count -- by one LHEVI ARK
 * step each, with one tableau and dt for all (Sec. 4.1; Sec. 4.3 eqs.
 * lhevi-ark-final-2/3):
 *     refactor A = I - a~_ii dt L_z                        (if requested)
 *     S_1 = L_z (q^n - q_ref)
 *     for i = 2..s:  Q_i = stage solve of hevi_stage_solve with
 *                        E = {q^n, S_1..S_{i-1}}, e = {1, dt a_i1, ..},
 *                        Qprev = {Q_1 = q^n, Q_2..Q_{i-1}}, c_j = (a~_ij - a_ij)/a~_ii
 *                    S_i = L_z (Q_i - q_ref)
 *     q^{n+1} = q^n + dt sum_i b_i S_i
 * Each phase of the step is one persistent launch over the 64-column tiles of
 * all members (HEVI_LAUNCH_ONE), one per distinct order (HEVI_LAUNCH_PER_ORDER)
 * or one plain launch per member (HEVI_LAUNCH_PER_MEMBER); the tiles are handed
 * out most expensive first.  The refactor runs one launch per distinct order in
 * both multi-problem plans.  Results do not depend on the plan.
 * Buffers: per member, caller-owned device state vectors [v][k][c] of the
 * member's shape.  d_Q[1..s-1] receive Q_2..Q_s (d_Q[0] is ignored: Q_1 = q^n),
 * d_S[0..s-1] receive S_1..S_s, d_out receives q^{n+1}; none may alias another
 * or q^n / q_ref.  The buffers are bound at creation and must stay valid until
 * hevi_group_free.  Factors (FP64 or FP32 by `prec`) and scratch are owned by
 * the group.  Steps of one group must not overlap in time (one stream, or
 * synchronised streams): the launches share the group's work counters. */
#define HEVI_MAX_STAGES 8
typedef struct hevi_group hevi_group;

typedef struct {
  const hevi_ops *ops;
  const double *d_qn;
  const double *d_qref;
  double *d_out;
  double *d_Q[HEVI_MAX_STAGES];
  double *d_S[HEVI_MAX_STAGES];
} hevi_group_member;

typedef enum {
  HEVI_LAUNCH_ONE = 0,        /* one launch per phase over every member             */
  HEVI_LAUNCH_PER_ORDER = 1,  /* one launch per phase and distinct order N          */
  HEVI_LAUNCH_PER_MEMBER = 2  /* one single-problem launch per phase and member     */
} hevi_launch_mode;

typedef struct {
  int32_t mode;       /* hevi_launch_mode                                          */
  int32_t grid;       /* workgroups (one wavefront each) per persistent launch;
                         0 = one per tile.  Ignored for HEVI_LAUNCH_PER_MEMBER.     */
  int32_t use_graph;  /* replay the step from a captured HIP graph                 */
} hevi_group_plan;

typedef struct {
  hevi_group_plan plan;
  double ms_per_step; /* mean over the timed steps                                */
} hevi_tune_result;

/* Create a group of n >= 1 members (tableau as hevi_tableau; dt > 0) and factor
 * every member once (enqueued on `stream`).  refine: NULL = {4, 1e-13, 0};
 * full_sweeps must be 0.  The initial plan is {HEVI_LAUNCH_ONE, 0, 0}. */
hevi_status hevi_group_create(hevi_ctx *ctx, int32_t n, const hevi_group_member *members,
                              const char *tableau, double dt, hevi_precision prec,
                              const hevi_refine *refine, hevi_group **out, hipStream_t stream);
hevi_status hevi_group_set_plan(hevi_ctx *ctx, hevi_group *g, const hevi_group_plan *plan);
hevi_status hevi_group_get_plan(const hevi_group *g, hevi_group_plan *plan);
/* One ARK step of every member, enqueued on `stream` (refactor != 0: factor
 * A = I - a~_ii dt L_z first).  With use_graph the first call of each refactor
 * flag captures the step into a HIP graph; later calls launch the graph. */
hevi_status hevi_group_step(hevi_ctx *ctx, hevi_group *g, int32_t refactor, hipStream_t stream);
/* Wait for `stream` and report, per member, the worst kernel-detected problem
 * of every step since the previous check (h_infos: n entries); then reset. */
hevi_status hevi_group_check(hevi_ctx *ctx, hevi_group *g, hevi_info *h_infos,
                             hipStream_t stream);
/* Autotuner: time `reps` steps (after one untimed step) of each candidate plan
 * -- launch modes x persistent grid sizes x graph on/off -- keep the fastest
 * as the group's plan and write up to `cap` results (n_results = candidates
 * timed).  It runs real steps: the members' d_out, d_Q and d_S are
 * overwritten (q^n is not), and the factors are refreshed. */
hevi_status hevi_group_autotune(hevi_ctx *ctx, hevi_group *g, int32_t reps,
                                hevi_tune_result *results, int32_t cap, int32_t *n_results,
                                hipStream_t stream);
void hevi_group_free(hevi_group *g);

/* ---- serving: continuous batching of stage solves over resident factors -----
 * A server keeps the factors of registered simulations resident in HBM and
 * runs stage-solve requests (each exactly hevi_stage_solve of one simulation,
 * Sec. 4.3 eq. lhevi-ark-final-3) from any host thread.  A worker thread
 * gathers the queued requests into batches -- at most one request per
 * simulation per batch, first come first served -- and runs each batch as
 * one persistent launch per kernel phase over the tiles of all its requests
 * (FP64 simulations of at most 106 nodes per column, which take the fused stage
 * kernel, other FP64 simulations and FP32-factor simulations in separate
 * launches), on the server's own stream, with up to 3 batches in flight.  Requests of one simulation run in
 * submission order.
 *
 * hevi_serve_create: hbm_budget_bytes bounds the library-owned memory of all
 *   registered simulations (factors and scratch); max_inflight bounds the
 *   requests submitted and not yet completed; `refine` (NULL = {4, 1e-13, 0};
 *   full_sweeps must be 0) is the refinement of every FP32-factor simulation.
 * hevi_serve_register: factor A = I - lambda L_z of `ops` (enqueued on the
 *   server's stream) and return a simulation id.  HEVI_E_NOMEM: not admitted
 *   now (the budget is used up; release a simulation and retry).  `ops` must
 *   stay valid until hevi_serve_release.
 * hevi_serve_submit: queue one stage solve of simulation sim_id (arguments as
 *   in hevi_stage_solve).  The device buffers must stay valid and unchanged
 *   until the ticket completes; the stage-solve operands are read when the
 *   batch runs.  HEVI_E_BUSY: max_inflight requests are pending (retry later);
 *   HEVI_E_CLOSED: unknown or released simulation, or server shut down.
 * hevi_serve_poll / hevi_serve_wait: report a ticket's completion (poll: *done
 *   = 0 or 1; wait: blocks).  On completion the ticket's kernel report and the
 *   latency in seconds from submit to observed completion (latency_s may be
 *   NULL) are written, and the ticket is retired: a second poll or wait of it
 *   returns HEVI_E_CLOSED, as does an unknown ticket.
 * hevi_serve_release: wait for the simulation's requests, then free its
 *   factors and return its budget.  hevi_serve_destroy: finish every queued
 *   request, stop the worker and free everything.
 * All server calls are thread-safe.  If the device fails, pending and later
 * tickets complete with status HEVI_E_DEVICE. */
hevi_status hevi_serve_create(hevi_ctx *ctx, size_t hbm_budget_bytes, int32_t max_inflight,
                              const hevi_refine *refine, hevi_server **out);
hevi_status hevi_serve_register(hevi_server *srv, const hevi_ops *ops, double lambda,
                                hevi_precision prec, int32_t *sim_id);
hevi_status hevi_serve_submit(hevi_server *srv, int32_t sim_id, int32_t n_e,
                              const double *const *h_dE, const double *h_e, int32_t n_prev,
                              const double *const *h_dQprev, const double *h_c, double *d_Qi,
                              uint64_t *ticket);
hevi_status hevi_serve_poll(hevi_server *srv, uint64_t ticket, int32_t *done, hevi_info *info,
                            double *latency_s);
hevi_status hevi_serve_wait(hevi_server *srv, uint64_t ticket, hevi_info *info,
                            double *latency_s);
hevi_status hevi_serve_release(hevi_server *srv, int32_t sim_id);
void hevi_serve_destroy(hevi_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* HEVI_H */
